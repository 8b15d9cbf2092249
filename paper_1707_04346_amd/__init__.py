"""Python binding of libcisigma (the C ABI in include/cisigma.h).

Argument marshalling only: every step of sigma = H C and of the Davidson
solver runs in the library's HIP kernels.  PyTorch supplies device memory
(tensor data pointers) and streams.  Importing this module loads the built
library and raises if it is missing -- there is no fallback path.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcisigma.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOCONV, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
FP64, FP32 = 0, 1
OPT_PRECISION, OPT_MAX_SPACE, OPT_MAX_ITER, OPT_REFINE_EVERY, OPT_RESID_TOL, OPT_VERBOSE, OPT_PROFILE = 1, 2, 3, 4, 5, 6, 7
PASSES = ["layout_in", "clear", "sigma_aa", "sigma_ab", "sigma_bb", "layout_out"]
OPT_SIGMA_PATH = 8
OPT_SS_CHUNK = 9
OPT_SPIN_PARITY = 10
OPT_GRAPH = 11
OPT_OVERLAP = 12
OPT_THICK_RESTART = 13
OPT_PSPACE = 14
OPT_LOW_MEMORY = 15
OPT_GAS_UNIT_ORDER = 16
OPT_SS_SPLIT = 17
OPT_UNIT_COLS = 18
OPT_DETERMINISTIC = 20
OPT_UNIT_LAUNCH = 19

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libcisigma.so is not built ({LIB_PATH}); run __graft_entry__.build()")

# PyTorch ships its own HIP runtime; when torch is present it must be loaded
# before this library so that the process holds a single HIP runtime.
try:
    import torch  # noqa: F401
except ImportError:
    pass


class _Gas(ctypes.Structure):
    _fields_ = [("ngas", ctypes.c_int), ("norb", ctypes.c_void_p), ("min_cum", ctypes.c_void_p),
                ("max_cum", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("sigma_fp32", ctypes.c_int), ("sigma_fp64", ctypes.c_int),
                ("refinements", ctypes.c_int), ("residual", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = ctypes.CDLL(LIB_PATH)
_vp, _i32, _i64, _u32, _f64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint32, ctypes.c_double
_lib.cisigma_init.restype = _i32
_lib.cisigma_init.argtypes = [ctypes.POINTER(_vp), _i32, _i32, _i32, _vp, _vp, _vp]
_lib.cisigma_init_sym.restype = _i32
_lib.cisigma_init_sym.argtypes = [ctypes.POINTER(_vp), _i32, _i32, _i32, _vp, _vp, _i32, _vp, _vp]
_lib.cisigma_free.restype = None
_lib.cisigma_free.argtypes = [_vp]
_lib.cisigma_ndet.restype = _i64
_lib.cisigma_ndet.argtypes = [_vp]
_lib.cisigma_layout.restype = _i32
_lib.cisigma_layout.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.cisigma_address.restype = _i32
_lib.cisigma_address.argtypes = [_vp, _u32, _u32, ctypes.POINTER(_i64)]
_lib.cisigma_strings.restype = _i32
_lib.cisigma_strings.argtypes = [_vp, _i32, _vp, ctypes.POINTER(_i32)]
_lib.cisigma_excitations.restype = _i32
_lib.cisigma_excitations.argtypes = [_vp, _i32, _vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]
_lib.cisigma_set_option.restype = _i32
_lib.cisigma_set_option.argtypes = [_vp, _i32, _f64]
_lib.cisigma_apply.restype = _i32
_lib.cisigma_apply.argtypes = [_vp, _vp, _vp, _i32, _vp]
_lib.cisigma_hdiag.restype = _i32
_lib.cisigma_hdiag.argtypes = [_vp, _vp, _vp]
_lib.cisigma_autotune.restype = _i32
_lib.cisigma_autotune.argtypes = [_vp, _i32, _i32, ctypes.c_char_p, _i32]
_lib.cisigma_hmat_block.restype = _i32
_lib.cisigma_hmat_block.argtypes = [_vp, _i32, _vp, _i32, _vp, _vp]
_lib.cisigma_davidson.restype = _i32
_lib.cisigma_davidson.argtypes = [_vp, _i32, _f64, _vp, _vp, ctypes.POINTER(Stats)]
_lib.cisigma_rdm.restype = _i32
_lib.cisigma_rdm.argtypes = [_vp, _vp, _i32, _vp, _vp, _vp]
_lib.cisigma_last_path.restype = _i32
_lib.cisigma_last_path.argtypes = [_vp, _i32, ctypes.POINTER(_i32)]
_lib.cisigma_set_log.restype = _i32
_lib.cisigma_set_log.argtypes = [_vp, ctypes.c_char_p]
_lib.cisigma_apply_noalloc.restype = _i32
_lib.cisigma_apply_noalloc.argtypes = [_vp, _vp, _vp, _i32, _vp]
_lib.cisigma_last_shape.restype = _i32
_lib.cisigma_last_shape.argtypes = [_vp, _i32, _vp]
_lib.cisigma_pass_times.restype = _i32
_lib.cisigma_pass_times.argtypes = [_vp, _vp, ctypes.POINTER(_i32)]
_lib.cisigma_last_error.restype = ctypes.c_char_p
_lib.cisigma_last_error.argtypes = [_vp]
_lib.cisigma_strerror.restype = ctypes.c_char_p
_lib.cisigma_strerror.argtypes = [_i32]

EXPORTS = ["cisigma_init", "cisigma_free", "cisigma_ndet", "cisigma_layout", "cisigma_address", "cisigma_strings",
           "cisigma_excitations", "cisigma_set_option", "cisigma_apply", "cisigma_hdiag", "cisigma_davidson",
           "cisigma_pass_times", "cisigma_last_path", "cisigma_last_error", "cisigma_strerror", "cisigma_rdm",
           "cisigma_hmat_block", "cisigma_autotune", "cisigma_last_shape",
           "cisigma_apply_noalloc", "cisigma_set_log", "cisigma_init_sym"]
PATH_AB_OWNER, PATH_SS_MATERIALISED, PATH_AB_SHARED_CU = 1, 2, 4


class CisigmaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"cisigma status {status} ({_lib.cisigma_strerror(status).decode()}): {msg}")
        self.status = status


def strerror(status):
    return _lib.cisigma_strerror(int(status)).decode()


def _ptr(x):
    """Raw pointer of a torch tensor or numpy array (or an int / None)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    return x.ctypes.data


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Context:
    """cisigma_init (cisigma_init_sym with orbsym) / cisigma_free around one
    (norb, nalpha, nbeta[, gas][, orbsym, target]) problem."""

    def __init__(self, norb, nalpha, nbeta, h1e, eri, gas=None, orbsym=None, target=0):
        h1e = np.ascontiguousarray(h1e, dtype=np.float64)
        eri = np.ascontiguousarray(eri, dtype=np.float64)
        self._keep = []
        gp = None
        if gas is not None:
            gn, gmin, gmax = (np.ascontiguousarray(a, dtype=np.int32) for a in gas)
            self._keep += [gn, gmin, gmax]
            g = _Gas(len(gn), gn.ctypes.data, gmin.ctypes.data, gmax.ctypes.data)
            self._keep.append(g)
            gp = ctypes.addressof(g)
        h = _vp()
        if orbsym is None:
            st = _lib.cisigma_init(ctypes.byref(h), int(norb), int(nalpha), int(nbeta), gp, h1e.ctypes.data,
                                   eri.ctypes.data)
        else:
            osym = np.ascontiguousarray(orbsym, dtype=np.int32)
            if osym.size != int(norb):
                raise CisigmaError(EINVAL, "orbsym needs one irrep per orbital")
            self._keep.append(osym)
            st = _lib.cisigma_init_sym(ctypes.byref(h), int(norb), int(nalpha), int(nbeta), gp, osym.ctypes.data,
                                       int(target), h1e.ctypes.data, eri.ctypes.data)
        if st != OK:
            raise CisigmaError(st, "cisigma_init failed")
        self._h = h
        self.norb, self.nalpha, self.nbeta = int(norb), int(nalpha), int(nbeta)
        self.ndet = int(_lib.cisigma_ndet(self._h))

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.cisigma_free(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, st):
        if st != OK:
            raise CisigmaError(st, _lib.cisigma_last_error(self._h).decode())
        return st

    @property
    def handle(self):
        return self._h.value

    def layout(self):
        nb = _i32()
        self._check(_lib.cisigma_layout(self._h, ctypes.byref(nb), None, None, None, None, None))
        n = nb.value
        off = np.zeros(n + 1, np.int64)
        ta, tb, na, nbs = (np.zeros(max(n, 1), np.int32) for _ in range(4))
        self._check(_lib.cisigma_layout(self._h, ctypes.byref(nb), off.ctypes.data, ta.ctypes.data, tb.ctypes.data,
                                        na.ctypes.data, nbs.ctypes.data))
        return dict(offset=off, alpha_type=ta[:n], beta_type=tb[:n], nalpha_str=na[:n], nbeta_str=nbs[:n])

    def address(self, abits, bbits):
        idx = _i64()
        self._check(_lib.cisigma_address(self._h, int(abits), int(bbits), ctypes.byref(idx)))
        return idx.value

    def strings(self, spin):
        n = _i32()
        self._check(_lib.cisigma_strings(self._h, int(spin), None, ctypes.byref(n)))
        out = np.zeros(max(n.value, 1), np.uint32)
        self._check(_lib.cisigma_strings(self._h, int(spin), out.ctypes.data, ctypes.byref(n)))
        return out[:n.value]

    def excitations(self, spin):
        per, n = _i32(), _i32()
        self._check(_lib.cisigma_excitations(self._h, int(spin), None, ctypes.byref(per), ctypes.byref(n)))
        out = np.zeros(max(per.value * n.value, 1), np.uint32)
        self._check(_lib.cisigma_excitations(self._h, int(spin), out.ctypes.data, ctypes.byref(per),
                                             ctypes.byref(n)))
        return out[:per.value * n.value].reshape(n.value, per.value)

    def set_option(self, key, value):
        self._check(_lib.cisigma_set_option(self._h, int(key), float(value)))

    def apply(self, C, sigma, stream=None):
        """sigma = H C on device tensors (float32 or float64), asynchronous on stream."""
        dt = FP32 if str(C.dtype).endswith("float32") else FP64
        if str(sigma.dtype) != str(C.dtype) or C.numel() != self.ndet or sigma.numel() != self.ndet:
            raise CisigmaError(EINVAL, "C and sigma must be device tensors of ndet elements of one dtype")
        if not (C.is_contiguous() and sigma.is_contiguous()):
            raise CisigmaError(EINVAL, "C and sigma must be contiguous")
        self._check(_lib.cisigma_apply(self._h, _ptr(C), _ptr(sigma), dt, _stream_ptr(stream)))
        return sigma

    def apply_noalloc(self, C, sigma, stream=None):
        """sigma = H C through cisigma_apply_noalloc (workspace in the library's
        static device scratch; no allocation)."""
        dt = FP32 if str(C.dtype).endswith("float32") else FP64
        if str(sigma.dtype) != str(C.dtype) or C.numel() != self.ndet or sigma.numel() != self.ndet:
            raise CisigmaError(EINVAL, "C and sigma must be device tensors of ndet elements of one dtype")
        if not (C.is_contiguous() and sigma.is_contiguous()):
            raise CisigmaError(EINVAL, "C and sigma must be contiguous")
        self._check(_lib.cisigma_apply_noalloc(self._h, _ptr(C), _ptr(sigma), dt, _stream_ptr(stream)))
        return sigma

    def apply_raw(self, c_ptr, s_ptr, dtype, stream_ptr=None):
        return _lib.cisigma_apply(self._h, c_ptr, s_ptr, int(dtype), stream_ptr)

    def hdiag(self, out, stream=None):
        self._check(_lib.cisigma_hdiag(self._h, _ptr(out), _stream_ptr(stream)))
        return out

    def autotune(self, dtype=FP32, reps=3):
        """Time the apply launch parameters of this space for dtype and keep the
        fastest; returns the library's report (one line per timing and choice)."""
        buf = ctypes.create_string_buffer(8192)
        self._check(_lib.cisigma_autotune(self._h, int(dtype), int(reps), buf, len(buf)))
        return buf.value.decode()

    def hmat_block(self, rows, cols):
        """H(rows[i], cols[j]) (numpy, n x m) between determinants given by vector index."""
        r = np.ascontiguousarray(rows, dtype=np.int64)
        c = np.ascontiguousarray(cols, dtype=np.int64)
        out = np.zeros((r.size, c.size), np.float64)
        self._check(_lib.cisigma_hmat_block(self._h, int(r.size), r.ctypes.data, int(c.size), c.ctypes.data,
                                            out.ctypes.data))
        return out

    def davidson(self, nroots=1, tol=1e-10, vecs=None, allow_noconv=False):
        """Lowest nroots energies (numpy), Stats, status."""
        e = np.zeros(int(nroots), np.float64)
        st = Stats()
        status = _lib.cisigma_davidson(self._h, int(nroots), float(tol), e.ctypes.data, _ptr(vecs), ctypes.byref(st))
        if status != OK and not (allow_noconv and status == ENOCONV):
            self._check(status)
        return e, st.as_dict(), status

    def rdm(self, C, rdm1, rdm2, stream=None):
        """Spin-summed density matrices of C into device FP64 tensors rdm1 (n*n) and
        rdm2 (n**4), asynchronous on stream."""
        dt = FP32 if str(C.dtype).endswith("float32") else FP64
        n = self.norb
        if C.numel() != self.ndet or not C.is_contiguous():
            raise CisigmaError(EINVAL, "C must be a contiguous device tensor of ndet elements")
        if rdm1.numel() != n * n or rdm2.numel() != n ** 4 or not str(rdm1.dtype).endswith("float64") \
                or not str(rdm2.dtype).endswith("float64") or not (rdm1.is_contiguous() and rdm2.is_contiguous()):
            raise CisigmaError(EINVAL, "rdm1 and rdm2 must be contiguous float64 device tensors of n^2 and n^4 elements")
        self._check(_lib.cisigma_rdm(self._h, _ptr(C), dt, _ptr(rdm1), _ptr(rdm2), _stream_ptr(stream)))
        return rdm1, rdm2

    def pass_times(self):
        """Summed milliseconds per apply pass since profiling was enabled, and the call count."""
        ms = np.zeros(len(PASSES), np.float64)
        n = _i32()
        self._check(_lib.cisigma_pass_times(self._h, ms.ctypes.data, ctypes.byref(n)))
        return dict(zip(PASSES, ms.tolist())), n.value

    def last_path(self, dtype=FP32):
        """CISIGMA_PATH_* flags of the most recent apply of dtype."""
        f = _i32()
        self._check(_lib.cisigma_last_path(self._h, int(dtype), ctypes.byref(f)))
        return f.value

    def last_shape(self, dtype=FP32):
        """(k steps, pair row blocks, plan entries per lane, variant) of the
        owner-computes sigma_3 kernel of the most recent apply of dtype;
        variant 0: general kernel, 1: own row in a k step, 2: rank-1 own row,
        3: GAS units."""
        sh = np.zeros(4, np.int32)
        self._check(_lib.cisigma_last_shape(self._h, int(dtype), sh.ctypes.data))
        return tuple(int(x) for x in sh)

    def set_log(self, path):
        """Davidson JSON-lines log file (None: off)."""
        self._check(_lib.cisigma_set_log(self._h, None if path is None else str(path).encode()))

    def last_error(self):
        return _lib.cisigma_last_error(self._h).decode()
