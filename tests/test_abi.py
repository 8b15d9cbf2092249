"""CPU-side checks of the C-ABI library: it loads, exports every entry point
declared in include/cisigma.h, and its host-only calls behave."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cisigma.h")
LIB = os.path.join(ROOT, "paper_1707_04346_amd", "libcisigma.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cisigma_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["cisigma_init", "cisigma_apply", "cisigma_davidson", "cisigma_free", "cisigma_ndet"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (cisigma_\w+)", out))
    assert exported == set(_declared())


def test_binding_names_match_header():
    import paper_1707_04346_amd as cis
    assert sorted(cis.EXPORTS) == _declared()


def test_strerror_and_null_handling():
    import paper_1707_04346_amd as cis
    assert cis.strerror(0) == "ok"
    assert "invalid" in cis.strerror(-1)
    assert "converge" in cis.strerror(-4)
    lib = cis._lib
    assert lib.cisigma_ndet(None) == -1
    assert lib.cisigma_apply(None, None, None, 0, None) == cis.EINVAL
    assert lib.cisigma_davidson(None, 1, 1e-8, None, None, None) == cis.EINVAL
    assert lib.cisigma_hmat_block(None, 0, None, 0, None, None) == cis.EINVAL
    assert lib.cisigma_autotune(None, cis.FP32, 1, None, 0) == cis.EINVAL
    assert b"NULL" in lib.cisigma_last_error(None)
    h = ctypes.c_void_p()
    # bad sizes are rejected before any device work
    assert lib.cisigma_init(ctypes.byref(h), 0, 1, 1, None, None, None) == cis.EINVAL
    assert lib.cisigma_init(ctypes.byref(h), 33, 1, 1, None, None, None) == cis.EINVAL
    assert lib.cisigma_init(None, 4, 1, 1, None, None, None) == cis.EINVAL


def test_device_code_has_no_packed_fp32():
    """The library is built without packed-FP32 instructions (v_pk_{add,mul,fma}_f32);
    the sigma kernels do use the matrix cores."""
    llvm = "/opt/rocm/llvm/bin"
    if not os.path.exists(os.path.join(llvm, "llvm-objdump")):
        pytest.skip("llvm tools not available")
    d = os.path.join(ROOT, "paper_1707_04346_amd", "_build")
    mfma = 0
    for f in sorted(os.listdir(d)):
        if not f.endswith(".o"):
            continue
        fb, dev = f"/tmp/_cis_{os.getpid()}_{f}.fatbin", f"/tmp/_cis_{os.getpid()}_{f}.co"
        r = subprocess.run([os.path.join(llvm, "llvm-objcopy"), f"--dump-section=.hip_fatbin={fb}",
                            os.path.join(d, f), f"/tmp/_cis_{os.getpid()}_junk.o"], capture_output=True, text=True)
        if r.returncode != 0:
            assert "not found" in r.stderr, r.stderr   # host-only object
            continue
        subprocess.check_call([os.path.join(llvm, "clang-offload-bundler"), "--unbundle", "--type=o",
                               f"--input={fb}", f"--output={dev}", "--targets=hipv4-amdgcn-amd-amdhsa--gfx950"])
        asm = subprocess.run([os.path.join(llvm, "llvm-objdump"), "-d", dev], capture_output=True, text=True).stdout
        for x in (fb, dev, f"/tmp/_cis_{os.getpid()}_junk.o"):
            if os.path.exists(x):
                os.remove(x)
        assert "gfx950" in asm or "amdgcn" in asm or asm
        for bad in ("v_pk_add_f32", "v_pk_mul_f32", "v_pk_fma_f32"):
            assert bad not in asm, (f, bad)
        mfma += asm.count("v_mfma_")
    assert mfma > 0


def _init(norb, na, nb, h, g, gas=None):
    import numpy as np
    import paper_1707_04346_amd as cis
    hh = np.ascontiguousarray(h, dtype=np.float64)
    gg = np.ascontiguousarray(g, dtype=np.float64)
    handle = ctypes.c_void_p()
    gp = None
    keep = []
    if gas is not None:
        arrs = [np.ascontiguousarray(a, dtype=np.int32) for a in gas]
        keep += arrs
        gs = cis._Gas(len(arrs[0]), arrs[0].ctypes.data, arrs[1].ctypes.data, arrs[2].ctypes.data)
        keep.append(gs)
        gp = ctypes.addressof(gs)
    st = cis._lib.cisigma_init(ctypes.byref(handle), norb, na, nb, gp, hh.ctypes.data, gg.ctypes.data)
    if handle.value:
        cis._lib.cisigma_free(handle)
    return st


def test_init_rejects_bad_integrals_before_device_work():
    """NaN, asymmetric h1e, integrals without 8-fold symmetry and inconsistent
    GAS definitions are EINVAL (checked on the host, no GPU needed)."""
    import numpy as np
    import paper_1707_04346_amd as cis
    import synth_inputs as si
    h, g = si.integrals(4, 8, 0)
    bad = h.copy(); bad[0, 1] += 1e-3
    assert _init(4, 2, 2, bad, g) == cis.EINVAL
    bad = h.copy(); bad[2, 2] = np.nan
    assert _init(4, 2, 2, bad, g) == cis.EINVAL
    gb = g.copy(); gb[0, 1, 2, 3] += 1e-3
    assert _init(4, 2, 2, h, gb) == cis.EINVAL
    gb = g.copy(); gb[1, 1, 1, 1] = np.inf
    assert _init(4, 2, 2, h, gb) == cis.EINVAL
    # GAS orbital counts must sum to norb; the space must not be empty
    assert _init(4, 2, 2, h, g, gas=([2, 1], [0, 4], [4, 4])) == cis.EINVAL
    assert _init(4, 2, 2, h, g, gas=([2, 2], [5, 5], [5, 5])) == cis.EINVAL
