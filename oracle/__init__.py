"""CPU oracle for the determinant-basis sigma = H C and the Davidson CI solver.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library never loads it and shares no code with it.

* ``Space`` wraps ``oracle.c`` (plain Slater-Condon sigma of Eqs. 4-7 of
  Vogiatzis et al., arXiv:1707.04346, Sec. 2.1; FP64; OpenMP over output
  determinants).
* ``davidson`` is a plain Davidson-Liu eigensolver written from Sec. 3.3
  (steps 1-4: initial subspace and sigma, diagonal preconditioner,
  preconditioned correction orthogonalised against all previous vectors, new
  sigma and re-diagonalisation of the projected matrix), with numpy's ``eigh``
  for the small projected problem.

* ``Space.rdm``: one- and two-particle density matrices by applying every
  creation/annihilation operator to every determinant (the plain definition).
* ``parity_basis`` / ``parity_spectrum``: the M_S = 0 sectors of Sec. 3.1 and
  Sec. 3.3 (vectors symmetric or antisymmetric under alpha <-> beta string
  exchange) and the dense spectrum of H inside them.

Parity status: pinned (see ``tests/test_oracle.py``) against a brute-force
second-quantised construction of Eq. 6, the two-site Hubbard closed form, the
non-interacting closed form, spin and transposition symmetry, GAS = projected
CAS, and dense ``eigh``; the sectors against the full spectrum, total spin
(even S in the symmetric sector, odd S in the antisymmetric one) and the
Hubbard closed form; the density matrices against the energy from sigma, traces,
index symmetries and the single-determinant closed form.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(verbose=False):
    """Compile oracle.c into liboracle.so (gcc, -O2, OpenMP)."""
    import subprocess
    src = os.path.join(_HERE, "oracle.c")
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall",
           "-o", _LIB_PATH + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i64, i32, u32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_uint32
    lib.or_create.restype = vp
    lib.or_create.argtypes = [i32, i32, i32, i32, vp, vp, vp, vp, vp]
    lib.or_create_sym.restype = vp
    lib.or_create_sym.argtypes = [i32, i32, i32, i32, vp, vp, vp, vp, i32, vp, vp]
    lib.or_free.argtypes = [vp]
    lib.or_ndet.restype = i64
    lib.or_ndet.argtypes = [vp]
    lib.or_nstr.restype = i32
    lib.or_nstr.argtypes = [vp, i32]
    lib.or_ntype.restype = i32
    lib.or_ntype.argtypes = [vp, i32]
    lib.or_nblocks.restype = i32
    lib.or_nblocks.argtypes = [vp]
    lib.or_blocks.argtypes = [vp, vp, vp, vp]
    lib.or_strings.argtypes = [vp, i32, vp, vp]
    lib.or_address.restype = i64
    lib.or_address.argtypes = [vp, u32, u32]
    lib.or_det.argtypes = [vp, i64, vp, vp]
    lib.or_h_elem.restype = ctypes.c_double
    lib.or_h_elem.argtypes = [vp, i64, i64]
    lib.or_sigma.argtypes = [vp, vp, vp]
    lib.or_sigma_rows.argtypes = [vp, i64, vp, vp, vp]
    lib.or_hdiag.argtypes = [vp, vp]
    lib.or_hmat.restype = i32
    lib.or_hmat.argtypes = [vp, vp]
    lib.or_set_threads.argtypes = [i32]
    lib.or_rdm.restype = i32
    lib.or_rdm.argtypes = [vp, vp, vp, vp]
    lib.or_max_threads.restype = i32
    _lib = lib
    return lib


def set_threads(n):
    _load().or_set_threads(int(n))


def max_threads():
    return int(_load().or_max_threads())


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class Space:
    """Determinant space of (norb, nalpha, nbeta[, GAS]) with its integrals.

    ``gas`` is None (CAS) or ``(norb_per_space, min_cum, max_cum)`` with
    cumulative bounds on the total (alpha+beta) electron count of spaces
    1..g (Sec. 3.1 occupation types).  ``orbsym`` (irrep 0..7 of each
    orbital, D2h products as XOR) with ``target`` keeps only determinants
    whose string irreps multiply to the target (the S of Sec. 3.1, Eq. 9).
    """

    def __init__(self, norb, nalpha, nbeta, h1e, eri, gas=None, orbsym=None, target=0):
        lib = _load()
        self.norb, self.nalpha, self.nbeta = int(norb), int(nalpha), int(nbeta)
        if gas is None:
            gas = ([norb], [nalpha + nbeta], [nalpha + nbeta])
        gn, gmin, gmax = (np.ascontiguousarray(x, dtype=np.int32) for x in gas)
        self.gas = (gn.copy(), gmin.copy(), gmax.copy())
        self.h1e = np.ascontiguousarray(h1e, dtype=np.float64).reshape(norb, norb)
        self.eri = np.ascontiguousarray(eri, dtype=np.float64).reshape(norb, norb, norb, norb)
        self.orbsym = None if orbsym is None else np.ascontiguousarray(orbsym, dtype=np.int32).copy()
        self.target = int(target)
        if self.orbsym is None:
            self._h = lib.or_create(self.norb, self.nalpha, self.nbeta, len(gn), _ptr(gn), _ptr(gmin),
                                    _ptr(gmax), _ptr(self.h1e), _ptr(self.eri))
        else:
            assert self.orbsym.size == self.norb
            self._h = lib.or_create_sym(self.norb, self.nalpha, self.nbeta, len(gn), _ptr(gn), _ptr(gmin),
                                        _ptr(gmax), _ptr(self.orbsym), self.target, _ptr(self.h1e),
                                        _ptr(self.eri))
        if not self._h:
            raise ValueError("oracle: invalid space definition")
        self.ndet = int(lib.or_ndet(self._h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.or_free(h)
            self._h = None

    # -- layout ------------------------------------------------------------
    def strings(self, spin):
        lib = _load()
        n = lib.or_nstr(self._h, spin)
        nt = lib.or_ntype(self._h, spin)
        out = np.zeros(max(n, 1), dtype=np.uint32)
        cnt = np.zeros(max(nt, 1), dtype=np.int32)
        lib.or_strings(self._h, spin, _ptr(out), _ptr(cnt))
        return out[:n], cnt[:nt]

    def blocks(self):
        lib = _load()
        nb = lib.or_nblocks(self._h)
        ta = np.zeros(max(nb, 1), dtype=np.int32)
        tb = np.zeros(max(nb, 1), dtype=np.int32)
        off = np.zeros(nb + 1, dtype=np.int64)
        lib.or_blocks(self._h, _ptr(ta), _ptr(tb), _ptr(off))
        return ta[:nb], tb[:nb], off

    def address(self, abits, bbits):
        return int(_load().or_address(self._h, int(abits), int(bbits)))

    def det(self, idx):
        a = ctypes.c_uint32()
        b = ctypes.c_uint32()
        _load().or_det(self._h, int(idx), ctypes.byref(a), ctypes.byref(b))
        return a.value, b.value

    def dets(self):
        """(alpha bits, beta bits) of every determinant, in vector order."""
        out = np.zeros((self.ndet, 2), dtype=np.uint64)
        for i in range(self.ndet):
            out[i] = self.det(i)
        return out

    # -- numerics ----------------------------------------------------------
    def h_elem(self, i, j):
        return float(_load().or_h_elem(self._h, int(i), int(j)))

    def sigma(self, C):
        C = np.ascontiguousarray(C, dtype=np.float64).reshape(-1)
        assert C.size == self.ndet
        out = np.empty(self.ndet, dtype=np.float64)
        _load().or_sigma(self._h, _ptr(C), _ptr(out))
        return out

    def sigma_rows(self, rows, C):
        rows = np.ascontiguousarray(rows, dtype=np.int64).reshape(-1)
        C = np.ascontiguousarray(C, dtype=np.float64).reshape(-1)
        assert C.size == self.ndet
        assert rows.size == 0 or (rows.min() >= 0 and rows.max() < self.ndet)
        out = np.empty(rows.size, dtype=np.float64)
        _load().or_sigma_rows(self._h, rows.size, _ptr(rows), _ptr(C), _ptr(out))
        return out

    def rdm(self, C):
        """Spin-summed one- and two-particle density matrices of C, normalised
        by <C|C>: gamma[p,q] = sum_s <a+_ps a_qs>, Gamma[p,q,r,s] =
        sum_(s,t) <a+_ps a+_rt a_st a_qs> (chemists' order: the energy is
        sum h gamma + 1/2 sum (pq|rs) Gamma).  Every operator is applied to
        every determinant of the space (plain definition; small spaces)."""
        C = np.ascontiguousarray(C, dtype=np.float64).reshape(-1)
        assert C.size == self.ndet
        n = self.norb
        g1 = np.empty((n, n), dtype=np.float64)
        g2 = np.empty((n, n, n, n), dtype=np.float64)
        rc = _load().or_rdm(self._h, _ptr(C), _ptr(g1), _ptr(g2))
        if rc != 0:
            raise ValueError("oracle: zero vector")
        return g1, g2

    def hdiag(self):
        out = np.empty(self.ndet, dtype=np.float64)
        _load().or_hdiag(self._h, _ptr(out))
        return out

    def hmat(self):
        if self.ndet > 20000:
            raise ValueError("dense H only for tiny spaces")
        out = np.empty((self.ndet, self.ndet), dtype=np.float64)
        rc = _load().or_hmat(self._h, _ptr(out))
        assert rc == 0
        return out


def parity_basis(nside, parity):
    """Orthonormal basis (rows) of the M_S = 0 sector of a one-block space of
    nside x nside determinants: vectors with C(Ib, Ia) = parity * C(Ia, Ib)
    (Sec. 3.1, Sec. 3.3: for M_S = 0 the work is done on combinations of a
    determinant and its alpha <-> beta exchanged partner).  The basis holds
    (|Ia Ib> + parity |Ib Ia>)/sqrt(2) for Ia < Ib and, for parity = +1, the
    diagonal determinants |Ia Ia>."""
    rows = []
    r2 = 1.0 / np.sqrt(2.0)
    for a in range(nside):
        for b in range(a, nside):
            if a == b and parity < 0:
                continue
            v = np.zeros(nside * nside)
            if a == b:
                v[a * nside + a] = 1.0
            else:
                v[a * nside + b] = r2
                v[b * nside + a] = parity * r2
            rows.append(v)
    return np.array(rows).reshape(len(rows), nside * nside)


def parity_spectrum(space, parity):
    """Eigenvalues (ascending) of H restricted to the M_S = 0 sector of
    ``parity_basis``: dense eigh of Q H Q^T (tiny spaces only)."""
    n = int(round(np.sqrt(space.ndet)))
    if n * n != space.ndet:
        raise ValueError("the sector needs a one-block space with n_alpha = n_beta")
    Q = parity_basis(n, parity)
    return np.linalg.eigvalsh(Q @ space.hmat() @ Q.T)


def parity_basis_dets(space, parity):
    """Orthonormal basis (rows) of the M_S = 0 sector of any space with
    n_alpha = n_beta whose determinant set is closed under exchanging the alpha
    and beta strings (GAS bounds on alpha + beta totals and point-group targets
    both are): (|Ia Ib> + parity |Ib Ia>)/sqrt(2) for each exchanged pair,
    the member of the pair with the lower vector index first, and for
    parity = +1 the determinants with Ia = Ib (Sec. 3.1, Sec. 3.3).  For
    one-block spaces it is ``parity_basis`` row for row."""
    d = space.dets()
    where = {(int(a), int(b)): i for i, (a, b) in enumerate(d)}
    r2 = 1.0 / np.sqrt(2.0)
    rows = []
    for i, (a, b) in enumerate(d):
        j = where[(int(b), int(a))]          # KeyError: the space is not closed under the exchange
        if j < i or (j == i and parity < 0):
            continue
        v = np.zeros(space.ndet)
        if j == i:
            v[i] = 1.0
        else:
            v[i] = r2
            v[j] = parity * r2
        rows.append(v)
    return np.array(rows).reshape(len(rows), space.ndet)


def parity_spectrum_dets(space, parity):
    """Eigenvalues (ascending) of H restricted to the sector of
    ``parity_basis_dets`` (tiny spaces only)."""
    Q = parity_basis_dets(space, parity)
    return np.linalg.eigvalsh(Q @ space.hmat() @ Q.T)


def davidson(space, nroots=1, tol=1e-10, rtol=None, max_iter=200, max_space=None,
             sigma=None, hdiag=None, verbose=False):
    """Lowest ``nroots`` eigenpairs of H by Davidson-Liu (Sec. 3.3, steps 1-4).

    1. Initial subspace: unit vectors on the ``nroots`` lowest diagonal
       elements (ties: lowest index); their sigma vectors; diagonalise B^T H B.
    2. Preconditioner: the diagonal H_II.
    3. Correction t = r / (theta - H_II) (denominator kept away from zero with
       its sign), orthogonalised against all previous vectors by classical
       Gram-Schmidt applied twice, normalised; dropped if it vanishes.
    4. Sigma of the new vectors, re-diagonalise the projected matrix.
    Converged when every root has |delta theta| <= tol and ||r|| <= rtol
    (default sqrt(tol)).  At ``max_space`` the basis collapses to the current
    Ritz vectors.  Returns (energies, vectors[nroots, ndet], info dict).
    """
    N = space.ndet
    nroots = min(nroots, N)
    if rtol is None:
        rtol = np.sqrt(tol)
    if max_space is None:
        max_space = max(8 * nroots, 24)
    max_space = max(max_space, 2 * nroots)
    sig = sigma if sigma is not None else space.sigma
    hd = space.hdiag() if hdiag is None else hdiag
    order = np.argsort(hd, kind="stable")[:nroots]
    B = np.zeros((0, N))
    S = np.zeros((0, N))
    new = np.zeros((nroots, N))
    for k, i in enumerate(order):
        new[k, i] = 1.0
    theta_old = np.full(nroots, np.inf)
    it = 0
    nsigma = 0
    conv = False
    while True:
        if new.shape[0]:
            snew = np.stack([sig(v) for v in new])
            nsigma += new.shape[0]
            B = np.vstack([B, new])
            S = np.vstack([S, snew])
        Gm = B @ S.T
        Gm = 0.5 * (Gm + Gm.T)
        w, y = np.linalg.eigh(Gm)
        theta = w[:nroots]
        Y = y[:, :nroots]
        X = Y.T @ B
        R = Y.T @ S - theta[:, None] * X
        rnorm = np.linalg.norm(R, axis=1)
        dtheta = np.abs(theta - theta_old)
        theta_old = theta.copy()
        it += 1
        if verbose:
            print(f"it {it:3d} dim {B.shape[0]:3d} theta {theta} |r| {rnorm}")
        if np.all(dtheta <= tol) and np.all(rnorm <= rtol):
            conv = True
            break
        if it >= max_iter or B.shape[0] >= N:
            conv = bool(np.all(rnorm <= rtol)) or B.shape[0] >= N
            break
        if B.shape[0] + nroots > max_space:
            B = X.copy()
            S = Y.T @ S
            # re-orthonormalise the collapsed basis (Ritz vectors already are)
        cand = []
        for k in range(nroots):
            if rnorm[k] <= rtol and dtheta[k] <= tol:
                continue
            den = theta[k] - hd
            small = np.abs(den) < 1e-8
            den = np.where(small, np.where(den < 0, -1e-8, 1e-8), den)
            cand.append(R[k] / den)
        new_list = []
        for t in cand:
            Q = np.vstack([B] + new_list) if new_list else B
            for _ in range(2):
                t = t - Q.T @ (Q @ t)
            nt = np.linalg.norm(t)
            if nt < 1e-12:
                continue
            new_list.append(t / nt)
        new = np.stack(new_list) if new_list else np.zeros((0, N))
        if new.shape[0] == 0:
            conv = bool(np.all(rnorm <= rtol))
            break
    return theta, X, {"iterations": it, "nsigma": nsigma, "rnorm": rnorm, "converged": conv}
