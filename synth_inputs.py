"""Seeded synthetic inputs shared by the tests, the oracle checks and the benchmark.

This module draws random numbers and shapes them into integrals and CI vectors.
It holds none of the method's arithmetic (no strings, no excitation lists, no
Hamiltonian elements), so both the GPU path's tests and the CPU oracle can use
it without sharing method code.

Integral recipe (the paper's Cr3 / pentacene / Cr4 integrals are not
available, so these stand in for them; active-space shapes follow the paper's
CAS(n,n) workloads, Sec. 4-5):

  rng = numpy.random.default_rng(seed)            (PCG64)
  eps = sort(rng.uniform(-2, 1, n))               orbital energies, ascending
  O   = rng.normal(0, 0.1, (n, n))
  h   = triu(O, 1) + triu(O, 1)^T + diag(eps)      symmetric one-electron matrix
  L   = rng.normal(0, 0.15, (P, n, n));  L^P <- triu(L^P) + triu(L^P, 1)^T
  (ij|kl) = sum_P L^P_ij L^P_kl                    8-fold symmetric, PSD over (ij),(kl)

CI vectors: ``default_rng(seed + 1000).standard_normal(ndet)``, normalised; or
the paper's benchmark convention (Sec. 5): every coefficient 1/ndet.
"""
import numpy as np


def integrals(norb, nchol, seed=0, orbsym=None):
    """(h1e[n,n], eri[n,n,n,n]) in FP64 from the recipe above.

    With ``orbsym`` (irrep 0..7 of each orbital; D2h products as XOR) the same
    draws are made and then shaped to the point group: h_pq is zeroed unless
    orbsym[p] == orbsym[q], and factor P carries irrep P % 8, so L^P_pq is
    zeroed unless orbsym[p] ^ orbsym[q] == P % 8.  (pq|rs) = sum_P L^P_pq L^P_rs
    is then nonzero only when the four irreps multiply to the totally symmetric
    one, and stays 8-fold symmetric and PSD."""
    n = int(norb)
    rng = np.random.default_rng(seed)
    eps = np.sort(rng.uniform(-2.0, 1.0, n))
    O = rng.normal(0.0, 0.1, (n, n))
    h = np.triu(O, 1)
    h = h + h.T + np.diag(eps)
    L = rng.normal(0.0, 0.15, (int(nchol), n, n))
    L = np.triu(L) + np.transpose(np.triu(L, 1), (0, 2, 1))
    if orbsym is not None:
        s = np.asarray(orbsym, dtype=np.int64)
        pq = s[:, None] ^ s[None, :]
        h = np.where(pq == 0, h, 0.0)
        L = np.where(pq[None, :, :] == (np.arange(int(nchol)) % 8)[:, None, None], L, 0.0)
    Lf = L.reshape(int(nchol), n * n)
    eri = (Lf.T @ Lf).reshape(n, n, n, n)
    return np.ascontiguousarray(h), np.ascontiguousarray(eri)


def ci_vector(ndet, seed=0, kind="normal"):
    """Normalised FP64 CI vector of length ndet."""
    if kind == "uniform":
        return np.full(int(ndet), 1.0 / int(ndet))
    rng = np.random.default_rng(seed + 1000)
    c = rng.standard_normal(int(ndet))
    return c / np.linalg.norm(c)


# Workloads of the paper's active-space shapes (Sec. 4-5), as synthetic stand-ins.
WORKLOADS = {
    "cas6": dict(norb=6, nalpha=3, nbeta=3, nchol=12, gas=None),
    "cas8": dict(norb=8, nalpha=4, nbeta=4, nchol=16, gas=None),
    "cas12": dict(norb=12, nalpha=6, nbeta=6, nchol=24, gas=None),
    "cas16": dict(norb=16, nalpha=8, nbeta=8, nchol=32, gas=None),
    "cas18": dict(norb=18, nalpha=9, nbeta=9, nchol=36, gas=None),
    # 20 electrons in 20 orbitals split 6/8/6 with at most two holes in space 1
    # and at most two particles in space 3 (cumulative total-electron bounds).
    "gas20": dict(norb=20, nalpha=10, nbeta=10, nchol=40,
                  gas=([6, 8, 6], [10, 18, 20], [12, 20, 20])),
    # D2h-labelled active spaces (the point-group blocking of Sec. 3.1; the paper's
    # spaces are all D2h, Sec. 4-5): orbital p in irrep p % 8, totally symmetric target
    "cas12_d2h": dict(norb=12, nalpha=6, nbeta=6, nchol=24, gas=None, orbsym=[p % 8 for p in range(12)], target=0),
    "cas16_d2h": dict(norb=16, nalpha=8, nbeta=8, nchol=32, gas=None, orbsym=[p % 8 for p in range(16)], target=0),
    "cas18_d2h": dict(norb=18, nalpha=9, nbeta=9, nchol=36, gas=None, orbsym=[p % 8 for p in range(18)], target=0),
}
