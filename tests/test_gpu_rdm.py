"""Density matrices on the GPU (cisigma_rdm) against the oracle's plain
operator-by-operator construction, and identities that hold at any size.

* small spaces: every element of rdm1 and rdm2 against ``oracle.Space.rdm``
  (relative 2-norm, FP64 1e-10, FP32 1e-5), including n_alpha != n_beta, one
  or no electrons of a spin, ragged beta tiles, and more alpha strings than
  workgroups (grid-stride);
* CAS(12,12) and CAS(16,16): the energy identity
  sum h gamma + 1/2 sum (pq|rs) Gamma = <C|H C>/<C|C> with H C from the
  library's sigma, traces N and N(N-1), the partial trace (N-1) gamma and the
  index symmetries;
* GAS spaces are refused (EUNSUPPORTED).
"""
import numpy as np
import pytest
import torch

import oracle
import synth_inputs as si
from tolerance import rel

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-10, torch.float32: 1e-5}


def _cis():
    import paper_1707_04346_amd as cis
    return cis


def make(norb, na, nb, nchol=None, seed=0, gas=None):
    h, g = si.integrals(norb, nchol or 2 * norb, seed)
    return _cis().Context(norb, na, nb, h, g, gas=gas), oracle.Space(norb, na, nb, h, g, gas=gas), h, g


def gpu_rdm(ctx, C):
    n = ctx.norb
    g1 = torch.full((n, n), float("nan"), dtype=torch.float64, device="cuda")
    g2 = torch.full((n, n, n, n), float("nan"), dtype=torch.float64, device="cuda")
    ctx.rdm(C, g1, g2)
    torch.cuda.synchronize()
    return g1.cpu().numpy(), g2.cpu().numpy()




SMALL = [(4, 2, 2), (6, 3, 3), (6, 3, 2), (5, 1, 3), (5, 0, 2), (8, 4, 4), (9, 5, 4), (10, 4, 4)]


@pytest.mark.parametrize("case", SMALL, ids=[f"n{c[0]}a{c[1]}b{c[2]}" for c in SMALL])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_rdm_matches_oracle(case, dtype):
    norb, na, nb = case
    ctx, ref, _, _ = make(norb, na, nb, seed=3)
    c = si.ci_vector(ctx.ndet, 4)
    w1, w2 = ref.rdm(c)
    g1, g2 = gpu_rdm(ctx, torch.tensor(c, dtype=dtype, device="cuda"))
    assert rel(g1, w1) <= TOL[dtype]
    assert rel(g2, w2) <= TOL[dtype]
    # a second call on the same context reuses its buffers
    g1b, g2b = gpu_rdm(ctx, torch.tensor(2.0 * c, dtype=dtype, device="cuda"))
    assert rel(g2b, w2) <= TOL[dtype]


def _identities(ctx, h, g, C, tol):
    N = ctx.nalpha + ctx.nbeta
    g1, g2 = gpu_rdm(ctx, C)
    S = torch.empty_like(C)
    ctx.apply(C, S)
    torch.cuda.synchronize()
    e_sig = float((C.double() @ S.double()) / (C.double() @ C.double()))
    e_rdm = np.einsum("pq,pq", h, g1) + 0.5 * np.einsum("pqrs,pqrs", g, g2)
    assert abs(e_rdm - e_sig) <= tol * abs(e_sig), (e_rdm, e_sig)
    assert abs(np.trace(g1) - N) <= tol * N
    assert abs(np.einsum("pprr", g2) - N * (N - 1)) <= tol * N * N
    assert np.abs(np.einsum("pqrr->pq", g2) - (N - 1) * g1).max() <= tol * N * N
    assert np.abs(g2 - g2.transpose(2, 3, 0, 1)).max() <= tol * N
    assert np.abs(g1 - g1.T).max() <= tol * N


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_rdm_identities_cas12(dtype):
    w = si.WORKLOADS["cas12"]
    ctx, _, h, g = make(w["norb"], w["nalpha"], w["nbeta"], w["nchol"])
    c = si.ci_vector(ctx.ndet, 0)
    _identities(ctx, h, g, torch.tensor(c, dtype=dtype, device="cuda"), 1e-10 if dtype == torch.float64 else 1e-5)


def test_rdm_identities_cas16_fp32():
    w = si.WORKLOADS["cas16"]
    h, g = si.integrals(w["norb"], w["nchol"], 0)
    ctx = _cis().Context(w["norb"], w["nalpha"], w["nbeta"], h, g)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    C = torch.randn(ctx.ndet, dtype=torch.float32, device="cuda", generator=gen)
    _identities(ctx, h, g, C, 1e-5)
    del C
    ctx.close()


def test_rdm_refuses_gas_and_bad_arguments():
    cis = _cis()
    gas = ([2, 3, 2], [3, 5, 6], [4, 6, 6])
    ctx, _, _, _ = make(7, 3, 3, gas=gas)
    C = torch.zeros(ctx.ndet, dtype=torch.float64, device="cuda")
    g1 = torch.empty(49, dtype=torch.float64, device="cuda")
    g2 = torch.empty(7 ** 4, dtype=torch.float64, device="cuda")
    with pytest.raises(cis.CisigmaError) as ei:
        ctx.rdm(C, g1, g2)
    assert ei.value.status == cis.EUNSUPPORTED
    ctx2, _, _, _ = make(4, 2, 2)
    C2 = torch.ones(ctx2.ndet, dtype=torch.float64, device="cuda")
    with pytest.raises(cis.CisigmaError):
        ctx2.rdm(C2, torch.empty(15, dtype=torch.float64, device="cuda"), torch.empty(256, dtype=torch.float64, device="cuda"))
    assert cis._lib.cisigma_rdm(ctx2.handle, C2.data_ptr(), cis.FP64, None, None, None) == cis.EINVAL
