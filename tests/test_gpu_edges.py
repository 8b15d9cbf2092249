"""Edge shapes on the GPU against the oracle: the largest orbital counts the
32-bit strings allow (norb = 32), orbital counts just past the one-block fast
kernels (norb = 17, 20, 24: the general kernels), and the density matrices and
spin sector at their own limits (norb = 16 with few electrons)."""
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


def make(norb, na, nb, seed=0):
    h, g = si.integrals(norb, 2 * norb, seed)
    return _cis().Context(norb, na, nb, h, g), oracle.Space(norb, na, nb, h, g)




EDGE = [(32, 1, 1), (32, 2, 1), (32, 0, 3), (24, 2, 2), (20, 1, 3), (17, 2, 2), (17, 3, 1)]


@pytest.mark.parametrize("case", EDGE, ids=[f"n{c[0]}a{c[1]}b{c[2]}" for c in EDGE])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_sigma_edge_shapes(case, dtype):
    ctx, ref = make(*case, seed=5)
    c = si.ci_vector(ctx.ndet, 6)
    C = torch.tensor(c, dtype=dtype, device="cuda")
    S = torch.full_like(C, float("nan"))
    ctx.apply(C, S)
    torch.cuda.synchronize()
    assert rel(S.double().cpu().numpy(), ref.sigma(c)) <= TOL[dtype]


def test_davidson_norb32():
    ctx, ref = make(32, 1, 1, seed=2)
    w = np.linalg.eigvalsh(ref.hmat())
    e, st, status = ctx.davidson(2, 1e-10)
    assert status == 0
    assert np.allclose(e, w[:2], atol=1e-8), (e, w[:2])


@pytest.mark.parametrize("case", [(16, 1, 1), (16, 2, 2), (16, 2, 1)], ids=["n16a1b1", "n16a2b2", "n16a2b1"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_rdm_norb16_few_electrons(case, dtype):
    """17 row blocks of M (n^2 + 1 = 257 rows), fewer alpha strings than workgroups."""
    ctx, ref = make(*case, seed=7)
    c = si.ci_vector(ctx.ndet, 8)
    w1, w2 = ref.rdm(c)
    n = ctx.norb
    g1 = torch.empty(n * n, dtype=torch.float64, device="cuda")
    g2 = torch.empty(n ** 4, dtype=torch.float64, device="cuda")
    ctx.rdm(torch.tensor(c, dtype=dtype, device="cuda"), g1, g2)
    torch.cuda.synchronize()
    assert rel(g1.cpu().numpy().reshape(n, n), w1) <= TOL[dtype]
    assert rel(g2.cpu().numpy().reshape(n, n, n, n), w2) <= TOL[dtype]


@pytest.mark.parametrize("parity", [1, -1], ids=["even", "odd"])
def test_parity_sigma_general_kernels(parity):
    """M_S = 0 sector on a one-block space served by the general kernels (norb = 17)."""
    cis = _cis()
    ctx, ref = make(17, 2, 2, seed=9)
    n = int(round(np.sqrt(ctx.ndet)))
    M = si.ci_vector(ctx.ndet, 10).reshape(n, n)
    c = (0.5 * (M + parity * M.T)).reshape(-1)
    ctx.set_option(cis.OPT_SPIN_PARITY, parity)
    C = torch.tensor(c, dtype=torch.float64, device="cuda")
    S = torch.empty_like(C)
    ctx.apply(C, S)
    torch.cuda.synchronize()
    assert rel(S.cpu().numpy(), ref.sigma(c)) <= 1e-10
