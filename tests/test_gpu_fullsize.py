"""Parity at the full workload sizes, in the configuration bench.py times.

The oracle cannot build whole sigma vectors of 1.6e8 determinants in test
time, so it computes sampled output determinants one by one (its row-sampled
Slater-Condon sigma) and the GPU vector is compared there; properties that hold
at any size check every element:

* symmetry of H:  <C2|H C1> = <C1|H C2> for two random vectors;
* alpha <-> beta exchange (n_alpha = n_beta):  sigma(C^T) = sigma(C)^T, which
  runs the alpha and beta halves of every pass on exchanged data.

Tolerances, 1e-10 (FP64) and 1e-5 (FP32), on the larger of the relative
2-norm error over the sample and the largest element error over the largest
reference element (tests/tolerance.py).
"""
import numpy as np
import pytest
import torch

import oracle
import synth_inputs as si
from tolerance import rel, rel_t

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-10, torch.float32: 1e-5}


def _cis():
    import paper_1707_04346_amd as cis
    return cis


def workload(name):
    w = si.WORKLOADS[name]
    h, g = si.integrals(w["norb"], w["nchol"], 0)
    ctx = _cis().Context(w["norb"], w["nalpha"], w["nbeta"], h, g, gas=w["gas"])
    ref = oracle.Space(w["norb"], w["nalpha"], w["nbeta"], h, g, gas=w["gas"])
    return ctx, ref


def sample_rows(ndet, nrand, seed, extra=()):
    rng = np.random.default_rng(seed)
    rows = np.concatenate([rng.integers(0, ndet, nrand), np.asarray(extra, dtype=np.int64)])
    return np.unique(np.clip(rows, 0, ndet - 1))


@pytest.fixture(scope="module")
def cas16():
    ctx, ref = workload("cas16")
    c = si.ci_vector(ctx.ndet, 0)
    yield ctx, ref, c
    ctx.close()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_cas16_sampled_rows(cas16, dtype):
    """CAS(16,16), 165,636,900 determinants: 4096 random rows plus the first and
    last rows and the ends of the first and last 32-column tiles."""
    cis = _cis()
    ctx, ref, c = cas16
    n = 12870
    extra = [0, 1, 31, 32, n - 1, n, ctx.ndet - 1, ctx.ndet - n, (n - 1) * n + 31, (n - 1) * n + n - 32]
    rows = sample_rows(ctx.ndet, 4096, 21, extra)
    C = torch.tensor(c, dtype=dtype, device="cuda")
    S = torch.empty_like(C)
    ctx.apply(C, S)
    torch.cuda.synchronize()
    # FP32: the one-W-tile form of the owner kernel, two workgroups per compute unit
    shared = cis.PATH_AB_SHARED_CU if dtype == torch.float32 else 0
    assert ctx.last_path(cis.FP32 if dtype == torch.float32 else cis.FP64) == \
        cis.PATH_AB_OWNER | cis.PATH_SS_MATERIALISED | shared
    assert ctx.last_shape(cis.FP32 if dtype == torch.float32 else cis.FP64) == (16, 9, 10, 2)
    got = S[torch.tensor(rows, device="cuda")].double().cpu().numpy()
    want = ref.sigma_rows(rows, c)
    err = rel(got, want)
    assert err <= TOL[dtype], err


def test_cas16_symmetric_operator(cas16):
    ctx, _, _ = cas16
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    C1 = torch.randn(ctx.ndet, dtype=torch.float64, device="cuda", generator=g)
    C2 = torch.randn(ctx.ndet, dtype=torch.float64, device="cuda", generator=g)
    S1, S2 = torch.empty_like(C1), torch.empty_like(C2)
    ctx.apply(C1, S1)
    ctx.apply(C2, S2)
    a, b = float(C2 @ S1), float(C1 @ S2)
    scale = float(torch.linalg.vector_norm(C1) * torch.linalg.vector_norm(S2))
    assert abs(a - b) <= 1e-12 * scale, (a, b)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_cas16_alpha_beta_exchange(cas16, dtype):
    """sigma(C^T) = sigma(C)^T for every element: the exchanged vector runs the
    beta data through the alpha kernels and the other way round."""
    ctx, _, _ = cas16
    n = 12870
    g = torch.Generator(device="cuda")
    g.manual_seed(6)
    C = torch.randn(n, n, dtype=dtype, device="cuda", generator=g)
    Ct = C.t().contiguous()
    S, St = torch.empty_like(C), torch.empty_like(C)
    ctx.apply(C.reshape(-1), S.reshape(-1))
    ctx.apply(Ct.reshape(-1), St.reshape(-1))
    err = rel_t(St, S.t())
    assert err <= TOL[dtype], err


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_gas20_sampled_rows(dtype):
    """GAS(20,20) 6/8/6 with cumulative bounds [10,12], [18,20], [20,20]:
    22,065,484 determinants in 36 blocks; random rows plus the first and last
    determinant of every block."""
    ctx, ref = workload("gas20")
    c = si.ci_vector(ctx.ndet, 0)
    offs = ctx.layout()["offset"]
    extra = list(offs[:-1]) + [int(o) - 1 for o in offs[1:]]
    rows = sample_rows(ctx.ndet, 2048, 22, extra)
    C = torch.tensor(c, dtype=dtype, device="cuda")
    S = torch.empty_like(C)
    ctx.apply(C, S)
    torch.cuda.synchronize()
    # the owner-computes GAS kernel in both precisions (FP64: long sigma rows split over
    # several units), the same-spin parts as stored pair-product rows plus a gather
    assert ctx.last_path(_cis().FP32 if dtype == torch.float32 else _cis().FP64) == \
        _cis().PATH_AB_OWNER | _cis().PATH_SS_MATERIALISED
    got = S[torch.tensor(rows, device="cuda")].double().cpu().numpy()
    want = ref.sigma_rows(rows, c)
    err = rel(got, want)
    ctx.close()
    assert err <= TOL[dtype], err


@pytest.fixture(scope="module")
def cas18():
    ctx, ref = workload("cas18")
    c = si.ci_vector(ctx.ndet, 0)
    yield ctx, ref, c
    ctx.close()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_cas18_sampled_rows(cas18, dtype):
    """CAS(18,18), 2,363,904,400 determinants (9.5 GB per FP32 vector, 18.9 GB
    per FP64 vector; element offsets beyond 2^31): 1024 random rows, plus the
    first and last element of every 32-column tile of the first and the last
    alpha row."""
    ctx, ref, c = cas18
    n = 48620
    ends = [t * 32 for t in range(-(-n // 32))] + [min(t * 32 + 31, n - 1) for t in range(-(-n // 32))]
    extra = ends + [(n - 1) * n + e for e in ends]
    rows = sample_rows(ctx.ndet, 1024, 23, extra)
    C = torch.tensor(c, dtype=dtype, device="cuda")
    S = torch.empty_like(C)
    ctx.apply(C, S)
    torch.cuda.synchronize()
    got = S[torch.tensor(rows, device="cuda")].double().cpu().numpy()
    del C, S
    torch.cuda.empty_cache()
    want = ref.sigma_rows(rows, c)
    err = rel(got, want)
    assert err <= TOL[dtype], err
