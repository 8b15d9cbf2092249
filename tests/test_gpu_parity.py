"""M_S = 0 spin-parity sector (Sec. 3.1, Sec. 3.3) on the GPU, through the C ABI.

With CISIGMA_OPT_SPIN_PARITY p the library assumes C(Ib, Ia) = p C(Ia, Ib)
and takes the beta-beta part of sigma as p times the transposed alpha-alpha
part.  Checked here:

* sigma of sector vectors against the oracle's plain sigma (FP64 1e-10, FP32
  1e-5 relative), and that the result lies in the sector;
* at CAS(16,16) against the library's own full sigma on the same vector and
  the oracle on sampled rows;
* Davidson in each sector against the dense spectrum of H restricted to the
  sector (``oracle.parity_spectrum``), FP64 and mixed;
* GAS and point-group spaces (blocks (ta, tb) and (tb, ta) mirror each
  other): sector sigma against the oracle, and Davidson against the dense
  spectrum of H restricted to the sector (``oracle.parity_spectrum_dets``);
* the option's error paths (n_alpha != n_beta, out-of-range values, more
  roots than the sector holds).
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


def make(norb, na, nb, nchol=None, seed=0, gas=None):
    h, g = si.integrals(norb, nchol or 2 * norb, seed)
    return _cis().Context(norb, na, nb, h, g, gas=gas), oracle.Space(norb, na, nb, h, g, gas=gas)


def sector_vector(ndet, seed, parity):
    n = int(round(np.sqrt(ndet)))
    M = si.ci_vector(ndet, seed).reshape(n, n)
    M = 0.5 * (M + parity * M.T)
    return (M / np.linalg.norm(M)).reshape(-1), n


def gpu_sigma(ctx, c, dtype):
    C = torch.tensor(c, dtype=dtype, device="cuda")
    S = torch.full_like(C, float("nan"))
    ctx.apply(C, S)
    torch.cuda.synchronize()
    return S.double().cpu().numpy()




CASES = [(2, 1, 0), (6, 3, 0), (8, 4, 1), (9, 4, 2), (10, 5, 3)]


@pytest.mark.parametrize("case", CASES, ids=[f"cas{c[0]}" for c in CASES])
@pytest.mark.parametrize("parity", [1, -1], ids=["even", "odd"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_parity_sigma_matches_oracle(case, parity, dtype):
    norb, ne, seed = case
    cis = _cis()
    ctx, ref = make(norb, ne, ne, seed=seed)
    c, n = sector_vector(ctx.ndet, seed + 10, parity)
    want = ref.sigma(c)
    ctx.set_option(cis.OPT_SPIN_PARITY, parity)
    got = gpu_sigma(ctx, c, dtype)
    assert rel(got, want) <= TOL[dtype]
    G = got.reshape(n, n)
    assert np.abs(G - parity * G.T).max() <= TOL[dtype] * np.abs(G).max() * 10
    # switching the option off gives the plain path again
    ctx.set_option(cis.OPT_SPIN_PARITY, 0)
    assert rel(gpu_sigma(ctx, c, dtype), want) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_parity_sigma_cas16(dtype):
    """CAS(16,16), 165,636,900 determinants, symmetric vector: the sector path
    against the full path on every element and against the oracle on 512
    sampled rows."""
    cis = _cis()
    w = si.WORKLOADS["cas16"]
    ctx, ref = make(w["norb"], w["nalpha"], w["nbeta"], w["nchol"])
    n = 12870
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    M = torch.randn(n, n, dtype=dtype, device="cuda", generator=g)
    M = (M + M.t()) * 0.5
    C = M.reshape(-1)
    S_full, S_par = torch.empty_like(C), torch.empty_like(C)
    ctx.apply(C, S_full)
    ctx.set_option(cis.OPT_SPIN_PARITY, 1)
    ctx.apply(C, S_par)
    torch.cuda.synchronize()
    err = rel_t(S_par, S_full)
    assert err <= TOL[dtype], err
    rows = np.unique(np.random.default_rng(24).integers(0, ctx.ndet, 512))
    got = S_par[torch.tensor(rows, device="cuda")].double().cpu().numpy()
    c = C.double().cpu().numpy()
    want = ref.sigma_rows(rows, c)
    del M, C, S_full, S_par
    ctx.close()
    assert rel(got, want) <= TOL[dtype]


@pytest.mark.parametrize("case", [(6, 3, 3), (8, 4, 2), (4, 2, 2)], ids=["cas6", "cas8", "cas4"])
@pytest.mark.parametrize("parity", [1, -1], ids=["even", "odd"])
def test_davidson_parity_fp64(case, parity):
    norb, ne, nroots = case
    cis = _cis()
    ctx, ref = make(norb, ne, ne)
    want = oracle.parity_spectrum(ref, parity)[:nroots]
    ctx.set_option(cis.OPT_SPIN_PARITY, parity)
    X = torch.empty(nroots, ctx.ndet, dtype=torch.float64, device="cuda")
    e, st, status = ctx.davidson(nroots, 1e-10, vecs=X)
    assert status == 0
    assert np.allclose(e, want, atol=1e-8), (e, want)
    n = int(round(np.sqrt(ctx.ndet)))
    for r in range(nroots):
        V = X[r].cpu().numpy().reshape(n, n)
        assert np.abs(V - parity * V.T).max() < 1e-10


@pytest.mark.parametrize("parity", [1, -1], ids=["even", "odd"])
def test_davidson_parity_mixed(parity):
    cis = _cis()
    ctx, ref = make(8, 4, 4)
    want = oracle.parity_spectrum(ref, parity)[:3]
    ctx.set_option(cis.OPT_SPIN_PARITY, parity)
    ctx.set_option(cis.OPT_PRECISION, cis.FP32)
    e, st, status = ctx.davidson(3, 1e-10)
    assert status == 0
    assert np.allclose(e, want, atol=1e-6), (e - want)
    assert st["sigma_fp32"] > 0 and st["sigma_fp64"] > 0


def test_parity_sectors_hold_the_full_spectrum():
    """The lowest root over both sectors is the lowest root of the full space."""
    cis = _cis()
    ctx, ref = make(6, 3, 3)
    e_full, _, _ = ctx.davidson(1, 1e-10)
    lows = []
    for parity in (1, -1):
        ctx.set_option(cis.OPT_SPIN_PARITY, parity)
        e, _, status = ctx.davidson(1, 1e-10)
        assert status == 0
        lows.append(e[0])
    assert abs(min(lows) - e_full[0]) < 1e-8


def test_parity_option_errors():
    cis = _cis()
    ctx, _ = make(6, 3, 2)
    with pytest.raises(cis.CisigmaError) as ei:
        ctx.set_option(cis.OPT_SPIN_PARITY, 1)
    assert ei.value.status == cis.EINVAL
    ctx.set_option(cis.OPT_SPIN_PARITY, 0)
    gas = ([2, 3, 2], [3, 5, 6], [4, 6, 6])
    ctx_g, _ = make(7, 3, 3, gas=gas)
    ctx_g.set_option(cis.OPT_SPIN_PARITY, -1)     # GAS blocks mirror each other when n_alpha = n_beta
    ctx_g.set_option(cis.OPT_SPIN_PARITY, 0)
    ctx_u, _ = make(7, 3, 2, gas=([2, 3, 2], [2, 4, 5], [3, 5, 5]))
    with pytest.raises(cis.CisigmaError) as ei:
        ctx_u.set_option(cis.OPT_SPIN_PARITY, 1)
    assert ei.value.status == cis.EINVAL
    ctx2, _ = make(2, 1, 1)
    for bad in (2, 0.5, -3):
        with pytest.raises(cis.CisigmaError):
            ctx2.set_option(cis.OPT_SPIN_PARITY, bad)
    ctx2.set_option(cis.OPT_SPIN_PARITY, -1)   # the odd sector of 2 x 2 determinants has one state
    with pytest.raises(cis.CisigmaError) as ei:
        ctx2.davidson(2, 1e-10)
    assert ei.value.status == cis.EINVAL
    e, _, status = ctx2.davidson(1, 1e-10)
    assert status == 0


# spaces with several blocks: (norb, n per spin, gas, orbsym, target)
BLOCKED = [
    (7, 3, ([2, 3, 2], [3, 5, 6], [4, 6, 6]), None, 0),
    (6, 3, ([2, 2, 2], [0, 0, 6], [6, 6, 6]), None, 0),
    (8, 4, None, [p % 8 for p in range(8)], 0),
    (8, 4, None, [p % 8 for p in range(8)], 5),
]


def make_blocked(case, seed=2):
    norb, ne, gas, orbsym, target = case
    h, g = si.integrals(norb, 2 * norb, seed, orbsym=orbsym)
    ctx = _cis().Context(norb, ne, ne, h, g, gas=gas, orbsym=orbsym, target=target)
    ref = oracle.Space(norb, ne, ne, h, g, gas=gas, orbsym=orbsym, target=target)
    swap = np.array([ref.address(int(b), int(a)) for a, b in ref.dets()])
    return ctx, ref, swap


def _bid(c):
    return f"n{c[0]}e{c[1]}" + ("gas" if c[2] else f"sym{c[4]}")


@pytest.mark.parametrize("case", BLOCKED, ids=[_bid(c) for c in BLOCKED])
@pytest.mark.parametrize("parity", [1, -1], ids=["even", "odd"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_parity_sigma_blocked_spaces(case, parity, dtype):
    """Sector sigma of GAS and point-group spaces: the beta-beta part as the
    transposed alpha-alpha part read from the mirror block."""
    cis = _cis()
    ctx, ref, swap = make_blocked(case)
    c = si.ci_vector(ctx.ndet, 40)
    c = 0.5 * (c + parity * c[swap])
    c /= np.linalg.norm(c)
    want = ref.sigma(c)
    ctx.set_option(cis.OPT_SPIN_PARITY, parity)
    got = gpu_sigma(ctx, c, dtype)
    assert rel(got, want) <= TOL[dtype]
    assert np.abs(got - parity * got[swap]).max() <= TOL[dtype] * np.abs(got).max() * 10
    ctx.set_option(cis.OPT_SPIN_PARITY, 0)
    assert rel(gpu_sigma(ctx, c, dtype), want) <= TOL[dtype]


@pytest.mark.parametrize("case", BLOCKED[:3], ids=[_bid(c) for c in BLOCKED[:3]])
@pytest.mark.parametrize("parity", [1, -1], ids=["even", "odd"])
def test_davidson_parity_blocked_spaces(case, parity):
    """Sector Davidson of GAS and point-group spaces (FP64 and mixed) against
    the dense spectrum of H restricted to the sector; the FP64 eigenvectors lie
    in the sector."""
    cis = _cis()
    ctx, ref, swap = make_blocked(case)
    want = oracle.parity_spectrum_dets(ref, parity)[:2]
    ctx.set_option(cis.OPT_SPIN_PARITY, parity)
    X = torch.empty(2, ctx.ndet, dtype=torch.float64, device="cuda")
    e, st, status = ctx.davidson(2, 1e-10, vecs=X)
    assert status == 0
    assert np.allclose(e, want, atol=1e-8), (e, want)
    for r in range(2):
        v = X[r].cpu().numpy()
        assert np.abs(v - parity * v[swap]).max() < 1e-10
    ctx.set_option(cis.OPT_PRECISION, cis.FP32)
    e32, st32, status = ctx.davidson(2, 1e-10)
    assert status == 0
    assert np.allclose(e32, want, atol=1e-6), (e32 - want)

