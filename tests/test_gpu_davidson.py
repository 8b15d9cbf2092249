"""Davidson on the GPU against dense diagonalisation of the oracle's H, and
against oracle-certified Rayleigh quotients for spaces too large for eigh."""
import numpy as np
import pytest
import torch

import oracle
import synth_inputs as si
from tolerance import rel

pytestmark = pytest.mark.gpu


def _cis():
    import paper_1707_04346_amd as cis
    return cis


def make(norb, na, nb, nchol=None, seed=0, gas=None):
    h, g = si.integrals(norb, nchol or 2 * norb, seed)
    return _cis().Context(norb, na, nb, h, g, gas=gas), oracle.Space(norb, na, nb, h, g, gas=gas)


@pytest.mark.parametrize("case", [(6, 3, 3, 1, None), (8, 4, 4, 3, None), (7, 4, 2, 2, None),
                                  (7, 3, 3, 2, ([2, 3, 2], [3, 5, 6], [4, 6, 6]))])
def test_davidson_fp64_vs_dense(case):
    norb, na, nb, nroots, gas = case
    ctx, ref = make(norb, na, nb, gas=gas)
    w = np.linalg.eigvalsh(ref.hmat())
    e, st, status = ctx.davidson(nroots, 1e-10)
    assert status == 0
    assert np.allclose(e, w[:nroots], atol=1e-8), (e, w[:nroots])
    assert st["sigma_fp64"] > 0 and st["sigma_fp32"] == 0


@pytest.mark.parametrize("case", [(6, 3, 3, 1), (8, 4, 4, 3)])
def test_davidson_mixed_vs_dense(case):
    norb, na, nb, nroots = case
    cis = _cis()
    ctx, ref = make(norb, na, nb)
    w = np.linalg.eigvalsh(ref.hmat())
    ctx.set_option(cis.OPT_PRECISION, cis.FP32)
    e, st, status = ctx.davidson(nroots, 1e-10)
    assert status == 0
    assert np.allclose(e, w[:nroots], atol=1e-6), (e - w[:nroots])
    assert st["sigma_fp32"] > 0 and st["sigma_fp64"] > 0 and st["refinements"] >= 1


@pytest.mark.parametrize("case", [(4, 2, 2, None), (5, 3, 2, None), (6, 1, 4, None),
                                  (7, 3, 3, ([2, 3, 2], [3, 5, 6], [4, 6, 6]))],
                         ids=["cas4", "n5a3b2", "n6a1b4", "gas7"])
def test_hmat_block_matches_oracle(case):
    """cisigma_hmat_block (the P-space Hamiltonian) against the oracle's dense H:
    every element of the space for small cases, bit-level agreement not required
    (same rules, different summation order): 1e-12 absolute."""
    norb, na, nb, gas = case
    ctx, ref = make(norb, na, nb, seed=3, gas=gas)
    H = ref.hmat()
    idx = np.arange(ctx.ndet)
    got = ctx.hmat_block(idx, idx)
    assert np.abs(got - H).max() <= 1e-12 * max(1.0, np.abs(H).max())
    # a rectangular block with repeated and permuted indices
    rng = np.random.default_rng(1)
    r, c = rng.integers(0, ctx.ndet, 7), rng.permutation(ctx.ndet)[:5]
    assert np.abs(ctx.hmat_block(r, c) - H[np.ix_(r, c)]).max() <= 1e-12 * max(1.0, np.abs(H).max())
    cis = _cis()
    with pytest.raises(cis.CisigmaError):
        ctx.hmat_block([ctx.ndet], [0])


@pytest.mark.parametrize("pspace", [64, 0], ids=["pspace64", "nopspace"])
@pytest.mark.parametrize("thick", [1, 0], ids=["thick", "plain"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_davidson_thick_and_plain_restarts_vs_dense(thick, prec, pspace):
    """A subspace of 3 nroots vectors forces a collapse every iteration or two:
    thick restarts (current + previous Ritz vectors) and plain ones (current
    only) both reach the dense eigenvalues."""
    cis = _cis()
    ctx, ref = make(8, 4, 4, seed=6)
    w = np.linalg.eigvalsh(ref.hmat())
    nroots = 2
    ctx.set_option(cis.OPT_THICK_RESTART, thick)
    ctx.set_option(cis.OPT_PSPACE, pspace)
    ctx.set_option(cis.OPT_MAX_SPACE, 3 * nroots)
    ctx.set_option(cis.OPT_MAX_ITER, 600)
    ctx.set_option(cis.OPT_PRECISION, cis.FP64 if prec == "fp64" else cis.FP32)
    e, st, status = ctx.davidson(nroots, 1e-10)
    assert status == 0
    assert np.allclose(e, w[:nroots], atol=1e-8 if prec == "fp64" else 1e-6), (e - w[:nroots])


@pytest.mark.parametrize("case", [(4, 2, 2, 2), (5, 2, 3, 3), (2, 1, 1, 1)], ids=["cas4", "n5a2b3", "n2"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_davidson_pspace_covers_the_space(case, prec):
    """Spaces smaller than the P-space: the guess is already exact, the
    corrections vanish, and the driver still ends with the dense eigenvalues."""
    norb, na, nb, nroots = case
    cis = _cis()
    ctx, ref = make(norb, na, nb, seed=5)
    w = np.linalg.eigvalsh(ref.hmat())
    assert ctx.ndet <= 256
    ctx.set_option(cis.OPT_PRECISION, cis.FP64 if prec == "fp64" else cis.FP32)
    e, st, status = ctx.davidson(nroots, 1e-10)
    assert status == 0
    assert np.allclose(e, w[:nroots], atol=1e-8 if prec == "fp64" else 1e-6), (e - w[:nroots])


def test_davidson_mixed_low_memory_swaps_workspaces():
    """CISIGMA_OPT_LOW_MEMORY: the FP32 and FP64 sigma workspaces are released
    and re-created around every refinement (forced here with a refinement every
    8 iterations).  Same arithmetic in fresh buffers: the run matches the one
    without the option exactly, and the dense energies; plain apply calls of
    both precisions work afterwards."""
    cis = _cis()
    ctx, ref = make(8, 4, 4, seed=8)
    w = np.linalg.eigvalsh(ref.hmat())
    runs = []
    for low in (0, 1):
        ctx.set_option(cis.OPT_LOW_MEMORY, low)
        ctx.set_option(cis.OPT_REFINE_EVERY, 8)
        ctx.set_option(cis.OPT_MAX_ITER, 400)
        ctx.set_option(cis.OPT_PRECISION, cis.FP32)
        e, st, status = ctx.davidson(2, 1e-10)
        assert status == 0 and st["refinements"] >= 2
        assert np.allclose(e, w[:2], atol=1e-6), (e - w[:2])
        runs.append((e, st["iterations"], st["sigma_fp32"], st["sigma_fp64"]))
    assert np.array_equal(runs[0][0], runs[1][0]) and runs[0][1:] == runs[1][1:], runs
    c = si.ci_vector(ctx.ndet, 2)
    for dt, tol in ((torch.float32, 1e-5), (torch.float64, 1e-10)):
        C = torch.tensor(c, dtype=dt, device="cuda")
        S = torch.empty_like(C)
        ctx.apply(C, S)
        torch.cuda.synchronize()
        s_ref = ref.sigma(c)
        assert rel(S.double().cpu().numpy(), s_ref) <= tol


def test_davidson_vectors_and_certificate_cas12():
    """CAS(12,12): GPU FP64 eigenvector; the oracle's sigma of it gives a
    Rayleigh quotient equal to the GPU energy and a small residual."""
    w = si.WORKLOADS["cas12"]
    ctx, ref = make(w["norb"], w["nalpha"], w["nbeta"], w["nchol"])
    cis = _cis()
    # this synthetic Hamiltonian is strongly correlated (E0 - min H_II ~ -2.6 Eh): many iterations
    ctx.set_option(cis.OPT_MAX_ITER, 400)
    ctx.set_option(cis.OPT_MAX_SPACE, 48)
    X = torch.empty(ctx.ndet, dtype=torch.float64, device="cuda")
    e, st, status = ctx.davidson(1, 1e-10, vecs=X)
    assert status == 0
    x = X.cpu().numpy()
    s = ref.sigma(x)
    rq = x @ s / (x @ x)
    r = np.linalg.norm(s - rq * x) / np.linalg.norm(x)
    assert abs(rq - e[0]) < 1e-9
    assert r < 1e-4


def test_davidson_max_iter_gives_enoconv():
    cis = _cis()
    ctx, _ = make(8, 4, 4)
    ctx.set_option(cis.OPT_MAX_ITER, 1)
    e, st, status = ctx.davidson(1, 1e-12, allow_noconv=True)
    assert status == cis.ENOCONV
    assert np.isfinite(e[0]) and st["iterations"] == 1


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("nroots,max_space", [(5, 15), (3, 9), (4, 12)], ids=["r5s15", "r3s9", "r4s12"])
@pytest.mark.parametrize("space", [(8, 4, 4), (7, 4, 3)], ids=["cas8_quad", "n7a4b3_plain"])
def test_davidson_restarts_vs_dense(prec, nroots, max_space, space):
    """A small subspace, so the thick restart runs many times: 5 roots keep up
    to 10 vectors per restart (the 16-coefficient in-place combination) and take
    two passes of the four-root Ritz kernel; 3 and 4 roots keep up to 6 and 8
    (the 8-coefficient combination).  CAS(8,8) has 4,900 determinants (the
    vector kernels' four-element form), n7a4b3 1,225 (their plain form).
    Energies against dense eigh of the oracle's H."""
    cis = _cis()
    ctx, ref = make(*space)
    assert (ctx.ndet % 4 == 0) == (space == (8, 4, 4))
    w = np.linalg.eigvalsh(ref.hmat())
    ctx.set_option(cis.OPT_MAX_SPACE, max_space)
    ctx.set_option(cis.OPT_THICK_RESTART, 1)
    ctx.set_option(cis.OPT_MAX_ITER, 400)
    if prec == "mixed":
        ctx.set_option(cis.OPT_PRECISION, cis.FP32)
    e, st, status = ctx.davidson(nroots, 1e-10)
    assert status == 0
    assert st["iterations"] > max_space // nroots   # at least one restart happened
    assert np.allclose(e, w[:nroots], atol=1e-8 if prec == "fp64" else 1e-6), (e - w[:nroots])


@pytest.mark.parametrize("case", [((8, 4, 4), 16), ((7, 4, 3), 40), ((10, 5, 5), 256)],
                         ids=["cas8_np16", "n7a4b3_np40", "cas10_np256"])
def test_pspace_is_the_lowest_diagonal(case):
    """The P-space is the np determinants of lowest (H_II, index), H_II as the
    library computes it (cisigma_hdiag; n_alpha = n_beta puts pairs of equal or
    nearly equal H_II at the boundary): after one FP64 iteration the Ritz values
    are the lowest eigenvalues of H over exactly that set, built from the
    oracle's matrix elements."""
    (norb, na, nb), npp = case
    cis = _cis()
    ctx, ref = make(norb, na, nb, seed=2)
    hd = torch.empty(ctx.ndet, dtype=torch.float64, device="cuda")
    ctx.hdiag(hd)
    torch.cuda.synchronize()
    h = hd.cpu().numpy()
    P = np.lexsort((np.arange(h.size), h))[:npp]
    Hpp = np.array([[ref.h_elem(int(i), int(j)) for j in P] for i in P])
    lam = np.linalg.eigvalsh(Hpp)
    ctx.set_option(cis.OPT_PSPACE, npp)
    ctx.set_option(cis.OPT_MAX_ITER, 1)
    nroots = 3
    e, st, status = ctx.davidson(nroots, 1e-12, allow_noconv=True)
    assert status == cis.ENOCONV and st["iterations"] == 1
    assert np.allclose(e, lam[:nroots], atol=1e-9, rtol=0), (e - lam[:nroots])
