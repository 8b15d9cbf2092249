"""Spatial (point-group) symmetry -- the S of the TTSS blocks, Sec. 3.1 Eq. 9;
the paper's spaces are D2h (Sec. 4-5) -- through cisigma_init_sym, against the
oracle restricted by the same selection rule (the plain Slater-Condon sigma
over the determinants whose string irreps multiply to the target):

* string tables, type counts and block layout bit-exact;
* sigma element by element on whole vectors (FP64 1e-10, FP32 1e-5, both
  error measures of tests/tolerance.py), CAS and GAS, n_alpha != n_beta,
  every target irrep of a small space;
* the D2h CAS(16,16) workload on sampled rows plus the ends of every block;
* H_II, determinant addresses, the Davidson energies against dense eigh of
  the oracle's symmetric H, and the refusal of integrals that break the
  symmetry.
"""
import numpy as np
import pytest
import torch

import oracle
import synth_inputs as si
from tolerance import rel

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-10, torch.float32: 1e-5}
D2H8 = [p % 8 for p in range(8)]
CASES = [
    (6, 3, 3, [0, 1, 2, 3, 0, 1], 0, None),
    (8, 4, 4, D2H8, 0, None),
    (8, 4, 4, D2H8, 5, None),
    (9, 4, 5, [0, 1, 2, 3, 0, 1, 2, 3, 0], 2, None),     # C2v-like labels (two generators)
    (10, 3, 4, [p % 8 for p in range(10)], 3, None),
    (7, 3, 3, [0, 1, 1, 2, 3, 0, 5], 1, ([2, 3, 2], [3, 5, 6], [4, 6, 6])),
    (12, 6, 6, [p % 8 for p in range(12)], 0, None),
]


def _cis():
    import paper_1707_04346_amd as cis
    return cis


def make(norb, na, nb, orbsym, target, gas, seed=0):
    h, g = si.integrals(norb, 2 * norb, seed, orbsym=orbsym)
    ctx = _cis().Context(norb, na, nb, h, g, gas=gas, orbsym=orbsym, target=target)
    ref = oracle.Space(norb, na, nb, h, g, gas=gas, orbsym=orbsym, target=target)
    return ctx, ref


def _ids(c):
    return f"n{c[0]}a{c[1]}b{c[2]}t{c[4]}" + ("gas" if c[5] else "")


@pytest.mark.parametrize("case", CASES, ids=[_ids(c) for c in CASES])
def test_symmetric_tables_and_layout(case):
    ctx, ref = make(*case)
    assert ctx.ndet == ref.ndet
    for spin in (0, 1):
        s_ref, cnt_ref = ref.strings(spin)
        assert np.array_equal(ctx.strings(spin), s_ref)
    lay = ctx.layout()
    ta, tb, off = ref.blocks()
    assert np.array_equal(lay["offset"], off)
    assert np.array_equal(lay["alpha_type"], ta) and np.array_equal(lay["beta_type"], tb)
    # excitation lists: every entry against the string list
    norb = case[0]
    for spin, ne in ((0, case[1]), (1, case[2])):
        s_ref, _ = ref.strings(spin)
        index = {int(x): i for i, x in enumerate(s_ref)}
        exc = ctx.excitations(spin)
        for I, x in enumerate(int(v) for v in s_ref[:200]):
            occ = [p for p in range(norb) if (x >> p) & 1]
            emp = [p for p in range(norb) if not (x >> p) & 1]
            for ko, k in enumerate(occ):
                for lv, l in enumerate(emp):
                    y = (x & ~(1 << k)) | (1 << l)
                    w = int(exc[I, ko * len(emp) + lv])
                    if y not in index:
                        assert w == 0xFFFFFFFF
                        continue
                    lo, hi = min(k, l), max(k, l)
                    neg = bin(x & (((1 << hi) - 1) & ~((1 << (lo + 1)) - 1))).count("1") & 1
                    assert w == (index[y] << 11) | (k << 6) | (l << 1) | neg


@pytest.mark.parametrize("case", CASES, ids=[_ids(c) for c in CASES])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_symmetric_sigma_matches_oracle(case, dtype):
    ctx, ref = make(*case, seed=1)
    c = si.ci_vector(ctx.ndet, 2)
    C = torch.tensor(c, dtype=dtype, device="cuda")
    S = torch.full_like(C, float("nan"))
    ctx.apply(C, S)
    torch.cuda.synchronize()
    assert rel(S.double().cpu().numpy(), ref.sigma(c)) <= TOL[dtype]


def test_every_target_of_a_small_space():
    """Each of the eight symmetric spaces of CAS(8,8) with D2h labels (empty
    ones refused), FP64 sigma against the oracle; their sizes add up to the
    whole space."""
    cis = _cis()
    h, g = si.integrals(8, 16, 3, orbsym=D2H8)
    total = 0
    for t in range(8):
        ref = oracle.Space(8, 4, 4, h, g, orbsym=D2H8, target=t)
        if ref.ndet == 0:
            with pytest.raises(cis.CisigmaError):
                cis.Context(8, 4, 4, h, g, orbsym=D2H8, target=t)
            continue
        ctx = cis.Context(8, 4, 4, h, g, orbsym=D2H8, target=t)
        assert ctx.ndet == ref.ndet
        total += ctx.ndet
        c = si.ci_vector(ctx.ndet, t)
        C = torch.tensor(c, dtype=torch.float64, device="cuda")
        S = torch.empty_like(C)
        ctx.apply(C, S)
        torch.cuda.synchronize()
        assert rel(S.cpu().numpy(), ref.sigma(c)) <= 1e-10
    assert total == 70 * 70


@pytest.mark.parametrize("case", CASES[:4], ids=[_ids(c) for c in CASES[:4]])
def test_symmetric_hdiag_address_davidson(case):
    cis = _cis()
    ctx, ref = make(*case, seed=4)
    d = torch.empty(ctx.ndet, dtype=torch.float64, device="cuda")
    ctx.hdiag(d)
    torch.cuda.synchronize()
    assert np.allclose(d.cpu().numpy(), ref.hdiag(), atol=1e-12)
    dets = ref.dets()
    for i in np.random.default_rng(0).integers(0, ref.ndet, 50):
        assert ctx.address(int(dets[i][0]), int(dets[i][1])) == i
    # a determinant of another irrep is not in the space
    a0, b0 = (int(v) for v in dets[0])
    norb, orbsym = case[0], case[3]
    for k in range(norb):
        for l in range(norb):
            if (a0 >> k) & 1 and not (a0 >> l) & 1 and orbsym[k] != orbsym[l]:
                assert ctx.address((a0 & ~(1 << k)) | (1 << l), b0) == -1
                break
    w = np.linalg.eigvalsh(ref.hmat())
    nroots = min(2, ref.ndet)
    e, st, status = ctx.davidson(nroots, 1e-10)
    assert status == 0
    assert np.allclose(e, w[:nroots], atol=1e-8), (e, w[:nroots])


def test_symmetry_breaking_integrals_refused():
    cis = _cis()
    h, g = si.integrals(6, 12, 0)           # no point-group shaping
    with pytest.raises(cis.CisigmaError) as ei:
        cis.Context(6, 3, 3, h, g, orbsym=[0, 1, 2, 3, 0, 1], target=0)
    assert ei.value.status == cis.EINVAL


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_cas16_d2h_sampled_rows(dtype):
    """CAS(16,16) with D2h labels (orbital p in irrep p % 8, target A_g): 4096
    random rows plus the first and last determinant of every block."""
    w = si.WORKLOADS["cas16_d2h"]
    h, g = si.integrals(w["norb"], w["nchol"], 0, orbsym=w["orbsym"])
    ctx = _cis().Context(w["norb"], w["nalpha"], w["nbeta"], h, g, orbsym=w["orbsym"], target=w["target"])
    ref = oracle.Space(w["norb"], w["nalpha"], w["nbeta"], h, g, orbsym=w["orbsym"], target=w["target"])
    assert ctx.ndet == ref.ndet
    c = si.ci_vector(ctx.ndet, 0)
    offs = ctx.layout()["offset"]
    rng = np.random.default_rng(31)
    rows = np.unique(np.concatenate([rng.integers(0, ctx.ndet, 4096), offs[:-1], offs[1:] - 1]))
    C = torch.tensor(c, dtype=dtype, device="cuda")
    S = torch.empty_like(C)
    ctx.apply(C, S)
    torch.cuda.synchronize()
    got = S[torch.tensor(rows, device="cuda")].double().cpu().numpy()
    want = ref.sigma_rows(rows, c)
    ctx.close()
    assert rel(got, want) <= TOL[dtype]


OWNER_CASES = [CASES[0], CASES[1], CASES[2], CASES[5]]


@pytest.mark.parametrize("case", OWNER_CASES, ids=[_ids(c) for c in OWNER_CASES])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_symmetric_spaces_take_the_owner_paths(case, dtype):
    """Spaces with irreps run sigma_3 on the owner-computes units (every k step
    multiplied, tiles and row blocks from the plans) and the same-spin parts as
    stored pair-product rows: no atomics, bit-identical repeats."""
    cis = _cis()
    norb, na, nb, orbsym, target, gas = case
    ctx, ref = make(norb, na, nb, orbsym, target, gas, seed=31)
    c = si.ci_vector(ctx.ndet, 32)
    C = torch.tensor(c, dtype=dtype, device="cuda")
    S1, S2 = torch.empty_like(C), torch.empty_like(C)
    ctx.apply(C, S1)
    ctx.apply(C, S2)
    torch.cuda.synchronize()
    prec = cis.FP32 if dtype == torch.float32 else cis.FP64
    assert ctx.last_path(prec) == cis.PATH_AB_OWNER | cis.PATH_SS_MATERIALISED
    assert ctx.last_shape(prec)[3] == (5 if dtype == torch.float32 else 3)   # GAS form: eight waves in FP32
    got = S1.double().cpu().numpy()
    assert rel(got, ref.sigma(c)) <= TOL[dtype]
    assert torch.equal(S1, S2)

