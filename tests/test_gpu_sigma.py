"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

* string and single-excitation tables: bit-exact against the oracle's string
  order (itself pinned to an itertools enumeration) and a Python brute force
  of the excitation lists;
* sigma = H C: element by element against the oracle on the same seeded
  inputs; FP64 within 1e-10 and FP32 within 1e-5 relative (2-norm), the
  tolerances of the FP64 and FP32 modes;
* H_II against the oracle diagonal.
"""
import numpy as np
import pytest
import torch

import oracle
import synth_inputs as si
from tolerance import rel

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-10, 1e-5


def _cis():
    import paper_1707_04346_amd as cis
    return cis


def make(norb, na, nb, nchol=None, seed=0, gas=None):
    h, g = si.integrals(norb, nchol or 2 * norb, seed)
    return _cis().Context(norb, na, nb, h, g, gas=gas), oracle.Space(norb, na, nb, h, g, gas=gas)


def gpu_sigma(ctx, c, dtype):
    C = torch.tensor(c, dtype=dtype, device="cuda")
    S = torch.full_like(C, float("nan"))
    ctx.apply(C, S)
    torch.cuda.synchronize()
    return S.double().cpu().numpy()




# (norb, nalpha, nbeta, gas)
SMALL = [
    (6, 3, 3, None),            # CAS(6,6), 400 determinants
    (6, 3, 2, None),
    (7, 2, 4, None),
    (5, 1, 3, None),            # one alpha electron: one-electron same-spin kernel
    (5, 0, 2, None),            # no alpha electrons: no alpha-beta part
    (4, 4, 1, None),            # full alpha shell
    (8, 4, 4, None),            # CAS(8,8)
    (9, 5, 4, None),            # 126 x 126: ragged column tiles
    (10, 3, 3, None),
    (7, 3, 3, ([2, 3, 2], [3, 5, 6], [4, 6, 6])),      # GAS, three spaces
    (8, 3, 4, ([3, 5], [5, 7], [6, 7])),               # GAS, two spaces, n_a != n_b
    (6, 3, 3, ([2, 2, 2], [0, 0, 6], [6, 6, 6])),      # unrestricted GAS (= CAS)
]


def _ids(c):
    return f"n{c[0]}a{c[1]}b{c[2]}" + ("gas" if c[3] else "")


@pytest.mark.parametrize("case", SMALL, ids=[_ids(c) for c in SMALL])
def test_tables_bit_exact(case):
    norb, na, nb, gas = case
    ctx, ref = make(norb, na, nb, gas=gas)
    assert ctx.ndet == ref.ndet
    for spin, ne in ((0, na), (1, nb)):
        s_ref, _ = ref.strings(spin)
        s_gpu = ctx.strings(spin)
        assert np.array_equal(s_gpu, s_ref)
        index = {int(x): i for i, x in enumerate(s_ref)}
        exc = ctx.excitations(spin)
        assert exc.shape == (len(s_ref), ne * (norb - ne))
        brute = np.zeros_like(exc)
        for I, x in enumerate(int(v) for v in s_ref):
            occ = [p for p in range(norb) if (x >> p) & 1]
            vir = [p for p in range(norb) if not (x >> p) & 1]
            e = 0
            for k in occ:
                for l in vir:
                    y = (x & ~(1 << k)) | (1 << l)
                    J = index.get(y)
                    if J is None:
                        brute[I, e] = 0xFFFFFFFF
                    else:
                        lo, hi = min(k, l), max(k, l)
                        between = bin(x & (((1 << hi) - 1) & ~((1 << (lo + 1)) - 1))).count("1")
                        brute[I, e] = (J << 11) | (k << 6) | (l << 1) | (between & 1)
                    e += 1
        assert np.array_equal(exc, brute)
    # host-side address agrees with the oracle's order
    for i in range(0, ref.ndet, max(1, ref.ndet // 97)):
        assert ctx.address(*ref.det(i)) == i


@pytest.mark.parametrize("case", SMALL, ids=[_ids(c) for c in SMALL])
def test_sigma_fp64_full(case):
    norb, na, nb, gas = case
    ctx, ref = make(norb, na, nb, gas=gas, seed=3)
    c = si.ci_vector(ctx.ndet, 5)
    s_ref = ref.sigma(c)
    s = gpu_sigma(ctx, c, torch.float64)
    assert rel(s, s_ref) <= TOL64, rel(s, s_ref)


@pytest.mark.parametrize("case", SMALL, ids=[_ids(c) for c in SMALL])
def test_sigma_fp32_full(case):
    norb, na, nb, gas = case
    ctx, ref = make(norb, na, nb, gas=gas, seed=4)
    c = si.ci_vector(ctx.ndet, 6)
    s_ref = ref.sigma(c)
    s = gpu_sigma(ctx, c, torch.float32)
    assert rel(s, s_ref) <= TOL32, rel(s, s_ref)


def test_sigma_cas12_fp64_and_fp32():
    """CAS(12,12), 853,776 determinants: the full vector in both precisions."""
    w = si.WORKLOADS["cas12"]
    ctx, ref = make(w["norb"], w["nalpha"], w["nbeta"], w["nchol"], seed=0)
    c = si.ci_vector(ctx.ndet, 0)
    s_ref = ref.sigma(c)
    assert rel(gpu_sigma(ctx, c, torch.float64), s_ref) <= TOL64
    assert rel(gpu_sigma(ctx, c, torch.float32), s_ref) <= TOL32


def test_sigma_uniform_vector_and_repeat():
    """The paper's timing input (every coefficient 1/N, Sec. 5); two calls in a
    row give the same FP64 result (the accumulators are cleared each call)."""
    ctx, ref = make(8, 4, 4, seed=9)
    c = si.ci_vector(ctx.ndet, kind="uniform")
    s_ref = ref.sigma(c)
    s1 = gpu_sigma(ctx, c, torch.float64)
    s2 = gpu_sigma(ctx, c, torch.float64)
    assert rel(s1, s_ref) <= TOL64 and rel(s2, s_ref) <= TOL64


def test_hdiag():
    for norb, na, nb, gas in [(6, 3, 3, None), (7, 3, 3, ([2, 3, 2], [3, 5, 6], [4, 6, 6])), (5, 1, 3, None)]:
        ctx, ref = make(norb, na, nb, gas=gas)
        out = torch.empty(ctx.ndet, dtype=torch.float64, device="cuda")
        ctx.hdiag(out)
        torch.cuda.synchronize()
        assert np.abs(out.cpu().numpy() - ref.hdiag()).max() < 1e-12


def test_apply_rejects_aliasing_and_bad_dtype():
    cis = _cis()
    ctx, _ = make(6, 3, 3)
    C = torch.zeros(ctx.ndet, dtype=torch.float64, device="cuda")
    assert ctx.apply_raw(C.data_ptr(), C.data_ptr(), cis.FP64) == cis.EINVAL
    assert ctx.apply_raw(C.data_ptr(), C.data_ptr() + 8, cis.FP64) == cis.EINVAL
    S = torch.zeros_like(C)
    assert ctx.apply_raw(C.data_ptr(), S.data_ptr(), 7) == cis.EINVAL
    assert ctx.apply_raw(0, S.data_ptr(), cis.FP64) == cis.EINVAL
    assert "overlap" in ctx.last_error() or "NULL" in ctx.last_error()


def test_apply_on_a_side_stream():
    ctx, ref = make(8, 4, 3, seed=2)
    c = si.ci_vector(ctx.ndet, 1)
    s_ref = ref.sigma(c)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        C = torch.tensor(c, dtype=torch.float64, device="cuda")
        S = torch.empty_like(C)
        ctx.apply(C, S, stream=st)
    st.synchronize()
    assert rel(S.cpu().numpy(), s_ref) <= TOL64


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_cas_sigma_is_bitwise_reproducible(dtype):
    """One-block spaces take the owner-computes alpha-beta kernel (fixed scatter
    plan) and the materialised same-spin form (plain stores, fixed gather
    order): no atomics, so repeated applies agree bit for bit."""
    cis = _cis()
    ctx, _ = make(10, 5, 5, seed=3)
    c = si.ci_vector(ctx.ndet, 4)
    C = torch.tensor(c, dtype=dtype, device="cuda")
    S1, S2 = torch.empty_like(C), torch.empty_like(C)
    ctx.apply(C, S1)
    for _ in range(3):
        ctx.apply(C, S2)
        torch.cuda.synchronize()
        assert torch.equal(S1, S2)
    prec = cis.FP32 if dtype == torch.float32 else cis.FP64
    assert ctx.last_path(prec) & ~cis.PATH_AB_SHARED_CU == cis.PATH_AB_OWNER | cis.PATH_SS_MATERIALISED


@pytest.mark.parametrize("case", [(8, 4, 4), (9, 5, 4), (10, 5, 5)], ids=lambda c: f"n{c[0]}a{c[1]}b{c[2]}")
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_overlap_option_matches_oracle(case, dtype):
    """CISIGMA_OPT_OVERLAP: the beta-beta pass on the context's second stream,
    joined before the output gather; repeated calls on a caller stream, each
    checked against the oracle, then the option switched off again."""
    cis = _cis()
    ctx, ref = make(*case, seed=4)
    tol = TOL64 if dtype == torch.float64 else TOL32
    st = torch.cuda.Stream()
    ctx.set_option(cis.OPT_OVERLAP, 1)
    for k in range(3):
        c = si.ci_vector(ctx.ndet, 20 + k)
        C = torch.tensor(c, dtype=dtype, device="cuda")
        S = torch.full_like(C, float("nan"))
        torch.cuda.synchronize()
        ctx.apply(C, S, stream=st)
        st.synchronize()
        assert rel(S.double().cpu().numpy(), ref.sigma(c)) <= tol, k
    ctx.set_option(cis.OPT_OVERLAP, 0)
    S2 = torch.empty_like(C)
    ctx.apply(C, S2)
    torch.cuda.synchronize()
    assert rel(S2.double().cpu().numpy(), ref.sigma(c)) <= tol


@pytest.mark.parametrize("case", [(6, 3, 3), (8, 4, 4), (9, 5, 4), (7, 2, 4), (10, 5, 5)],
                         ids=lambda c: f"n{c[0]}a{c[1]}b{c[2]}")
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_sigma_general_path_matches_oracle(case, dtype):
    """The general kernels (scatter with float atomics) that GAS spaces use,
    forced on CAS spaces that would otherwise take the owner-computes path."""
    cis = _cis()
    norb, na, nb = case
    ctx, ref = make(norb, na, nb, seed=11)
    ctx.set_option(cis.OPT_SIGMA_PATH, 1)
    c = si.ci_vector(ctx.ndet, 12)
    s_ref = ref.sigma(c)
    tol = TOL64 if dtype == torch.float64 else TOL32
    assert rel(gpu_sigma(ctx, c, dtype), s_ref) <= tol


@pytest.mark.parametrize("case", [(6, 3, 3), (8, 4, 4), (10, 5, 5), (12, 6, 6)], ids=lambda c: f"n{c[0]}")
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_cas_takes_the_fast_paths(case, dtype):
    """One-block spaces run the owner-computes sigma_3 kernel and the
    materialised same-spin products (no silent fallback), and stay exact."""
    cis = _cis()
    norb, na, nb = case
    ctx, ref = make(norb, na, nb, seed=13)
    c = si.ci_vector(ctx.ndet, 14)
    s = gpu_sigma(ctx, c, dtype)
    flags = ctx.last_path(cis.FP32 if dtype == torch.float32 else cis.FP64)
    assert flags & ~cis.PATH_AB_SHARED_CU == cis.PATH_AB_OWNER | cis.PATH_SS_MATERIALISED, flags
    if dtype == torch.float64:
        assert not flags & cis.PATH_AB_SHARED_CU   # the shared-CU form is FP32 only
    tol = TOL64 if dtype == torch.float64 else TOL32
    assert rel(s, ref.sigma(c)) <= tol


# One-block spaces whose alpha excitation count n_a (n - n_a) is a multiple of 4
# start the alpha-beta accumulators from the rank-1 term of Ia's own row
# instead of giving that row a k step: one space per compiled shape of that
# form not already run above (n = 8, 12 there; n = 16 in the full-size tests).
# The expected shape (k steps, pair row blocks, plan entries per lane, variant)
# is the compiled kernel each space must get: variant 2 = rank-1 own row,
# 1 = own row in a k step.  The plan width is the narrow one unless a target's
# contributions within a 32-column tile would span more than four lanes at it
# (then 16).
SHAPES = [((4, 2, 2), (1, 1, 2, 2)), ((6, 2, 3), (2, 2, 16, 2)), ((10, 4, 5), (6, 4, 16, 2)),
          ((8, 4, 4), (4, 3, 16, 2)), ((12, 6, 6), (9, 5, 16, 2)), ((7, 2, 4), (3, 2, 16, 1)),
          ((9, 5, 4), (6, 3, 16, 1)), ((7, 4, 2), (4, 2, 4, 1))]


@pytest.mark.parametrize("case,shape", SHAPES, ids=[f"n{c[0]}a{c[1]}b{c[2]}" for c, _ in SHAPES])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_rank1_self_row_shapes(case, shape, dtype):
    cis = _cis()
    norb, na, nb = case
    ctx, ref = make(norb, na, nb, seed=17)
    c = si.ci_vector(ctx.ndet, 18)
    s = gpu_sigma(ctx, c, dtype)
    dt = cis.FP32 if dtype == torch.float32 else cis.FP64
    assert ctx.last_path(dt) & cis.PATH_AB_OWNER
    assert ctx.last_shape(dt) == shape, ctx.last_shape(dt)
    tol = TOL64 if dtype == torch.float64 else TOL32
    assert rel(s, ref.sigma(c)) <= tol


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_rank1_self_row_cas14_sampled(dtype):
    """14 orbitals, 6 alpha + 7 beta electrons (3003 x 3432 determinants, 48
    alpha excitations): 2048 random rows plus the ends of the first and last
    alpha rows and of their first and last 32-column tiles, against the oracle."""
    cis = _cis()
    ctx, ref = make(14, 6, 7, seed=19)
    c = si.ci_vector(ctx.ndet, 20)
    nb = 3432
    extra = [0, 31, 32, nb - 32, nb - 1, ctx.ndet - nb, ctx.ndet - nb + 31, ctx.ndet - 1]
    rng = np.random.default_rng(22)
    rows = np.unique(np.concatenate([rng.integers(0, ctx.ndet, 2048), np.array(extra)])).astype(np.int64)
    C = torch.tensor(c, dtype=dtype, device="cuda")
    S = torch.empty_like(C)
    ctx.apply(C, S)
    torch.cuda.synchronize()
    dt = cis.FP32 if dtype == torch.float32 else cis.FP64
    assert ctx.last_path(dt) & cis.PATH_AB_OWNER
    assert ctx.last_shape(dt) == (12, 7, 8, 2), ctx.last_shape(dt)
    got = S[torch.tensor(rows, device="cuda")].double().cpu().numpy()
    want = ref.sigma_rows(rows, c)
    tol = TOL64 if dtype == torch.float64 else TOL32
    assert rel(got, want) <= tol


@pytest.mark.parametrize("case", [(7, 3, 3, ([2, 3, 2], [3, 5, 6], [4, 6, 6])),
                                  (8, 3, 4, ([3, 5], [5, 7], [6, 7])),
                                  (6, 3, 3, ([2, 2, 2], [0, 0, 6], [6, 6, 6]))], ids=["gas7", "gas8", "gas6open"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_gas_takes_the_owner_path(case, dtype):
    """GAS spaces run the owner-computes sigma_3 kernel with per-type source
    tiles and the same-spin parts as stored pair-product rows plus a gather (no
    atomics anywhere), stay exact, and repeat bit for bit."""
    cis = _cis()
    norb, na, nb, gas = case
    ctx, ref = make(norb, na, nb, gas=gas, seed=16)
    c = si.ci_vector(ctx.ndet, 17)
    s = gpu_sigma(ctx, c, dtype)
    assert ctx.last_path(cis.FP32 if dtype == torch.float32 else cis.FP64) == \
        cis.PATH_AB_OWNER | cis.PATH_SS_MATERIALISED
    tol = TOL64 if dtype == torch.float64 else TOL32
    assert rel(s, ref.sigma(c)) <= tol
    assert np.array_equal(gpu_sigma(ctx, c, dtype), s)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_gas_general_path_matches_oracle(dtype):
    """The general (atomic) sigma_3 kernel on GAS spaces, forced."""
    cis = _cis()
    for norb, na, nb, gas in [(7, 3, 3, ([2, 3, 2], [3, 5, 6], [4, 6, 6])), (8, 3, 4, ([3, 5], [5, 7], [6, 7]))]:
        ctx, ref = make(norb, na, nb, gas=gas, seed=18)
        ctx.set_option(cis.OPT_SIGMA_PATH, 1)
        c = si.ci_vector(ctx.ndet, 19)
        s = gpu_sigma(ctx, c, dtype)
        assert ctx.last_path(cis.FP32 if dtype == torch.float32 else cis.FP64) == 0
        tol = TOL64 if dtype == torch.float64 else TOL32
        assert rel(s, ref.sigma(c)) <= tol


# One-block spaces on the owner-computes units of the GAS form (path 2): sigma
# rows cut at the occupation classes of the two highest orbitals, and inside a
# class where the unit width asks for it; W rows grouped so that a source tile
# of another class multiplies only the row blocks leading into the unit.  This
# is the form CAS(18,18) runs at full size.  (norb, na, nb, gas), unit width,
# expected (k steps, row blocks); GAS rows are cut at beta-type ends.
UNITS = [((8, 4, 4, None), 0, (5, 4)), ((8, 4, 4, None), 64, (5, 4)), ((10, 5, 5, None), 64, (7, 5)),
         ((10, 5, 5, None), 128, (7, 5)), ((7, 3, 3, ([2, 3, 2], [3, 5, 6], [4, 6, 6])), 64, None)]


@pytest.mark.parametrize("case,cols,shape", UNITS,
                         ids=[f"{_ids(c)}_w{w}" for c, w, _ in UNITS])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_owner_units_match_oracle(case, cols, shape, dtype):
    cis = _cis()
    norb, na, nb, gas = case
    ctx, ref = make(norb, na, nb, gas=gas, seed=23)
    if gas is None:
        ctx.set_option(cis.OPT_SIGMA_PATH, 2)
    if cols:
        ctx.set_option(cis.OPT_UNIT_COLS, cols)
    c = si.ci_vector(ctx.ndet, 24)
    s = gpu_sigma(ctx, c, dtype)
    dt = cis.FP32 if dtype == torch.float32 else cis.FP64
    assert ctx.last_path(dt) & cis.PATH_AB_OWNER
    got = ctx.last_shape(dt)
    # FP32 one-block rows: the eight-wave unit kernel; FP32 GAS: the eight-wave GAS
    # form; FP64: the four-wave GAS form
    assert got[3] == (3 if dtype == torch.float64 else 4 if gas is None else 5), got
    if shape is not None:
        assert got[:2] == shape, got
    tol = TOL64 if dtype == torch.float64 else TOL32
    assert rel(s, ref.sigma(c)) <= tol
    assert np.array_equal(gpu_sigma(ctx, c, dtype), s)   # one writer per target: bitwise repeatable


def test_unit_cols_option_rejects_bad_values():
    cis = _cis()
    ctx, _ = make(6, 3, 3, seed=1)
    for bad in (-1, 1, 63, 70000, 100.5):
        with pytest.raises(Exception):
            ctx.set_option(cis.OPT_UNIT_COLS, bad)
    for bad in (-1, 4):
        with pytest.raises(Exception):
            ctx.set_option(cis.OPT_SIGMA_PATH, bad)


@pytest.mark.parametrize("case", [(10, 5, 5), (12, 6, 6), (9, 5, 4)], ids=["cas10", "cas12", "n9a5b4"])
def test_one_block_two_w_form_matches_oracle(case):
    """FP32 one-block sigma_3 in both forms: by default the one-W-tile kernel with
    two workgroups per compute unit (PATH_AB_SHARED_CU); with CISIGMA_OPT_SIGMA_PATH
    = 3 the double-buffered two-W-tile kernel, one workgroup per CU (the form the
    shapes whose registers leave room for one workgroup take).  Both against the
    oracle's sigma, each repeating bit for bit."""
    cis = _cis()
    norb, na, nb = case
    ctx, ref = make(norb, na, nb, seed=29)
    c = si.ci_vector(ctx.ndet, 30)
    want = ref.sigma(c)
    s1 = gpu_sigma(ctx, c, torch.float32)
    assert ctx.last_path(cis.FP32) == cis.PATH_AB_OWNER | cis.PATH_SS_MATERIALISED | cis.PATH_AB_SHARED_CU
    ctx.set_option(cis.OPT_SIGMA_PATH, 3)
    s2 = gpu_sigma(ctx, c, torch.float32)
    assert ctx.last_path(cis.FP32) == cis.PATH_AB_OWNER | cis.PATH_SS_MATERIALISED
    assert ctx.last_shape(cis.FP32)[3] in (1, 2)
    assert rel(s1, want) <= TOL32 and rel(s2, want) <= TOL32
    assert np.array_equal(gpu_sigma(ctx, c, torch.float32), s2)
    s64 = gpu_sigma(ctx, c, torch.float64)   # FP64 has one form: path 3 changes nothing there
    assert ctx.last_path(cis.FP64) == cis.PATH_AB_OWNER | cis.PATH_SS_MATERIALISED
    assert rel(s64, want) <= TOL64


@pytest.mark.parametrize("case,cols", [((7, 3, 3, ([2, 3, 2], [3, 5, 6], [4, 6, 6])), 0), ((10, 5, 5, None), 64)],
                         ids=["gas7", "n10_w64"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_one_launch_per_unit_is_the_same_sigma(case, cols, dtype):
    """CISIGMA_OPT_UNIT_LAUNCH = 1 (one launch per unit, the per-block baseline)
    runs the same workgroups as the single launch: the same sigma bit for bit."""
    cis = _cis()
    norb, na, nb, gas = case
    ctx, ref = make(norb, na, nb, gas=gas, seed=27)
    if gas is None:
        ctx.set_option(cis.OPT_SIGMA_PATH, 2)
    if cols:
        ctx.set_option(cis.OPT_UNIT_COLS, cols)
    c = si.ci_vector(ctx.ndet, 28)
    one = gpu_sigma(ctx, c, dtype)
    ctx.set_option(cis.OPT_UNIT_LAUNCH, 1)
    per = gpu_sigma(ctx, c, dtype)
    dt = cis.FP32 if dtype == torch.float32 else cis.FP64
    assert ctx.last_path(dt) & cis.PATH_AB_OWNER
    assert np.array_equal(one, per)
    assert rel(per, ref.sigma(c)) <= (TOL64 if dtype == torch.float64 else TOL32)
    with pytest.raises(Exception):
        ctx.set_option(cis.OPT_UNIT_LAUNCH, 2)



@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_deterministic_mode(dtype):
    """CISIGMA_OPT_DETERMINISTIC = 1: spaces the atomic-free kernels cover give the
    same sigma as before, bit for bit, and a converged Davidson; an apply that
    would need a float-atomic kernel is refused (EUNSUPPORTED) and leaves the
    output untouched -- sigma_3 forced onto the general kernel (SIGMA_PATH = 1),
    and a space without stored same-spin rows (one-block, 15 orbitals, 2 beta
    electrons: its same-spin passes take the atomic kernel)."""
    cis = _cis()
    ctx, ref = make(8, 4, 4, seed=31)
    c = si.ci_vector(ctx.ndet, 32)
    plain = gpu_sigma(ctx, c, dtype)
    ctx.set_option(cis.OPT_DETERMINISTIC, 1)
    det = gpu_sigma(ctx, c, dtype)
    assert np.array_equal(det, plain)
    assert rel(det, ref.sigma(c)) <= (TOL64 if dtype == torch.float64 else TOL32)
    if dtype == torch.float64:
        w = np.linalg.eigvalsh(ref.hmat())
        e, st, status = ctx.davidson(2, 1e-10)
        assert status == 0 and np.allclose(e, w[:2], atol=1e-8)
    ctx.set_option(cis.OPT_SIGMA_PATH, 1)
    C = torch.tensor(c, dtype=dtype, device="cuda")
    S = torch.full_like(C, 7.0)
    with pytest.raises(cis.CisigmaError) as err:
        ctx.apply(C, S)
    assert err.value.status == cis.EUNSUPPORTED
    torch.cuda.synchronize()
    assert bool((S == 7.0).all())
    ctx.set_option(cis.OPT_SIGMA_PATH, 0)
    assert np.array_equal(gpu_sigma(ctx, c, dtype), plain)
    for bad in (-1, 2):
        with pytest.raises(cis.CisigmaError):
            ctx.set_option(cis.OPT_DETERMINISTIC, bad)
    h, g = si.integrals(15, 30, 0)
    ctx2 = cis.Context(15, 7, 2, h, g)
    C2 = torch.ones(ctx2.ndet, dtype=dtype, device="cuda")
    S2 = torch.empty_like(C2)
    ctx2.apply(C2, S2)
    prec = cis.FP32 if dtype == torch.float32 else cis.FP64
    assert not ctx2.last_path(prec) & cis.PATH_SS_MATERIALISED   # the atomic same-spin kernel ran
    ctx2.set_option(cis.OPT_DETERMINISTIC, 1)
    S2.fill_(7.0)
    with pytest.raises(cis.CisigmaError) as err:
        ctx2.apply(C2, S2)
    assert err.value.status == cis.EUNSUPPORTED
    torch.cuda.synchronize()
    assert bool((S2 == 7.0).all())
