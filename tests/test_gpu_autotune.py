"""cisigma_autotune and the launch parameters it sets (GAS owner-unit order,
same-spin column split): every value gives sigma equal to the oracle's (FP64
1e-10, FP32 1e-5 relative), and the tuner reports its timings and choices."""
import numpy as np
import pytest
import torch

import oracle
import synth_inputs as si
from tolerance import rel

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-10, torch.float32: 1e-5}
GAS7 = ([2, 3, 2], [3, 5, 6], [4, 6, 6])
GAS8 = ([3, 3, 2], [4, 7, 8], [6, 8, 8])


def _cis():
    import paper_1707_04346_amd as cis
    return cis




def sigma(ctx, c, dtype):
    C = torch.tensor(c, dtype=dtype, device="cuda")
    S = torch.full_like(C, float("nan"))
    ctx.apply(C, S)
    torch.cuda.synchronize()
    return S.double().cpu().numpy()


@pytest.mark.parametrize("case", [(7, 3, 3, GAS7), (8, 4, 4, GAS8)], ids=["gas7", "gas8"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_knobs_keep_sigma(case, dtype):
    cis = _cis()
    norb, na, nb, gas = case
    h, g = si.integrals(norb, 2 * norb, 2)
    ctx = cis.Context(norb, na, nb, h, g, gas=gas)
    ref = oracle.Space(norb, na, nb, h, g, gas=gas)
    c = si.ci_vector(ctx.ndet, 5)
    want = ref.sigma(c)
    # unit launch orders 0-5 (4, 5: the batch weights of Sec. 3.1 Eqs. 10 and 11):
    # only the order of independent workgroups changes, so sigma is the same bit for bit
    first = None
    for order in range(6):
        ctx.set_option(cis.OPT_GAS_UNIT_ORDER, order)
        got = sigma(ctx, c, dtype)
        assert rel(got, want) <= TOL[dtype], order
        if first is None:
            first = got
        assert np.array_equal(got, first), order
    for split in (1, 3, 16, 0):
        ctx.set_option(cis.OPT_SS_SPLIT, split)
        assert rel(sigma(ctx, c, dtype), want) <= TOL[dtype], split
    with pytest.raises(cis.CisigmaError):
        ctx.set_option(cis.OPT_GAS_UNIT_ORDER, 6)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_autotune_reports_and_keeps_sigma(dtype):
    cis = _cis()
    h, g = si.integrals(8, 16, 3)
    ctx = cis.Context(8, 4, 4, h, g, gas=GAS8)
    ref = oracle.Space(8, 4, 4, h, g, gas=GAS8)
    prec = cis.FP64 if dtype == torch.float64 else cis.FP32
    report = ctx.autotune(prec, reps=2)
    assert "as set:" in report
    assert "same_spin_split ->" in report
    if ctx.last_path(prec) & cis.PATH_AB_OWNER:
        assert "gas_unit_order ->" in report
        assert "unit_cols ->" in report
    c = si.ci_vector(ctx.ndet, 9)
    assert rel(sigma(ctx, c, dtype), ref.sigma(c)) <= TOL[dtype]


def test_autotune_on_cas_and_bad_arguments():
    """A one-block space has no GAS units and uses the materialised same-spin
    form: nothing but the baseline timing to report."""
    cis = _cis()
    h, g = si.integrals(8, 16, 4)
    ctx = cis.Context(8, 4, 4, h, g)
    report = ctx.autotune(cis.FP32, reps=1)
    assert report.startswith("as set:") and "->" not in report
    assert cis._lib.cisigma_autotune(ctx.handle, 9, 1, None, 0) == cis.EINVAL
    assert cis._lib.cisigma_autotune(ctx.handle, cis.FP32, 0, None, 0) == cis.EINVAL
