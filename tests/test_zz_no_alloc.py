"""cisigma_apply_noalloc against cisigma_apply, through the C ABI.

The no-allocation entry point runs the same kernels on a workspace carved from
the library's static device scratch.  Two calls in a row, the second on a
smaller space (a different context, so the scratch holds the first call's
layout when the second starts), each compared element by element with
cisigma_apply on the same vector and with the oracle; plus the refusal of a
space too large for the scratch.
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


def _pair(ctx, c, dtype):
    C = torch.tensor(c, dtype=dtype, device="cuda")
    S_ref = torch.full_like(C, float("nan"))
    S_na = torch.full_like(C, float("nan"))
    ctx.apply(C, S_ref)
    torch.cuda.synchronize()
    ctx.apply_noalloc(C, S_na)
    torch.cuda.synchronize()
    return S_na.double().cpu().numpy(), S_ref.double().cpu().numpy()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_noalloc_matches_apply_two_calls(dtype):
    cis = _cis()
    cases = [(12, 6, 6, None),                                   # CAS(12,12): 853,776 determinants
             (7, 3, 3, ([2, 3, 2], [3, 5, 6], [4, 6, 6]))]       # a GAS space, far smaller
    for norb, na, nb, gas in cases:
        h, g = si.integrals(norb, 2 * norb, 5)
        ctx = cis.Context(norb, na, nb, h, g, gas=gas)
        c = si.ci_vector(ctx.ndet, 6)
        got, want = _pair(ctx, c, dtype)
        assert not np.isnan(got).any()
        assert rel(got, want) <= TOL[dtype], (norb, rel(got, want))
        if ctx.ndet <= 5000:
            assert rel(got, oracle.Space(norb, na, nb, h, g, gas=gas).sigma(c)) <= TOL[dtype]
        ctx.close()


def test_noalloc_refuses_spaces_beyond_the_scratch():
    cis = _cis()
    h, g = si.integrals(14, 28, 0)
    ctx = cis.Context(14, 7, 7, h, g)          # 3432^2 determinants: the copies alone exceed 64 MiB
    C = torch.zeros(ctx.ndet, dtype=torch.float32, device="cuda")
    S = torch.zeros_like(C)
    with pytest.raises(cis.CisigmaError) as ei:
        ctx.apply_noalloc(C, S)
    assert ei.value.status == cis.EUNSUPPORTED
    assert "static scratch" in ctx.last_error()
    ctx.close()
