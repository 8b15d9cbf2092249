"""cisigma_apply replayed from a captured HIP graph (CISIGMA_OPT_GRAPH).

The graph is captured at the first call with given buffers and replayed by
later calls; the buffers' contents change between replays, with the caller's
own eager GPU work and synchronisations in between.  Every replay is checked
against the oracle's sigma of the current contents (FP64 1e-10, FP32 1e-5), and
against the library's eager result on the same vector.
"""
import numpy as np
import pytest
import torch

import oracle
import synth_inputs as si
from tolerance import rel

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-10, torch.float32: 1e-5}
CASES = [(8, 4, 4, None), (6, 3, 2, None), (7, 3, 3, ([2, 3, 2], [3, 5, 6], [4, 6, 6]))]


def _cis():
    import paper_1707_04346_amd as cis
    return cis




@pytest.mark.parametrize("case", CASES, ids=["cas8", "cas6a3b2", "gas7"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_graph_replays_match_oracle_and_eager(case, dtype):
    norb, na, nb, gas = case
    cis = _cis()
    h, g = si.integrals(norb, 2 * norb, 1)
    ctx = cis.Context(norb, na, nb, h, g, gas=gas)
    ref = oracle.Space(norb, na, nb, h, g, gas=gas)
    stream = torch.cuda.Stream()
    C = torch.empty(ctx.ndet, dtype=dtype, device="cuda")
    S = torch.empty_like(C)
    S_eager = torch.empty_like(C)
    ctx.set_option(cis.OPT_GRAPH, 1)
    for it in range(5):
        c = si.ci_vector(ctx.ndet, 100 + it)
        C.copy_(torch.tensor(c, dtype=dtype))
        junk = torch.randn(4096, device="cuda") @ torch.randn(4096, device="cuda")   # the caller's own work
        torch.cuda.synchronize()
        ctx.apply(C, S, stream=stream)            # it 0: eager + capture; later: replay
        stream.synchronize()
        got = S.double().cpu().numpy()
        assert rel(got, ref.sigma(c)) <= TOL[dtype], it
        ctx.apply(C, S_eager)                     # NULL stream: always eager
        torch.cuda.synchronize()
        assert rel(got, S_eager.double().cpu().numpy()) <= TOL[dtype], it
        del junk
    ctx.close()


def test_graph_dropped_when_the_sector_changes():
    """Switching the spin-parity option drops the captured graphs: the next call
    captures the sector form."""
    cis = _cis()
    h, g = si.integrals(6, 12, 2)
    ctx = cis.Context(6, 3, 3, h, g)
    ref = oracle.Space(6, 3, 3, h, g)
    n = 20
    M = si.ci_vector(ctx.ndet, 3).reshape(n, n)
    c = (0.5 * (M + M.T)).reshape(-1)
    stream = torch.cuda.Stream()
    C = torch.tensor(c, dtype=torch.float64, device="cuda")
    S = torch.empty_like(C)
    ctx.set_option(cis.OPT_GRAPH, 1)
    for parity in (0, 1, 0, 1):
        ctx.set_option(cis.OPT_SPIN_PARITY, parity)
        for _ in range(2):
            ctx.apply(C, S, stream=stream)
            stream.synchronize()
            assert rel(S.cpu().numpy(), ref.sigma(c)) <= 1e-10
