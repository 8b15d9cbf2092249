"""Failure handling and logging through the C ABI on the GPU.

* ENOMEM: the host fills the device with a torch allocation, leaving 1 GiB,
  then asks for sigma (FP64 workspace of CAS(16,16): 5.3 GB) and for a
  Davidson run; both return CISIGMA_ENOMEM with a message and no fault, and
  both work once the memory is handed back.
* The Davidson JSON-lines log: one parseable line per iteration (and per FP64
  refinement in mixed mode) whose last energies are the returned ones.
"""
import json

import numpy as np
import pytest
import torch

import synth_inputs as si

pytestmark = pytest.mark.gpu


def _cis():
    import paper_1707_04346_amd as cis
    return cis


def test_enomem_when_the_device_is_full():
    cis = _cis()
    w = si.WORKLOADS["cas16"]
    h, g = si.integrals(w["norb"], w["nchol"], 0)
    ctx = cis.Context(w["norb"], w["nalpha"], w["nbeta"], h, g)
    C = torch.zeros(ctx.ndet, dtype=torch.float64, device="cuda")
    C[0] = 1.0
    S = torch.empty_like(C)
    torch.cuda.synchronize()
    free, _ = torch.cuda.mem_get_info()
    hog = torch.empty(free - (1 << 30), dtype=torch.uint8, device="cuda")
    with pytest.raises(cis.CisigmaError) as ei:
        ctx.apply(C, S)
    assert ei.value.status == cis.ENOMEM, ei.value
    assert "memory" in ctx.last_error()
    with pytest.raises(cis.CisigmaError) as ei:
        ctx.davidson(1, 1e-8)
    assert ei.value.status == cis.ENOMEM, ei.value
    del hog
    torch.cuda.empty_cache()
    ctx.apply(C, S)
    torch.cuda.synchronize()
    assert abs(float(S[0]) - float(np.dot(C.cpu().numpy(), S.cpu().numpy()))) < 1e-12
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_davidson_jsonl_log(tmp_path, prec):
    cis = _cis()
    h, g = si.integrals(8, 16, 0)
    ctx = cis.Context(8, 4, 4, h, g)
    if prec == "mixed":
        ctx.set_option(cis.OPT_PRECISION, cis.FP32)
    path = tmp_path / "dav.jsonl"
    ctx.set_log(path)
    e, st, status = ctx.davidson(2, 1e-10)
    assert status == 0
    lines = [json.loads(x) for x in open(path)]
    its = [x for x in lines if "iteration" in x]
    assert len(its) == st["iterations"]
    assert [x["iteration"] for x in its] == list(range(1, st["iterations"] + 1))
    assert all(x["precision"] == prec and len(x["energies"]) == 2 for x in lines)
    if prec == "mixed":
        refs = [x for x in lines if "refinement" in x]
        assert len(refs) == st["refinements"]
        assert np.allclose(refs[-1]["energies"], e, atol=1e-12)
    else:
        assert np.allclose(its[-1]["energies"], e, atol=1e-12)
    ctx.set_log(None)
    ctx.davidson(1, 1e-8)
    assert len(open(path).readlines()) == len(lines)
