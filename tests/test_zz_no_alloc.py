"""cryo_forward_noalloc (the forward with its workspace in the library's own
device array) against cryo_forward with a caller workspace: the same
fields and surface traces bit for bit, on two calls in a row whose second
cell is smaller than the first (the array keeps the first call's contents),
for FP64 and FP32 pairs; refusals of an oversized cell and of a plan
without device tables."""
import numpy as np
import pytest

import cellgen
from gpu_util import say

pytestmark = pytest.mark.gpu


def _reference(P, plan, n):
    import torch
    T = plan.init()
    S = torch.zeros(n, dtype=torch.float64, device="cuda")
    plan.forward(T, 0, n, surf=S)
    return T, S


def _noalloc(P, plan, n):
    import torch
    T = plan.init()
    S = torch.zeros(n, dtype=torch.float64, device="cuda")
    plan.forward_noalloc(T, 0, n, surf=S)
    return T, S


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_equals_forward_two_calls_second_smaller(dtype):
    import torch

    import paper_1408_5853_amd as P
    # the first cell's workspace (66 MiB) nearly fills the array
    big = cellgen.device_cell(0, z_active=True)
    small = cellgen.small_cell(1, z_active=True)
    for c, n in ((big, 60), (small, 250)):
        say("noalloc %s nr=%d nz=%d steps=%d" % (dtype, c["nr"], c["nz"], n))
        plan = P.Plan(c, dtype)
        T1, S1 = _reference(P, plan, n)          # also makes the plan's device tables
        T2, S2 = _noalloc(P, plan, n)
        torch.cuda.synchronize()
        assert torch.equal(T1, T2)
        assert torch.equal(S1, S2)
        assert np.all(np.isfinite(plan.field_values(T2)))


def test_noalloc_refusals():
    import paper_1408_5853_amd as P
    lib = P._abi.lib()
    dc = cellgen.device_cell(0)
    huge = cellgen.scaled(cellgen.with_nz(dc, 8192), height=2 * dc["height"])
    plan = P.Plan(huge, "f64")
    assert plan.workspace_bytes(0) > (72 << 20)
    T = plan.init()
    st = lib.cryo_forward_noalloc(plan._h, P._ptr(T), 0, 1, None, P._stream(None))
    assert st == 5, lib.cryo_last_error()                     # CRYO_ERR_WORKSPACE
    fresh = P.Plan(cellgen.small_cell(0), "f64")               # no device tables yet
    T = fresh.init()
    st = lib.cryo_forward_noalloc(fresh._h, P._ptr(T), 0, 1, None, P._stream(None))
    assert st == 1, lib.cryo_last_error()                     # CRYO_ERR_ARG
