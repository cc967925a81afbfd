"""The resident state (cryo_state_*): the field kept in the kernels' internal
layout between calls gives the same fields and surface traces, bit for bit,
as single cryo_forward calls over the same steps, for FP64 and FP32 pairs,
with the turn-on model's sub-steps inside a call, and reports a non-finite
field through cryo_poll on its memory."""
import numpy as np
import pytest

import cellgen
from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("make", ["small_z_active", "tiny_ragged", "turn_on"])
def test_state_calls_equal_one_forward(dtype, make):
    import torch

    import paper_1408_5853_amd as P
    if make == "small_z_active":
        c, splits = cellgen.small_cell(1, z_active=True), [1, 7, 300, 2, 1100]
    elif make == "tiny_ragged":
        c = cellgen.tiny(3, nr=333, nz=9, n_layers=4, nsteps=60, z_active=True, dt=2e-7,
                         amplitude=5e9)
        splits = [3, 1, 1, 40, 15]
    else:
        c = cellgen.with_nz(cellgen.small_cell(2), 12)
        c.update(turn_on=True, period=20 * c["dt"], width=5 * c["dt"], t_on=3 * c["dt"])
        splits = [2, 2, 19, 21, 40]
    n = sum(splits)
    say("case %s %s nr=%d nz=%d steps=%s" % (make, dtype, c["nr"], c["nz"], splits))
    plan = P.Plan(c, dtype)
    T = plan.init()
    S1 = torch.zeros(n, dtype=torch.float64, device="cuda")
    plan.forward(T, 0, n, surf=S1)
    st = P.State(plan, plan.init())
    S2 = torch.zeros(n, dtype=torch.float64, device="cuda")
    k = 0
    for m in splits:
        st.forward(k, m, surf=S2[k:])
        k += m
    T2 = st.store()
    st.poll()
    torch.cuda.synchronize()
    assert torch.equal(T, T2)
    assert torch.equal(S1, S2)
    # store is repeatable and leaves the state as it was
    T3 = st.store()
    st.forward(k, 5)
    plan.forward(T3, k, 5)
    assert torch.equal(st.store(), T3)


def test_state_reload_and_nonfinite_flag():
    import torch

    import paper_1408_5853_amd as P
    c = cellgen.tiny(4, nr=70, nz=5, n_layers=3, nsteps=10, z_active=True, dt=2e-7)
    plan = P.Plan(c, "f64")
    st = P.State(plan, plan.init())
    st.forward(0, 10)
    st.poll()
    bad = plan.init()
    bad[2, 7] = float("nan")
    st.load(bad)
    st.forward(10, 3)
    with pytest.raises(P.CryoError) as e:
        st.poll()
    assert e.value.status == 4
    st.load(plan.init())                     # a load clears the error word
    st.forward(0, 3)
    st.poll()
    T = plan.init()
    plan.forward(T, 0, 3)
    torch.cuda.synchronize()
    assert torch.equal(st.store(), T)
