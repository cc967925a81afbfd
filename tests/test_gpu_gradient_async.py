"""The stream-ordered gradient (device target, J, grad and trace; no host
wait): bit for bit the host entry point's results, within the oracle
adjoint's tolerance, with the turn-on model and a stepped domain, and
replayed from a captured HIP graph."""
import numpy as np
import pytest

import cellgen
import oracle
from gpu_util import say

pytestmark = pytest.mark.gpu


def _norm_err(g, ref, theta):
    P = np.abs(theta)
    return float(np.max(np.abs(g - ref) * P / np.max(np.abs(ref * P))))


def _case(kind):
    c = cellgen.tiny(31, nr=140, nz=9, n_layers=3, nsteps=40, z_active=True, dt=2e-6,
                     amplitude=4e9, heater=2)
    dt = c["dt"]
    if kind in ("turn_on", "both"):
        c.update(t_on=3 * dt, period=20 * dt, width=4.6 * dt, turn_on=True)
    if kind in ("stepped", "both"):
        c["stepped"] = dict(z_full=5, nr_top=90)
    _, S = oracle.forward(c, nsteps=40, surf=True)
    tgt = S + np.random.default_rng(2).normal(scale=0.05, size=40) + 0.02
    return c, tgt


@pytest.mark.parametrize("kind", ["plain", "turn_on", "stepped", "both"])
def test_async_gradient_equals_host_call_and_oracle(kind):
    import torch

    import paper_1408_5853_amd as P
    c, tgt = _case(kind)
    say("case gradient_async %s" % kind)
    plan = P.gradient_plan(c)
    J0, g0, S0 = plan.gradient(tgt, ckpt=6)
    T0 = plan.init()
    td = torch.tensor(tgt, dtype=torch.float64, device="cuda")
    J, g, S, ws = plan.gradient_async(td, T0, ckpt=6)
    plan.poll(ws)
    J, g, S = J.item(), g.cpu().numpy(), S.cpu().numpy()
    assert J == J0 and np.array_equal(g, g0) and np.array_equal(S, S0)
    Jo, go, So = oracle.gradient(c, tgt)
    assert J == pytest.approx(Jo, rel=1e-9)
    assert np.max(np.abs(S - So) / So) < 1e-10
    e = _norm_err(g, go, P.params_of(c))
    say("  normalised gradient error %.3e" % e)
    assert e < 1e-8, (g, go)


@pytest.mark.parametrize("store", [0, 17, 40])
def test_async_gradient_replays_from_a_graph(store):
    # the whole gradient captured once and replayed three times, with other
    # device work and host synchronisation between the replays; every replay
    # against the eager call, bit for bit; with checkpoints only, with part
    # of the run's states stored and with all of them
    import torch

    import paper_1408_5853_amd as P
    c, tgt = _case("plain")
    plan = P.gradient_plan(c)
    plan.set_gradient_store(store)
    T0 = plan.init()
    td = torch.tensor(tgt, dtype=torch.float64, device="cuda")
    ws = torch.empty(plan.gradient_workspace_bytes(40, 6), dtype=torch.uint8, device="cuda")
    J0, g0, S0, _ = plan.gradient_async(td, T0, ckpt=6, ws=ws)
    torch.cuda.synchronize()
    ref = (J0.item(), g0.cpu().numpy(), S0.cpu().numpy())
    other = P.gradient_plan(_case("stepped")[0])
    To = other.init()
    wo = other.workspace(50)
    say("case gradient_async graph capture, store %d" % store)
    gr = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(gr, stream=s):
            J, g, S, _ = plan.gradient_async(td, T0, ckpt=6, ws=ws)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        # clobber the outputs and the workspace's gradient areas first
        J.fill_(-1.0)
        g.fill_(-1.0)
        S.fill_(-1.0)
        ws.fill_(7)
        other.forward(To, 0, 50, ws=wo)
        torch.cuda.synchronize()
        gr.replay()
        torch.cuda.synchronize()
        plan.poll(ws)
        assert J.item() == ref[0], rep
        assert np.array_equal(g.cpu().numpy(), ref[1]), rep
        assert np.array_equal(S.cpu().numpy(), ref[2]), rep
    say("  3 replays equal to the eager call")


def test_async_gradient_refuses_bad_arguments():
    import torch

    import paper_1408_5853_amd as P
    c, tgt = _case("plain")
    plan = P.gradient_plan(c)
    T0 = plan.init()
    td = torch.tensor(tgt, dtype=torch.float64, device="cuda")
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(P.CryoError):
        plan.gradient_async(td, T0, ckpt=6, ws=small)
    f32 = P.Plan(c, "f32")
    with pytest.raises(P.CryoError):
        f32.gradient_async(td, f32.init(), ckpt=6)
