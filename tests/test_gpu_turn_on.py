"""Parity of the transient turn-on model (Sec. 3.2, eq. (22)) on the GPU with
the FP64 CPU oracle.

Each pulse-start step runs as 100 sub-steps of dt/100 through a second set of
step tables; FP64 must agree to 1e-10 relative and FP32 to 1e-4 K, on the
field and on the per-step surface trace, over runs that cross several pulse
starts, with a gate shorter than a step, under a non-default launch shape,
and on the cold-start cell of the paper's Fig. 3.
"""
import numpy as np
import pytest

import cellgen
import oracle
from gpu_util import rel_err, run_gpu, say
from test_oracle_pins import fig3_cell

pytestmark = pytest.mark.gpu

F64_TOL = 1e-10
F32_TOL_K = 1e-4


def _pulsed(seed, nz, z_active, width_steps=5.0):
    c = cellgen.with_nz(cellgen.small_cell(seed, z_active=z_active), nz)
    dt = c["dt"]
    c.update(t_on=3 * dt, width=width_steps * dt, period=20 * dt, turn_on=True,
             amplitude=3 * c["amplitude"])
    return c


def _check64(c, nsteps, k0=0):
    say("case turn-on nr=%d nz=%d steps=%d k0=%d width=%.3g dt" %
        (c["nr"], c["nz"], nsteps, k0, c["width"] / c["dt"]))
    Tg, Sg = run_gpu(c, nsteps, k0=k0)
    To, So = oracle.forward(c, k0=k0, nsteps=nsteps, surf=True)
    e, es = rel_err(Tg, To), rel_err(Sg, So)
    say("  max rel err field %.3e surface %.3e" % (e, es))
    assert e < F64_TOL and es < F64_TOL
    return Tg, To, Sg


@pytest.mark.parametrize("seed,nz,z_active", [(0, 4, False), (1, 9, True), (3, 6, True)])
def test_turn_on_matches_oracle_f64(seed, nz, z_active):
    c = _pulsed(seed, nz, z_active)
    Tg, To, _ = _check64(c, 60)              # pulse starts at steps 3, 23, 43
    off = oracle.forward(dict(c, turn_on=False), nsteps=60)
    assert rel_err(off, To) > 1e-6           # the model changed the result


def test_turn_on_gate_shorter_than_a_step_f64():
    _check64(_pulsed(2, 5, True, width_steps=0.375), 45, k0=1)


def test_turn_on_f32():
    c = _pulsed(1, 7, True)
    say("case turn-on f32 nr=%d nz=%d" % (c["nr"], c["nz"]))
    Tg, Sg = run_gpu(c, 60, dtype="f32")
    To, So = oracle.forward(c, nsteps=60, surf=True)
    e, es = np.max(np.abs(Tg - To)), np.max(np.abs(Sg - So))
    say("  max abs err field %.3e K surface %.3e K" % (e, es))
    assert e < F32_TOL_K and es < F32_TOL_K


def test_turn_on_follows_launch_shape():
    import torch

    import paper_1408_5853_amd as P
    c = _pulsed(4, 6, True)
    plan = P.Plan(c)
    plan.set_shape(4, 2, 2)
    say("case turn-on shape", plan.shape())
    T = plan.init()
    ws = plan.workspace(40)
    S = torch.zeros(40, dtype=torch.float64, device="cuda")
    plan.forward(T, 0, 40, ws=ws, surf=S)
    plan.poll(ws)
    torch.cuda.synchronize()
    To, So = oracle.forward(c, nsteps=40, surf=True)
    assert rel_err(plan.field_values(T), To) < F64_TOL
    assert rel_err(S.cpu().numpy(), So) < F64_TOL


@pytest.mark.parametrize("mult", [20, 100])
def test_turn_on_fig3_cold_start(mult):
    c = fig3_cell(mult, True)
    n = int(round(1e-3 / c["dt"]))
    say("case fig3 cold start, steps of %d us, %d steps" % (mult, n))
    Tg, Sg = run_gpu(c, n)
    To, So = oracle.forward(c, nsteps=n, surf=True)
    assert rel_err(Tg, To) < F64_TOL and rel_err(Sg, So) < F64_TOL
    assert np.all(np.diff(Sg) >= 0)         # heating without the start jump
