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


def _batch_cells():
    # instances with their own dt and pulse: turn-on model with starts at
    # steps 3, 73, 143 and at 40, on a plain cell; the model with the
    # polynomial laws and a stepped domain; one instance without it (its
    # pulse still starts at step 3); two radial sizes (two launch groups)
    def pulsed(c, t_on, period, width, on=True):
        dt = c["dt"]
        c = dict(c, t_on=t_on * dt, period=period * dt, width=width * dt,
                 amplitude=3 * c["amplitude"])
        if on:
            c["turn_on"] = True
        return c
    a = pulsed(cellgen.with_nz(cellgen.small_cell(0, z_active=True), 24), 3, 70, 5.0)
    b = pulsed(cellgen.with_nz(cellgen.small_cell(1, z_active=True), 20), 40, 1000, 0.37)
    p = pulsed(cellgen.poly_variant(cellgen.with_nz(cellgen.small_cell(2, z_active=True), 30), 2,
                                    joule_tref=30.0), 3, 70, 4.6)
    p["stepped"] = {"z_full": 18, "nr_top": 40}
    plain = pulsed(cellgen.with_nz(cellgen.small_cell(3, z_active=True), 16), 3, 70, 5.0, on=False)
    big = pulsed(cellgen.tiny(4, nr=200, nz=12, n_layers=3, z_active=True, dt=2e-6,
                              amplitude=4e9, heater=2), 40, 1000, 2.5)
    return [a, b, p, plain, big]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("k0,n", [(2, 150), (0, 75)])
def test_batch_with_turn_on_instances(dtype, k0, n):
    # the batch splits its step range at the pulse starts of its turn-on
    # instances (captured blocks and single steps between them, from either
    # buffer): every instance equals a single plan with the same shape and
    # options bit for bit, and the oracle within the tolerances
    import torch

    import paper_1408_5853_amd as P
    cells = _batch_cells()
    say("case batch with turn-on instances %s k0=%d steps=%d" % (dtype, k0, n))
    b = P.Batch(cells, dtype)
    T = b.init()
    ws = b.workspace()
    b.forward(T, k0, n, ws)
    b.poll(ws)
    torch.cuda.synchronize()
    for i, c in enumerate(cells):
        got = P.Plan.field_values(b.field(T, i))
        plan = P.Plan(c, dtype)
        plan.set_shape(*b.shape(i))
        Ts = plan.init()
        plan.forward(Ts, k0, n)
        torch.cuda.synchronize()
        assert np.array_equal(got, plan.field_values(Ts)), i
        To = oracle.forward(c, k0=k0, nsteps=n)
        if dtype == "f64":
            assert rel_err(got, To) < F64_TOL, i
        else:
            assert np.max(np.abs(got - To)) < F32_TOL_K, i
