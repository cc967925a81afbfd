"""The gradient store: the states of a run's last kernel steps kept from the
gradient's forward, so that only the steps before them are checkpointed and
recomputed.  The store changes where states live, not how they are computed:
J, the gradient and the surface trace must equal those of the checkpoints-only
sweep bit for bit for every store and checkpoint interval (with the turn-on
model's sub-steps, a stepped domain and the polynomial laws), through the
synchronous, stream-ordered and many-design calls, and at the adjoint
workload's full size; one case is also held against the oracle adjoint."""
import numpy as np
import pytest

import cellgen
import oracle
from gpu_util import say

pytestmark = pytest.mark.gpu


def _target(cell, n, T0=None):
    _, S = oracle.forward(cell, T0, nsteps=n, surf=True)
    rng = np.random.default_rng(1)
    return S + rng.normal(scale=0.05, size=n) + 0.02


def _same(a, b):
    Ja, ga, Sa = a
    Jb, gb, Sb = b
    return Ja == Jb and np.array_equal(ga, gb) and np.array_equal(Sa, Sb)


def _sweep(c, tgt, stores, ckpts, shape=None, T0=None):
    import paper_1408_5853_amd as P
    plan = P.Plan(c)
    if shape:
        plan.set_shape(*shape)
    ref = plan.gradient(tgt, T0=T0, ckpt=0, store=0)
    for ck in ckpts:
        for st in stores:
            say("  store=%d ckpt=%d" % (st, ck))
            got = plan.gradient(tgt, T0=T0, ckpt=ck, store=st)
            assert _same(got, ref), (st, ck)
    return ref


def test_store_equals_checkpoints_bitwise_and_oracle():
    import paper_1408_5853_amd as P
    c = cellgen.tiny(11, nr=40, nz=7, n_layers=3, nsteps=30, z_active=True, dt=2e-6,
                     amplitude=4e9, heater=2)
    tgt = _target(c, 30)
    say("case gradient store nr=40 nz=7 30 steps")
    # no store, one stored step, a tail cut inside a segment, all but one,
    # all, and more than the run has
    J, g, S = _sweep(c, tgt, [0, 1, 13, 29, 30, 10 ** 6], [0, 1, 7, 30])
    Jo, go, So = oracle.gradient(c, tgt)
    assert J == pytest.approx(Jo, rel=1e-9)
    assert np.max(np.abs(S - So) / So) < 1e-10
    sc = np.max(np.abs(go * P.params_of(c)))
    assert np.max(np.abs(g - go) * np.abs(P.params_of(c))) / sc < 1e-8


@pytest.mark.parametrize("shape", [None, (4, 2, 1), (8, 1, 2)])
def test_store_with_turn_on_sub_steps(shape):
    # 30 steps with two pulse starts make 228 kernel steps; stores that end
    # inside the first and the second start's sub-steps, and at a step edge
    c = cellgen.tiny(12, nr=40, nz=7, n_layers=3, nsteps=30, z_active=True, dt=2e-6,
                     amplitude=4e9, heater=2)
    dt = c["dt"]
    c.update(t_on=3 * dt, period=20 * dt, width=4.6 * dt, turn_on=True)
    tgt = _target(c, 30)
    say("case gradient store turn-on shape=%s" % (shape,))
    _sweep(c, tgt, [40, 107, 150, 227, 228], [0, 9], shape=shape)


def test_store_with_stepped_domain_and_polynomial_laws():
    c = cellgen.tiny(13, nr=40, nz=9, n_layers=3, nsteps=24, z_active=True, dt=2e-6,
                     amplitude=4e9, heater=2)
    c["stepped"] = dict(z_full=5, nr_top=30)
    rng = np.random.default_rng(13)
    T0 = 28.0 + rng.uniform(0, 3, size=(9, 40))
    tgt = _target(c, 24, T0)
    say("case gradient store stepped")
    _sweep(c, tgt, [5, 24], [0, 6], T0=T0)
    p = cellgen.poly_variant(cellgen.tiny(14, nr=300, nz=9, n_layers=3, nsteps=30, z_active=True,
                                          dt=2e-6, amplitude=4e9, heater=2), 14, joule_tref=30.0)
    tgt = _target(p, 30)
    say("case gradient store poly + Joule")
    _sweep(p, tgt, [11, 30], [0, 7])


def test_store_async_and_many():
    import torch

    import paper_1408_5853_amd as P
    cells = [cellgen.tiny(15 + i, nr=64 * (i + 1), nz=8, n_layers=3, nsteps=40, z_active=True,
                          dt=2e-6, amplitude=4e9, heater=2) for i in range(3)]
    tgs = [_target(c, 40) for c in cells]
    refs = [P.gradient(c, t, ckpt=6) for c, t in zip(cells, tgs)]
    say("case gradient store async")
    plan = P.gradient_plan(cells[0])
    T0 = plan.init()
    td = torch.tensor(tgs[0], dtype=torch.float64, device="cuda")
    for st in (0, 17, 40):
        J, g, S, ws = plan.gradient_async(td, T0, ckpt=6, store=st)
        torch.cuda.synchronize()
        plan.poll(ws)
        assert _same((float(J.item()), g.cpu().numpy(), S.cpu().numpy()), refs[0]), st
    say("case gradient store many")
    J, grads, surfs = P.gradient_many(cells, tgs, ckpt=6, streams=2, store=[40, 0, 23])
    for i in range(3):
        assert _same((J[i], grads[i], surfs[i]), refs[i]), i


def test_store_full_size_adjoint_cell():
    # the adjoint workload's grid (512 x 2048) over a 1,200-step prefix: half
    # the steps stored, and all of them
    import paper_1408_5853_amd as P
    c = cellgen.adjoint_cell(0)
    n = 1200
    tgt = cellgen.tracking_target(c, n)
    say("case gradient store adjoint cell 512x2048, %d steps" % n)
    plan = P.gradient_plan(c)
    ref = plan.gradient(tgt, nsteps=n, store=0)
    assert np.all(np.isfinite(ref[1]))
    for st in (600, n):
        assert _same(plan.gradient(tgt, nsteps=n, store=st), ref), st
