"""The concurrent design loop (many gradients in one call) against single
gradient calls (bit for bit), against the oracle adjoint on small designs and,
at full size (64 designs' shape: 512 x 1024 nodes), against the oracle on
the exactly z-invariant reduction; and the first Adam step of the design loop
descends."""
import numpy as np
import pytest

import cellgen
import oracle
from gpu_util import say

pytestmark = pytest.mark.gpu


def _norm_err(g, ref, theta):
    P = np.abs(theta)
    scale = np.max(np.abs(ref * P))
    return float(np.max(np.abs(g - ref) * P / scale))


def _small_designs(n, nsteps):
    out = []
    for i in range(n):
        L = 3 + (i % 3)
        # heater in the outer layer: the surface sees the pulse within the run
        c = cellgen.tiny(20 + i, nr=40 + 57 * i, nz=5 + (i % 3), n_layers=L,
                         nsteps=nsteps, z_active=bool(i % 2), dt=2e-6, amplitude=3e9 + 5e8 * i,
                         heater=L - 1)
        out.append(c)
    return out


def _targets(cells, n):
    return [cellgen.tracking_target(c, n) for c in cells]


def test_gradient_many_equals_single_calls_bitwise():
    import paper_1408_5853_amd as P
    cells = _small_designs(5, 24)
    tg = _targets(cells, 24)
    say("case gradient_many 5 designs, 3 streams")
    J, grads, surfs = P.gradient_many(cells, tg, ckpt=5, streams=3)
    for i, c in enumerate(cells):
        Ji, gi, Si = P.gradient(c, tg[i], ckpt=5)
        assert J[i] == Ji
        assert np.array_equal(grads[i], gi)
        assert np.array_equal(surfs[i], Si)


@pytest.mark.parametrize("shared,store,streams", [(1, 0, 0), (2, 24, 0), (2, [24, 0, 7, 24, 3], 4),
                                                  (3, 10, 2)])
def test_gradient_many_shared_workspaces_bitwise(shared, store, streams):
    # designs sharing a workspace run one after another on one stream (with
    # or without gradient stores, mixed per design); every result equals the
    # single call's bit for bit
    import paper_1408_5853_amd as P
    cells = _small_designs(5, 24)
    tg = _targets(cells, 24)
    say("case gradient_many shared=%d store=%s streams=%d" % (shared, store, streams))
    J, grads, surfs = P.gradient_many(cells, tg, ckpt=5, streams=streams, store=store,
                                      shared=shared)
    for i, c in enumerate(cells):
        Ji, gi, Si = P.gradient(c, tg[i], ckpt=5)
        assert J[i] == Ji, i
        assert np.array_equal(grads[i], gi), i
        assert np.array_equal(surfs[i], Si), i


@pytest.mark.parametrize("streams", [0, 1, 4])
def test_gradient_many_matches_oracle_adjoint(streams):
    import paper_1408_5853_amd as P
    cells = _small_designs(3, 20)
    tg = _targets(cells, 20)
    say("case gradient_many vs oracle, streams %d" % streams)
    J, grads, _ = P.gradient_many(cells, tg, streams=streams)
    for i, c in enumerate(cells):
        Jo, go, _ = oracle.gradient(c, tg[i])
        assert J[i] == pytest.approx(Jo, rel=1e-9)
        e = _norm_err(grads[i], go, P.params_of(c))
        say("  design %d normalised gradient error %.3e" % (i, e))
        assert e < 1e-8


def test_design_cells_full_size_against_reduced_oracle():
    # two of the 64 designs at full size (512 x 1024 nodes), 400 steps; the
    # designs are exactly z-invariant, so J and its gradient equal those of
    # the 4-line reduction.  Designs 0 and 9: their surfaces respond within
    # 400 steps (in several others the pulse has not reached the surface yet
    # and the gradient is zero up to rounding)
    import paper_1408_5853_amd as P
    allc = cellgen.design_cells(0, n_designs=10, nsteps=400)
    cells = [allc[0], allc[9]]
    n = 400
    tg = _targets(cells, n)
    say("case design cells 2 x 512x1024, %d steps" % n)
    J, grads, _ = P.gradient_many(cells, tg, streams=2)
    for i, c in enumerate(cells):
        Jo, go, _ = oracle.gradient(cellgen.with_nz(c, 4), tg[i])
        e = _norm_err(grads[i], go, P.params_of(c))
        say("  design %d J gpu %.12e oracle %.12e, gradient error %.3e" % (i, J[i], Jo, e))
        assert J[i] == pytest.approx(Jo, rel=1e-9)
        assert e < 1e-6


def test_design_adam_first_step_descends():
    from paper_1408_5853_amd.design import design_adam, design_params
    cells = _small_designs(3, 30)
    tg = [t + 3.0 for t in _targets(cells, 30)]          # reachable by more heat
    say("case design loop, 1 Adam step, lr 0.01")
    new, hist = design_adam(cells, tg, iters=1, lr=0.01, streams=2)
    assert hist.shape == (2, 3)
    for i in range(3):
        say("  design %d J %.6e -> %.6e" % (i, hist[0, i], hist[1, i]))
        assert hist[1, i] < hist[0, i]
        ratio = design_params(new[i]) / design_params(cells[i])
        assert np.all(np.abs(np.log(ratio)) <= 0.0101)   # Adam steps at most lr


def test_gradient_many_with_turn_on_and_stepped_plans_bitwise():
    # designs with the turn-on model's sub-steps and with a stepped domain
    # in one call: each run keeps its own kernel-step list and tables
    import paper_1408_5853_amd as P
    cells = []
    for i in range(4):
        c = cellgen.tiny(30 + i, nr=24, nz=8, n_layers=3, nsteps=24, z_active=True, dt=2e-6,
                         amplitude=4e9, heater=2)
        dt = c["dt"]
        if i % 2 == 0:
            c.update(t_on=3 * dt, period=20 * dt, width=4.6 * dt, turn_on=True)
        if i >= 2:
            c["stepped"] = dict(z_full=4, nr_top=15)
        cells.append(c)
    tg = _targets(cells, 24)
    say("case gradient_many, turn-on and stepped designs")
    J, grads, surfs = P.gradient_many(cells, tg, ckpt=6, streams=2)
    for i, c in enumerate(cells):
        Ji, gi, Si = P.gradient(c, tg[i], ckpt=6)
        assert J[i] == Ji and np.array_equal(grads[i], gi) and np.array_equal(surfs[i], Si)
    Jo, go, _ = oracle.gradient(cells[3], tg[3])
    assert J[3] == pytest.approx(Jo, rel=1e-9)
    assert _norm_err(grads[3], go, P.params_of(cells[3])) < 1e-8


def test_gradient_many_names_the_design_with_a_nonfinite_field():
    # three designs on one shared workspace, the middle one started from a
    # field with a NaN: the error names it, although the design after it
    # reuses (and clears) the workspace's error word
    import paper_1408_5853_amd as P
    cells = _small_designs(3, 12)
    tg = _targets(cells, 12)
    bad = np.full((cells[1]["nz"], cells[1]["nr"]), 28.0)
    bad[1, 3] = np.nan
    say("case gradient_many shared workspace, design 1 non-finite")
    with pytest.raises(P.CryoError) as e:
        P.gradient_many(cells, tg, ckpt=4, shared=1, T0s=[None, bad, None])
    assert e.value.status == 4 and "design 1" in str(e.value)
