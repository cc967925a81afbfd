"""The GPU discrete adjoint against the oracle adjoint (itself pinned by
finite differences of the oracle forward), finite differences of the GPU
forward, checkpoint invariance, the autograd boundary, and the full-size
adjoint workload (512 x 2048, 50,000 steps) against the oracle on its
exactly z-invariant reduction."""
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


def _target(cell, n):
    _, S = oracle.forward(cell, nsteps=n, surf=True)
    rng = np.random.default_rng(0)
    return S + rng.normal(scale=0.05, size=n) + 0.02


@pytest.mark.parametrize("seed,nr,nz,zact", [(0, 14, 6, True), (1, 40, 9, True),
                                              (2, 100, 5, False), (3, 300, 7, True)])
def test_gpu_gradient_matches_oracle_adjoint(seed, nr, nz, zact):
    import paper_1408_5853_amd as P
    c = cellgen.tiny(seed, nr=nr, nz=nz, n_layers=3, nsteps=30, z_active=zact, dt=2e-6,
                     amplitude=4e9, heater=2)
    n = c["nsteps"]
    tgt = _target(c, n)
    say("case adjoint nr=%d nz=%d" % (nr, nz))
    Jo, go, So = oracle.gradient(c, tgt)
    Jg, gg, Sg = P.gradient(c, tgt, ckpt=7)
    assert Jg == pytest.approx(Jo, rel=1e-9)
    assert np.max(np.abs(Sg - So) / So) < 1e-10
    e = _norm_err(gg, go, P.params_of(c))
    say("  normalised gradient error %.3e" % e)
    assert e < 1e-8, (gg, go)


def test_gpu_gradient_every_chunk_shape_and_checkpoint_stride():
    import paper_1408_5853_amd as P
    c = cellgen.tiny(5, nr=200, nz=6, n_layers=4, nsteps=25, z_active=True, dt=2e-6,
                     amplitude=4e9, heater=3)
    tgt = _target(c, 25)
    ref = None
    for shape in [(4, 1, 1), (4, 2, 1), (8, 1, 2), (4, 4, 3)]:
        for ck in (1, 6, 0):
            plan = P.Plan(c)
            plan.set_shape(*shape)
            J, g, _ = plan.gradient(tgt, ckpt=ck)
            if ref is None:
                ref = (J, g)
            assert J == pytest.approx(ref[0], rel=1e-12)
            assert _norm_err(g, ref[1], P.params_of(c)) < 1e-11


def test_gpu_gradient_central_differences():
    import paper_1408_5853_amd as P
    c = cellgen.tiny(6, nr=64, nz=6, n_layers=3, nsteps=40, z_active=True, dt=2e-6,
                     amplitude=4e9, heater=2)
    tgt = _target(c, 40)
    J, g, _ = P.gradient(c, tgt)
    th = P.params_of(c)
    fd = np.zeros_like(g)
    for q in range(len(th)):
        h = 1e-4 * abs(th[q])
        f = []
        for k in (1, -1, 2, -2):
            t2 = th.copy()
            t2[q] += k * h
            Jk, _, _ = P.gradient(P.with_params(c, t2), tgt)
            f.append(Jk)
        fd[q] = (8 * (f[0] - f[1]) - (f[2] - f[3])) / (12 * h)
    assert _norm_err(g, fd, th) < 1e-6


def test_autograd_function_returns_adjoint_gradient():
    import torch

    import paper_1408_5853_amd as P
    c = cellgen.tiny(7, nr=50, nz=5, n_layers=3, nsteps=20, z_active=True, dt=2e-6,
                     amplitude=4e9, heater=2)
    tgt = _target(c, 20)
    theta = torch.tensor(P.params_of(c), dtype=torch.float64, requires_grad=True)
    J = P.CryoSolve.apply(theta, c, tgt, 20, 0)
    J.backward()
    Jr, gr, _ = P.gradient(c, tgt)
    assert float(J) == pytest.approx(Jr, rel=1e-14)
    assert np.allclose(theta.grad.numpy(), gr, rtol=1e-14, atol=0)
    # with every state stored: the same J and gradient bit for bit
    th2 = torch.tensor(P.params_of(c), dtype=torch.float64, requires_grad=True)
    J2 = P.CryoSolve.apply(th2, c, tgt, 20, 0, 20)
    J2.backward()
    assert float(J2) == float(J) and torch.equal(th2.grad, theta.grad)


@pytest.fixture(scope="module")
def adjoint_workload():
    # 512 x 2048 nodes, 6 layers, 50,000 steps; the cell is exactly
    # z-invariant, so J and its gradient equal those of the 4-line reduction
    import paper_1408_5853_amd as P
    c = cellgen.adjoint_cell(0)
    n = c["nsteps"]
    tgt = cellgen.tracking_target(c, n)
    say("case adjoint workload 512x2048, %d steps" % n)
    Jg, gg, _ = P.gradient(c, tgt)
    Jo, go, _ = oracle.gradient(cellgen.with_nz(c, 4), tgt, ckpt=250)
    return c, tgt, Jg, gg, Jo, go


def test_adjoint_workload_full_size_against_reduced_oracle(adjoint_workload):
    import paper_1408_5853_amd as P
    c, _, Jg, gg, Jo, go = adjoint_workload
    e = _norm_err(gg, go, P.params_of(c))
    say("  J gpu %.12e oracle %.12e, normalised gradient error %.3e" % (Jg, Jo, e))
    assert Jg == pytest.approx(Jo, rel=1e-9)
    assert e < 1e-6


# components whose log-sensitivity |g theta| is at least this fraction of the
# largest must match the oracle adjoint to 1e-6 relative, each on its own
SENS_FLOOR = 1e-3


def test_adjoint_workload_per_component(adjoint_workload):
    """Per-component bounds: 1e-6 relative for every component whose
    log-sensitivity is at least SENS_FLOOR of the largest; below the floor
    (sensitivities the objective barely feels) the error, scaled as a
    log-sensitivity, must stay below 1e-9 of the largest log-sensitivity,
    which is a relative bound of 1e-9 / (its fraction of the largest)."""
    import paper_1408_5853_amd as P
    c, _, _, gg, _, go = adjoint_workload
    th = np.abs(P.params_of(c))
    ls = np.abs(go * th)
    frac = ls / ls.max()
    rel = np.abs(gg - go) / np.abs(go)
    scaled = np.abs(gg - go) * th / ls.max()
    for q in range(len(th)):
        say("  theta[%d] log-sensitivity fraction %.2e, relative error %.2e" % (q, frac[q], rel[q]))
    big = frac >= SENS_FLOOR
    assert big.sum() >= 8
    assert np.all(rel[big] < 1e-6), rel[big]
    assert np.all(scaled[~big] < 1e-9), scaled[~big]


def test_adjoint_workload_central_differences(adjoint_workload):
    """Central differences of the GPU forward's J (h = 1e-6 relative, one
    component at a time) on the components whose log-sensitivity is at
    least 1e-2 of the largest: there the difference quotient is accurate to
    about 1e-7 (the rounding of J over 50,000 steps against a 2e-6 change)."""
    import torch

    import paper_1408_5853_amd as P
    c, tgt, _, gg, _, _ = adjoint_workload
    n = c["nsteps"]
    th = P.params_of(c)
    ls = np.abs(gg * th)
    sh = P._gradient_shape(c)

    def J_of(theta):
        cc = P.with_params(c, theta)
        plan = P.Plan(cc, "f64")
        plan.set_shape(*sh)
        st = P.State(plan, plan.init())
        S = torch.zeros(n, dtype=torch.float64, device="cuda")
        st.forward(0, n, surf=S)
        st.poll()
        return float(np.sum((S.cpu().numpy() - tgt) ** 2))

    picked = [q for q in range(len(th)) if ls[q] >= 1e-2 * ls.max()]
    assert len(picked) >= 4
    for q in picked:
        h = 1e-6 * abs(th[q])
        tp, tm = th.copy(), th.copy()
        tp[q] += h
        tm[q] -= h
        fd = (J_of(tp) - J_of(tm)) / (2 * h)
        e = abs(fd - gg[q]) / abs(gg[q])
        say("  theta[%d] adjoint %.10e central difference %.10e, relative %.2e" % (q, gg[q], fd, e))
        assert e < 1e-5


@pytest.mark.parametrize("shape", [(4, 1, 1), (8, 1, 2), (4, 2, 1)])
def test_gpu_gradient_general_power_laws(shape):
    """Capacity exponents other than 3 (the general power path of both
    adjoint passes) and conductivity exponents far apart across layers."""
    import paper_1408_5853_amd as P
    c = cellgen.tiny(9, nr=120, nz=7, n_layers=3, nsteps=25, z_active=True, dt=2e-6,
                     amplitude=4e9, heater=2)
    for m, (q, p) in enumerate([(2.0, -1.5), (3.5, 2.5), (1.5, 0.3)]):
        c["layers"][m]["q"] = q
        c["layers"][m]["p"] = p
    tgt = _target(c, c["nsteps"])
    say("case adjoint general laws shape %s" % (shape,))
    Jo, go, _ = oracle.gradient(c, tgt)
    plan = P.Plan(c)
    plan.set_shape(*shape)
    Jg, gg, _ = plan.gradient(tgt, ckpt=6)
    assert Jg == pytest.approx(Jo, rel=1e-9)
    e = _norm_err(gg, go, P.params_of(c))
    say("  normalised gradient error %.3e" % e)
    assert e < 1e-8, (gg, go)


@pytest.mark.parametrize("seed,w_steps,ckpt,shape", [(0, 7.3, 7, None), (1, 0.374, 0, (4, 2, 1)),
                                                     (2, 4.6, 60, (8, 1, 2))])
def test_gpu_gradient_turn_on_matches_oracle_adjoint(seed, w_steps, ckpt, shape):
    # the turn-on model's sub-steps (eq. (22)) inside the checkpointed sweep:
    # pulse ends inside a regular step and inside a sub-step, fused passes
    # with one and with two lines per group, segments cut inside sub-steps
    import paper_1408_5853_amd as P
    c = cellgen.tiny(seed, nr=40, nz=7, n_layers=3, nsteps=30, z_active=True, dt=2e-6,
                     amplitude=4e9, heater=2)
    dt = c["dt"]
    c.update(t_on=3 * dt, period=20 * dt, width=w_steps * dt, turn_on=True)
    tgt = _target(c, 30)
    say("case adjoint turn-on width=%g dt ckpt=%d shape=%s" % (w_steps, ckpt, shape))
    Jo, go, So = oracle.gradient(c, tgt)
    plan = P.Plan(c)
    if shape:
        plan.set_shape(*shape)
    Jg, gg, Sg = plan.gradient(tgt, ckpt=ckpt)
    assert Jg == pytest.approx(Jo, rel=1e-9)
    assert np.max(np.abs(Sg - So) / So) < 1e-10
    e = _norm_err(gg, go, P.params_of(c))
    say("  normalised gradient error %.3e" % e)
    assert e < 1e-8, (gg, go)


@pytest.mark.parametrize("seed,nr,nz,z_full,nr_top,shape,ckpt,turn_on", [
    (0, 14, 8, 4, 9, None, 7, False), (1, 14, 8, 4, 6, (4, 2, 1), 0, False),
    (2, 40, 9, 5, 30, (8, 1, 2), 5, False), (3, 40, 9, 3, 22, None, 0, True)])
def test_gpu_gradient_stepped_matches_oracle_adjoint(seed, nr, nz, z_full, nr_top, shape, ckpt,
                                                     turn_on):
    # the stepped domain (eq. (9)) in the adjoint passes: the terminal's
    # tables, the closed step face, the surface over the layered section;
    # one and two waves per line, one and two lines per group, with the
    # turn-on model's sub-steps; random start fields
    import paper_1408_5853_amd as P
    c = cellgen.tiny(20 + seed, nr=nr, nz=nz, n_layers=3, nsteps=24, z_active=True, dt=2e-6,
                     amplitude=4e9, heater=2)
    c["stepped"] = dict(z_full=z_full, nr_top=nr_top)
    if turn_on:
        dt = c["dt"]
        c.update(t_on=3 * dt, period=20 * dt, width=4.6 * dt, turn_on=True)
    rng = np.random.default_rng(seed)
    T0 = 28.0 + rng.uniform(0, 3, size=(nz, nr))
    _, S = oracle.forward(c, T0, nsteps=24, surf=True)
    tgt = S + rng.normal(scale=0.05, size=24) + 0.02
    say("case adjoint stepped nr=%d nz=%d z_full=%d nr_top=%d shape=%s turn_on=%s" %
        (nr, nz, z_full, nr_top, shape, turn_on))
    Jo, go, So = oracle.gradient(c, tgt, T0=T0)
    plan = P.Plan(c)
    if shape:
        plan.set_shape(*shape)
    Jg, gg, Sg = plan.gradient(tgt, T0=T0, ckpt=ckpt)
    assert Jg == pytest.approx(Jo, rel=1e-9)
    assert np.max(np.abs(Sg - So) / So) < 1e-10
    e = _norm_err(gg, go, P.params_of(c))
    say("  normalised gradient error %.3e" % e)
    assert e < 1e-8, (gg, go)


@pytest.mark.parametrize("seed,nr,joule,shape,extra", [
    (0, 40, 0.0, None, None), (1, 40, 30.0, (4, 2, 1), None), (2, 40, 30.0, (8, 1, 2), "stepped"),
    (3, 40, 30.0, None, "turn_on"), (4, 300, 30.0, None, None), (5, 300, 0.0, (4, 4, 1), None)])
def test_gpu_gradient_poly_matches_oracle_adjoint(seed, nr, joule, shape, extra):
    # the polynomial laws of eqs. (23), (24) and the Joule source of eq. (25)
    # in the adjoint passes: derivative polynomials, the interface row's
    # quotient of two laws, the source's sqrt(tref / T) factor in lam^n and
    # in the amplitude and width sums; with a stepped domain and with the
    # turn-on model's sub-steps; one, two and four waves per line
    import paper_1408_5853_amd as P
    c = cellgen.poly_variant(cellgen.tiny(40 + seed, nr=nr, nz=9, n_layers=3, nsteps=30,
                                          z_active=True, dt=2e-6, amplitude=4e9, heater=2),
                             seed, joule_tref=joule)
    if extra == "stepped":
        c["stepped"] = dict(z_full=5, nr_top=30)
    if extra == "turn_on":
        dt = c["dt"]
        c.update(t_on=3 * dt, period=20 * dt, width=4.6 * dt, turn_on=True)
    tgt = _target(c, 30)
    say("case adjoint poly nr=%d joule=%g shape=%s %s" % (nr, joule, shape, extra))
    Jo, go, So = oracle.gradient(c, tgt)
    plan = P.Plan(c)
    if shape:
        plan.set_shape(*shape)
    Jg, gg, Sg = plan.gradient(tgt, ckpt=7)
    assert Jg == pytest.approx(Jo, rel=1e-9)
    assert np.max(np.abs(Sg - So) / So) < 1e-10
    e = _norm_err(gg, go, P.params_of(c))
    say("  normalised gradient error %.3e" % e)
    assert e < 1e-8, (gg, go)


def test_adjoint_workload_with_the_bench_store(adjoint_workload):
    """The full workload as the bench times its stored-tail variant (the
    states of the last steps kept in up to 200 GiB, at most 85 % of the free
    device memory): J and the gradient equal the checkpoints-only sweep's
    bit for bit, so the oracle comparison above covers it."""
    import torch

    import paper_1408_5853_amd as P
    c, tgt, Jg, gg, _, _ = adjoint_workload
    n = c["nsteps"]
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    plan = P.gradient_plan(c)
    d = plan.gradient_store_for(n, int(min(200 * 2**30, 0.85 * free)))
    say("case adjoint workload with a store of %d steps" % d)
    assert d > 0
    Js, gs, _ = plan.gradient(tgt, store=d)
    assert Js == Jg and np.array_equal(gs, gg)
    plan.set_gradient_store(0)
    torch.cuda.empty_cache()
