"""Pins of the oracle's discrete adjoint against central finite differences of
the oracle forward (which the forward pins tie to the paper), and of its
checkpoint/recompute against storing every state."""
import copy

import numpy as np
import pytest

import cellgen
import oracle


def _J(cell, target, T0=None):
    _, S = oracle.forward(cell, T0, nsteps=cell["nsteps"], surf=True)
    return float(np.sum((S - target[: cell["nsteps"]]) ** 2))


def _perturbed(cell, q, h):
    """cell with parameter q (gradient ordering) moved by h (absolute)."""
    c = copy.deepcopy(cell)
    L = len(c["layers"])
    if q == 0:
        c["amplitude"] += h
    elif q == 1:
        c["width"] += h
    elif q < 2 + L:
        c["layers"][q - 2]["thickness"] += h
    else:
        c["layers"][q - 2 - L]["k_scale"] += h
    return c


def _param(cell, q):
    L = len(cell["layers"])
    if q == 0:
        return cell["amplitude"]
    if q == 1:
        return cell["width"]
    if q < 2 + L:
        return cell["layers"][q - 2]["thickness"]
    return cell["layers"][q - 2 - L]["k_scale"]


def _target(cell, rng):
    n = cell["nsteps"]
    _, S = oracle.forward(cell, nsteps=n, surf=True)
    # a target the trajectory does not hit, so J has a nonzero gradient
    return S + rng.normal(scale=0.05, size=n) + 0.02


def _fd(cell, q, target, T0=None, rel=1e-4):
    """fourth-order central difference of J in parameter q"""
    h = rel * abs(_param(cell, q))
    f = lambda a: _J(_perturbed(cell, q, a * h), target, T0)
    return (8 * (f(1) - f(-1)) - (f(2) - f(-2))) / (12 * h)


def _fd_check(cell, seed, rtol, T0=None, target=None):
    """Compare every gradient entry with a finite difference.  Errors are
    measured on log-sensitivities p dJ/dp and normalised by the largest one:
    a weakly coupled parameter's difference quotient is limited by the
    rounding of J, not by the adjoint."""
    rng = np.random.default_rng(seed)
    if target is None:
        target = _target(cell, rng)
    J, g, _ = oracle.gradient(cell, target, T0=T0)
    assert J == pytest.approx(_J(cell, target, T0), rel=1e-14)
    P = np.array([abs(_param(cell, q)) for q in range(len(g))])
    fd = np.array([_fd(cell, q, target, T0) for q in range(len(g))])
    scale = np.max(np.abs(g * P))
    err = np.abs(g - fd) * P / scale
    assert np.max(err) <= rtol, (err, g, fd)
    return g, fd


@pytest.mark.parametrize("seed", range(3))
def test_gradient_matches_central_differences_z_active(seed):
    # heater in the outer layer, so that the surface responds within the run
    c = cellgen.tiny(seed, nr=14, nz=6, n_layers=3, nsteps=24, z_active=True,
                     dt=2e-6, amplitude=4e9, heater=2)
    _fd_check(c, seed, 1e-6)


@pytest.mark.parametrize("seed", range(2))
def test_gradient_matches_central_differences_insulated_z(seed):
    # all-insulated z ends: the boundary lines are copies, whose
    # sensitivities the adjoint moves back onto the copied lines
    c = cellgen.tiny(10 + seed, nr=13, nz=5, n_layers=4, nsteps=20,
                     z_active=False, dt=2e-6, amplitude=4e9)
    rng = np.random.default_rng(seed)
    T0 = 28.0 + rng.uniform(0, 3, size=(c["nz"], c["nr"]))
    T0[0], T0[-1] = T0[1], T0[-2]
    _fd_check(c, seed, 1e-6, T0=T0)


def test_state_adjoint_matches_directional_difference():
    c = cellgen.tiny(5, nr=12, nz=7, n_layers=3, nsteps=16, z_active=True,
                     dt=2e-6, amplitude=4e9)
    rng = np.random.default_rng(0)
    T0 = 28.0 + rng.uniform(0, 2, size=(c["nz"], c["nr"]))
    T0[-1] = 28.0
    target = _target(c, rng)
    J, g, S, lam0 = oracle.gradient(c, target, T0=T0, want_lam0=True)
    for trial in range(3):
        v = rng.normal(size=T0.shape)
        h = 1e-5
        fd = (_J(c, target, T0 + h * v) - _J(c, target, T0 - h * v)) / (2 * h)
        assert np.sum(lam0 * v) == pytest.approx(fd, rel=1e-6)


def test_width_gradient_on_step_aligned_pulse_edge():
    # pulse end exactly on a step boundary: J has a kink in the width there,
    # and the adjoint returns the mean of the two one-sided derivatives (what
    # a central difference of vanishing step measures)
    c = cellgen.tiny(3, nr=12, nz=5, n_layers=3, nsteps=30, dt=2e-6,
                     amplitude=4e9, heater=2)
    c["t_on"] = 0.0
    c["width"] = 11 * c["dt"]
    c["period"] = 25 * c["dt"]
    target = _target(c, np.random.default_rng(7))
    J, g, _ = oracle.gradient(c, target)
    h = 1e-4 * c["width"]
    f = lambda a: _J(_perturbed(c, 1, a * h), target)
    right = (-3 * f(0) + 4 * f(1) - f(2)) / (2 * h)     # second-order one-sided
    left = (3 * f(0) - 4 * f(-1) + f(-2)) / (2 * h)
    assert abs(right - left) > 1e-3 * abs(right)         # a real kink
    assert g[1] == pytest.approx(0.5 * (right + left), rel=1e-6)


def test_checkpointing_is_bitwise_equal_to_storing_all():
    c = cellgen.tiny(2, nr=12, nz=6, n_layers=3, nsteps=23, dt=2e-6,
                     amplitude=4e9)
    target = _target(c, np.random.default_rng(1))
    J0, g0, S0 = oracle.gradient(c, target, ckpt=0)
    for K in (1, 5, 7, 23):
        J1, g1, S1 = oracle.gradient(c, target, ckpt=K)
        assert J1 == J0 and np.array_equal(g1, g0) and np.array_equal(S1, S0)


def test_gradient_threads_bitwise_deterministic():
    c = cellgen.tiny(4, nr=16, nz=9, n_layers=3, nsteps=12, dt=2e-6,
                     amplitude=4e9)
    target = _target(c, np.random.default_rng(2))
    a = oracle.gradient(c, target, nthreads=1)
    b = oracle.gradient(c, target, nthreads=4)
    assert a[0] == b[0] and np.array_equal(a[1], b[1])


def _turn_on_cell(seed, w_steps, nsteps=24):
    c = cellgen.tiny(seed, nr=14, nz=6, n_layers=3, nsteps=nsteps, z_active=True,
                     dt=2e-6, amplitude=4e9, heater=2)
    dt = c["dt"]
    c.update(t_on=3 * dt, period=20 * dt, width=w_steps * dt, turn_on=True)
    return c


@pytest.mark.parametrize("seed,w_steps", [(0, 7.3), (1, 0.374)])
def test_turn_on_gradient_matches_central_differences(seed, w_steps):
    # the turn-on model's sub-steps inside the adjoint sweep (eq. (22)); a
    # pulse end inside a regular step, and one inside sub-step 37 of a pulse
    # start (the width derivative of a sub-step's source factor)
    _fd_check(_turn_on_cell(seed, w_steps), seed, 1e-6)


def test_turn_on_checkpointing_over_sub_steps_bitwise():
    c = _turn_on_cell(2, 4.6, nsteps=23)
    target = _target(c, np.random.default_rng(3))
    J0, g0, S0 = oracle.gradient(c, target, ckpt=0)
    for K in (1, 7, 60, 217):                 # 23 steps + 2 x 99 sub-steps = 221 launches
        J1, g1, S1 = oracle.gradient(c, target, ckpt=K)
        assert J1 == J0 and np.array_equal(g1, g0) and np.array_equal(S1, S0)


@pytest.mark.parametrize("seed,nr_top", [(0, 9), (1, 6)])
def test_stepped_gradient_matches_central_differences(seed, nr_top):
    # the stepped domain (eq. (9)): shorter terminal lines, the closed step
    # face, the surface mean over the layered section; a random start field
    # so that the terminal and the step face carry heat
    c = cellgen.tiny(20 + seed, nr=14, nz=8, n_layers=3, nsteps=24, z_active=True,
                     dt=2e-6, amplitude=4e9, heater=2)
    c["stepped"] = dict(z_full=4, nr_top=nr_top)
    rng = np.random.default_rng(seed)
    T0 = 28.0 + rng.uniform(0, 3, size=(c["nz"], c["nr"]))
    _fd_check(c, seed, 1e-6, T0=T0)


@pytest.mark.parametrize("seed,joule,z_active", [(0, 0.0, True), (1, 30.0, True), (2, 30.0, False)])
def test_poly_gradient_matches_central_differences(seed, joule, z_active):
    # the polynomial laws of eqs. (23), (24) (their derivative polynomials in
    # the adjoint) and the Joule source of eq. (25), whose sqrt(tref / T)
    # factor depends on the old temperature of each heater node
    c = cellgen.poly_variant(
        cellgen.tiny(30 + seed, nr=14, nz=6, n_layers=3, nsteps=30, z_active=z_active,
                     dt=2e-6, amplitude=4e9, heater=2), seed, joule_tref=joule)
    _fd_check(c, seed, 1e-6)


def test_poly_gradient_checkpointing_bitwise():
    c = cellgen.poly_variant(cellgen.tiny(33, nr=14, nz=6, n_layers=3, nsteps=25, z_active=True,
                                          dt=2e-6, amplitude=4e9, heater=2), 3, joule_tref=30.0)
    target = _target(c, np.random.default_rng(4))
    J0, g0, S0 = oracle.gradient(c, target, ckpt=0)
    for K in (1, 6):
        J1, g1, S1 = oracle.gradient(c, target, ckpt=K)
        assert J1 == J0 and np.array_equal(g1, g0) and np.array_equal(S1, S0)
