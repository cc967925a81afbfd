"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed-form
continuum solutions (Bessel series, layered logarithmic steady state), exact
discrete eigenmodes of the explicit z operator, exact heat balance, dense
brute-force solves, the paper's own sweep formulas, exact rational schedule
values and invariants.  All run on the CPU.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.integrate as si
import scipy.optimize as sp_opt
import scipy.special as sp

import cellgen
import oracle

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def layer(thickness, intervals, k0=1.0, p=0.0, c0=1.0, q=0.0, rho=1e3,
          tref=30.0, k_scale=1.0):
    return dict(thickness=thickness, intervals=intervals, k0=k0, p=p,
                k_scale=k_scale, c0=c0, q=q, rho=rho, tref=tref)


def cell(layers, nz=3, r_inner=1e-3, height=1.0, dt=1e-6, heater=0,
         amplitude=0.0, width=0.0, period=1.0, t_on=0.0, bc=None,
         T_init=28.0, nsteps=10):
    nr = 1 + sum(l["intervals"] for l in layers)
    if bc is None:
        bc = [[0, 0.0]] * 4
    return dict(r_inner=r_inner, height=height, nr=nr, nz=nz, layers=layers,
                heater=heater, amplitude=amplitude, width=width, period=period,
                t_on=t_on, bc=[list(b) for b in bc], dt=dt, T_init=T_init,
                nsteps=nsteps)


# --------------------------------------------------------------------------
# Source schedule, eq. (4): exact step averages by rational arithmetic
# --------------------------------------------------------------------------

def _exact_fraction(dt, t_on, w, P, k):
    lo, hi = Fraction(k), Fraction(k + 1)
    b0, W, Pp = (Fraction(t_on) / Fraction(dt), Fraction(w) / Fraction(dt),
                 Fraction(P) / Fraction(dt))
    s = Fraction(0)
    n = 0
    while b0 + n * Pp < hi:
        b, e = b0 + n * Pp, b0 + n * Pp + W
        s += max(Fraction(0), min(hi, e) - max(lo, b))
        n += 1
    return s


@pytest.mark.parametrize("dt,t_on,w,P", [
    (0.25, 0.0, 1.0, 4.0),           # edges on step boundaries
    (0.25, 0.625, 0.875, 2.5),       # edges inside steps
    (0.5, 0.25, 0.25, 1.5),          # pulse inside one step
])
def test_schedule_exact_fractions(dt, t_on, w, P):
    # dyadic inputs: every quantity is exact in binary floating point
    c = cell([layer(1e-3, 4)], dt=dt, t_on=t_on, width=w, period=P)
    for k in range(40):
        want = float(_exact_fraction(dt, t_on, w, P, k))
        assert oracle.source_fraction(c, k) == want, k


def test_schedule_workload_edges_snap():
    # 1 ms pulse every 10 ms at dt = 1 us: exactly 1000 on-steps per period,
    # despite 1e-3/1e-6 not being exact in binary
    c = cellgen.small_cell(0)
    s = np.array([oracle.source_fraction(c, k) for k in range(20_500)])
    want = np.zeros_like(s)
    for n0 in (0, 10_000, 20_000):
        want[n0:n0 + 1000] = 1.0
    assert np.array_equal(s, want)


def test_schedule_width_derivative_matches_central_difference():
    c = cell([layer(1e-3, 4)], dt=1e-6, t_on=2.5e-6, width=3.3e-5,
             period=1e-4)
    for k in range(0, 300):
        h = 1e-9
        cp = dict(c, width=c["width"] + h)
        cm = dict(c, width=c["width"] - h)
        fd = (oracle.source_fraction(cp, k) - oracle.source_fraction(cm, k)) / (2 * h)
        assert abs(oracle.source_fraction_dwidth(c, k) - fd) < 1e-3 / c["dt"], k


def test_schedule_derivative_half_on_exact_edges():
    # pulse end on a step boundary: half the one-sided slope on each side
    c = cell([layer(1e-3, 4)], dt=0.25, width=1.0, period=4.0)
    d = [oracle.source_fraction_dwidth(c, k) for k in range(6)]
    assert d == [0.0, 0.0, 0.0, 2.0, 2.0, 0.0]


# --------------------------------------------------------------------------
# Line solve: dense brute force; paper's own sweep formulas
# --------------------------------------------------------------------------

def _random_field(c, seed, lo=28.0, hi=40.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(c["nz"], c["nr"]))


@pytest.mark.parametrize("seed", range(4))
def test_step_equals_dense_solve_of_assembled_rows(seed):
    c = cellgen.tiny(seed, nr=17, nz=6, n_layers=3)
    T = _random_field(c, seed)
    T[0], T[-1] = T[1], c["bc"][3][1]
    k = 3
    Tn = oracle.forward(c, T, k0=k, nsteps=1)
    for j in range(1, c["nz"] - 1):
        A, B, Cc, F = oracle.line_rows(c, T, k, j)
        n = c["nr"]
        M = np.diag(B) + np.diag(A[1:], -1) + np.diag(Cc[:-1], 1)
        # interface rows are ~1e16 times smaller than capacity rows: equilibrate
        # the rows first, or LU would not enforce them
        D = 1.0 / np.abs(B)
        x = np.linalg.solve(M * D[:, None], F * D)
        assert np.max(np.abs(Tn[j] - x) / np.abs(x)) < 1e-13
        assert A[0] == 0 and Cc[n - 1] == 0


@pytest.mark.parametrize("seed", range(4))
def test_generic_thomas_reproduces_paper_interface_sweep(seed):
    # eq. (12) applied to the interface row of eq. (18) must give eq. (20);
    # eqs. (16)/(17) must follow from eq. (15)
    c = cellgen.tiny(seed, nr=19, nz=5, n_layers=4, z_active=False)
    c["bc"][0] = [0, 0.0]
    T = _random_field(c, 10 + seed)
    T[0], T[-1] = T[1], T[-2]
    Tn = oracle.forward(c, T, k0=1, nsteps=1)
    for j in range(1, c["nz"] - 1):
        x = oracle.line_paper_sweep(c, T, 1, j)
        assert np.max(np.abs(x - Tn[j]) / np.abs(x)) < 1e-14


def test_thomas_against_dense_random_dominant():
    rng = np.random.default_rng(0)
    n = 50
    A = -rng.uniform(0, 1, n); A[0] = 0
    Cc = -rng.uniform(0, 1, n); Cc[-1] = 0
    B = -A - Cc + rng.uniform(0.1, 1, n)
    F = rng.normal(size=n)
    M = np.diag(B) + np.diag(A[1:], -1) + np.diag(Cc[:-1], 1)
    assert np.allclose(oracle.thomas(A, B, Cc, F), np.linalg.solve(M, F),
                       rtol=1e-13, atol=1e-13)


# --------------------------------------------------------------------------
# Explicit z operator, eq. (11): exact discrete cosine modes
# --------------------------------------------------------------------------

@pytest.mark.parametrize("z_high_fixed", [False, True])
def test_z_operator_exact_discrete_modes(z_high_fixed):
    # constant coefficients (p = q = 0) and a radially uniform field: each
    # step multiplies a discrete cosine mode of the axial Laplacian by
    # 1 - (4 kappa dt / eta^2) sin^2(theta / 2)
    nz, M = 18, 16
    k0, rho, c0 = 2.0, 4e3, 5.0
    height = 8e-3
    eta = height / (nz - 1)
    kappa = k0 / (rho * c0)
    dt = 0.4 * eta ** 2 / kappa / 2
    bc = [[0, 0.0], [0, 0.0], [0, 0.0], [1 if z_high_fixed else 0, 28.0]]
    c = cell([layer(1e-3, 6, k0=k0, c0=c0, rho=rho)], nz=nz, height=height,
             dt=dt, bc=bc)
    jj = np.arange(1, M + 1)
    for k in (1, 3, 7):
        theta = (math.pi * (k - 0.5) / (M + 0.5)) if z_high_fixed else (math.pi * k / M)
        v = np.cos(theta * (jj - 0.5))
        T = np.full((nz, c["nr"]), 28.0)
        T[1:M + 1] += 0.5 * v[:, None]
        T[0] = T[1]
        T[-1] = 28.0 if z_high_fixed else T[-2]
        n = 25
        Tn = oracle.forward(c, T, nsteps=n)
        g = (1 - 4 * kappa * dt / eta ** 2 * math.sin(theta / 2) ** 2) ** n
        want = 28.0 + 0.5 * g * v
        assert np.max(np.abs(Tn[1:M + 1] - want[:, None])) < 1e-12
        assert np.array_equal(Tn[0], Tn[1])


# --------------------------------------------------------------------------
# Continuum closed forms
# --------------------------------------------------------------------------

def _bessel_solid_cylinder(r, t, R, kappa, T0, Ts, nterms=80):
    mu = sp.jn_zeros(0, nterms)
    out = np.zeros_like(r)
    for m in mu:
        out += 2 * sp.j0(m * r / R) / (m * sp.j1(m)) * math.exp(-kappa * m * m * t / R ** 2)
    return Ts + (T0 - Ts) * out


def test_bessel_series_solid_cylinder_convergence():
    # single layer, constant coefficients, r from the axis to R with a held
    # outer wall: the classical Bessel series solution.  The first-order
    # boundary approximation (eq. (15)) limits the order to about 1 (the
    # paper's accuracy statement).
    R, k0, rho, c0 = 1e-3, 1.0, 1e3, 1.0
    kappa = k0 / (rho * c0)
    t_end, dt = 2e-4, 2e-8
    errs = []
    for n in (16, 32, 64):
        c = cell([layer(R, n, k0=k0, rho=rho, c0=c0)], r_inner=0.0, dt=dt,
                 bc=[[0, 0.0], [1, 20.0], [0, 0.0], [0, 0.0]], T_init=30.0,
                 height=1.0)
        steps = int(round(t_end / dt))
        T = oracle.forward(c, nsteps=steps)
        r = oracle.radii(c)
        ex = _bessel_solid_cylinder(r, t_end, R, kappa, 30.0, 20.0)
        errs.append(np.max(np.abs(T[1] - ex)[1:-1]))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 2e-2
    assert min(orders) > 0.9, (errs, orders)


def _annulus_modes(a, b, nmodes):
    f = lambda lam: sp.j1(lam * b) * sp.y0(lam * a) - sp.y1(lam * b) * sp.j0(lam * a)
    xs = np.linspace(1e-3, 60.0, 200000) / (b - a)
    v = f(xs)
    roots = []
    from scipy.optimize import brentq
    for i in range(len(xs) - 1):
        if v[i] * v[i + 1] < 0:
            roots.append(brentq(f, xs[i], xs[i + 1], xtol=1e-14))
            if len(roots) == nmodes:
                break
    return np.array(roots)


def test_bessel_series_annulus_inner_wall_held():
    # the workloads' boundary set: inner wall held, outer wall insulated
    a, d = 1.2e-3, 0.8e-3
    b = a + d
    k0, rho, c0 = 1.0, 1e3, 1.0
    kappa = k0 / (rho * c0)
    lams = _annulus_modes(a, b, 40)
    U = lambda lam, r: sp.j0(lam * r) * sp.y0(lam * a) - sp.y0(lam * r) * sp.j0(lam * a)
    coef = []
    for lam in lams:
        num = si.quad(lambda r: r * U(lam, r), a, b, limit=400, epsabs=0, epsrel=1e-13)[0]
        den = si.quad(lambda r: r * U(lam, r) ** 2, a, b, limit=400, epsabs=0, epsrel=1e-13)[0]
        coef.append(num / den)
    t_end, dt = 1e-4, 1e-8
    errs = []
    for n in (16, 32, 64):
        c = cell([layer(d, n, k0=k0, rho=rho, c0=c0)], r_inner=a, dt=dt,
                 bc=[[1, 20.0], [0, 0.0], [0, 0.0], [0, 0.0]], T_init=30.0)
        T = oracle.forward(c, nsteps=int(round(t_end / dt)))
        r = oracle.radii(c)
        ex = 20.0 + 10.0 * sum(cf * U(l, r) * math.exp(-kappa * l * l * t_end)
                               for cf, l in zip(coef, lams))
        errs.append(np.max(np.abs(T[1] - ex)))
    # the insulated outer row (eq. (15)) is first order: it puts the wall half
    # an interval early, and the whole solution converges at order ~1, the
    # accuracy the paper states for its scheme
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 5e-2, errs
    assert min(orders) > 0.9, (errs, orders)


def _layered_steady_state(c, r):
    """Piecewise steady state with the heater always on, inner wall held at
    Tw, other faces insulated; power-law conductivities by the Kirchhoff
    transform U_m(T) = k0 tref/(p+1) (T/tref)^(p+1) within each layer."""
    Ls = c["layers"]
    R = [c["r_inner"]]
    for l in Ls:
        R.append(R[-1] + l["thickness"])
    h0, h1 = R[c["heater"]], R[c["heater"] + 1]
    Q = c["amplitude"]

    def Gint(x0, x1):
        # integral of G(s)/s, G(s) = int_s^rout Q(u) u du
        tot = 0.0
        lo, hi = x0, min(x1, h0)
        if hi > lo:
            tot += Q * (h1 ** 2 - h0 ** 2) / 2 * math.log(hi / lo)
        lo, hi = max(x0, h0), min(x1, h1)
        if hi > lo:
            tot += Q / 2 * (h1 ** 2 * math.log(hi / lo) - (hi ** 2 - lo ** 2) / 2)
        return tot

    def Uf(l, T):
        return l["k0"] * l["tref"] / (l["p"] + 1) * (T / l["tref"]) ** (l["p"] + 1)

    def Uinv(l, U):
        return l["tref"] * ((l["p"] + 1) * U / (l["k0"] * l["tref"])) ** (1 / (l["p"] + 1))

    Tb = [c["bc"][0][1]]
    for m, l in enumerate(Ls):
        Tb.append(Uinv(l, Uf(l, Tb[-1]) + Gint(R[m], R[m + 1])))
    out = np.zeros_like(r)
    for i, x in enumerate(r):
        m = min(np.searchsorted(R, x, side="right") - 1, len(Ls) - 1)
        l = Ls[m]
        out[i] = Uinv(l, Uf(l, Tb[m]) + Gint(R[m], x))
    return out


@pytest.mark.parametrize("nonlinear", [False, True])
def test_layered_logarithmic_steady_state(nonlinear):
    # heater on all the time (width = period), inner wall held: the
    # steady state is piecewise logarithmic in r (Kirchhoff-transformed for
    # power-law conductivities), continuous T and flux at the interfaces
    # (eq. (7)).  The paper's first-order interface rows give order ~1.
    th = [0.4e-3, 0.3e-3, 0.2e-3, 0.5e-3]
    k0s = [5.0, 0.5, 2.0, 0.8]
    ps = [1.2, 0.6, 1.8, 0.9] if nonlinear else [0.0] * 4
    errs = []
    for base in (16, 32, 64):
        Ls = [layer(t, base * w, k0=k, p=p, c0=100.0, q=3.0 if nonlinear else 0.0,
                    rho=5e3)
              for t, w, k, p in zip(th, (2, 2, 1, 2), k0s, ps)]
        c = cell(Ls, r_inner=1.2e-3, heater=2, amplitude=2e8, width=1.0,
                 period=1.0, dt=5.0, height=1.0,
                 bc=[[1, 28.0], [0, 0.0], [0, 0.0], [0, 0.0]])
        T = oracle.forward(c, nsteps=800)
        T2 = oracle.forward(c, T, k0=800, nsteps=1)
        assert np.max(np.abs(T2 - T)) < 1e-9           # converged
        r = oracle.radii(c)
        ex = _layered_steady_state(c, r)
        errs.append(np.max(np.abs(T[1] - ex)) / (ex.max() - 28.0))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    # interface rows hold no capacity and no source, so the heater loses a
    # fraction O(h) of its volume: first order, as the paper states
    assert errs[-1] < 2e-2, errs
    assert min(orders) > 0.9, (errs, orders)


# --------------------------------------------------------------------------
# Heat balance and invariants
# --------------------------------------------------------------------------

def _heat_balance_defect(c, T, Tn, k):
    r = oracle.radii(c)
    h = np.diff(r)
    hb = 0.5 * (h[:-1] + h[1:])          # hbar_i, i = 1..nr-2
    eta = c["height"] / (c["nz"] - 1)
    l = c["layers"][0]
    rc = l["rho"] * l["c0"] * (T[1:-1, 1:-1] / l["tref"]) ** l["q"]
    w = r[1:-1] * hb * eta
    lhs = np.sum(w * rc * (Tn[1:-1, 1:-1] - T[1:-1, 1:-1]))
    s = oracle.source_fraction(c, k)
    rhs = c["dt"] * c["amplitude"] * s * np.sum(w * np.ones_like(rc))
    return lhs, rhs


def test_heat_balance_exact_single_layer_insulated():
    # insulated on all sides: the r- and z-fluxes telescope, so the capacity-
    # weighted heat content changes by exactly the injected source
    Ls = [layer(1e-3, 40, k0=3.0, p=1.3, c0=80.0, q=3.0, rho=4e3)]
    c = cell(Ls, nz=12, height=5e-3, dt=2e-7, amplitude=3e8, width=4e-6,
             period=1e-5, heater=0)
    T = _random_field(c, 3, 28.0, 34.0)
    T[0], T[-1] = T[1], T[-2]
    for k in range(0, 60, 7):
        Tn = oracle.forward(c, T, k0=k, nsteps=1)
        lhs, rhs = _heat_balance_defect(c, T, Tn, k)
        scale = np.sum(np.abs(Tn - T)) + abs(rhs) + 1e-30
        if rhs != 0:
            assert abs(lhs - rhs) <= 1e-11 * abs(rhs)
        else:
            # no source this step: content is conserved to rounding
            rc = Ls[0]["rho"] * Ls[0]["c0"] * 1.0
            assert abs(lhs) <= 1e-11 * rc * scale
        T = Tn


def test_zero_source_keeps_uniform_field():
    # with no source a uniform field is a fixed point of eq. (8); only the
    # rounding of the row sums moves it
    c = cellgen.small_cell(1)
    c["amplitude"] = 0.0
    T = oracle.forward(c, nsteps=3000)
    assert np.max(np.abs(T - 28.0)) < 1e-11


def test_as_written_config_is_exactly_z_invariant():
    c = cellgen.small_cell(2)
    T = oracle.forward(c, nsteps=1500)
    assert np.all(T == T[1][None, :])
    assert T.max() > 28.0
    # and a short-axis copy gives the same lines
    T4 = oracle.forward(cellgen.with_nz(c, 4), nsteps=1500)
    assert np.array_equal(T4[1], T[1])


def test_maximum_principle_and_heating():
    c = cellgen.small_cell(3, z_active=True)
    T, S = oracle.forward(c, nsteps=3000, surf=True)
    assert T.min() > 28.0 - 1e-9
    assert np.all(np.diff(S[:900]) >= -1e-12)     # heating phase: surface rises


# --------------------------------------------------------------------------
# Transient turn-on model, Sec. 3.2, eq. (22) (decaying exponential reading)
# --------------------------------------------------------------------------

def _p2_sum(m):
    # sum_{i<m} (1 - exp(-i/7)) by the geometric series
    return m - (1.0 - math.exp(-m / 7.0)) / (1.0 - math.exp(-1.0 / 7.0))


@pytest.mark.parametrize("w_steps,open_frac", [
    # gate open over the whole step: all 100 sub-steps
    (3.0, _p2_sum(100) / 100.0),
    # gate closing at 0.375 of the step: sub-steps 0..36 open, 37 half open
    (0.375, (_p2_sum(37) + 0.5 * (1.0 - math.exp(-37.0 / 7.0))) / 100.0),
])
def test_turn_on_heat_balance_closed_form(w_steps, open_frac):
    # constant capacity, nonlinear conductivity, insulated on all sides: over
    # the 100 sub-steps the fluxes telescope and the capacity-weighted content
    # grows by exactly Q tau* sum_i (gate_i p2_i)
    dt = 2e-7
    Ls = [layer(1e-3, 30, k0=3.0, p=1.3, c0=80.0, q=0.0, rho=4e3)]
    c = cell(Ls, nz=8, height=5e-3, dt=dt, amplitude=3e9, width=w_steps * dt,
             period=50 * dt, heater=0)
    c["turn_on"] = True
    T = _random_field(c, 5, 28.0, 34.0)
    T[0], T[-1] = T[1], T[-2]
    Tn = oracle.forward(c, T, k0=50, nsteps=1)          # step 50 starts pulse 1
    r = oracle.radii(c)
    h = np.diff(r)
    w = r[1:-1] * 0.5 * (h[:-1] + h[1:]) * (c["height"] / (c["nz"] - 1))
    wc = w * Ls[0]["rho"] * Ls[0]["c0"] * np.ones((c["nz"] - 2, 1))
    lhs = np.sum(wc * (Tn[1:-1, 1:-1] - T[1:-1, 1:-1]))
    rhs = dt * c["amplitude"] * open_frac * np.sum(w * np.ones((c["nz"] - 2, 1)))
    # rounding: each of the 100 sub-steps stores every temperature (<= 40 K)
    # to within 2 ulp
    rnd = 100 * 2 * np.finfo(float).eps * 40.0 * np.sum(wc)
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs) + rnd
    assert rnd < 1e-8 * abs(rhs)
    # without the model the same step injects the plain step average
    c["turn_on"] = False
    Tp = oracle.forward(c, T, k0=50, nsteps=1)
    lhs_p = np.sum(w * Ls[0]["rho"] * Ls[0]["c0"] * (Tp[1:-1, 1:-1] - T[1:-1, 1:-1]))
    rhs_p = dt * c["amplitude"] * min(w_steps, 1.0) * np.sum(w * np.ones((c["nz"] - 2, 1)))
    assert abs(lhs_p - rhs_p) <= 1e-11 * abs(rhs_p)
    assert abs(lhs - lhs_p) > 0.05 * abs(lhs_p)


def test_turn_on_leaves_other_steps_alone():
    c = cellgen.with_nz(cellgen.small_cell(1), 4)
    dt = c["dt"]
    c.update(t_on=3 * dt, width=5 * dt, period=20 * dt)
    on = dict(c, turn_on=True)
    T = oracle.forward(c, nsteps=3)                      # steps 0..2: no pulse starts
    assert np.array_equal(oracle.forward(on, nsteps=3), T)
    # steps 4..22 start no pulse either
    T5 = oracle.forward(c, T, k0=3, nsteps=1)
    assert np.array_equal(oracle.forward(on, T5, k0=4, nsteps=19),
                          oracle.forward(c, T5, k0=4, nsteps=19))
    # the pulse-start step 3 does change
    assert not np.array_equal(oracle.forward(on, T, k0=3, nsteps=1), T5)


def test_turn_on_substeps_are_hundredth_steps():
    # with no source a pulse-start step is 100 plain steps of dt / 100
    c = cellgen.with_nz(cellgen.small_cell(2, z_active=True), 6)
    c["amplitude"] = 0.0
    T0 = _random_field(c, 9, 28.0, 31.0)
    on = dict(c, turn_on=True)
    fine = dict(c, dt=c["dt"] / 100.0)
    k = int(round(c["t_on"] / c["dt"]))
    assert np.array_equal(oracle.forward(on, T0, k0=k, nsteps=1),
                          oracle.forward(fine, T0, k0=0, nsteps=100))


def test_turn_on_factor_shape():
    # p^2 starts at zero, rises, and is saturated about halfway through the
    # step (Sec. 3.2, Fig. 2)
    c = cellgen.small_cell(0)
    c.update(turn_on=True, width=10 * c["dt"])
    f = np.array([oracle.turn_on_source(c, 0, i) for i in range(100)])
    assert f[0] == 0.0
    assert np.all(np.diff(f) > 0)
    assert 0.999 < f[50] < 1.0 and f[99] < 1.0
    assert f[10] < 0.8


def test_turn_on_needs_pulse_starts_on_steps():
    c = cellgen.with_nz(cellgen.small_cell(0), 4)
    c.update(turn_on=True, t_on=2.5 * c["dt"])
    with pytest.raises(ValueError):
        oracle.forward(c, nsteps=2)
    c.update(t_on=0.0, period=1000.5 * c["dt"])
    with pytest.raises(ValueError):
        oracle.forward(c, nsteps=2)
    with pytest.raises(ValueError):
        oracle.gradient(c, np.zeros(2), nsteps=2)


def fig3_cell(mult, turn_on):
    """A cold start (4.2 K, inner wall held there) with a strong pulse, the
    setting of the paper's Fig. 3: steps of mult x 1 us."""
    c = cellgen.with_nz(cellgen.small_cell(0), 4)
    c.update(T_init=4.2, amplitude=3e9, dt=1e-6 * mult, turn_on=turn_on)
    c["bc"][0] = [1, 4.2]
    return c


def _heater_trace(c, t_end=1e-3):
    T = oracle.initial_field(c)
    out = []
    for k in range(int(round(t_end / c["dt"]))):
        T = oracle.forward(c, T, k0=k, nsteps=1)
        out.append(T[1].max())
    return np.array(out)


def test_turn_on_removes_start_jump_fig3():
    # Fig. 3: with long steps and no turn-on model the first step overshoots
    # and the cell then cools while the heater is still on; with the model it
    # heats monotonically and ends near the short-step solution
    ref = _heater_trace(fig3_cell(1, False))[-1]
    for mult in (20, 100):
        off = _heater_trace(fig3_cell(mult, False))
        on = _heater_trace(fig3_cell(mult, True))
        assert np.any(np.diff(off) < -0.1)
        assert off[0] > ref * 0.5 and off.max() > on.max()
        assert np.all(np.diff(on) >= 0)
        assert abs(on[-1] - ref) < abs(off[-1] - ref)
        assert abs(on[-1] - ref) < 0.03 * ref


# --------------------------------------------------------------------------
# Polynomial laws (eqs. (23), (24)) and the Joule source (eqs. (2), (25))
# --------------------------------------------------------------------------

def poly_layer(thickness, intervals, a, b, rho=5e3):
    l = layer(thickness, intervals, rho=rho)
    l.update(poly_a=[float(x) for x in a], poly_b=[float(x) for x in b])
    return l


def poly_cell(Ls, **kw):
    c = cell(Ls, **kw)
    c["poly"] = True
    return c


def test_polynomial_laws_reduce_to_power_laws():
    # integer exponents: lambda = k0 (T/tref)^p and c = c0 (T/tref)^3 are
    # polynomials; both law paths must give the same run to rounding
    ps, k0s, c0s = [0, 1, 2], [3.0, 40.0, 0.7], [50.0, 120.0, 30.0]
    Ls = [layer(t, n, k0=k, p=float(p), c0=c0, q=3.0, rho=4e3)
          for t, n, k, p, c0 in zip([4e-4, 3e-4, 5e-4], [12, 10, 14], k0s, ps, c0s)]
    c = cell(Ls, nz=7, height=4e-3, dt=2e-7, heater=1, amplitude=2e9, width=2e-6,
             period=1e-5, bc=[[1, 28.0], [0, 0.0], [0, 0.0], [1, 30.0]])
    T0 = _random_field(c, 4, 28.0, 33.0)
    Tp = oracle.forward(c, T0, nsteps=150)
    Pl = []
    for l, k, p, c0 in zip(Ls, k0s, ps, c0s):
        b = [0.0] * 5
        b[p] = k / 30.0 ** p
        Pl.append(poly_layer(l["thickness"], l["intervals"], [0, 0, 0, c0 / 30.0 ** 3], b,
                             rho=l["rho"]))
    cp = dict(c, layers=Pl, poly=True)
    Tq = oracle.forward(cp, T0, nsteps=150)
    assert np.max(np.abs(Tq - Tp) / Tp) < 1e-12
    assert np.max(np.abs(Tp - T0)) > 0.1


def _poly_U(b, T):
    # Kirchhoff transform of a polynomial conductivity: int_0^T lambda
    return sum(bk * T ** (k + 1) / (k + 1) for k, bk in enumerate(b))


def _poly_Uinv(b, U):
    return sp_opt.brentq(lambda T: _poly_U(b, T) - U, 1e-3, 1e4, xtol=1e-14, rtol=1e-15)


def test_polynomial_layered_steady_state():
    # the layered logarithmic steady state of a held-wall cell with the heater
    # on all the time, for quartic conductivities (Kirchhoff transform of each
    # layer's polynomial, inverted numerically): first-order convergence
    th = [0.4e-3, 0.3e-3, 0.2e-3, 0.5e-3]
    bs = [[4.0, 0.03, 2e-4, 1e-6, 3e-9], [0.3, 0.01, 1e-4, 0.0, 1e-9],
          [1.5, 0.0, 5e-4, 2e-6, 0.0], [0.6, 0.02, 0.0, 1e-6, 2e-9]]
    a = [20.0, 1.0, 0.05, 1e-3]
    errs = []
    for base in (16, 32, 64):
        Ls = [poly_layer(t, base * w, a, b) for t, w, b in zip(th, (2, 2, 1, 2), bs)]
        c = poly_cell(Ls, r_inner=1.2e-3, heater=2, amplitude=2e8, width=1.0,
                      period=1.0, dt=5.0, height=1.0,
                      bc=[[1, 28.0], [0, 0.0], [0, 0.0], [0, 0.0]])
        T = oracle.forward(c, nsteps=800)
        T2 = oracle.forward(c, T, k0=800, nsteps=1)
        assert np.max(np.abs(T2 - T)) < 1e-9
        r = oracle.radii(c)
        R = [c["r_inner"]]
        for l in Ls:
            R.append(R[-1] + l["thickness"])
        h0, h1, Q = R[2], R[3], c["amplitude"]

        def G(x0, x1):
            tot = 0.0
            lo, hi = x0, min(x1, h0)
            if hi > lo:
                tot += Q * (h1 ** 2 - h0 ** 2) / 2 * math.log(hi / lo)
            lo, hi = max(x0, h0), min(x1, h1)
            if hi > lo:
                tot += Q / 2 * (h1 ** 2 * math.log(hi / lo) - (hi ** 2 - lo ** 2) / 2)
            return tot

        Tb = [28.0]
        for m in range(4):
            Tb.append(_poly_Uinv(bs[m], _poly_U(bs[m], Tb[-1]) + G(R[m], R[m + 1])))
        ex = np.array([_poly_Uinv(bs[m], _poly_U(bs[m], Tb[m]) + G(R[m], x))
                       for x in r for m in [min(np.searchsorted(R, x, side="right") - 1, 3)]])
        errs.append(np.max(np.abs(T[1] - ex)) / (ex.max() - 28.0))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 2e-2, errs
    assert min(orders) > 0.9, (errs, orders)


def test_polynomial_heat_balance_with_joule_source():
    # insulated single layer, polynomial capacity, Joule source: per step the
    # capacity-weighted content (c at the old level) grows by exactly
    # dt A s sum w sqrt(T_J / T_old)
    Ls = [poly_layer(1e-3, 36, [15.0, 0.8, 0.03, 2e-4], [2.0, 0.05, 1e-3, 0.0, 1e-8], rho=3e3)]
    c = poly_cell(Ls, nz=10, height=5e-3, dt=2e-7, amplitude=3e8, width=4e-6,
                  period=1e-5, heater=0)
    c["joule_tref"] = 30.0
    T = _random_field(c, 7, 28.0, 36.0)
    T[0], T[-1] = T[1], T[-2]
    r = oracle.radii(c)
    h = np.diff(r)
    w = r[1:-1] * 0.5 * (h[:-1] + h[1:]) * (c["height"] / (c["nz"] - 1))
    a = Ls[0]["poly_a"]
    for k in range(0, 40, 9):
        Tn = oracle.forward(c, T, k0=k, nsteps=1)
        Ti = T[1:-1, 1:-1]
        cap = a[0] + a[1] * Ti + a[2] * Ti ** 2 + a[3] * Ti ** 3
        lhs = np.sum(w * Ls[0]["rho"] * cap * (Tn[1:-1, 1:-1] - Ti))
        s = oracle.source_fraction(c, k)
        rhs = c["dt"] * c["amplitude"] * s * np.sum(w * np.sqrt(30.0 / Ti))
        if s > 0:
            assert abs(lhs - rhs) <= 1e-11 * abs(rhs)
        else:
            assert abs(lhs) <= 1e-11 * np.sum(w * Ls[0]["rho"] * cap * np.abs(Tn[1:-1, 1:-1] - Ti)) + 1e-30
        T = Tn


def test_joule_uniform_field_converges_to_closed_form():
    # a uniform, insulated, all-heater cell with constant c: the field stays
    # uniform and follows dT/dt = A sqrt(T_J / T) / (rho c), whose solution is
    # T^(3/2) = T0^(3/2) + (3/2) A sqrt(T_J) t / (rho c); the lagged source
    # makes the scheme first order in dt
    t_end, A, TJ, rho, c0, T0 = 2e-3, 4e7, 30.0, 2e3, 5.0, 28.0
    exact = (T0 ** 1.5 + 1.5 * A * math.sqrt(TJ) * t_end / (rho * c0)) ** (2.0 / 3.0)
    errs = []
    for n in (50, 100, 200):
        Ls = [poly_layer(1e-3, 12, [c0, 0, 0, 0], [1.0, 0.01, 0, 0, 0], rho=rho)]
        c = poly_cell(Ls, nz=5, height=2e-3, dt=t_end / n, amplitude=A, width=1.0,
                      period=1.0, heater=0, T_init=T0)
        c["joule_tref"] = TJ
        T = oracle.forward(c, nsteps=n)
        assert np.ptp(T) <= 1e-12 * T.max()
        errs.append(abs(T[2, 5] - exact))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert exact - T0 > 5.0
    assert errs[-1] < 5e-3 * (exact - T0), errs
    assert min(orders) > 0.9, (errs, orders)


# --------------------------------------------------------------------------
# Stepped domain (eq. (9): N_j radial nodes on line j)
# --------------------------------------------------------------------------

def test_stepped_domain_full_radius_is_rectangular():
    # the terminal spanning every radial node leaves the field unchanged bit
    # for bit; only the surface mean is restricted to the layered section
    c = cellgen.with_nz(cellgen.small_cell(2, z_active=True), 14)
    T0 = _random_field(c, 3, 28.0, 32.0)
    Tr = oracle.forward(c, T0, nsteps=120)
    st = dict(c, stepped=dict(z_full=8, nr_top=c["nr"]))
    Ts, S = oracle.forward(st, T0, nsteps=120, surf=True)
    assert np.array_equal(Ts, Tr)
    w = np.ones(9)
    w[0] = w[-1] = 0.5
    assert S[-1] == pytest.approx(np.dot(w, Tr[:9, -1]) / 8, rel=1e-15)


def test_stepped_domain_heat_balance_exact():
    # insulated everywhere, random field: over the domain's capacity nodes the
    # content changes by exactly the injected source each step, so the step
    # face and the terminal's outer wall pass no heat; nodes outside the
    # domain are left alone
    Ls = [layer(1e-3, 40, k0=3.0, p=1.3, c0=80.0, q=3.0, rho=4e3)]
    c = cell(Ls, nz=12, height=5e-3, dt=2e-7, amplitude=3e8, width=4e-6,
             period=1e-5, heater=0)
    j0, nt = 5, 15
    c["stepped"] = dict(z_full=j0, nr_top=nt)
    T = _random_field(c, 11, 28.0, 34.0)
    T[0], T[-1] = T[1], T[-2]
    r = oracle.radii(c)
    h = np.diff(r)
    w = r[1:-1] * 0.5 * (h[:-1] + h[1:]) * (c["height"] / (c["nz"] - 1))
    mask = np.zeros((c["nz"], c["nr"]), bool)
    mask[1:j0 + 1, 1:-1] = True
    mask[j0 + 1:-1, 1:nt - 1] = True
    W = np.zeros_like(T)
    W[:, 1:-1] = w
    l = Ls[0]
    for k in range(0, 40, 9):
        Tn = oracle.forward(c, T, k0=k, nsteps=1)
        rc = l["rho"] * l["c0"] * (T / l["tref"]) ** l["q"]
        lhs = np.sum((W * rc * (Tn - T))[mask])
        rhs = c["dt"] * c["amplitude"] * oracle.source_fraction(c, k) * np.sum(W[mask])
        scale = np.sum((W * rc * np.abs(Tn - T))[mask])
        assert abs(lhs - rhs) <= 1e-11 * max(abs(rhs), scale)
        assert np.array_equal(Tn[j0 + 1:-1, nt:], T[j0 + 1:-1, nt:])
        assert scale > 0
        T = Tn


@pytest.mark.parametrize("nt_from_outer", [0, 6])
def test_stepped_domain_held_outer_wall_heat_balance(nt_from_outer):
    # Outer wall held at T_w: on the layered lines (j <= z_full) heat enters
    # through the wall face of the last capacity node (the r-operator is
    # implicit, eq. (10): flux r_{i+1/2} lam (T_w - T^_{nr-2}) / h_{nr-1} with
    # lam at the old face mean); the terminal's own outer wall is insulated
    # (eq. (15)), also when the terminal spans every radial node, so its lines
    # take no wall flux.  Insulated elsewhere, one layer (no interfaces), so
    # the capacity-weighted content changes by exactly source + wall heat.
    Ls = [layer(1e-3, 30, k0=3.0, p=1.3, c0=80.0, q=3.0, rho=4e3)]
    Tw = 31.0
    bc = [[0, 0.0], [1, Tw], [0, 0.0], [0, 0.0]]
    c = cell(Ls, nz=11, height=5e-3, dt=2e-7, amplitude=3e8, width=4e-6,
             period=1e-5, heater=0, bc=bc)
    nr, nz = c["nr"], c["nz"]
    j0, nt = 6, nr - nt_from_outer
    c["stepped"] = dict(z_full=j0, nr_top=nt)
    T = _random_field(c, 5, 28.0, 34.0)
    T[:j0 + 1, -1] = Tw                          # held wall on the layered lines
    T[j0 + 1:, nt - 1] = T[j0 + 1:, nt - 2]      # insulated terminal wall
    T[0], T[-1] = T[1], T[-2]
    r = oracle.radii(c)
    h = np.diff(r)
    eta = c["height"] / (nz - 1)
    W = np.zeros_like(T)
    W[:, 1:-1] = r[1:-1] * 0.5 * (h[:-1] + h[1:]) * eta
    mask = np.zeros((nz, nr), bool)
    mask[1:j0 + 1, 1:-1] = True
    mask[j0 + 1:-1, 1:nt - 1] = True
    l = Ls[0]
    lam = lambda x: l["k_scale"] * l["k0"] * (x / l["tref"]) ** l["p"]
    r_face = 0.5 * (r[-1] + r[-2])
    wall_heat_seen = 0.0
    for k in range(0, 36, 7):
        Tn = oracle.forward(c, T, k0=k, nsteps=1)
        rc = l["rho"] * l["c0"] * (T / l["tref"]) ** l["q"]
        lhs = np.sum((W * rc * (Tn - T))[mask])
        src = c["amplitude"] * oracle.source_fraction(c, k) * np.sum(W[mask])
        jl = np.arange(1, j0 + 1)
        flux = r_face * lam(0.5 * (T[jl, -2] + T[jl, -1])) * (Tw - Tn[jl, -2]) / h[-1]
        wall = eta * np.sum(flux)
        rhs = c["dt"] * (src + wall)
        scale = np.sum((W * rc * np.abs(Tn - T))[mask])
        assert abs(lhs - rhs) <= 1e-11 * max(abs(rhs), scale), (lhs, rhs)
        # the held wall stays held on the layered lines only
        assert np.all(Tn[:j0 + 1, -1] == Tw)
        np.testing.assert_allclose(Tn[j0 + 1:-1, nt - 1], Tn[j0 + 1:-1, nt - 2],
                                   rtol=1e-14, atol=0)
        wall_heat_seen = max(wall_heat_seen, abs(c["dt"] * wall) / max(scale, 1e-300))
        T = Tn
    assert wall_heat_seen > 1e-3             # the wall term is not negligible


def test_stepped_domain_rejects_bad_steps():
    c = cellgen.with_nz(cellgen.small_cell(0), 6)
    for bad in (dict(z_full=5, nr_top=10), dict(z_full=2, nr_top=2),
                dict(z_full=2, nr_top=c["nr"] + 1)):
        with pytest.raises(ValueError):
            oracle.forward(dict(c, stepped=bad), nsteps=1)
