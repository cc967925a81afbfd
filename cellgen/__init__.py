"""Seeded synthetic problem descriptions for the multilayer cryogenic cell.

This module only draws numbers and lays them out as plain dictionaries; it
computes no part of the finite-difference method.  Both the CPU oracle and the
GPU library consume the same dictionary, so the dictionary (not the RNG) is the
contract between them.

Problem dictionary (SI units throughout):

    r_inner, height        inner radius and cell height [m]
    nr, nz                 radial / axial node counts (boundary nodes included)
    layers                 list, inner to outer, of
                           {thickness [m], intervals, k0 [W/m/K], p, k_scale,
                            c0 [J/kg/K], q, rho [kg/m^3], tref [K]}
                           lambda(T) = k_scale*k0*(T/tref)^p, c(T) = c0*(T/tref)^q
    heater                 index of the heated layer
    amplitude              volumetric source while the pulse is on [W/m^3]
    width, period, t_on    rectangular pulse train [s]
    bc                     4 x [kind, value] for r_inner, r_outer, z_low, z_high;
                           kind 0 = insulated (zero normal derivative), 1 = fixed T
    dt, T_init             time step [s], uniform initial temperature [K]
    nsteps                 step count of the workload

The geometry of the cell and the property families follow the paper's model
(Sec. 2, eq. (1), eqs. (4)-(6)): layers stacked along r, a heater layer second
from the outside, a periodic rectangular pulse, a uniform start and insulated
boundaries except for one held at T0.  The draw ranges are those of the
workloads this project measures.
"""
from __future__ import annotations

import copy
import math

import numpy as np

TREF = 30.0          # reference temperature of the power laws [K]
T0 = 28.0            # initial / wall temperature [K]
R_INNER = 1.2e-3     # inner wall radius [m] (the paper's cooler radius, 0.12 cm)
HEIGHT = 10e-3       # cell height [m]
NEUMANN, DIRICHLET = 0, 1


def _log_uniform(rng, lo, hi):
    return float(math.exp(rng.uniform(math.log(lo), math.log(hi))))


def allot_intervals(thicknesses, total, minimum=10):
    """Split `total` radial intervals over layers: `minimum` each, the rest in
    proportion to thickness (largest remainder, ties to the inner layer)."""
    L = len(thicknesses)
    if total < minimum * L:
        raise ValueError("too few radial intervals for %d layers" % L)
    spare = total - minimum * L
    tsum = float(sum(thicknesses))
    share = [spare * t / tsum for t in thicknesses]
    base = [int(math.floor(s)) for s in share]
    left = spare - sum(base)
    order = sorted(range(L), key=lambda m: (-(share[m] - base[m]), m))
    for m in order[:left]:
        base[m] += 1
    return [minimum + b for b in base]


def _draw_material(rng, eta, dt, margin, k_lo=0.1, k_hi=400.0):
    """Draw (p, c0, rho) first, then k0 log-uniformly below the explicit-z
    stability cap evaluated at the coldest temperature T0 (the diffusivity
    k/(rho c) grows as T falls because p < q).  `margin` < 1 keeps a safety
    factor.  Redraw when the cap falls below k_lo."""
    q = 3.0
    for _ in range(1000):
        p = float(rng.uniform(0.5, 2.0))
        c0 = _log_uniform(rng, 10.0, 300.0)
        rho = float(rng.uniform(2e3, 9e3))
        x = T0 / TREF
        kmax = min(k_hi, margin * eta * eta * rho * c0 * x ** q / (2.0 * dt * x ** p))
        if kmax >= k_lo:
            k0 = _log_uniform(rng, k_lo, kmax)
            return dict(k0=k0, p=p, k_scale=1.0, c0=c0, q=q, rho=rho, tref=TREF)
    raise RuntimeError("could not draw a stable material")


def _bc(z_active):
    bc = [[DIRICHLET, T0], [NEUMANN, 0.0], [NEUMANN, 0.0], [NEUMANN, 0.0]]
    if z_active:
        bc[3] = [DIRICHLET, T0]
    return bc


def _cell(rng, nr, nz, n_layers, thick, dt, nsteps, amplitude, width, period,
          z_active=False, heater=None, height=HEIGHT):
    eta = height / (nz - 1)
    margin = 0.5 if z_active else 0.9
    mats = [_draw_material(rng, eta, dt, margin) for _ in range(n_layers)]
    ints = allot_intervals(thick, nr - 1)
    layers = []
    for m in range(n_layers):
        d = dict(thickness=float(thick[m]), intervals=int(ints[m]))
        d.update(mats[m])
        layers.append(d)
    return dict(r_inner=R_INNER, height=height, nr=int(nr), nz=int(nz),
                layers=layers,
                heater=int(n_layers - 2 if heater is None else heater),
                amplitude=float(amplitude), width=float(width),
                period=float(period), t_on=0.0,
                bc=_bc(z_active), dt=float(dt), T_init=T0, nsteps=int(nsteps))


def _weights_2mm(rng, n_layers, heater):
    w = [float(rng.uniform(0.2, 1.0)) for _ in range(n_layers)]
    w[heater] = float(rng.uniform(0.02, 0.1))
    s = sum(w)
    return [2e-3 * x / s for x in w]


def small_cell(seed=0, z_active=False, nsteps=10_000):
    """64 x 128 nodes, 4 layers (substrate, insulator, heater film, outer
    shell) summing to 2 mm, dt = 1 us, 1 ms pulse every 10 ms."""
    rng = np.random.default_rng([1, seed])
    thick = _weights_2mm(rng, 4, 2)
    amp = _log_uniform(rng, 1e8, 1e9)
    return _cell(rng, 64, 128, 4, thick, 1e-6, nsteps, amp, 1e-3, 10e-3,
                 z_active=z_active, heater=2)


def device_cell(seed=0, z_active=False, nsteps=100_000, nr=1024, nz=4096):
    """1024 x 4096 nodes, 8 layers summing to 2 mm, dt = 0.2 us, 2 ms pulse
    every 20 ms, amplitude 5e8 W/m^3, 100,000 steps (one period)."""
    rng = np.random.default_rng([2, seed])
    thick = _weights_2mm(rng, 8, 6)
    # the stability cap uses the full-size axial spacing so that a reduced-nz
    # copy of this problem keeps the same materials
    cell = _cell(rng, nr, 4096, 8, thick, 2e-7, nsteps, 5e8, 2e-3, 20e-3,
                 z_active=z_active, heater=6)
    cell["nz"] = int(nz)
    return cell


def paper_shape(seed=0, nsteps=100_000):
    """631 x 1201 nodes with the small cell's laws, dt = 0.25 us, 100,000 steps: the
    grid and run length of the paper's timing table (Table 4, last column)."""
    rng = np.random.default_rng([6, seed])
    thick = _weights_2mm(rng, 4, 2)
    amp = _log_uniform(rng, 1e8, 1e9)
    return _cell(rng, 631, 1201, 4, thick, 2.5e-7, nsteps, amp, 1e-3, 10e-3,
                 heater=2)


def sweep_cells(seed=0, n_instances=256, nsteps=20_000):
    """Batched design sweep: uneven grids from 128x256 to 512x2048, 4-8
    layers of 20 um - 1 mm, per-instance amplitude, width, period;
    dt_i = period_i / 20,000."""
    rng = np.random.default_rng([3, seed])
    out = []
    for _ in range(n_instances):
        nr = int(rng.choice(np.arange(128, 513, 32)))
        nz = int(rng.choice(np.arange(256, 2049, 64)))
        L = int(rng.integers(4, 9))
        thick = [_log_uniform(rng, 20e-6, 1e-3) for _ in range(L)]
        amp = _log_uniform(rng, 1e8, 1e9)
        width = float(rng.uniform(0.5e-3, 3e-3))
        period = float(rng.uniform(5e-3, 50e-3))
        dt = period / 20_000
        out.append(_cell(rng, nr, nz, L, thick, dt, nsteps, amp, width, period))
    return out


def adjoint_cell(seed=0, z_active=False, nsteps=50_000, nr=512, nz=2048):
    """Adjoint workload: 512 x 2048 nodes, 6 layers of 20 um - 1 mm, 5e8
    W/m^3, 1 ms pulse every 10 ms, dt = 0.2 us, 50,000 steps."""
    rng = np.random.default_rng([4, seed])
    thick = [_log_uniform(rng, 20e-6, 1e-3) for _ in range(6)]
    cell = _cell(rng, nr, 2048, 6, thick, 2e-7, nsteps, 5e8, 1e-3, 10e-3,
                 z_active=z_active)
    cell["nz"] = int(nz)
    return cell


def design_cells(seed=0, n_designs=64, nsteps=100_000, nr=512, nz=1024):
    """Batched adjoint: 64 designs of 512 x 1024, period 10 ms, dt = 0.5 us,
    100,000 steps; per-design amplitude, width, layer count and
    thicknesses from the design-sweep ranges."""
    rng = np.random.default_rng([5, seed])
    out = []
    for _ in range(n_designs):
        L = int(rng.integers(4, 9))
        thick = [_log_uniform(rng, 20e-6, 1e-3) for _ in range(L)]
        amp = _log_uniform(rng, 1e8, 1e9)
        width = float(rng.uniform(0.5e-3, 3e-3))
        out.append(_cell(rng, nr, 1024, L, thick, 5e-7, nsteps, amp, width,
                         10e-3))
        out[-1]["nz"] = int(nz)
    return out


def tracking_target(cell, nsteps, t_hot=42.0, t_cold=T0):
    """Target surface temperature after each step n = 1..nsteps: t_hot while
    the nominal pulse is on at the end time n*dt of the step, else t_cold."""
    dt, P, w, t0 = cell["dt"], cell["period"], cell["width"], cell["t_on"]
    n = np.arange(1, nsteps + 1, dtype=np.float64)
    t = n * dt - t0
    phase = t - np.floor(t / P) * P
    on = (t >= 0) & (phase < w - 1e-9 * dt)
    return np.where(on, t_hot, t_cold).astype(np.float64)


def with_nz(cell, nz):
    """Copy of `cell` with a different axial node count; the axial spacing
    changes, the materials do not."""
    c = copy.deepcopy(cell)
    c["nz"] = int(nz)
    return c


def scaled(cell, **kw):
    """Copy of `cell` with top-level fields replaced."""
    c = copy.deepcopy(cell)
    c.update(kw)
    return c


def tiny(seed=0, nr=12, nz=6, n_layers=3, nsteps=20, z_active=True,
         dt=2e-7, amplitude=5e8, heater=None):
    """Small random cell for brute-force and derivative checks; the heater
    defaults to the second layer from the outside."""
    rng = np.random.default_rng([7, seed])
    thick = [_log_uniform(rng, 50e-6, 400e-6) for _ in range(n_layers)]
    eta = HEIGHT / (nz - 1)
    mats = [_draw_material(rng, eta, dt, 0.5) for _ in range(n_layers)]
    ints = allot_intervals(thick, nr - 1, minimum=2)
    layers = []
    for m in range(n_layers):
        d = dict(thickness=thick[m], intervals=ints[m])
        d.update(mats[m])
        layers.append(d)
    return dict(r_inner=R_INNER, height=HEIGHT, nr=nr, nz=nz, layers=layers,
                heater=max(0, n_layers - 2) if heater is None else heater,
                amplitude=float(amplitude),
                width=float(rng.uniform(0.3, 0.7) * nsteps * dt),
                period=float(nsteps * dt * 0.9), t_on=float(2.5 * dt),
                bc=_bc(z_active), dt=dt, T_init=T0, nsteps=nsteps)


def poly_variant(cell, seed=0, joule_tref=0.0):
    """Copy of `cell` with polynomial laws (the form of the paper's fits,
    Sec. 5: cubic capacity, quartic conductivity) drawn around each layer's
    power laws: c(T) = sum_k a_k T^k and lambda(T) = sum_k b_k T^k with
    positive coefficients whose terms share the power law's value at tref,
    lambda scaled by 0.8 so that it stays below the power law (and within
    the explicit-z bound the power law was drawn for) near T0.  joule_tref
    > 0 switches on the T^(-1/2) Joule source."""
    rng = np.random.default_rng([11, seed])
    c = copy.deepcopy(cell)
    for l in c["layers"]:
        wa = rng.dirichlet(np.ones(4)) * np.array([0.05, 0.1, 0.25, 1.0])
        wa /= wa.sum()
        wb = rng.dirichlet(np.ones(5))
        l["poly_a"] = [float(l["c0"] * wa[k] / l["tref"] ** k) for k in range(4)]
        l["poly_b"] = [float(0.8 * l["k0"] * wb[k] / l["tref"] ** k) for k in range(5)]
    c["poly"] = True
    c["joule_tref"] = float(joule_tref)
    return c


def frozen(name):
    """The problem dictionaries of a frozen workload (cellgen/frozen/NAME.json,
    written by cellgen/freeze.py): small_cell, small_cell_z_active,
    device_cell, device_cell_z_active, sweep_cells, adjoint_cell,
    design_cells, paper_shape."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "frozen", name + ".json")
    with open(path) as f:
        return json.load(f)["problems"]
