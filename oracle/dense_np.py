"""Second, independent oracle: the explicit-implicit step in plain NumPy.

TEST INFRASTRUCTURE ONLY (tests call it; nothing else does).  Written from
the paper's equations, not from ``oracle.c``: each interior line's rows are
assembled into a dense matrix, divided row by row by its diagonal, and
solved with ``numpy.linalg.solve``.  Every
operation is analytic in the temperatures and in the parameters (thickness,
conductivity scale, amplitude, pulse width away from step-aligned edges), so
running it in complex arithmetic gives complex-step derivatives,
Im J(theta + i h e_k) / h, exact to rounding.  For tiny grids only.

Scheme (Sec. 3):
  * grid, eq. (9): r_i = r_inner + sum of the interval widths, layer m has
    n_m equal intervals of d_m / n_m; eta = H / (nz - 1);
  * capacity rows, eqs. (8), (11), (13): rho c(T)/tau (T^_i - T_i) =
    Lambda_i[T^] + Lambda_j[T] + X, with
    Lambda_i[T] = [r_{i+1/2} lam_{i+1/2} (T_{i+1}-T_i)/h_{i+1}
                   - r_{i-1/2} lam_{i-1/2} (T_i-T_{i-1})/h_i] / (r_i hbar_i),
    Lambda_j[T] = [lam_{j+1/2} (T_{j+1}-T_j) - lam_{j-1/2} (T_j-T_{j-1})] / eta^2,
    face conductivities at the face-mean temperature of the old level, an
    r-face in the layer of its interval, a z-face in the node's layer;
  * interface rows, eq. (18): lam*_m h_{i+1} (T^_i - T^_{i-1}) =
    lam*_{m+1} h_i (T^_{i+1} - T^_i), lam* of the two layers at the old node
    temperature;
  * radial boundary rows, eq. (15) or a held value; z-boundary lines copied
    (insulated) or held after the interior lines, eq. (6);
  * source, eq. (4): amplitude times the pulse average over the step on the
    heater layer's capacity nodes;
  * objective: J = sum_n (S_n - target_n)^2 with S_n the trapezoid mean over
    z of T^ on r = r_max.
"""
from __future__ import annotations

import numpy as np


def _snap(x):
    """Pulse times in step units: snapped to the nearest integer within 1e-9
    relative (real values only; a complex value is left as it is)."""
    if np.iscomplexobj(x) and np.imag(x) != 0:
        return x
    x = float(np.real(x))
    n = round(x)
    return float(n) if abs(x - n) <= 1e-9 * max(abs(x), 1.0) else x


def pulse_average(cell, k, width=None):
    """Average over step k (time [k dt, (k+1) dt)) of the pulse gate."""
    dt = cell["dt"]
    b0 = _snap(cell["t_on"] / dt)
    W = _snap((cell["width"] if width is None else width) / dt)
    P = _snap(cell["period"] / dt)
    lo, hi = float(k), float(k + 1)
    s = 0.0
    n = 0
    while True:
        b = b0 + n * P
        if np.real(b) >= hi:
            break
        e = b + W
        # overlap of [lo, hi) with [b, e), branches chosen on real parts
        a = b if np.real(b) > lo else lo
        z = e if np.real(e) < hi else hi
        if np.real(z) > np.real(a):
            s = s + (z - a)
        n += 1
    return s


def grid(cell, thick=None):
    """Node radii, interval widths h (h[0] unused) and the layer of each
    interval (lay[i] for the interval (r_{i-1}, r_i))."""
    Ls = cell["layers"]
    th = [l["thickness"] for l in Ls] if thick is None else thick
    widths, lay = [], []
    for m, l in enumerate(Ls):
        for _ in range(l["intervals"]):
            widths.append(th[m] / l["intervals"])
            lay.append(m)
    nr = cell["nr"]
    assert len(widths) == nr - 1
    dt = np.result_type(*[np.asarray(w) for w in widths], float)
    h = np.zeros(nr, dtype=dt)
    h[1:] = widths
    r = np.zeros(nr, dtype=dt)
    r[0] = cell["r_inner"]
    for i in range(1, nr):
        r[i] = r[i - 1] + h[i]
    return r, h, [None] + lay


def _k(l, ks, T):
    return ks * l["k0"] * (T / l["tref"]) ** l["p"]


def _rc(l, T, dt):
    return l["rho"] * l["c0"] * (T / l["tref"]) ** l["q"] / dt


class _Setup:
    """Grid, node classes and parameters of a cell (thickness, conductivity
    scale, amplitude and width may be overridden, e.g. by complex values)."""

    def __init__(self, cell, thick=None, kscale=None, amplitude=None, width=None):
        Ls = cell["layers"]
        self.cell, self.Ls = cell, Ls
        self.nr, self.nz = cell["nr"], cell["nz"]
        self.ks = [l["k_scale"] for l in Ls] if kscale is None else kscale
        self.amp = cell["amplitude"] if amplitude is None else amplitude
        self.width = width
        self.r, self.h, self.lay = grid(cell, thick)
        self.dt, self.eta = cell["dt"], cell["height"] / (self.nz - 1)
        nr = self.nr
        # layer of a node = layer of its intervals; interface nodes sit
        # between intervals of two layers
        self.node_layer = [self.lay[1]] + [self.lay[i] for i in range(1, nr - 1)] + [self.lay[nr - 1]]
        self.iface = [False] * nr
        for i in range(1, nr - 1):
            if self.lay[i] != self.lay[i + 1]:
                self.iface[i] = True


def assemble(st, T, j, X):
    """Dense matrix M and right-hand side F of interior line j (rows of
    eqs. (13), (18) and (15)), coefficients from the old field T."""
    cell, Ls, ks, r, h, lay = st.cell, st.Ls, st.ks, st.r, st.h, st.lay
    nr, bc = st.nr, cell["bc"]
    M = np.zeros((nr, nr), dtype=T.dtype)
    F = np.zeros(nr, dtype=T.dtype)
    for i in range(nr):
        if i == 0 or i == nr - 1:
            side = 0 if i == 0 else 1
            M[i, i] = 1.0
            if bc[side][0] == 1:
                F[i] = bc[side][1]
            else:
                M[i, 1 if i == 0 else nr - 2] = -1.0
            continue
        if st.iface[i]:
            a, b = lay[i], lay[i + 1]
            la = _k(Ls[a], ks[a], T[j, i])
            lb = _k(Ls[b], ks[b], T[j, i])
            M[i, i - 1] = -la * h[i + 1]
            M[i, i] = la * h[i + 1] + lb * h[i]
            M[i, i + 1] = -lb * h[i]
            continue
        m = st.node_layer[i]
        lw = _k(Ls[lay[i]], ks[lay[i]], 0.5 * (T[j, i] + T[j, i - 1]))
        le = _k(Ls[lay[i + 1]], ks[lay[i + 1]], 0.5 * (T[j, i] + T[j, i + 1]))
        hb = 0.5 * (h[i] + h[i + 1])
        gw = 0.5 * (r[i] + r[i - 1]) / (r[i] * hb * h[i])
        ge = 0.5 * (r[i] + r[i + 1]) / (r[i] * hb * h[i + 1])
        rc = _rc(Ls[m], T[j, i], st.dt)
        ln = _k(Ls[m], ks[m], 0.5 * (T[j, i] + T[j + 1, i]))
        ls = _k(Ls[m], ks[m], 0.5 * (T[j, i] + T[j - 1, i]))
        lz = (ln * (T[j + 1, i] - T[j, i]) - ls * (T[j, i] - T[j - 1, i])) / st.eta ** 2
        M[i, i - 1] = -gw * lw
        M[i, i + 1] = -ge * le
        M[i, i] = rc + gw * lw + ge * le
        F[i] = rc * T[j, i] + lz + (X if m == cell["heater"] else 0.0)
    return M, F


def forward(cell, T0=None, nsteps=None, thick=None, kscale=None, amplitude=None, width=None,
            dtype=np.float64):
    """(final field [nz][nr], surface trace S[n]) after nsteps steps."""
    st = _Setup(cell, thick, kscale, amplitude, width)
    nr, nz, bc = st.nr, st.nz, cell["bc"]
    n = int(cell["nsteps"] if nsteps is None else nsteps)
    T = (np.full((nz, nr), cell["T_init"], dtype=dtype) if T0 is None
         else np.array(T0, dtype=dtype))
    wz = np.full(nz, 1.0 / (nz - 1))
    wz[0] = wz[-1] = 0.5 / (nz - 1)
    S = []
    for k in range(n):
        X = st.amp * pulse_average(cell, k, width)
        Tn = T.copy()
        for j in range(1, nz - 1):
            M, F = assemble(st, T, j, X)
            # rows differ in scale by ~1e15 (interface rows vs capacity rows):
            # divide each by its diagonal before the pivoted dense solve
            d = np.diag(M).copy()
            Tn[j] = np.linalg.solve(M / d[:, None], F / d)
        for side, jb, js in ((2, 0, 1), (3, nz - 1, nz - 2)):
            Tn[jb] = bc[side][1] if bc[side][0] == 1 else Tn[js]
        T = Tn
        S.append(np.dot(wz, T[:, nr - 1]))
    return T, np.array(S)


def objective(cell, target, **kw):
    _, S = forward(cell, **kw)
    return np.sum((S - np.asarray(target[: len(S)])) ** 2)


def complex_step_gradient(cell, target, nsteps, h=1e-30, include_width=True):
    """dJ/d[amplitude, width, thickness_m, k_scale_m] by complex steps."""
    Ls = cell["layers"]
    L = len(Ls)
    th = [l["thickness"] for l in Ls]
    ks = [l["k_scale"] for l in Ls]
    base = dict(nsteps=nsteps, dtype=np.complex128)
    g = np.zeros(2 + 2 * L)
    amp = cell["amplitude"]
    g[0] = np.imag(objective(cell, target, amplitude=amp * (1 + 1j * h), **base)) / (amp * h)
    if include_width:
        w = cell["width"]
        g[1] = np.imag(objective(cell, target, width=w * (1 + 1j * h), **base)) / (w * h)
    else:
        g[1] = np.nan
    for m in range(L):
        t2 = [complex(x) for x in th]
        t2[m] = th[m] * (1 + 1j * h)
        g[2 + m] = np.imag(objective(cell, target, thick=t2, **base)) / (th[m] * h)
        k2 = [complex(x) for x in ks]
        k2[m] = ks[m] * (1 + 1j * h)
        g[2 + L + m] = np.imag(objective(cell, target, kscale=k2, **base)) / (ks[m] * h)
    return g
