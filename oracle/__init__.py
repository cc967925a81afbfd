"""Python access to the plain FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product path never imports this
package.  The oracle follows the paper's scheme (eqs. (8)-(20)) literally; see
the header of ``oracle.c`` for the readings it takes.  ``dense_np`` is a second,
independent implementation (dense NumPy solves, complex-step capable) that
pins this one.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")


def build(force=True):
    """Compile liboracle.so with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-Wextra", "-o", _SO, _SRC, "-lm"]
        subprocess.check_call(cmd, cwd=_HERE)
    return _SO


class _OCell(C.Structure):
    _fields_ = [
        ("r_inner", C.c_double), ("height", C.c_double),
        ("nr", C.c_int), ("nz", C.c_int), ("n_layers", C.c_int),
        ("heater", C.c_int),
        ("thick", C.POINTER(C.c_double)), ("intervals", C.POINTER(C.c_int)),
        ("k0", C.POINTER(C.c_double)), ("p", C.POINTER(C.c_double)),
        ("kscale", C.POINTER(C.c_double)),
        ("c0", C.POINTER(C.c_double)), ("q", C.POINTER(C.c_double)),
        ("rho", C.POINTER(C.c_double)), ("tref", C.POINTER(C.c_double)),
        ("amplitude", C.c_double), ("width", C.c_double),
        ("period", C.c_double), ("t_on", C.c_double),
        ("bc_kind", C.c_int * 4), ("bc_value", C.c_double * 4),
        ("dt", C.c_double), ("turn_on", C.c_int),
        ("poly_a", C.POINTER(C.c_double)), ("poly_b", C.POINTER(C.c_double)),
        ("joule_tref", C.c_double),
        ("z_full", C.c_int), ("nr_top", C.c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        dp = C.POINTER(C.c_double)
        cp = C.POINTER(_OCell)
        L.oc_radii.argtypes = [cp, dp]
        L.oc_source_fraction.argtypes = [cp, C.c_long]
        L.oc_source_fraction.restype = C.c_double
        L.oc_turn_on_source.argtypes = [cp, C.c_long, C.c_int]
        L.oc_turn_on_source.restype = C.c_double
        L.oc_source_fraction_dwidth.argtypes = [cp, C.c_long]
        L.oc_source_fraction_dwidth.restype = C.c_double
        L.oc_line_rows.argtypes = [cp, dp, C.c_long, C.c_int, dp, dp, dp, dp]
        L.oc_thomas.argtypes = [C.c_int, dp, dp, dp, dp, dp]
        L.oc_line_paper_sweep.argtypes = [cp, dp, C.c_long, C.c_int, dp]
        L.oc_forward.argtypes = [cp, dp, C.c_long, C.c_long, dp, C.c_int]
        L.oc_gradient.argtypes = [cp, dp, C.c_long, dp, C.c_long, dp, dp, dp,
                                  dp, C.c_int]
        _lib = L
    return _lib


class _Cell:
    """Keeps the numpy arrays behind an _OCell alive."""

    def __init__(self, cell):
        Ls = cell["layers"]
        f = lambda key: np.ascontiguousarray([float(l[key]) for l in Ls])
        self.arrs = dict(thick=f("thickness"), k0=f("k0"), p=f("p"),
                         kscale=f("k_scale"), c0=f("c0"), q=f("q"),
                         rho=f("rho"), tref=f("tref"))
        self.ints = np.ascontiguousarray([int(l["intervals"]) for l in Ls],
                                         dtype=np.int32)
        s = _OCell()
        s.r_inner = cell["r_inner"]
        s.height = cell["height"]
        s.nr, s.nz = int(cell["nr"]), int(cell["nz"])
        s.n_layers = len(Ls)
        s.heater = int(cell["heater"])
        dp = C.POINTER(C.c_double)
        for k, a in self.arrs.items():
            setattr(s, k, a.ctypes.data_as(dp))
        s.intervals = self.ints.ctypes.data_as(C.POINTER(C.c_int))
        s.amplitude = cell["amplitude"]
        s.width = cell["width"]
        s.period = cell["period"]
        s.t_on = cell["t_on"]
        for q in range(4):
            s.bc_kind[q] = int(cell["bc"][q][0])
            s.bc_value[q] = float(cell["bc"][q][1])
        s.dt = cell["dt"]
        s.turn_on = int(bool(cell.get("turn_on", False)))
        if cell.get("poly"):
            # eqs. (23), (24): per layer poly_a (4 values) and poly_b (5)
            self.pa = np.ascontiguousarray([float(x) for l in Ls for x in l["poly_a"]])
            self.pb = np.ascontiguousarray([float(x) for l in Ls for x in l["poly_b"]])
            assert self.pa.size == 4 * len(Ls) and self.pb.size == 5 * len(Ls)
            s.poly_a = self.pa.ctypes.data_as(dp)
            s.poly_b = self.pb.ctypes.data_as(dp)
        s.joule_tref = float(cell.get("joule_tref", 0.0))
        # eq. (9), stepped domain: {"z_full": j0, "nr_top": N_t}
        st = cell.get("stepped")
        if st:
            s.z_full, s.nr_top = int(st["z_full"]), int(st["nr_top"])
        self.s = s

    def ref(self):
        return C.byref(self.s)


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _check(rc, what):
    if rc != 0:
        raise ValueError("oracle: %s rejected the problem" % what)


def initial_field(cell):
    return np.full((cell["nz"], cell["nr"]), float(cell["T_init"]))


def radii(cell):
    c = _Cell(cell)
    r = np.zeros(cell["nr"])
    _check(lib().oc_radii(c.ref(), _dp(r)), "radii")
    return r


def source_fraction(cell, k):
    return lib().oc_source_fraction(_Cell(cell).ref(), int(k))


def turn_on_source(cell, k, i):
    """Source factor of sub-step i of pulse-start step k, eq. (22)."""
    return lib().oc_turn_on_source(_Cell(cell).ref(), int(k), int(i))


def source_fraction_dwidth(cell, k):
    return lib().oc_source_fraction_dwidth(_Cell(cell).ref(), int(k))


def line_rows(cell, T, k, j):
    c = _Cell(cell)
    T = np.ascontiguousarray(T, dtype=np.float64)
    out = [np.zeros(cell["nr"]) for _ in range(4)]
    _check(lib().oc_line_rows(c.ref(), _dp(T), int(k), int(j),
                              *[_dp(a) for a in out]), "line_rows")
    return out


def thomas(A, B, Cc, F):
    n = len(B)
    A, B, Cc, F = [np.ascontiguousarray(a, dtype=np.float64) for a in (A, B, Cc, F)]
    x = np.zeros(n)
    _check(lib().oc_thomas(n, _dp(A), _dp(B), _dp(Cc), _dp(F), _dp(x)), "thomas")
    return x


def line_paper_sweep(cell, T, k, j):
    c = _Cell(cell)
    T = np.ascontiguousarray(T, dtype=np.float64)
    x = np.zeros(cell["nr"])
    _check(lib().oc_line_paper_sweep(c.ref(), _dp(T), int(k), int(j), _dp(x)),
           "line_paper_sweep")
    return x


def forward(cell, T=None, k0=0, nsteps=None, surf=False, nthreads=0):
    """Advance T (default: the uniform initial field) by nsteps steps from
    global step k0.  Returns T, or (T, surface trace) when surf is set."""
    c = _Cell(cell)
    T = initial_field(cell) if T is None else np.array(T, dtype=np.float64)
    T = np.ascontiguousarray(T)
    n = int(cell["nsteps"] if nsteps is None else nsteps)
    S = np.zeros(max(n, 1)) if surf else None
    rc = lib().oc_forward(c.ref(), _dp(T), int(k0), n,
                          _dp(S) if surf else None, int(nthreads))
    _check(rc, "forward")
    return (T, S[:n]) if surf else T


def gradient(cell, target, T0=None, nsteps=None, ckpt=0, nthreads=0,
             want_lam0=False):
    """J and dJ/d[amplitude, width, thickness_m..., k_scale_m...] by the
    discrete adjoint; also the surface trace (and dJ/dT0 if asked)."""
    c = _Cell(cell)
    T0 = initial_field(cell) if T0 is None else np.ascontiguousarray(T0, dtype=np.float64)
    n = int(cell["nsteps"] if nsteps is None else nsteps)
    target = np.ascontiguousarray(target[:n], dtype=np.float64)
    ng = 2 + 2 * len(cell["layers"])
    J = np.zeros(1)
    g = np.zeros(ng)
    S = np.zeros(n)
    lam0 = np.zeros_like(T0) if want_lam0 else None
    rc = lib().oc_gradient(c.ref(), _dp(T0), n, _dp(target), int(ckpt), _dp(J),
                           _dp(g), _dp(S), _dp(lam0) if want_lam0 else None,
                           int(nthreads))
    _check(rc, "gradient")
    if want_lam0:
        return float(J[0]), g, S, lam0
    return float(J[0]), g, S
