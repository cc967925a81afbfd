"""Host-side checks of the C ABI (no device calls): the library loads and
exports every declared symbol, descriptors are validated, the explicit
stability bound (eq. (21)) is enforced, and the library's own grid and pulse
schedule agree with the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

import cellgen
import oracle
import paper_1408_5853_amd as P
from paper_1408_5853_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "cryocell.h")).read()
    return sorted(set(re.findall(r"\b(cryo_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_abi.LIB_PATH)
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_abi.SYMBOLS)


def test_validation_rejects_bad_descriptors():
    good = cellgen.small_cell(0)
    P.validate(good)
    bad = []
    c = cellgen.scaled(good); c["layers"] = [dict(l) for l in c["layers"]]
    c["layers"][0]["intervals"] = 1; bad.append(c)
    c = cellgen.scaled(good, nr=good["nr"] + 1); bad.append(c)
    c = cellgen.scaled(good, heater=7); bad.append(c)
    c = cellgen.scaled(good, width=2.0 * good["period"]); bad.append(c)
    c = cellgen.scaled(good, nz=2); bad.append(c)
    c = cellgen.scaled(good, bc=[[2, 0.0]] * 4); bad.append(c)
    c = cellgen.scaled(good, r_inner=0.0); bad.append(c)    # held axis
    for c in bad:
        with pytest.raises(P.CryoError) as e:
            P.validate(c)
        assert e.value.status == 1


def test_unstable_dt_is_refused():
    c = cellgen.small_cell(0)
    dmax = P.stability_dt_max(c, 28.0)
    assert c["dt"] <= dmax
    P.Plan(cellgen.scaled(c, dt=0.999 * dmax))
    with pytest.raises(P.CryoError) as e:
        P.Plan(cellgen.scaled(c, dt=1.01 * dmax))
    assert e.value.status == 2


def test_stability_bound_formula():
    # eq. (21): tau <= eta^2/2 * min rho c / lambda, here at T = tref
    c = cellgen.small_cell(1)
    eta = c["height"] / (c["nz"] - 1)
    want = min(l["rho"] * l["c0"] / (l["k_scale"] * l["k0"]) for l in c["layers"])
    assert P.stability_dt_max(c, 30.0) == pytest.approx(0.5 * eta * eta * want, rel=1e-14)


def _binom8_bound(e):
    # first term the degree-7 binomial series of (1 + u)^e drops, |u| <= 2^-7
    c = 1.0
    for k in range(1, 9):
        c *= (e - (k - 1)) / k
    return abs(c) * 2.0 ** -56


def with_exponents(c, ps):
    """Copy of `c` with conductivity exponents `ps`; k0 lowered where needed
    so that eq. (21) still holds at the coldest temperature (28 K)."""
    c = cellgen.scaled(c)
    c["layers"] = [dict(l) for l in c["layers"]]
    eta = c["height"] / (c["nz"] - 1)
    for l, p in zip(c["layers"], ps):
        l["p"] = float(p)
        x = 28.0 / l["tref"]
        cap = 0.5 * eta * eta * l["rho"] * l["c0"] * x ** l["q"] / (2 * c["dt"] * x ** p)
        l["k0"] = min(l["k0"], cap)
    return c


def test_power_law_exponents_outside_series_range_refused():
    # the FP64 table powers cut the binomial series of (1 + u)^e after degree
    # 7: exponents whose first dropped term exceeds 1e-14 are refused, for
    # the layers' own laws and for the interface ratio laws p_m - p_{m+1}
    base = cellgen.small_cell(0)
    assert _binom8_bound(-5.2) < 1e-14 < _binom8_bound(-5.5)
    assert _binom8_bound(12.3) < 1e-14 < _binom8_bound(12.6)
    P.validate(with_exponents(base, [1.0, -4.0, 1.2, 1.0]))       # ratios 5.0, -5.2
    P.validate(with_exponents(base, [0.5, 2.0, 0.5, 2.0]))
    for ps in ([1.0, -5.5, -5.5, 1.0],          # a layer's own exponent
               [1.0, -4.0, 1.5, 1.0],           # ratio -5.5 between layers 1 and 2
               [13.0, 13.0, 13.0, 13.0]):
        with pytest.raises(P.CryoError) as e:
            P.validate(with_exponents(base, ps))
        assert e.value.status == 6 and "series" in P.lib().cryo_last_error().decode()
    c = cellgen.scaled(base)
    c["layers"] = [dict(l) for l in c["layers"]]
    c["layers"][2]["q"] = -6.0                  # capacity exponent
    with pytest.raises(P.CryoError) as e:
        P.validate(c)
    assert e.value.status == 6


def test_nr_above_limit_unsupported():
    c = cellgen.small_cell(0)
    c = cellgen.scaled(c, nr=4097)
    c["layers"] = [dict(l) for l in c["layers"]]
    c["layers"][0]["intervals"] += 4097 - 64
    with pytest.raises(P.CryoError) as e:
        P.validate(c)
    assert e.value.status == 6


@pytest.mark.parametrize("make", [lambda: cellgen.small_cell(0), lambda: cellgen.device_cell(0),
                                  lambda: cellgen.sweep_cells(0, 3)[2],
                                  lambda: cellgen.tiny(1)])
def test_library_grid_and_schedule_match_oracle(make):
    c = make()
    pl = P.Plan(c)
    assert np.allclose(pl.radii(), oracle.radii(c), rtol=1e-15, atol=0)
    n = 5000
    s = pl.source_fraction(0, n)
    so = np.array([oracle.source_fraction(c, k) for k in range(n)])
    assert np.max(np.abs(s - so)) < 1e-9


def test_workspace_grows_with_grid():
    a = P.Plan(cellgen.small_cell(0)).workspace_bytes(100)
    b = P.Plan(cellgen.device_cell(0, nz=64)).workspace_bytes(100)
    assert 0 < a < b


def test_turn_on_model_host_checks():
    # eq. (22) needs pulse starts on step boundaries; host-only checks
    c = cellgen.with_nz(cellgen.small_cell(0), 4)
    dt = c["dt"]
    P.Plan(dict(c, turn_on=True))                                   # t_on = 0
    P.Plan(dict(c, turn_on=True, width=0.0, t_on=2.5 * dt))        # no pulse: nothing to expand
    for bad in (dict(t_on=2.5 * dt), dict(period=1000.5 * dt)):
        with pytest.raises(P.CryoError) as e:
            P.Plan(dict(c, turn_on=True, **bad))
        assert e.value.status == 6
    plan = P.Plan(dict(c, turn_on=True))
    plan.set_shape(4, 2, 1)                 # the sub-step tables follow
    plan.set_turn_on(False)
    plan.set_turn_on(True)
    # the gradient's workspace counts the sub-steps among its kernel steps
    plain = P.Plan(c)
    L = P.lib()
    b_on, b_off = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.cryo_gradient_workspace_bytes(plan._h, 40, 1, ctypes.byref(b_on)) == 0
    assert L.cryo_gradient_workspace_bytes(plain._h, 40, 1, ctypes.byref(b_off)) == 0
    assert b_on.value > b_off.value


def test_polynomial_laws_host_checks():
    c = cellgen.poly_variant(cellgen.with_nz(cellgen.small_cell(0), 4), 0, joule_tref=30.0)
    plan = P.Plan(c)                                        # FP64, laws accepted
    P.Plan(c, "f32")                                        # and FP32
    Ls = c["layers"]
    a = [l["poly_a"] for l in Ls]
    zero_b = [[0.0] * 5 for _ in Ls]
    with pytest.raises(P.CryoError) as e:
        P.Plan(dict(c, poly=False)).set_poly_laws(a, zero_b)          # lambda = 0
    assert e.value.status == 1
    big_b = [[1e6 * x for x in l["poly_b"]] for l in Ls]
    with pytest.raises(P.CryoError) as e:
        P.Plan(dict(c, poly=False)).set_poly_laws(a, big_b)           # eq. (21) bound
    assert e.value.status == 2
    with pytest.raises(ValueError):
        plan.set_poly_laws(a[:-1], zero_b)
    P.Plan(dict(c, turn_on=True))                           # with the turn-on model
    # the gradient takes the polynomial laws (FP64 plans; the host check
    # refuses an FP32 plan before any device work)
    L = P.lib()
    tgt = np.zeros(4)
    J, g = ctypes.c_double(), np.zeros(2 + 2 * len(Ls))
    dp = ctypes.POINTER(ctypes.c_double)
    f32 = P.Plan(c, "f32")
    st = L.cryo_gradient(f32._h, ctypes.c_void_p(256), 4, tgt.ctypes.data_as(dp), 0,
                         ctypes.c_void_p(256), 1 << 40, ctypes.byref(J), g.ctypes.data_as(dp),
                         None, None)
    assert st == 6 and "FP64" in P.lib().cryo_last_error().decode()


def test_stepped_domain_host_checks():
    c = cellgen.with_nz(cellgen.small_cell(0), 10)
    P.Plan(dict(c, stepped=dict(z_full=4, nr_top=20)))
    P.Plan(dict(c, stepped=dict(z_full=4, nr_top=20)), "f32")
    for bad in (dict(z_full=0, nr_top=20), dict(z_full=9, nr_top=20),
                dict(z_full=4, nr_top=2), dict(z_full=4, nr_top=c["nr"] + 1)):
        with pytest.raises(P.CryoError) as e:
            P.Plan(dict(c, stepped=bad))
        assert e.value.status == 1
    pc = cellgen.poly_variant(c, 0)
    P.Plan(dict(pc, stepped=dict(z_full=4, nr_top=20)))     # with polynomial laws
    plan = P.Plan(dict(c, stepped=dict(z_full=4, nr_top=20), turn_on=True))
    L = P.lib()
    tgt = np.zeros(4)
    J, g = ctypes.c_double(), np.zeros(2 + 2 * len(c["layers"]))
    dp = ctypes.POINTER(ctypes.c_double)
    # the adjoint's extra tables must fit a workgroup's LDS: refused up front
    big = cellgen.tiny(3, nr=1500, nz=6, n_layers=5, nsteps=10, z_active=True, dt=2e-7,
                       amplitude=5e9)
    bp = P.Plan(dict(big, stepped=dict(z_full=3, nr_top=500)))
    assert bp.shape()[:2] == (8, 4)
    st = L.cryo_gradient(bp._h, ctypes.c_void_p(256), 4, tgt.ctypes.data_as(dp), 0,
                         ctypes.c_void_p(256), 1 << 40, ctypes.byref(J), g.ctypes.data_as(dp),
                         None, None)
    assert st == 6 and "LDS" in P.lib().cryo_last_error().decode()


def test_batch_plan_options():
    # polynomial laws, the stepped domain and the turn-on model are
    # per-instance batch options (cryo_batch_create_with, host-side checks
    # only here; the batch tuner takes them too, on the GPU)
    base = cellgen.small_cell(0)
    poly = cellgen.poly_variant(base, 0, joule_tref=30.0)
    stepped = dict(base, stepped={"z_full": 60, "nr_top": 30})
    b = P.Batch([base, poly, stepped, dict(poly, stepped={"z_full": 60, "nr_top": 30})], "f64")
    assert len(b.offsets) == 5
    b.close()
    with pytest.raises(P.CryoError) as e:                          # nr_top > nr
        P.Batch([base, dict(base, stepped={"z_full": 60, "nr_top": base["nr"] + 1})], "f64")
    assert "instance 1" in str(e.value)
    b = P.Batch([base, dict(base, turn_on=True), dict(poly, turn_on=True, stepped={"z_full": 60,
                                                                                 "nr_top": 30})],
                "f32")
    assert len(b.offsets) == 4
    b.close()
    with pytest.raises(P.CryoError) as e:     # the turn-on model needs pulse starts on steps
        P.Batch([base, dict(base, turn_on=True, t_on=2.5 * base["dt"])], "f64")
    assert e.value.status == 6 and "instance 1" in str(e.value)


def test_gradient_store_host_checks():
    # the stored tail replaces checkpoints and the segment buffer: the
    # workspace changes by whole fields, and a store beyond the run's kernel
    # steps is the same as storing all of them
    plan = P.Plan(cellgen.with_nz(cellgen.adjoint_cell(0), 64))
    plan._gradient_ready()
    rpl, wpl, _ = plan.shape()
    F = (8 * 64 * 64 * wpl * rpl + 255) // 256 * 256
    N = 100

    def ws(store):
        plan.set_gradient_store(store)
        return plan.gradient_workspace_bytes(N)

    base = ws(0)          # 2 forward buffers, 10 checkpoints, 10 segment states, 6 adjoint fields
    assert ws(40) - base == ((2 + 8 + 8 + 41 + 6) - (2 + 10 + 10 + 6)) * F    # head 60: K = nck = 8
    assert ws(N) - base == ((2 + N + 1 + 6) - (2 + 10 + 10 + 6)) * F          # no head at all
    assert ws(10 ** 9) == ws(N)
    # the budget query is the largest fitting store, by brute force (the
    # workspace is not monotone in the store: the head's checkpoints and
    # segment shrink in steps)
    sizes = [ws(d) for d in range(N + 1)]
    for budget in [base - 1, base, base + 37 * F, base + 37 * F + 1, sizes[N] - 1, sizes[N],
                   sizes[N] + 10 * F]:
        want = max([d for d in range(N + 1) if sizes[d] <= budget], default=0)
        assert plan.gradient_store_for(N, budget) == want, budget
    plan.set_gradient_store(0)
    with pytest.raises(P.CryoError) as e:
        plan.set_gradient_store(-1)
    assert e.value.status == 1


def test_gradient_store_counts_turn_on_sub_steps():
    # the store counts kernel steps: with the turn-on model (eq. (22)) the
    # pulse start at step 0 adds 99 sub-steps, so storing everything of a
    # 100-step run means 199 states
    c = dict(cellgen.with_nz(cellgen.adjoint_cell(0), 64), turn_on=True)
    plan = P.Plan(c)
    assert plan.gradient_store_for(100, 1 << 50) == 199
    plan.set_gradient_store(199)
    all_stored = plan.gradient_workspace_bytes(100)
    plan.set_gradient_store(10 ** 6)
    assert plan.gradient_workspace_bytes(100) == all_stored
    plain = P.Plan(cellgen.with_nz(cellgen.adjoint_cell(0), 64))
    assert plain.gradient_store_for(100, 1 << 50) == 100


def test_new_entry_points_refuse_bad_arguments():
    # host-side argument checks of the gradient store calls and the batch
    # tuner with options (no device work happens before them)
    L = P.lib()
    plan = P.Plan(cellgen.with_nz(cellgen.adjoint_cell(0), 64))
    d = ctypes.c_int64()
    assert L.cryo_plan_set_gradient_store(None, 5) == 1
    assert L.cryo_gradient_store_steps(None, 10, 0, 1 << 30, ctypes.byref(d)) == 1
    assert L.cryo_gradient_store_steps(plan._h, 0, 0, 1 << 30, ctypes.byref(d)) == 1
    assert L.cryo_gradient_store_steps(plan._h, 10, -1, 1 << 30, ctypes.byref(d)) == 1
    assert L.cryo_gradient_store_steps(plan._h, 10, 0, 1 << 30, None) == 1
    assert L.cryo_gradient_store_steps(plan._h, 10, 0, 0, ctypes.byref(d)) == 0 and d.value == 0
    shapes = (ctypes.c_int32 * 3)()
    assert L.cryo_batch_autotune_with(0, None, 0, None, 32, None, None, shapes) == 1
    assert L.cryo_batch_autotune_with(1, plan._ps.ref(), 0, None, 0, None, None, shapes) == 1
