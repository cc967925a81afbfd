"""Parity of the HIP stepper with the FP64 CPU oracle, element by element.

FP64 must agree to 1e-10 relative, FP32 to 1e-4 K (absolute), on the field
after the run and on the surface-mean trace.  Sizes span one to several
register chunks per lane, ragged (non power-of-two) radial lengths, the
smallest axial extent and every boundary combination.
"""
import numpy as np
import pytest

import cellgen
import oracle
from gpu_util import rel_err, run_gpu, say

pytestmark = pytest.mark.gpu

F64_TOL = 1e-10
F32_TOL_K = 1e-4


def _check64(cell, nsteps, T0=None, k0=0):
    say("case nr=%d nz=%d steps=%d k0=%d" % (cell["nr"], cell["nz"], nsteps, k0))
    Tg, Sg = run_gpu(cell, nsteps, T0=T0, k0=k0)
    To, So = oracle.forward(cell, T0, k0=k0, nsteps=nsteps, surf=True)
    e, es = rel_err(Tg, To), rel_err(Sg, So)
    say("  max rel err field %.3e surface %.3e" % (e, es))
    assert e < F64_TOL and es < F64_TOL
    return Tg, To


def test_small_cell_full_run_f64():
    _check64(cellgen.small_cell(0), 10_000)


def test_small_cell_z_active_twin_full_run_f64():
    Tg, To = _check64(cellgen.small_cell(0, z_active=True), 10_000)
    assert np.ptp(To[:, -1]) > 1e-3      # the axial half is exercised


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_small_cell_seeds_f64(seed):
    _check64(cellgen.small_cell(seed, z_active=seed % 2 == 0), 3000)


@pytest.mark.parametrize("nr,nz", [(5, 3), (64, 4), (100, 7), (129, 5), (300, 9), (631, 6),
                                   (1024, 5), (1500, 4), (2048, 3)])
def test_ragged_shapes_random_fields_f64(nr, nz):
    c = cellgen.tiny(nr, nr=nr, nz=nz, n_layers=min(5, (nr - 1) // 2), nsteps=40,
                     z_active=True, dt=2e-7, amplitude=5e9)
    rng = np.random.default_rng(nr)
    T0 = 28.0 + rng.uniform(0, 6, size=(nz, nr))
    _check64(c, 40, T0=T0, k0=3)


@pytest.mark.parametrize("bc", [
    [[0, 0], [0, 0], [0, 0], [0, 0]],
    [[1, 28], [1, 29], [1, 30], [1, 31]],
    [[0, 0], [1, 28], [1, 28], [0, 0]],
    [[1, 27], [0, 0], [0, 0], [1, 33]],
])
def test_boundary_combinations_f64(bc):
    c = cellgen.tiny(9, nr=77, nz=6, n_layers=3, z_active=True, dt=2e-7, amplitude=5e9)
    c["bc"] = [list(map(float, b)) for b in bc]
    c["bc"] = [[int(b[0]), b[1]] for b in c["bc"]]
    rng = np.random.default_rng(5)
    T0 = 28.0 + rng.uniform(0, 4, size=(c["nz"], c["nr"]))
    _check64(c, 60, T0=T0)


def test_device_cell_reduced_axis_f64():
    # the as-written device cell is exactly z-invariant, so its oracle runs at
    # nz = 4 with the same radial grid, dt and steps
    c = cellgen.device_cell(0, nz=4)
    _check64(c, 3000)


def test_device_cell_full_size_z_invariant_and_matches_reduced():
    c = cellgen.device_cell(0)
    n = 200
    say("case device_cell full size, %d steps" % n)
    Tg, Sg = run_gpu(c, n)
    assert np.all(Tg == Tg[1][None, :]), "lines differ: a race or halo error"
    To, So = oracle.forward(cellgen.device_cell(0, nz=4), nsteps=n, surf=True)
    assert rel_err(Tg[1], To[1]) < F64_TOL
    assert rel_err(Sg, So) < F64_TOL


def test_paper_shape_prefix_f64():
    c = cellgen.with_nz(cellgen.paper_shape(0), 5)
    _check64(c, 2000)


def test_restart_is_bitwise_equal():
    c = cellgen.small_cell(0, z_active=True)
    T1, S1 = run_gpu(c, 700)
    Ta, Sa = run_gpu(c, 300)
    Tb, Sb = run_gpu(c, 400, T0=Ta, k0=300)
    assert np.array_equal(T1, Tb)
    assert np.array_equal(S1, np.concatenate([Sa, Sb]))


def test_run_to_run_bitwise_determinism():
    c = cellgen.small_cell(3, z_active=True)
    a = run_gpu(c, 500)
    b = run_gpu(c, 500)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_zero_steps_is_identity():
    c = cellgen.small_cell(0)
    rng = np.random.default_rng(0)
    T0 = 28 + rng.uniform(0, 1, size=(c["nz"], c["nr"]))
    T, _ = run_gpu(c, 0, T0=T0, surf=False)
    assert np.array_equal(T, T0)


def test_nonfinite_input_is_reported():
    import paper_1408_5853_amd as P
    c = cellgen.small_cell(0)
    T0 = np.full((c["nz"], c["nr"]), 28.0)
    T0[5, 7] = np.nan
    with pytest.raises(P.CryoError) as e:
        run_gpu(c, 3, T0=T0)
    assert e.value.status == 4


@pytest.mark.parametrize("make,n", [(lambda: cellgen.small_cell(0), 10_000),
                                    (lambda: cellgen.small_cell(0, z_active=True), 10_000),
                                    (lambda: cellgen.device_cell(0, nz=4), 20_000)])
def test_f32_within_1e4_kelvin(make, n):
    c = make()
    say("case f32 nr=%d nz=%d steps=%d" % (c["nr"], c["nz"], n))
    Tg, Sg = run_gpu(c, n, dtype="f32")
    To, So = oracle.forward(c, nsteps=n, surf=True)
    e, es = float(np.max(np.abs(Tg - To))), float(np.max(np.abs(Sg - So)))
    say("  max abs err field %.3e K surface %.3e K" % (e, es))
    assert e < F32_TOL_K and es < F32_TOL_K


SHAPES = [(2, 1), (3, 1), (4, 1), (5, 1), (6, 1), (7, 1), (8, 1), (10, 1), (12, 1), (16, 1),
          (4, 2), (8, 2), (4, 4), (8, 4)]


@pytest.mark.parametrize("shape", SHAPES)
def test_every_chunk_shape_matches_oracle(shape):
    import torch

    import paper_1408_5853_amd as P
    rpl, wpl = shape
    nr = min(64 * rpl * wpl, 300)
    c = cellgen.tiny(nr, nr=nr, nz=7, n_layers=4, z_active=True, dt=2e-7, amplitude=5e9)
    rng = np.random.default_rng(3)
    T0 = 28.0 + rng.uniform(0, 5, size=(c["nz"], c["nr"]))
    To = oracle.forward(c, T0, nsteps=30)
    for lpw in (1, 2, 5):
        say("case shape %s lines/wave %d nr %d" % (shape, lpw, nr))
        plan = P.Plan(c)
        plan.set_shape(rpl, wpl, lpw)
        T = plan.field_from(T0)
        ws = plan.workspace(30)
        plan.forward(T, 0, 30, ws=ws)
        plan.poll(ws)
        torch.cuda.synchronize()
        Tg = plan.field_values(T)
        assert rel_err(Tg, To) < F64_TOL
        if lpw == 1:
            ref = Tg
        else:
            assert np.array_equal(Tg, ref)      # the march order changes nothing


@pytest.mark.parametrize("shape", SHAPES)
def test_every_chunk_shape_f32_pairs_match_oracle(shape):
    """FP32 pairs through every kernel shape (with and without the LDS line
    ring), at ragged nr, against the FP64 oracle."""
    import torch

    import paper_1408_5853_amd as P
    rpl, wpl = shape
    nr = 64 * rpl * wpl - 37 if 64 * rpl * wpl > 200 else 64 * rpl * wpl - 5
    c = cellgen.tiny(nr + 1, nr=nr, nz=9, n_layers=4, z_active=True, dt=2e-7, amplitude=5e9)
    rng = np.random.default_rng(5)
    T0 = 28.0 + rng.uniform(0, 5, size=(c["nz"], c["nr"]))
    To = oracle.forward(c, T0, nsteps=40)
    for lpw in (1, 3):
        say("case f32 shape %s lines/wave %d nr %d" % (shape, lpw, nr))
        plan = P.Plan(c, "f32")
        plan.set_shape(rpl, wpl, lpw)
        T = plan.field_from(T0)
        ws = plan.workspace(40)
        plan.forward(T, 0, 40, ws=ws)
        plan.poll(ws)
        torch.cuda.synchronize()
        e = float(np.max(np.abs(plan.field_values(T) - To)))
        say("  max abs err %.3e K" % e)
        assert e < F32_TOL_K


def _general_exponents(c, qs, ps=None):
    """Capacity exponents other than 3 (the general power path instead of the
    cube) and, optionally, conductivity exponents far apart across layers
    (interface ratio laws of larger exponent)."""
    for m, l in enumerate(c["layers"]):
        l["q"] = qs[m % len(qs)]
        if ps is not None:
            l["p"] = ps[m % len(ps)]
    return c


@pytest.mark.parametrize("qs,ps", [((2.4,), None), ((1.0, 3.0, 0.5), None),
                                   ((2.0, 3.5, 1.5), (-1.5, 2.5, 0.3))])
@pytest.mark.parametrize("shape", [(3, 1), (16, 1), (4, 4)])
def test_general_power_laws_match_oracle_f64(qs, ps, shape):
    import torch

    import paper_1408_5853_amd as P
    rpl, wpl = shape
    nr = min(64 * rpl * wpl - 3, 300)
    c = _general_exponents(cellgen.tiny(17, nr=nr, nz=6, n_layers=3, z_active=True,
                                        dt=2e-7, amplitude=5e9), qs, ps)
    rng = np.random.default_rng(11)
    T0 = 28.0 + rng.uniform(0, 5, size=(c["nz"], c["nr"]))
    To = oracle.forward(c, T0, nsteps=40)
    for dtype in ("f64", "f32"):
        say("case general laws qs=%s ps=%s shape %s %s nr %d" % (qs, ps, shape, dtype, nr))
        plan = P.Plan(c, dtype)
        plan.set_shape(rpl, wpl, 2)
        T = plan.field_from(T0)
        ws = plan.workspace(40)
        plan.forward(T, 0, 40, ws=ws)
        plan.poll(ws)
        torch.cuda.synchronize()
        Tg = plan.field_values(T)
        if dtype == "f64":
            e = rel_err(Tg, To)
            say("  max rel err %.3e" % e)
            assert e < F64_TOL
        else:
            e = float(np.max(np.abs(Tg - To)))
            say("  max abs err %.3e K" % e)
            assert e < F32_TOL_K
