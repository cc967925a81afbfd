"""Parity at the workloads' full sizes and step counts.

* The device cell (1024 x 4096 nodes, 8 layers) over its whole run of
  100,000 steps (one pulse period), in FP64 (1e-10 relative) and in FP32
  pairs (1e-4 K), against the oracle on the cell's exact z-invariant
  reduction (4 axial nodes, same radial grid, dt and steps): every line of
  the GPU field must equal every other bit for bit, which is what makes the
  reduction exact.
* The z-active twins of the device cell and of the adjoint cell (the top
  line held, eq. (6), so the explicit axial half of eq. (11) is active) at
  full size over a 10,000-step prefix, against stored oracle runs
  (tests/golden/twin_*_10k.npz, written by tests/golden/make_twins.py from the
  oracle only): whole sampled lines and the surface trace.
* The design sweep's 4 smallest and 4 largest cells over their 20,000 steps:
  FP32 pairs inside the full 256-cell batch, FP64 in a batch of those 8,
  both with the launch shapes the batch autotuner picks; z-invariance bit
  for bit, the oracle on each cell's reduction.
* A batch of z-active cells (held top line) against single runs with the
  same launch shapes (bit for bit), with default shapes (rounding) and the
  oracle (the smallest cell, full grid).
* The axis case: a solid cylinder (r_inner = 0, insulated axis; the first
  row of the line is the symmetry row) against the oracle, FP64 and FP32.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import cellgen
import oracle
from gpu_util import rel_err, run_gpu, say

pytestmark = pytest.mark.gpu

F64_TOL = 1e-10
F32_TOL_K = 1e-4
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def device_oracle_100k():
    c = cellgen.device_cell(0, nz=4)
    say("oracle: device cell reduced to 4 lines, %d steps" % c["nsteps"])
    return oracle.forward(c, nsteps=c["nsteps"], surf=True)


def _state_run(cell, dtype, n):
    """n steps of `cell` with the field resident in the kernels' layout,
    surface trace on the device; returns (field [nz][nr] float64, trace)."""
    import torch

    import paper_1408_5853_amd as P
    plan = P.Plan(cell, dtype)
    st = P.State(plan, plan.init())
    S = torch.zeros(n, dtype=torch.float64, device="cuda")
    st.forward(0, n, surf=S)
    st.poll()
    T = st.store()
    torch.cuda.synchronize()
    return plan.field_values(T), S.cpu().numpy()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_device_cell_whole_run(dtype, device_oracle_100k):
    c = cellgen.device_cell(0)
    n = c["nsteps"]
    say("case device cell 1024x4096 %s, %d steps" % (dtype, n))
    Tg, Sg = _state_run(c, dtype, n)
    assert np.all(Tg == Tg[1][None, :]), "lines differ: a race or halo error"
    To, So = device_oracle_100k
    if dtype == "f64":
        e, es = rel_err(Tg[1], To[1]), rel_err(Sg, So)
        say("  max rel err line %.3e surface %.3e" % (e, es))
        assert e < F64_TOL and es < F64_TOL
    else:
        e, es = float(np.max(np.abs(Tg[1] - To[1]))), float(np.max(np.abs(Sg - So)))
        say("  max abs err line %.3e K surface %.3e K" % (e, es))
        assert e < F32_TOL_K and es < F32_TOL_K
    assert np.max(To[1]) - c["T_init"] > 0.05      # the pulse heated the cell


@pytest.mark.parametrize("name,make", [
    ("twin_device_cell", lambda: cellgen.device_cell(0, z_active=True)),
    ("twin_adjoint_cell", lambda: cellgen.adjoint_cell(0, z_active=True))])
def test_z_active_twin_full_size_prefix(name, make):
    c = make()
    with np.load(os.path.join(GOLDEN, name + "_10k.npz"), allow_pickle=False) as z:
        rec = {k: z[k] for k in z.files}
    n = int(rec["nsteps"])
    say("case %s %dx%d, %d steps" % (name, c["nr"], c["nz"], n))
    Tg, Sg = _state_run(c, "f64", n)
    lines = rec["lines"]
    e = rel_err(Tg[lines], rec["field"])
    es = rel_err(Sg[rec["steps"] - 1], rec["surface"])
    say("  max rel err sampled lines %.3e surface %.3e" % (e, es))
    assert e < F64_TOL and es < F64_TOL
    # the held top line draws heat: the axial half moved the lines below it
    assert np.max(np.abs(rec["field"][-1] - rec["field"][0])) > 1e-3


def _sweep_extremes():
    cells = cellgen.sweep_cells(0, 256)
    order = sorted(range(len(cells)), key=lambda i: cells[i]["nr"] * cells[i]["nz"])
    return cells, order[:4] + order[-4:]


def _oracle_reduced(cells, n):
    with ThreadPoolExecutor(8) as ex:
        return list(ex.map(lambda c: oracle.forward(cellgen.with_nz(c, 4), nsteps=n,
                                                     nthreads=1), cells))


def _batch_fields(cells, dtype, n, shapes=None):
    import torch

    import paper_1408_5853_amd as P
    b = P.Batch(cells, dtype, shapes=shapes)
    T = b.init()
    ws = b.workspace()
    b.forward(T, 0, n, ws)
    b.poll(ws)
    torch.cuda.synchronize()
    return b, T


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_sweep_extremes_whole_run(dtype):
    import paper_1408_5853_amd as P
    cells, idx = _sweep_extremes()
    n = cells[0]["nsteps"]
    run = cells if dtype == "f32" else [cells[i] for i in idx]
    pick = idx if dtype == "f32" else list(range(len(idx)))
    # the sweep as configured: launch shapes from the batch autotuner
    shapes = P.tune_batch(run, dtype)
    say("case sweep %s: batch of %d, %d steps, tuned shapes %s; checked %s" %
        (dtype, len(run), n, sorted(set(shapes)),
         [(cells[i]["nr"], cells[i]["nz"]) for i in idx]))
    b, T = _batch_fields(run, dtype, n, shapes)
    assert [b.shape(i) for i in range(len(run))] == shapes
    ref = _oracle_reduced([cells[i] for i in idx], n)
    for k, (i, To) in enumerate(zip(pick, ref)):
        g = P.Plan.field_values(b.field(T, i))
        assert np.all(g == g[1][None, :]), "instance %d: lines differ" % idx[k]
        if dtype == "f64":
            assert rel_err(g[1], To[1]) < F64_TOL, idx[k]
        else:
            assert np.max(np.abs(g[1] - To[1])) < F32_TOL_K, idx[k]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_z_active_batch(dtype):
    import paper_1408_5853_amd as P
    cells = cellgen.sweep_cells(1, 5)
    for c in cells:
        c["bc"][3] = [1, c["T_init"]]           # held top line: the axial half is active
    n = 600
    say("case z-active batch %s: %s" % (dtype, [(c["nr"], c["nz"]) for c in cells]))
    b, T = _batch_fields(cells, dtype, n)
    for i, c in enumerate(cells):
        g = P.Plan.field_values(b.field(T, i))
        # a single run with the instance's launch shape: the same kernels and
        # line blocks (another block partition changes rounding only: each
        # line sums its two axial fluxes in march order)
        plan = P.Plan(c, dtype)
        plan.set_shape(*b.shape(i))
        Ts = plan.init()
        plan.forward(Ts, 0, n)
        assert np.array_equal(g, plan.field_values(Ts)), i
        ref, _ = run_gpu(c, n, dtype=dtype, surf=False)          # default shape
        if dtype == "f64":
            assert rel_err(g, ref) < 1e-13, i
        else:
            assert np.max(np.abs(g - ref)) < 1e-5, i
    small = min(range(len(cells)), key=lambda i: cells[i]["nr"] * cells[i]["nz"])
    c = cells[small]
    g = P.Plan.field_values(b.field(T, small))
    To = oracle.forward(c, nsteps=n)
    assert np.max(np.abs(To[-2] - To[1])) > 1e-6           # not z-invariant
    if dtype == "f64":
        assert rel_err(g, To) < F64_TOL
    else:
        assert np.max(np.abs(g - To)) < F32_TOL_K


@pytest.mark.parametrize("dtype,z_active", [("f64", False), ("f64", True), ("f32", True)])
def test_solid_cylinder_axis(dtype, z_active):
    c = cellgen.small_cell(2, z_active=z_active)
    c["r_inner"] = 0.0
    c["bc"][0] = [0, 0.0]                       # the axis: symmetry (insulated) row
    c["heater"] = 0                             # heat the core: gradients at the axis
    if not z_active:
        c["bc"][1] = [1, c["T_init"]]           # held outer wall instead
    n = 4000
    say("case axis r_inner=0 %s z_active=%s, %d steps" % (dtype, z_active, n))
    Tg, Sg = run_gpu(c, n, dtype=dtype)
    To, So = oracle.forward(c, nsteps=n, surf=True)
    assert np.max(To[:, 0]) - c["T_init"] > 1e-3              # heat reached the axis
    if dtype == "f64":
        assert rel_err(Tg, To) < F64_TOL and rel_err(Sg, So) < F64_TOL
    else:
        assert np.max(np.abs(Tg - To)) < F32_TOL_K and np.max(np.abs(Sg - So)) < F32_TOL_K


def test_autotuners_pick_built_shapes_and_cache(tmp_path):
    import paper_1408_5853_amd as P
    cache = str(tmp_path / "tune.txt")
    c = cellgen.sweep_cells(2, 1)[0]
    sh, us = P.autotune(c, "f64", steps=8, cache=cache)
    assert us > 0 and sh[0] * sh[1] * 64 >= c["nr"] and 1 <= sh[2] <= 8
    sh2, us2 = P.autotune(c, "f64", steps=8, cache=cache)
    assert sh2 == sh and us2 == -1.0                       # from the cache
    cells = cellgen.sweep_cells(3, 12)
    shapes = P.tune_batch(cells, "f32", steps=32, cache=cache)
    assert all(r * w * 64 >= x["nr"] and 1 <= l <= x["nz"] - 2
               for (r, w, l), x in zip(shapes, cells))
    assert P.tune_batch(cells, "f32", steps=32, cache=cache) == shapes
    text = open(cache).read()
    assert "cube" in text and "batch f32" in text
