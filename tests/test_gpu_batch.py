"""Batched stepping of uneven cells: bitwise equal to the same instances run
one at a time, across captured graph blocks and remainders; FP32 within
1e-4 K and FP64 within 1e-10 of the oracle on the smallest and largest
instances of the design sweep."""
import numpy as np
import pytest

import cellgen
import oracle
from gpu_util import rel_err, run_gpu, say

pytestmark = pytest.mark.gpu


def _run_batch(cells, n, dtype, k0=0, shapes=None):
    import torch

    import paper_1408_5853_amd as P
    b = P.Batch(cells, dtype, shapes=shapes)
    T = b.init()
    ws = b.workspace()
    b.forward(T, k0, n, ws)
    b.poll(ws)
    torch.cuda.synchronize()
    out = [P.Plan.field_values(b.field(T, i)) for i in range(len(cells))]
    return out, b


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [5, 64, 77])
def test_batch_bitwise_equals_single_runs(dtype, n):
    cells = [cellgen.with_nz(c, 40) for c in cellgen.sweep_cells(0, 6)]
    say("case batch of %d, %s, %d steps" % (len(cells), dtype, n))
    got, b = _run_batch(cells, n, dtype, k0=11)
    for i, c in enumerate(cells):
        ref, _ = run_gpu(c, n, dtype=dtype, k0=11, surf=False)
        assert np.array_equal(got[i], ref), i


def _extremes(k=2):
    cells = cellgen.sweep_cells(0, 256)
    order = sorted(range(len(cells)), key=lambda i: cells[i]["nr"] * cells[i]["nz"])
    return [cells[i] for i in order[:k] + order[-k:]]


@pytest.mark.parametrize("dtype,tol", [("f64", None), ("f32", 1e-4)])
def test_batch_extreme_instances_match_oracle(dtype, tol):
    # the sweep's cells are exactly z-invariant (held inner wall, insulated
    # elsewhere): the oracle runs each on 4 axial nodes
    cells = _extremes()
    n = 2000
    say("case batch extremes %s: %s" % (dtype, [(c["nr"], c["nz"]) for c in cells]))
    got, _ = _run_batch(cells, n, dtype)
    for c, g in zip(cells, got):
        assert np.all(g == g[1][None, :]), "lines differ"
        To = oracle.forward(cellgen.with_nz(c, 4), nsteps=n)
        if tol is None:
            assert rel_err(g[1], To[1]) < 1e-10
        else:
            assert np.max(np.abs(g - To[1][None, :])) < tol


def _option_cells():
    # plain, polynomial laws with and without the Joule source (eqs.
    # (23)-(25)), the stepped domain (eq. (9)) and both, z-active, two
    # radial sizes (two chunk shapes)
    st = {"z_full": 80, "nr_top": 40}
    c = [cellgen.small_cell(0, z_active=True),
         cellgen.poly_variant(cellgen.small_cell(1, z_active=True), 1, joule_tref=30.0),
         cellgen.poly_variant(cellgen.small_cell(2, z_active=True), 2),
         dict(cellgen.small_cell(3, z_active=True), stepped=st),
         dict(cellgen.poly_variant(cellgen.small_cell(4, z_active=True), 4, joule_tref=40.0),
              stepped=st),
         cellgen.poly_variant(cellgen.tiny(5, nr=200, nz=40, n_layers=3, z_active=True,
                                           dt=2e-6, amplitude=4e9, heater=2), 5,
                              joule_tref=30.0)]
    return c


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_with_plan_options(dtype):
    # each instance equals a single plan with the same launch shape and
    # options, bit for bit (graph blocks and a remainder), and the oracle
    # within the tolerances
    import torch

    import paper_1408_5853_amd as P
    cells = _option_cells()
    n = 70
    say("case batch with plan options %s" % dtype)
    got, b = _run_batch(cells, n, dtype)
    for i, c in enumerate(cells):
        plan = P.Plan(c, dtype)
        plan.set_shape(*b.shape(i))
        T = plan.init()
        plan.forward(T, 0, n)
        torch.cuda.synchronize()
        assert np.array_equal(got[i], plan.field_values(T)), i
        To = oracle.forward(c, nsteps=n)
        if dtype == "f64":
            assert rel_err(got[i], To) < 1e-10, i
        else:
            assert np.max(np.abs(got[i] - To)) < 1e-4, i


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_tuned_batch_with_plan_options(dtype, tmp_path):
    # the batch tuner on instances with the polynomial laws and the stepped
    # domain: it groups them as the batch does, its shapes build, each
    # instance still equals a single plan of that shape bit for bit and the
    # oracle within the tolerances, and a second call reads the cache
    import torch

    import paper_1408_5853_amd as P
    cells = _option_cells()
    cache = str(tmp_path / "tune.txt")
    say("case tuned batch with plan options %s" % dtype)
    shapes = P.tune_batch(cells, dtype, steps=32, cache=cache)
    text = open(cache).read()
    assert " poly" in text and " stepped" in text
    assert P.tune_batch(cells, dtype, steps=32, cache=cache) == shapes
    n = 70
    got, b = _run_batch(cells, n, dtype, shapes=shapes)
    for i, c in enumerate(cells):
        assert tuple(b.shape(i)) == tuple(shapes[i]), i
        plan = P.Plan(c, dtype)
        plan.set_shape(*shapes[i])
        T = plan.init()
        plan.forward(T, 0, n)
        torch.cuda.synchronize()
        assert np.array_equal(got[i], plan.field_values(T)), i
        To = oracle.forward(c, nsteps=n)
        if dtype == "f64":
            assert rel_err(got[i], To) < 1e-10, i
        else:
            assert np.max(np.abs(got[i] - To)) < 1e-4, i
