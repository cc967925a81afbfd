"""Parity of the polynomial-law path (eqs. (23), (24)) and the Joule source
(eqs. (2), (25)) on the GPU with the FP64 CPU oracle, element by element:
1e-10 relative on the field and the surface trace in FP64 (1e-4 K in FP32),
over seeded cells with
interfaces, ragged radial lengths from 5 to 1024 nodes (every chunk length
the default shapes pick, the 16-row one included), a non-default launch shape
and the turn-on model.
"""
import numpy as np
import pytest

import cellgen
import oracle
from gpu_util import rel_err, run_gpu, say

pytestmark = pytest.mark.gpu

F64_TOL = 1e-10


def _check(c, nsteps, T0=None, k0=0):
    say("case poly nr=%d nz=%d steps=%d joule=%g turn_on=%s" %
        (c["nr"], c["nz"], nsteps, c.get("joule_tref", 0.0), bool(c.get("turn_on"))))
    Tg, Sg = run_gpu(c, nsteps, T0=T0, k0=k0)
    To, So = oracle.forward(c, T0, k0=k0, nsteps=nsteps, surf=True)
    e, es = rel_err(Tg, To), rel_err(Sg, So)
    say("  max rel err field %.3e surface %.3e" % (e, es))
    assert e < F64_TOL and es < F64_TOL
    return To


@pytest.mark.parametrize("seed,z_active,joule", [(0, False, 0.0), (1, True, 30.0),
                                                 (2, True, 0.0), (3, False, 45.0)])
def test_poly_small_cells_f64(seed, z_active, joule):
    c = cellgen.poly_variant(cellgen.small_cell(seed, z_active=z_active), seed, joule_tref=joule)
    c = cellgen.with_nz(c, 12 if z_active else 4)
    To = _check(c, 1500)
    assert To.max() > 28.05                        # the pulse heated the cell


@pytest.mark.parametrize("nr,nz", [(5, 3), (129, 5), (300, 9), (631, 6), (1024, 4)])
def test_poly_ragged_shapes_random_fields_f64(nr, nz):
    c = cellgen.tiny(nr, nr=nr, nz=nz, n_layers=min(5, (nr - 1) // 2), nsteps=40,
                     z_active=True, dt=2e-7, amplitude=5e9)
    c = cellgen.poly_variant(c, nr, joule_tref=30.0 if nr % 2 else 0.0)
    rng = np.random.default_rng(nr)
    T0 = 28.0 + rng.uniform(0, 6, size=(nz, nr))
    _check(c, 40, T0=T0, k0=3)


@pytest.mark.parametrize("seed,joule", [(1, 30.0), (2, 0.0)])
def test_poly_f32(seed, joule):
    c = cellgen.poly_variant(cellgen.with_nz(cellgen.small_cell(seed, z_active=True), 12), seed,
                             joule_tref=joule)
    say("case poly f32 nr=%d nz=%d joule=%g" % (c["nr"], c["nz"], joule))
    Tg, Sg = run_gpu(c, 1500, dtype="f32")
    To, So = oracle.forward(c, nsteps=1500, surf=True)
    e, es = np.max(np.abs(Tg - To)), np.max(np.abs(Sg - So))
    say("  max abs err field %.3e K surface %.3e K" % (e, es))
    assert e < 1e-4 and es < 1e-4
    assert To.max() > 28.05


def test_poly_non_default_shape_and_turn_on():
    import torch

    import paper_1408_5853_amd as P
    c = cellgen.poly_variant(cellgen.with_nz(cellgen.small_cell(4, z_active=True), 6), 4,
                             joule_tref=30.0)
    dt = c["dt"]
    c.update(t_on=3 * dt, width=5 * dt, period=20 * dt, turn_on=True, amplitude=3 * c["amplitude"])
    plan = P.Plan(c)
    plan.set_shape(4, 2, 2)
    say("case poly + turn-on, shape", plan.shape())
    T = plan.init()
    ws = plan.workspace(45)
    S = torch.zeros(45, dtype=torch.float64, device="cuda")
    plan.forward(T, 0, 45, ws=ws, surf=S)
    plan.poll(ws)
    torch.cuda.synchronize()
    To, So = oracle.forward(c, nsteps=45, surf=True)
    assert rel_err(plan.field_values(T), To) < F64_TOL
    assert rel_err(S.cpu().numpy(), So) < F64_TOL
