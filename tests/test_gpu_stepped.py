"""Parity of the stepped domain (eq. (9): a terminal of nr_top radial nodes
above line z_full) on the GPU with the FP64 CPU oracle, on the whole field
(nodes outside the domain included: both leave them alone) and the surface
trace: FP64 within 1e-10 relative, FP32 within 1e-4 K.  Cases put the step
at both ends and in the middle of the axis, the terminal's wall on an
interface node, a full-radius terminal, the step face inside and between
line groups marching either way (lines per wave 1..3), ragged radial
lengths, and the turn-on model.
"""
import numpy as np
import pytest

import cellgen
import oracle
from gpu_util import rel_err, say

pytestmark = pytest.mark.gpu

F64_TOL = 1e-10
F32_TOL_K = 1e-4


def _run(c, nsteps, shape=None, dtype="f64", T0=None):
    import torch

    import paper_1408_5853_amd as P
    plan = P.Plan(c, dtype)
    if shape:
        plan.set_shape(*shape)
    say("case stepped nr=%d nz=%d z_full=%d nr_top=%d shape=%s %s steps=%d" %
        (c["nr"], c["nz"], c["stepped"]["z_full"], c["stepped"]["nr_top"], plan.shape(), dtype,
         nsteps))
    T = plan.init() if T0 is None else plan.field_from(T0)
    ws = plan.workspace(nsteps)
    S = torch.zeros(nsteps, dtype=torch.float64, device="cuda")
    plan.forward(T, 0, nsteps, ws=ws, surf=S)
    plan.poll(ws)
    torch.cuda.synchronize()
    return plan.field_values(T), S.cpu().numpy()


@pytest.mark.parametrize("seed,nz,z_full,nr_top", [
    (0, 20, 7, 20), (0, 20, 1, 35), (0, 20, 18, 35), (3, 16, 9, 64), (3, 16, 6, 3)])
def test_stepped_matches_oracle_f64(seed, nz, z_full, nr_top):
    c = cellgen.with_nz(cellgen.small_cell(seed, z_active=True), nz)
    c["amplitude"] *= 3
    c["stepped"] = dict(z_full=z_full, nr_top=nr_top)
    Tg, Sg = _run(c, 800)
    To, So = oracle.forward(c, nsteps=800, surf=True)
    e, es = rel_err(Tg, To), rel_err(Sg, So)
    say("  max rel err field %.3e surface %.3e" % (e, es))
    assert e < F64_TOL and es < F64_TOL
    assert To.max() - 28.0 > 1e-3                   # the pulse heated the cell
    if nr_top < c["nr"]:                            # and the step mattered
        rect = oracle.forward(dict(c, stepped=None), nsteps=800)
        assert rel_err(rect, To) > 1e-9


@pytest.mark.parametrize("lpw", [1, 2, 3])
def test_stepped_face_inside_and_between_line_groups(lpw):
    c = cellgen.with_nz(cellgen.small_cell(1, z_active=True), 23)
    c["amplitude"] *= 3
    c["stepped"] = dict(z_full=10, nr_top=30)
    rng = np.random.default_rng(lpw)
    T0 = 28.0 + rng.uniform(0, 4, size=(c["nz"], c["nr"]))
    Tg, Sg = _run(c, 60, shape=(4, 1, lpw), T0=T0)
    To, So = oracle.forward(c, T0, nsteps=60, surf=True)
    assert rel_err(Tg, To) < F64_TOL and rel_err(Sg, So) < F64_TOL


def test_stepped_f32():
    c = cellgen.with_nz(cellgen.small_cell(2, z_active=True), 14)
    c["stepped"] = dict(z_full=6, nr_top=25)
    Tg, Sg = _run(c, 800, dtype="f32")
    To, So = oracle.forward(c, nsteps=800, surf=True)
    e, es = np.max(np.abs(Tg - To)), np.max(np.abs(Sg - So))
    say("  max abs err field %.3e K surface %.3e K" % (e, es))
    assert e < F32_TOL_K and es < F32_TOL_K


@pytest.mark.parametrize("nr,nz", [(129, 7), (631, 6), (1024, 5)])
def test_stepped_ragged_shapes_f64(nr, nz):
    c = cellgen.tiny(nr, nr=nr, nz=nz, n_layers=5, nsteps=40, z_active=True, dt=2e-7,
                     amplitude=5e9)
    c["stepped"] = dict(z_full=nz // 2, nr_top=nr // 3)
    rng = np.random.default_rng(nr)
    T0 = 28.0 + rng.uniform(0, 6, size=(nz, nr))
    Tg, Sg = _run(c, 40, T0=T0)
    To, So = oracle.forward(c, T0, nsteps=40, surf=True)
    assert rel_err(Tg, To) < F64_TOL and rel_err(Sg, So) < F64_TOL


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_stepped_with_polynomial_laws(dtype):
    c = cellgen.poly_variant(cellgen.with_nz(cellgen.small_cell(1, z_active=True), 15), 1,
                             joule_tref=30.0)
    c["amplitude"] *= 3
    c["stepped"] = dict(z_full=8, nr_top=38)          # the wall on an interface node
    Tg, Sg = _run(c, 800, dtype=dtype)
    To, So = oracle.forward(c, nsteps=800, surf=True)
    if dtype == "f64":
        assert rel_err(Tg, To) < F64_TOL and rel_err(Sg, So) < F64_TOL
    else:
        assert np.max(np.abs(Tg - To)) < F32_TOL_K and np.max(np.abs(Sg - So)) < F32_TOL_K


def test_stepped_with_turn_on():
    c = cellgen.with_nz(cellgen.small_cell(4, z_active=True), 12)
    dt = c["dt"]
    c.update(t_on=3 * dt, width=5 * dt, period=20 * dt, turn_on=True, amplitude=3 * c["amplitude"],
             stepped=dict(z_full=5, nr_top=22))
    Tg, Sg = _run(c, 45)
    To, So = oracle.forward(c, nsteps=45, surf=True)
    assert rel_err(Tg, To) < F64_TOL and rel_err(Sg, So) < F64_TOL
