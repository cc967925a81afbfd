"""The C oracle against a second, independent oracle (dense NumPy solves of
the paper's rows) and, through that oracle's complex-step derivatives,
its discrete adjoint: the gradient with respect to every parameter and the
state adjoint (a dot-product test).  CPU only."""
import numpy as np
import pytest

import cellgen
import oracle
from oracle import dense_np as D


def _cell(seed, zact, nr=14, nz=6, n_layers=3, nsteps=12, bc=None, heater=None):
    c = cellgen.tiny(seed, nr=nr, nz=nz, n_layers=n_layers, nsteps=nsteps, z_active=zact,
                     dt=2e-6, amplitude=4e9,
                     heater=n_layers - 1 if heater is None else heater)
    if bc is not None:
        c["bc"] = bc
    return c


BCS = [
    [[1, 28.0], [0, 0.0], [0, 0.0], [0, 0.0]],
    [[1, 28.0], [1, 29.0], [0, 0.0], [1, 27.5]],
    [[0, 0.0], [1, 28.5], [1, 28.0], [0, 0.0]],
    [[0, 0.0], [0, 0.0], [1, 28.0], [1, 28.0]],
]


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("bci", range(len(BCS)))
def test_dense_reference_matches_c_oracle_forward(seed, bci):
    c = _cell(seed, True, n_layers=2 + seed, nr=11 + 3 * seed, bc=BCS[bci], heater=seed % 2)
    Td, Sd = D.forward(c)
    To, So = oracle.forward(c, nsteps=c["nsteps"], surf=True)
    assert np.max(np.abs(Td - To) / np.abs(To)) < 1e-12
    assert np.max(np.abs(Sd - So) / np.abs(So)) < 1e-12


def test_dense_reference_rows_equal_c_oracle_rows():
    c = _cell(4, True, n_layers=4, nr=17)
    rng = np.random.default_rng(1)
    T = 28.0 + rng.uniform(0, 2, size=(c["nz"], c["nr"]))
    st = D._Setup(c)
    for k, j in [(0, 1), (3, 2), (7, c["nz"] - 2)]:
        A, B, Cc, F = oracle.line_rows(c, T, k, j)
        M, Fd = D.assemble(st, T, j, c["amplitude"] * D.pulse_average(c, k))
        Ad = np.r_[0.0, np.diag(M, -1)]
        Cd = np.r_[np.diag(M, 1), 0.0]
        for x, y in ((A, Ad), (B, np.diag(M)), (Cc, Cd), (F, Fd)):
            assert np.allclose(x, y, rtol=1e-14, atol=0.0)


def _norm_err(g, ref, theta):
    P = np.abs(theta)
    scale = np.max(np.abs(ref * P))
    return float(np.max(np.abs(g - ref) * P / scale))


@pytest.mark.parametrize("seed,zact", [(0, True), (1, False), (3, True), (5, False)])
def test_complex_step_pins_oracle_gradient(seed, zact):
    # amplitude, width (pulse edges off the step grid), thicknesses and
    # conductivity scales: complex steps are exact to rounding
    import paper_1408_5853_amd as Pk
    c = _cell(seed, zact, n_layers=3 + seed % 2, nr=13 + seed)
    n = c["nsteps"]
    assert abs(c["width"] / c["dt"] - round(c["width"] / c["dt"])) > 1e-3
    tg = cellgen.tracking_target(c, n) + 1.0
    Jo, go, _ = oracle.gradient(c, tg, nsteps=n)
    gc = D.complex_step_gradient(c, tg, n)
    assert Jo == pytest.approx(float(np.real(D.objective(c, tg, nsteps=n))), rel=1e-13)
    assert _norm_err(go, gc, Pk.params_of(c)) < 1e-12


@pytest.mark.parametrize("nsteps", [1, 4])
def test_state_adjoint_dot_product(nsteps):
    # <dJ/dT0, v> from the oracle's adjoint against Im J(T0 + i h v) / h
    c = _cell(7, True, n_layers=3, nr=12, nsteps=nsteps)
    rng = np.random.default_rng(3)
    T0 = 28.0 + rng.uniform(0, 1, size=(c["nz"], c["nr"]))
    tg = cellgen.tracking_target(c, nsteps) + 0.5
    Jo, go, So, lam0 = oracle.gradient(c, tg, T0=T0, nsteps=nsteps, want_lam0=True)
    for trial in range(3):
        v = rng.normal(size=T0.shape)
        h = 1e-30
        Jc = D.objective(c, tg, T0=T0 + 1j * h * v, nsteps=nsteps, dtype=np.complex128)
        lhs = float(np.sum(lam0 * v))
        rhs = float(np.imag(Jc) / h)
        assert lhs == pytest.approx(rhs, rel=1e-12, abs=1e-14 * np.sum(np.abs(lam0 * v)))
