"""Pins of the oracle's rigid-rod tension solve and corrector: the rigid
(K* -> infinity) limit of the semi-implicit spring update of Eqs. 13-17
(Section 3), with the tension forces acting along the bond directions at the
start of the step and coupled through the full diffusion tensor."""
import numpy as np
import pytest

from oracle import oracle as o
from paper_2208_06559_amd import inputs as I


def _a_par(hstar, a, R):
    # Eq. 8 (R >= 2a) / Eq. 9 (R < 2a), component of D_01 along the bond
    if R >= 2 * a:
        return 3 * hstar / (4 * R) * (2 - 4 * a * a / (3 * R * R))
    return 3 * hstar / (8 * a) * (8 / 3 - R / (2 * a))


@pytest.mark.parametrize("hstar", [0.0, 0.25, 0.5])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_dumbbell_closed_form(hstar, seed):
    # One rod: Q(T) = Q* - dt G_00 u T with G_00 u = 2 (1 - A_par) u, so
    # s = 2 dt (1 - A_par) T solves |Q* - s u| = b:
    #   s = (Q*.u) - sqrt((Q*.u)^2 - |Q*|^2 + b^2)
    rng = np.random.default_rng(seed)
    b, dt = 1.0, 1e-3
    x = np.array([[0.0, 0, 0], rng.normal(size=3)])
    x[1] *= b / np.linalg.norm(x[1])
    xs = x + 0.05 * rng.normal(size=(2, 3))
    p = o.make_params(2, hstar=hstar, dt=dt, b=b)
    xn, T, info = o.constrain(p, x, xs)
    assert info["status"] == o.OK
    u = x[1] - x[0]
    Qs = xs[1] - xs[0]
    qu = Qs @ u
    s = qu - np.sqrt(qu * qu - Qs @ Qs + b * b)
    scale = 2 * dt * (1 - _a_par(hstar, 0.5, b))
    # T is fixed only to the rod tolerance (1e-13) divided by dt (1 - A_par):
    # compare the displacement s = scale * T instead
    assert abs(scale * T[0] - s) <= 1e-13
    assert abs(np.linalg.norm(xn[1] - xn[0]) - b) <= 1e-13


def test_dumbbell_negative_discriminant_fails():
    # a predictor that moves the second bead far sideways has no root
    x = np.array([[0.0, 0, 0], [1.0, 0, 0]])
    xs = np.array([[0.0, 0, 0], [0.0, 5.0, 0]])
    p = o.make_params(2, dt=1e-3)
    _, _, info = o.constrain(p, x, xs)
    assert info["status"] == o.ERR_NO_CONVERGE


@pytest.mark.parametrize("N,hstar", [(8, 0.25), (20, 0.25), (30, 0.5), (25, 0.0)])
def test_gmres_newton_matches_dense_newton(N, hstar):
    rng = np.random.default_rng(N)
    x = I.random_walk(N, seed=N)
    xs = x + 0.02 * rng.normal(size=x.shape)
    p = o.make_params(N, hstar=hstar, dt=1e-3)
    xa, Ta, ia = o.constrain(p, x, xs)
    xb, Tb, ib = o.constrain(p, x, xs, dense=True)
    assert ia["status"] == o.OK and ib["status"] == o.OK
    np.testing.assert_allclose(Ta, Tb, rtol=0, atol=1e-12 * np.abs(Tb).max())
    np.testing.assert_allclose(xa, xb, rtol=0, atol=1e-13)
    assert np.abs(np.linalg.norm(np.diff(xa, axis=0), axis=1) - 1.0).max() <= 1e-13


def test_hi_off_band_preconditioner_is_exact():
    # h* = 0: G = Delta Delta^T is tridiagonal, so each GMRES solve takes one
    # iteration and Newton converges quadratically.
    N = 40
    rng = np.random.default_rng(3)
    x = I.random_walk(N, seed=3)
    xs = x + 0.02 * rng.normal(size=x.shape)
    p = o.make_params(N, hstar=0.0, dt=1e-3)
    _, _, info = o.constrain(p, x, xs)
    assert info["status"] == o.OK
    assert info["krylov_iters"] == info["newton_iters"]
    assert info["newton_iters"] <= 5


def test_fixed_point_without_noise_or_flow():
    x = I.random_walk(25, seed=4)
    xn, T, info = o.constrain(o.make_params(25), x, x.copy())
    assert info["status"] == o.OK and info["newton_iters"] == 0
    np.testing.assert_array_equal(T, 0.0)
    np.testing.assert_array_equal(xn, x)


def test_rotation_preserves_rods():
    # rigid-body rotation as the only motion: rods stay at length b
    N = 30
    x = I.random_walk(N, seed=5)
    w = 3.0
    K = np.array([[0, -w, 0], [w, 0, 0], [0, 0, 0]])
    dt = 1e-3
    xs = x + dt * x @ K.T
    xn, T, info = o.constrain(o.make_params(N, dt=dt), x, xs)
    assert info["status"] == o.OK
    assert np.abs(np.linalg.norm(np.diff(xn, axis=0), axis=1) - 1.0).max() <= 1e-13


@pytest.mark.parametrize("w", [I.SINGLE_SMALL])
def test_step_keeps_rod_lengths(w):
    p = o.make_params(w.n_beads, dt=w.dt, kappa=w.kappa, seed=w.seed)
    x = w.initial()
    for s in range(20):
        x, info = o.step(p, s, x)
        assert info["status"] == o.OK
        assert np.abs(np.linalg.norm(np.diff(x, axis=0), axis=1) - 1.0).max() <= 1e-10


def test_low_hstar_linear_response():
    # The paper's own check (Section 5, BR-100 at h* = 1e-5): vanishing h*
    # reproduces the HI-off dynamics.  Pathwise, with fixed noise, the
    # deviation after a few steps is linear in h*.
    N = 40
    x0 = I.random_walk(N, seed=6)
    k = I.kappa_for("uniaxial", 0.5)

    def traj(h):
        p = o.make_params(N, hstar=h, dt=1e-3, kappa=k, seed=6)
        return o.run(p, 0, 10, x0)[0]

    ref = traj(0.0)
    d = [np.abs(traj(h) - ref).max() for h in (1e-3, 1e-4, 1e-5)]
    assert 9.0 < d[0] / d[1] < 11.0
    assert 9.0 < d[1] / d[2] < 11.0


def test_invalid_params():
    x = I.random_walk(4, seed=0)
    for kw in ({"dt": 0.0}, {"b": -1.0}, {"hstar": 0.7}, {"newton_maxit": 0}):
        p = o.make_params(4, **kw)
        _, info = o.step(p, 0, x)
        assert info["status"] == o.ERR_PARAM
    p = o.make_params(1)
    assert o.step(p, 0, np.zeros((1, 3)))[1]["status"] == o.ERR_PARAM
