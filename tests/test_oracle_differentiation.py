"""Pins of the oracle's reverse-mode derivatives: the Cholesky adjoint
(Murray's matrix form of the backward of Eq. 10), the tension solve's
adjoint (implicit-function theorem on the rigid-rod constraint) and the
whole step's adjoint, each against central differences of the oracle's
forward routines (an independent route: the C oracle's factorisation,
constraint solve and step), plus closed forms."""
import numpy as np
import pytest

from oracle import oracle as o
from paper_2208_06559_amd import inputs as I


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    G = rng.normal(size=(n, n))
    return G @ G.T / n + np.eye(n)


def _sym(n, seed):
    S = np.random.default_rng(seed).normal(size=(n, n))
    return 0.5 * (S + S.T)


def _chol(A):
    L, info = o.cholesky(A)
    assert info == 0
    return np.tril(L)


@pytest.mark.parametrize("n,kind", [(1, "spd"), (2, "spd"), (21, "rpy"), (30, "spd"), (60, "rpy")])
def test_cholesky_adjoint_central_differences(n, kind):
    if kind == "rpy":
        N = n // 3
        A = o.rpy_assemble(o.make_params(N), I.random_walk(N, seed=n) * 0.7)
    else:
        A = _spd(n, n)
    L = _chol(A)
    Lbar = np.tril(np.random.default_rng(n + 1).normal(size=(n, n)))
    Abar = o.cholesky_adjoint(L, Lbar)
    S = _sym(n, n + 2)
    d = 1e-6
    fd = (np.sum(Lbar * _chol(A + d * S)) - np.sum(Lbar * _chol(A - d * S))) / (2 * d)
    np.testing.assert_allclose(np.sum(Abar * S), fd, rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(Abar, Abar.T, rtol=0, atol=0)


def test_cholesky_adjoint_of_half_squared_norm():
    # phi = <L, L> / 2 = tr(A) / 2 (since |L|_F^2 = tr(L L^T)): Abar = I / 2
    A = o.rpy_assemble(o.make_params(12), I.random_walk(12, seed=4))
    L = _chol(A)
    np.testing.assert_allclose(o.cholesky_adjoint(L, L), 0.5 * np.eye(36), rtol=0, atol=1e-13)


def test_cholesky_adjoint_two_by_two_by_hand():
    a, b, c = 2.0, 0.6, 1.5
    L = _chol(np.array([[a, b], [b, c]]))
    l11, l21, l22 = np.sqrt(a), b / np.sqrt(a), np.sqrt(c - b * b / a)
    np.testing.assert_allclose([L[0, 0], L[1, 0], L[1, 1]], [l11, l21, l22], rtol=1e-15)
    g11, g21, g22 = 0.3, -1.1, 0.7  # Lbar
    Abar = o.cholesky_adjoint(L, np.array([[g11, 0.0], [g21, g22]]))
    # d/da, d/db (b in both off-diagonal entries) and d/dc of
    # g11 l11 + g21 l21 + g22 l22, written out
    da = g11 / (2 * l11) - g21 * b / (2 * a ** 1.5) + g22 * (b * b / (a * a)) / (2 * l22)
    db = g21 / l11 - g22 * (b / a) / l22
    dc = g22 / (2 * l22)
    np.testing.assert_allclose([Abar[0, 0], 2 * Abar[1, 0], Abar[1, 1]], [da, db, dc], rtol=1e-14)


@pytest.mark.parametrize("N,hstar", [(2, 0.25), (6, 0.0), (6, 0.25), (17, 0.4)])
def test_constrain_adjoint_central_differences(N, hstar):
    p = o.make_params(N, hstar=hstar, dt=1e-3)
    rng = np.random.default_rng(N)
    x = I.random_walk(N, seed=N + 7)
    xs = x + 0.03 * rng.normal(size=x.shape)
    xnew, _, info = o.constrain(p, x, xs)
    assert info["status"] == o.OK
    xbar = rng.normal(size=x.shape)
    z = o.constrain_adjoint(p, x, xnew, xbar)
    d = rng.normal(size=x.shape)
    e = 1e-6
    fd = (np.sum(xbar * o.constrain(p, x, xs + e * d)[0])
          - np.sum(xbar * o.constrain(p, x, xs - e * d)[0])) / (2 * e)
    np.testing.assert_allclose(np.sum(z * d), fd, rtol=1e-6, atol=1e-9)


CASES = [(2, 0.25, "none", 0), (5, 0.25, "planar", 0), (8, 0.0, "planar", 0),
         (8, 0.25, "shear", 0), (7, 0.25, "uniaxial", 1)]


@pytest.mark.parametrize("N,hstar,flow,noise", CASES)
def test_step_adjoint_central_differences(N, hstar, flow, noise):
    kap = I.kappa_for(flow, 50.0) if flow != "none" else np.zeros((3, 3))
    K0 = np.diag([1.0, -1.0, 0.0])

    def params(h, k):
        return o.make_params(N, dt=1e-3, hstar=h, kappa=k, seed=3, noise=noise)

    x = I.random_walk(N, seed=N)
    rng = np.random.default_rng(N + 1)
    w = rng.normal(size=(N, 3))
    xb, hb, kb = o.step_adjoint(params(hstar, kap), 0, x, w)

    def phi(xx, h, k):
        xn, info = o.step(params(h, k), 0, xx)
        assert info["status"] == o.OK
        return np.sum(w * xn)

    e = 1e-6
    d = rng.normal(size=(N, 3))
    fd = (phi(x + e * d, hstar, kap) - phi(x - e * d, hstar, kap)) / (2 * e)
    np.testing.assert_allclose(np.sum(xb * d), fd, rtol=1e-5, atol=1e-8)
    fd = (phi(x, hstar, kap + e * K0) - phi(x, hstar, kap - e * K0)) / (2 * e)
    np.testing.assert_allclose(np.sum(kb * K0), fd, rtol=1e-5, atol=1e-8)
    if hstar > 0:
        fd = (phi(x, hstar + e, kap) - phi(x, hstar - e, kap)) / (2 * e)
        np.testing.assert_allclose(hb, fd, rtol=1e-5, atol=1e-8)


def test_stretch_gradient_small_ensemble():
    # the differentiation workload in miniature: 3 chains of 6 beads, planar
    # extension, 6 steps; gradient of the mean stretch in h* and the rate
    N, C_, steps, rate, hstar = 6, 3, 6, 30.0, 0.25
    K0 = I.kappa_for("planar", 1.0)

    def ps(h, r):
        return [o.make_params(N, dt=1e-3, hstar=h, kappa=r * K0, seed=5, chain_id=c)
                for c in range(C_)]

    X0 = np.stack([I.random_walk(N, seed=5, chain=c) for c in range(C_)])
    J, gh, ge = o.stretch_gradient(ps(hstar, rate), X0, steps, K0)

    def Jf(h, r):
        Xs = []
        for c, p in enumerate(ps(h, r)):
            x = X0[c].copy()
            for s in range(steps):
                x, info = o.step(p, s, x)
                assert info["status"] == o.OK
            Xs.append(x)
        return o.mean_stretch(np.stack(Xs), 1.0)

    assert J == pytest.approx(Jf(hstar, rate), rel=1e-14)
    e = 1e-6
    np.testing.assert_allclose(gh, (Jf(hstar + e, rate) - Jf(hstar - e, rate)) / (2 * e),
                               rtol=1e-5)
    np.testing.assert_allclose(ge, (Jf(hstar, rate + e) - Jf(hstar, rate - e)) / (2 * e),
                               rtol=1e-5)
