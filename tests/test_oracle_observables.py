"""Pins of the oracle's chain observables (end-to-end vector and radius of
gyration, the quantities of the paper's flow studies, Section 5) against
closed forms and invariances."""
import numpy as np
import pytest

from oracle import oracle as o
from paper_2208_06559_amd import inputs as I


@pytest.mark.parametrize("N,b", [(2, 1.0), (7, 0.5), (100, 1.0)])
def test_straight_chain_closed_forms(N, b):
    # N equally spaced points: R_ee = (N-1) b, R_g^2 = b^2 (N^2 - 1) / 12
    ob = o.observables(I.straight_chain(N, b))
    np.testing.assert_allclose(ob[:3], [(N - 1) * b, 0.0, 0.0], rtol=0, atol=1e-13)
    np.testing.assert_allclose(ob[3], b * b * (N * N - 1) / 12.0, rtol=1e-13)


def test_dumbbell():
    x = np.array([[0.3, -1.0, 2.0], [1.1, 0.5, 1.2]])
    q = x[1] - x[0]
    ob = o.observables(x)
    np.testing.assert_allclose(ob[:3], q, rtol=0, atol=1e-15)
    np.testing.assert_allclose(ob[3], q @ q / 4.0, rtol=1e-14)


def test_rigid_motion_invariance():
    x = I.random_walk(50, seed=3)
    ob = o.observables(x)
    th = 0.7
    Rz = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1.0]])
    y = x @ Rz.T + np.array([5.0, -2.0, 1.0])
    oy = o.observables(y)
    np.testing.assert_allclose(oy[:3], Rz @ ob[:3], rtol=0, atol=1e-12)
    np.testing.assert_allclose(oy[3], ob[3], rtol=1e-12)


# ---- Kramers stress (Section 5, Eqs. 28-29)

@pytest.mark.parametrize("N,ell,K", [(2, 1.1, 1e3), (10, 0.97, 1e4), (64, 1.003, 50.0)])
def test_stress_straight_stretched_springs(N, ell, K):
    # every connector along x with length ell: F_k Q_k^T = K (ell - b) ell xx^T
    M = N - 1
    st = o.kramers_stress(I.straight_chain(N, ell), 1.0, k_spring=K)
    np.testing.assert_allclose(st[0], M * K * (ell - 1.0) * ell - M, rtol=1e-12)
    np.testing.assert_allclose(st[1:3], [-M, -M], rtol=1e-15)
    np.testing.assert_allclose(st[3:6], 0.0, atol=1e-12)
    np.testing.assert_allclose(st[6], M * K * (ell - 1.0) * ell, rtol=1e-12)


def test_stress_springs_at_rest_length_are_isotropic():
    x = I.random_walk(40, b=0.8, seed=2)  # every bond exactly b
    st = o.kramers_stress(x, 0.8, k_spring=1e4)
    np.testing.assert_allclose(st[:3], -39.0, rtol=1e-9)
    np.testing.assert_allclose(st[3:], 0.0, atol=1e-8)


def test_stress_rigid_tensions_along_y():
    # rods of length b along y carrying tensions T_k: tau_yy = b sum T - M
    N, b = 9, 1.0
    T = np.linspace(-0.5, 3.0, N - 1)
    st = o.kramers_stress(I.straight_chain(N, b, axis=1), b, tensions=T)
    np.testing.assert_allclose(st[1], b * T.sum() - (N - 1), rtol=1e-13)
    np.testing.assert_allclose([st[0], st[2]], -(N - 1), rtol=1e-15)
    np.testing.assert_allclose(st[6], -b * T.sum(), rtol=1e-13)


def test_stress_dumbbell_and_rotation():
    # one connector: tau + I = c Q Q^T with c = T/|Q|; rotating the chain
    # rotates tau + M I
    x = np.array([[0.2, -0.4, 1.0], [0.9, 0.3, 0.1]])
    q = x[1] - x[0]
    T = 2.5
    st = o.kramers_stress(x, 1.0, tensions=[T])
    S = T / np.linalg.norm(q) * np.outer(q, q)
    np.testing.assert_allclose(st[:6], [S[0, 0] - 1, S[1, 1] - 1, S[2, 2] - 1, S[0, 1], S[0, 2],
                                        S[1, 2]], rtol=1e-14)
    y = I.random_walk(30, seed=5)
    th = 0.9
    R = np.array([[1.0, 0, 0], [0, np.cos(th), -np.sin(th)], [0, np.sin(th), np.cos(th)]])
    Tr = np.random.default_rng(1).normal(size=29)
    a, c = o.kramers_stress(y, 1.0, tensions=Tr), o.kramers_stress(y @ R.T, 1.0, tensions=Tr)

    def full(v):
        return np.array([[v[0], v[3], v[4]], [v[3], v[1], v[5]], [v[4], v[5], v[2]]]) + 29 * np.eye(3)
    np.testing.assert_allclose(full(c), R @ full(a) @ R.T, rtol=0, atol=1e-11)
