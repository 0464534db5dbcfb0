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
