"""Pins of the Brownian displacement y = c_B L xi (the noise term of Eq. 6
times dt; Eq. 2 for the paper's uniform noise)."""
import numpy as np

from oracle import oracle as o
from paper_2208_06559_amd import inputs as I


def test_matches_dense_product():
    N = 60
    p = o.make_params(N, dt=1e-4, seed=9, chain_id=2)
    D = o.rpy_assemble(p, I.random_walk(N, seed=7))
    L = np.linalg.cholesky(D)
    y, xi = o.brownian(p, 17, L)
    np.testing.assert_array_equal(xi, o.noise(p, 17, 3 * N))
    np.testing.assert_allclose(y, np.sqrt(2e-4) * (L @ xi), rtol=1e-13, atol=1e-16)
    pu = o.make_params(N, dt=1e-4, seed=9, chain_id=2, noise=o.NOISE_UNIFORM_PAPER)
    yu, nu = o.brownian(pu, 17, L)
    np.testing.assert_allclose(yu, np.sqrt(6e-4) * (L @ nu), rtol=1e-13, atol=1e-16)


def _sample_cov(noise_kind, nsamp=20000):
    N = 3
    x = np.array([[0.0, 0, 0], [1.0, 0, 0], [1.3, 0.8, 0.2]])
    dt = 1e-3
    p = o.make_params(N, dt=dt, noise=noise_kind)
    D = o.rpy_assemble(p, x)
    L = np.linalg.cholesky(D)
    Y = np.array([o.brownian(p, s, L)[0] for s in range(nsamp)])
    return np.cov(Y.T) / (2 * dt), D


def test_covariance_is_two_dt_D_gaussian():
    C, D = _sample_cov(o.NOISE_GAUSSIAN)
    # each entry of a sample covariance of unit-scale Gaussians has sd <= sqrt(2/n)
    assert np.abs(C - D).max() < 6 * np.sqrt(2.0 / 20000)


def test_covariance_is_two_dt_D_uniform():
    C, D = _sample_cov(o.NOISE_UNIFORM_PAPER)
    assert np.abs(C - D).max() < 6 * np.sqrt(2.0 / 20000)
