"""Pins of the oracle's adjoint of the noise product y = c_B L xi (Eq. 6's
noise term times dt): the gradients of <ybar, y> in the lower triangle of L
and in xi against central differences of the oracle's own forward product
(y is linear in each, so the differences are exact up to rounding)."""
import numpy as np
import pytest

from oracle import oracle as o


@pytest.mark.parametrize("noise", [o.NOISE_GAUSSIAN, o.NOISE_UNIFORM_PAPER])
def test_brownian_adjoint_matches_differences(noise):
    n = 12
    p = o.make_params(n // 3, dt=1e-3, noise=noise, seed=4)
    rng = np.random.default_rng(1)
    L = np.tril(rng.normal(size=(n, n))) + 3 * np.eye(n)
    ybar = rng.normal(size=n)
    _, xi = o.brownian(p, 5, L)
    Lbar, xibar = o.brownian_adjoint(p, L, xi, ybar)

    def phi(Lm):
        y, _ = o.brownian(p, 5, Lm)
        return float(ybar @ y)

    d = 1e-3
    for (i, j) in [(0, 0), (5, 2), (11, 11), (11, 0), (7, 6)]:
        Lp, Lm = L.copy(), L.copy()
        Lp[i, j] += d
        Lm[i, j] -= d
        np.testing.assert_allclose(Lbar[i, j], (phi(Lp) - phi(Lm)) / (2 * d), rtol=1e-9)
    assert np.all(np.triu(Lbar, 1) == 0)
    # y is linear in xi and in L: <ybar, y> = <xibar, xi> = <Lbar, L>, with
    # y from the forward product
    y, _ = o.brownian(p, 5, L)
    np.testing.assert_allclose(xibar @ xi, ybar @ y, rtol=1e-12)
    np.testing.assert_allclose(np.sum(Lbar * L), ybar @ y, rtol=1e-12)
