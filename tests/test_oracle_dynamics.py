"""Statistical pins of the whole oracle step against closed forms.

* Rigid dumbbell rotational diffusion (one rod, HI on and off): the bond
  direction u diffuses on the sphere with D_r = 2 (1 - A_perp) / b^2, where
  A_perp is the transverse RPY coefficient of Eq. 8 at R = b, so
  <u(t).u(0)> = exp(-2 D_r t).
* Freely-jointed equilibrium with HI off: <R_ee^2> = (N-1) b^2 (Section 5
  validates the code against the equilibrium scaling R_ee ~ N^0.5).
  Started from a straight chain so that the test does not pass trivially.
"""
import numpy as np
import pytest

from oracle import oracle as o
from paper_2208_06559_amd import inputs as I


@pytest.mark.slow
@pytest.mark.parametrize("hstar,a_perp", [(0.25, 7 / 32), (0.0, 0.0)])
def test_dumbbell_rotational_diffusion(hstar, a_perp):
    nch, dt, nsteps = 20000, 1e-3, 100
    X0 = np.stack([I.random_walk(2, seed=11, chain=c) for c in range(nch)])
    p = o.make_params(2, hstar=hstar, dt=dt, seed=21)
    X, st = o.run_many(p, np.arange(nch), 0, nsteps, X0)
    assert np.all(st == o.OK)
    u0 = X0[:, 1] - X0[:, 0]
    u1 = X[:, 1] - X[:, 0]
    c = np.einsum("ij,ij->i", u0, u1)
    Dr = 2.0 * (1.0 - a_perp)
    expect = np.exp(-2 * Dr * dt * nsteps)
    sigma = c.std() / np.sqrt(nch)
    # 4 sigma plus the O(dt) Euler bias, (1 - 2 D_r dt)^n vs exp(-2 D_r t)
    bias = abs((1 - 2 * Dr * dt) ** nsteps - expect)
    assert abs(c.mean() - expect) < 4 * sigma + 2 * bias + 1e-3


@pytest.mark.slow
def test_freely_jointed_end_to_end_hi_off():
    N, nch, dt = 4, 2000, 1e-3
    X0 = np.stack([I.straight_chain(N) for _ in range(nch)])
    p = o.make_params(N, hstar=0.0, dt=dt, seed=31)
    ids = np.arange(nch)
    X, st = o.run_many(p, ids, 0, 3000, X0)  # about 10 Rouse times
    assert np.all(st == o.OK)
    samples = []
    step = 3000
    for _ in range(30):
        X, st = o.run_many(p, ids, step, 100, X)
        step += 100
        samples.append(np.sum((X[:, -1] - X[:, 0]) ** 2, axis=1))
    per_chain = np.mean(samples, axis=0)
    mean = per_chain.mean()
    sigma = per_chain.std() / np.sqrt(nch)
    assert abs(mean - (N - 1)) < 4 * sigma + 0.02
    rods = np.linalg.norm(np.diff(X, axis=1), axis=2)
    assert np.abs(rods - 1.0).max() <= 1e-10
