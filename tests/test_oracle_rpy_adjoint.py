"""Pins of the oracle's adjoint of the RPY assembly (Eqs. 7-9): the
gradient of phi = sum_ij <Dbar_ij, D_ij(x)> with respect to the positions
and to h*, against central finite differences of the oracle's own forward
assembly (an independent route: no derivative formula is shared), with
pairs on both sides of R = 2a, where the tensor is C^1."""
import numpy as np
import pytest

from oracle import oracle as o
from paper_2208_06559_amd import inputs as I


def _phi(p, x, Dbar):
    return float(np.sum(Dbar * o.rpy_assemble(p, x, o.FILL_FULL)))


@pytest.mark.parametrize("N,seed,scale", [(2, 0, 1.0), (6, 1, 0.7), (12, 2, 1.0)])
def test_position_gradient_matches_central_differences(N, seed, scale):
    p = o.make_params(N, hstar=0.25, a=0.5)
    x = I.random_walk(N, seed=seed) * scale  # scale < 1: many near-field pairs
    rng = np.random.default_rng(seed)
    Dbar = rng.normal(size=(3 * N, 3 * N))
    xbar, _ = o.rpy_assemble_adjoint(p, x, Dbar)
    d = 1e-6
    fd = np.zeros_like(x)
    for i in range(N):
        for al in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, al] += d
            xm[i, al] -= d
            fd[i, al] = (_phi(p, xp, Dbar) - _phi(p, xm, Dbar)) / (2 * d)
    # adjacent beads sit exactly at R = 2a (unit bonds, a = b/2), where the
    # second derivative jumps: the central difference is then accurate only
    # to O(d), hence the absolute tolerance
    np.testing.assert_allclose(xbar, fd, rtol=1e-6, atol=1e-5 * np.abs(fd).max())


def test_hstar_gradient_matches_central_differences():
    N = 8
    x = I.random_walk(N, seed=5) * 0.8
    Dbar = np.random.default_rng(5).normal(size=(3 * N, 3 * N))
    _, hbar = o.rpy_assemble_adjoint(o.make_params(N, hstar=0.25, a=0.5), x, Dbar)
    d = 1e-6
    fd = (_phi(o.make_params(N, hstar=0.25 + d, a=0.5), x, Dbar)
          - _phi(o.make_params(N, hstar=0.25 - d, a=0.5), x, Dbar)) / (2 * d)
    np.testing.assert_allclose(hbar, fd, rtol=1e-7)


def test_symmetric_adjoint_of_two_beads_along_x():
    """Two beads along x, Dbar = identity on the off-diagonal blocks: phi
    = 2 (A_par + 2 A_perp) with A_par(R), A_perp(R) the two-bead
    coefficients of Eqs. 8-9; d phi / d x_1 = 2 (A_par' + 2 A_perp')."""
    a, hs = 0.5, 0.25
    for R in (0.8, 1.3):
        p = o.make_params(2, hstar=hs, a=a)
        x = np.array([[0.0, 0, 0], [R, 0, 0]])
        Dbar = np.zeros((6, 6))
        Dbar[:3, 3:] = np.eye(3)
        Dbar[3:, :3] = np.eye(3)
        xbar, _ = o.rpy_assemble_adjoint(p, x, Dbar)
        if R >= 2 * a:
            dpar = 0.75 * hs * (-2 / R ** 2 + 4 * a * a / R ** 4)
            dperp = 0.75 * hs * (-1 / R ** 2 - 2 * a * a / R ** 4)
        else:
            dpar = 3 * hs / (8 * a) * (-1 / (2 * a))
            dperp = 3 * hs / (8 * a) * (-3 / (4 * a))
        want = 2 * (dpar + 2 * dperp)
        np.testing.assert_allclose(xbar[1], [want, 0, 0], rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(xbar[0], [-want, 0, 0], rtol=1e-12, atol=1e-15)


def test_rejects_coincident_beads():
    p = o.make_params(3)
    x = np.array([[0.0, 0, 0], [1.0, 0, 0], [1.0, 0, 0]])
    with pytest.raises(ValueError):
        o.rpy_assemble_adjoint(p, x, np.ones((9, 9)))
