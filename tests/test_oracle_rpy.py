"""Pins of the oracle's RPY diffusion tensor (Eqs. 7-9, Section 3) against
closed forms and invariants that do not depend on the implementation."""
import os

import numpy as np
import pytest

from oracle import oracle as o
from paper_2208_06559_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rpy_two_bead.txt")


def _golden():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append(tuple(float(t) for t in line.split()))
    return rows


@pytest.mark.parametrize("hstar,a,R,apar,aperp", _golden())
def test_two_bead_closed_form(hstar, a, R, apar, aperp):
    # beads 0 and 1 on the x axis: D_01 = diag(A_par, A_perp, A_perp)
    B = o.rpy_block(hstar, a, [-R, 0.0, 0.0])
    np.testing.assert_allclose(B, np.diag([apar, aperp, aperp]), rtol=0, atol=1e-15)
    p = o.make_params(2, hstar=hstar, a=a)
    D = o.rpy_assemble(p, np.array([[0.0, 0, 0], [R, 0, 0]]))
    np.testing.assert_allclose(D[:3, 3:], np.diag([apar, aperp, aperp]), atol=1e-15)
    np.testing.assert_array_equal(D[:3, :3], np.eye(3))  # Eq. 7
    np.testing.assert_array_equal(D[3:, 3:], np.eye(3))


def test_block_layout_and_symmetry():
    x = I.random_walk(17, seed=2)
    p = o.make_params(17)
    D = o.rpy_assemble(p, x)
    for i in range(17):
        for j in range(17):
            blk = D[3 * i:3 * i + 3, 3 * j:3 * j + 3]
            ref = np.eye(3) if i == j else o.rpy_block(0.25, 0.5, x[i] - x[j])
            np.testing.assert_array_equal(blk, ref)
    # symmetric up to the rounding of the product order in R R^T
    np.testing.assert_allclose(D, D.T, rtol=0, atol=1e-16)


def test_lower_fill_is_tril_of_full():
    x = I.random_walk(9, seed=3)
    p = o.make_params(9)
    full = o.rpy_assemble(p, x, o.FILL_FULL)
    low = o.rpy_assemble(p, x, o.FILL_LOWER)
    np.testing.assert_array_equal(low, np.tril(full))


def test_translation_and_rotation():
    x = I.random_walk(20, seed=4)
    p = o.make_params(20)
    D = o.rpy_assemble(p, x)
    Dt = o.rpy_assemble(p, x + np.array([3.5, -7.25, 1.125]))
    np.testing.assert_allclose(Dt, D, atol=1e-13)
    th = 0.7
    Rz = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
    Rx = np.array([[1, 0, 0], [0, np.cos(1.1), -np.sin(1.1)], [0, np.sin(1.1), np.cos(1.1)]])
    Rot = Rz @ Rx
    Dr = o.rpy_assemble(p, x @ Rot.T)
    big = np.kron(np.eye(20), Rot)
    np.testing.assert_allclose(Dr, big @ D @ big.T, atol=1e-13)


def _block(h, a, R):
    return o.rpy_block(h, a, np.asarray(R, dtype=float))


def test_continuous_and_c1_at_contact():
    h, a = 0.25, 0.5
    d = np.array([0.3, -0.5, 0.81])
    d /= np.linalg.norm(d)
    eps = 1e-7
    inside = _block(h, a, (2 * a - eps) * d)
    outside = _block(h, a, (2 * a + eps) * d)
    np.testing.assert_allclose(inside, outside, atol=1e-6)
    # one-sided radial derivatives agree: I-part -9h/(32a^2), RR-part +3h/(32a^2)
    s = 1e-5
    din = (_block(h, a, (2 * a - s) * d) - _block(h, a, (2 * a - 2 * s) * d)) / s
    dout = (_block(h, a, (2 * a + 2 * s) * d) - _block(h, a, (2 * a + s) * d)) / s
    np.testing.assert_allclose(din, dout, atol=2e-4)
    dd = np.outer(d, d)
    expect = -9 * h / (32 * a * a) * np.eye(3) + 3 * h / (32 * a * a) * dd
    np.testing.assert_allclose(dout, expect, atol=2e-4)


def test_overlap_limit():
    h, a = 0.25, 0.5
    np.testing.assert_allclose(_block(h, a, [0.0, 0.0, 0.0]), (h / a) * np.eye(3), atol=0)
    np.testing.assert_allclose(_block(h, a, [1e-9, 0, 0]), (h / a) * np.eye(3), atol=1e-8)


@pytest.mark.parametrize("Rlen", [0.3, 0.9, 0.999, 1.001, 1.7, 4.0])
def test_divergence_free(Rlen):
    # sum_beta d D_{alpha beta} / d R_beta = 0 for both branches (RPY is
    # divergence-free, so Euler-Maruyama needs no drift term)
    h, a = 0.25, 0.5
    rng = np.random.default_rng(int(Rlen * 10))
    for _ in range(5):
        R = rng.normal(size=3)
        R *= Rlen / np.linalg.norm(R)
        s = 1e-6
        div = np.zeros(3)
        for beta in range(3):
            e = np.zeros(3)
            e[beta] = s
            dD = (_block(h, a, R + e) - _block(h, a, R - e)) / (2 * s)
            div += dD[:, beta]
        np.testing.assert_allclose(div, 0.0, atol=1e-8)


@pytest.mark.parametrize("N,seed,hstar", [(50, 0, 0.25), (200, 1, 0.25), (400, 2, 0.5), (120, 3, 0.1)])
def test_spd_lower_bound(N, seed, hstar):
    # D = (1 - h*/a) I + (h*/a) D_RPY(a) with D_RPY positive semi-definite
    x = I.random_walk(N, seed=seed)
    # compact the coil so many pairs fall inside the near field
    x = 0.35 * x
    p = o.make_params(N, hstar=hstar)
    ev = np.linalg.eigvalsh(o.rpy_assemble(p, x))
    assert ev.min() >= 1 - hstar / 0.5 - 1e-12


def test_hi_off_is_identity():
    x = I.random_walk(30, seed=5)
    D = o.rpy_assemble(o.make_params(30, hstar=0.0), x)
    np.testing.assert_array_equal(D, np.eye(90))


def test_invalid_params_rejected():
    x = I.random_walk(4, seed=0)
    with pytest.raises(ValueError):
        o.rpy_assemble(o.make_params(4, hstar=0.6, a=0.5), x)
    with pytest.raises(ValueError):
        o.rpy_assemble(o.make_params(4, a=0.0), x)
