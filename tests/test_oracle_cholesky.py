"""Pins of the oracle Cholesky (Eq. 10, Section 3): the lower factor with
positive diagonal is unique, so LAPACK (numpy / scipy) and closed forms fix
it independently of the implementation."""
import numpy as np
import pytest
import scipy.linalg as sl

from oracle import oracle as o
from paper_2208_06559_amd import inputs as I


@pytest.mark.parametrize("N,seed,hstar", [(16, 0, 0.25), (100, 1, 0.25), (512, 2, 0.25), (300, 3, 0.5)])
def test_matches_lapack(N, seed, hstar):
    x = I.random_walk(N, seed=seed)
    D = o.rpy_assemble(o.make_params(N, hstar=hstar), x)
    L, info = o.cholesky(D)
    assert info == 0
    L = np.tril(L)
    Ln = np.linalg.cholesky(D)
    Ls = sl.cholesky(D, lower=True)
    nrm = np.linalg.norm(Ln)
    assert np.linalg.norm(L - Ln) / nrm <= 1e-13
    assert np.linalg.norm(L - Ls) / nrm <= 1e-13
    assert np.all(np.diag(L) > 0)
    assert np.linalg.norm(L @ L.T - D) / np.linalg.norm(D) <= 1e-14


def test_random_spd_matches_lapack():
    rng = np.random.default_rng(11)
    A = rng.normal(size=(257, 257))
    S = A @ A.T + 257 * np.eye(257)
    L, info = o.cholesky(S)
    assert info == 0
    np.testing.assert_allclose(np.tril(L), np.linalg.cholesky(S), rtol=0, atol=1e-12)


def test_two_bead_closed_form():
    # D = [[I, B], [B, I]] with B = diag(A_par, A_perp, A_perp):
    # L = [[I, 0], [B, diag(sqrt(1 - A^2))]]
    apar, aperp = 0.3125, 0.21875  # h* = 1/4, a = 1/2, R = 1 (Eq. 8)
    D = o.rpy_assemble(o.make_params(2), np.array([[0.0, 0, 0], [1.0, 0, 0]]))
    L, info = o.cholesky(D)
    L = np.tril(L)
    expect = np.zeros((6, 6))
    expect[:3, :3] = np.eye(3)
    expect[3:, :3] = np.diag([apar, aperp, aperp])
    expect[3:, 3:] = np.diag(np.sqrt([1 - apar**2, 1 - aperp**2, 1 - aperp**2]))
    np.testing.assert_allclose(L, expect, atol=1e-15)


def test_hi_off_identity():
    D = o.rpy_assemble(o.make_params(10, hstar=0.0), I.random_walk(10, seed=1))
    L, info = o.cholesky(D)
    np.testing.assert_array_equal(np.tril(L), np.eye(30))


def test_upper_triangle_untouched():
    x = I.random_walk(8, seed=2)
    D = o.rpy_assemble(o.make_params(8), x, o.FILL_LOWER)
    n = D.shape[0]
    iu = np.triu_indices(n, 1)
    D[iu] = 12345.0
    L, info = o.cholesky(D)
    assert info == 0
    assert np.all(L[iu] == 12345.0)


def test_non_spd_reports_column():
    A = np.eye(5)
    A[3, 3] = -1.0
    L, info = o.cholesky(A)
    assert info == 4
    B = np.array([[1.0, 2.0], [2.0, 1.0]])  # second pivot 1 - 4 < 0
    L, info = o.cholesky(B)
    assert info == 2
    C = np.eye(3)
    C[0, 0] = 0.0
    assert o.cholesky(C)[1] == 1
