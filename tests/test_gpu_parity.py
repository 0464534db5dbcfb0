"""GPU (HIP, gfx950) path vs the CPU FP64 oracle, element by element, on the
same seeded inputs; every call goes through the C ABI.

Tolerances: FP64 path within 1e-10 relative per step (positions in units of
b); assembly and factor at the rounding level of FP64 (1e-13 relative);
mixed precision through its residual bound ||B B^T - D||_F / ||D||_F <= 1e-6.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as o
from paper_2208_06559_amd import binding as B
from paper_2208_06559_amd import inputs as I

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def h():
    torch.cuda.set_device(0)
    hh = B.Handle(0)
    yield hh
    hh.close()


def _params(N, **kw):
    return B.make_params(N, **kw), o.make_params(N, **kw)


def _to_dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _colmajor_buffer(M: np.ndarray, ld: int):
    """device (n, ld) buffer holding the column-major matrix M (n x n)."""
    n = M.shape[0]
    buf = np.full((n, ld), np.nan)
    buf[:, :n] = M.T
    return _to_dev(buf)


def _from_buffer(buf, n):
    return buf.cpu().numpy()[:, :n].T.copy()


@pytest.mark.parametrize("N,seed,fill", [(2, 0, 1), (32, 0, 0), (32, 0, 1), (333, 1, 0), (1001, 2, 1)])
def test_rpy_assemble(h, N, seed, fill):
    pg, po = _params(N)
    x = I.random_walk(N, seed=seed) * 0.6  # compact: many near-field pairs
    n = 3 * N
    ld = n + 5  # ragged leading dimension
    D = _to_dev(np.full((n, ld), 777.0))
    h.rpy_assemble(pg, _to_dev(x), D, ld, fill)
    torch.cuda.synchronize()
    got = D.cpu().numpy()
    ref = o.rpy_assemble(po, x, o.FILL_FULL)
    Dg = got[:, :n].T
    if fill == B.FILL_FULL:
        np.testing.assert_allclose(Dg, ref, rtol=1e-14, atol=1e-15)
    else:
        low = np.tril_indices(n)
        np.testing.assert_allclose(Dg[low], ref[low], rtol=1e-14, atol=1e-15)
        up = np.triu_indices(n, 1)
        assert np.all(Dg[up] == 777.0)
    assert np.all(got[:, n:] == 777.0)  # padding rows beyond n untouched


@pytest.mark.parametrize("N,seed", [(2, 0), (32, 0), (43, 3), (512, 1), (1001, 2)])
def test_cholesky_fp64(h, N, seed):
    pg, po = _params(N)
    x = I.random_walk(N, seed=seed)
    n = 3 * N
    Dref = o.rpy_assemble(po, x, o.FILL_FULL)
    Lref, info = o.cholesky(Dref)
    assert info == 0
    ld = n + 3
    A = _colmajor_buffer(np.tril(Dref) + np.triu(np.full((n, n), 5.0), 1), ld)
    h.cholesky(A, n, ld, B.PREC_FP64)
    st = h.info()
    assert st["status"] == B.OK and st["potrf_info"] == 0
    L = _from_buffer(A, n)
    low = np.tril_indices(n)
    scale = np.abs(Lref[low]).max()
    err = np.abs(L[low] - Lref[low]).max() / scale
    assert err <= 1e-13, err
    up = np.triu_indices(n, 1)
    assert np.all(L[up] == 5.0)


@pytest.mark.parametrize("N,seed", [(43, 3), (512, 1), (1001, 2)])
def test_cholesky_mixed_residual(h, N, seed):
    pg, po = _params(N)
    x = I.random_walk(N, seed=seed)
    n = 3 * N
    Dref = o.rpy_assemble(po, x, o.FILL_FULL)
    ld = n
    A = _colmajor_buffer(np.tril(Dref), ld)
    h.cholesky(A, n, ld, B.PREC_MIXED)
    assert h.info()["status"] == B.OK
    L = np.tril(_from_buffer(A, n))
    res = np.linalg.norm(L @ L.T - Dref) / np.linalg.norm(Dref)
    assert res <= 1e-6, res
    assert np.all(np.diag(L) > 0)


# (most panels per trailing pass, rows below which steps narrow to two
# panels): one, two or four panels throughout, and four turning to two
@pytest.mark.parametrize("steps", [("1", "0"), ("2", "0"), ("4", "0"), ("4", "600")])
@pytest.mark.parametrize("lookahead", ["0", "1"])
@pytest.mark.parametrize("prec", [B.PREC_FP64, B.PREC_MIXED])
@pytest.mark.parametrize("potrf", ["tile", "reg"])
def test_cholesky_schedules(monkeypatch, steps, lookahead, prec, potrf):
    """Every factorisation schedule (one, two or four panels per trailing
    pass, or four turning to two, with or without the lookahead stream,
    diagonal blocks on matrix cores or in register tiles) on a ragged n
    spanning several steps: FP64 to the rounding level of the oracle's
    factor, MIXED through its residual bound."""
    monkeypatch.setenv("BDRPY_STEP_PANELS", steps[0])
    monkeypatch.setenv("BDRPY_WIDE_ROWS", steps[1])
    monkeypatch.setenv("BDRPY_LOOKAHEAD", lookahead)
    monkeypatch.setenv("BDRPY_POTRF", potrf)
    hh = B.Handle(0)
    try:
        N = 367  # n = 1101: eight full panels and a 77-column tail
        pg, po = _params(N)
        x = I.random_walk(N, seed=5)
        n = 3 * N
        Dref = o.rpy_assemble(po, x, o.FILL_FULL)
        ld = n + 1
        A = _colmajor_buffer(np.tril(Dref), ld)
        hh.cholesky(A, n, ld, prec)
        assert hh.info()["status"] == B.OK
        L = np.tril(_from_buffer(A, n))
        if prec == B.PREC_FP64:
            Lref, info = o.cholesky(Dref)
            assert info == 0
            Lref = np.tril(Lref)  # the oracle leaves the strict upper part as given
            err = np.abs(L - Lref).max() / np.abs(Lref).max()
            assert err <= 1e-13, err
        else:
            res = np.linalg.norm(L @ L.T - Dref) / np.linalg.norm(Dref)
            assert res <= 1e-6, res
    finally:
        hh.close()


def test_cholesky_not_spd_reports_column(h):
    n = 300
    M = np.eye(n)
    M[200, 200] = -1.0
    A = _colmajor_buffer(M, n)
    h.cholesky(A, n, n, B.PREC_FP64)
    st = h.info()
    assert st["status"] == B.ERR_NOT_SPD
    assert st["potrf_info"] == 201


@pytest.mark.parametrize("noise", [B.NOISE_GAUSSIAN, B.NOISE_UNIFORM_PAPER])
@pytest.mark.parametrize("N", [2, 32, 700])
def test_brownian(h, N, noise):
    kw = dict(dt=1e-4, seed=123, chain_id=5, noise=noise)
    pg, po = _params(N, **kw)
    x = I.random_walk(N, seed=N)
    n = 3 * N
    L = np.linalg.cholesky(o.rpy_assemble(po, x, o.FILL_FULL))
    yref, xiref = o.brownian(po, 77, L)
    ld = n + 1
    Ld = _colmajor_buffer(np.tril(L), ld)
    y = torch.zeros(n, dtype=torch.float64, device=DEV)
    xi = torch.zeros(n, dtype=torch.float64, device=DEV)
    h.brownian(pg, 77, Ld, ld, y, xi)
    torch.cuda.synchronize()
    xi_g = xi.cpu().numpy()
    if noise == B.NOISE_UNIFORM_PAPER:
        np.testing.assert_array_equal(xi_g, xiref)
    else:
        np.testing.assert_allclose(xi_g, xiref, rtol=1e-14, atol=1e-15)
    scale = np.abs(yref).max()
    np.testing.assert_allclose(y.cpu().numpy(), yref, rtol=0, atol=1e-13 * scale)


@pytest.mark.parametrize("N,hstar", [(2, 0.25), (2, 0.0), (32, 0.25), (200, 0.5), (1000, 0.25)])
def test_constrain(h, N, hstar):
    pg, po = _params(N, hstar=hstar, dt=1e-3)
    rng = np.random.default_rng(N)
    x = I.random_walk(N, seed=N + 7)
    xs = x + 0.03 * rng.normal(size=x.shape)
    xref, Tref, iref = o.constrain(po, x, xs)
    assert iref["status"] == o.OK
    xg = _to_dev(xs)
    T = torch.zeros(N - 1, dtype=torch.float64, device=DEV)
    h.constrain(pg, _to_dev(x), xg, T)
    st = h.info()
    assert st["status"] == B.OK, st
    xn = xg.cpu().numpy()
    assert np.abs(xn - xref).max() <= 1e-11
    rods = np.linalg.norm(np.diff(xn, axis=0), axis=1)
    assert np.abs(rods - 1.0).max() <= 1e-12
    assert st["max_rod_err"] <= 1e-13


def test_constrain_no_root_reports(h):
    pg, po = _params(2, dt=1e-3)
    x = np.array([[0.0, 0, 0], [1.0, 0, 0]])
    xs = np.array([[0.0, 0, 0], [0.0, 5.0, 0]])
    h.constrain(pg, _to_dev(x), _to_dev(xs))
    assert h.info()["status"] == B.ERR_NO_CONVERGE


def _trajectory_parity(h, w, nsteps):
    """Every step twice: from the oracle's state (one-step parity) and along
    the GPU's own trajectory (free-running parity), both within 1e-10 b of
    the oracle's trajectory.  Returns the worst (one-step, free-running)
    errors in units of b."""
    kw = dict(dt=w.dt, kappa=w.kappa, seed=w.seed, hstar=w.hstar, a=w.a, b=w.b)
    pg, po = _params(w.n_beads, **kw)
    x0 = w.initial()
    xg = _to_dev(x0)
    xo = x0.copy()
    worst_one = worst_free = 0.0
    for s in range(nsteps):
        # one step from the common (oracle) state ...
        x1 = _to_dev(xo)
        h.step(pg, s, x1, B.PREC_FP64)
        # ... and the free-running GPU trajectory
        h.step(pg, s, xg, B.PREC_FP64)
        st = h.info()
        assert st["status"] == B.OK, (s, st)
        xo, io = o.step(po, s, xo)
        assert io["status"] == o.OK
        one = np.abs(x1.cpu().numpy() - xo).max() / w.b
        free = np.abs(xg.cpu().numpy() - xo).max() / w.b
        assert one <= 1e-10, (s, one)
        assert free <= 1e-10, (s, free)
        worst_one = max(worst_one, one)
        worst_free = max(worst_free, free)
    rods = np.linalg.norm(np.diff(xg.cpu().numpy(), axis=0), axis=1)
    assert np.abs(rods - w.b).max() <= 1e-10
    print(f"{w.name}: {nsteps} steps, worst one-step {worst_one:.3e} b, "
          f"worst free-running {worst_free:.3e} b", flush=True)
    return worst_one, worst_free


def test_step_trajectory_small(h):
    _trajectory_parity(h, I.SINGLE_SMALL, I.SINGLE_SMALL.steps)


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_step_trajectory_planar_512(h):
    """N = 512 beads, planar extension at Wi = 1, dt = 1e-4: all 1000 steps
    of the workload, each against the oracle."""
    _trajectory_parity(h, I.SINGLE_PLANAR, I.SINGLE_PLANAR.steps)


def test_step_mixed_keeps_rods(h):
    w = I.SINGLE_PLANAR
    kw = dict(dt=w.dt, kappa=w.kappa, seed=w.seed)
    pg, po = _params(w.n_beads, **kw)
    x0 = w.initial()
    xg = _to_dev(x0)
    xo = x0.copy()
    for s in range(5):
        h.step(pg, s, xg, B.PREC_MIXED)
        st = h.info()
        assert st["status"] == B.OK
        xo, _ = o.step(po, s, xo)
    xn = xg.cpu().numpy()
    rods = np.linalg.norm(np.diff(xn, axis=0), axis=1)
    assert np.abs(rods - 1.0).max() <= 1e-10
    # mixed precision changes the noise realisation only at the 1e-7 level
    assert np.abs(xn - xo).max() <= 1e-6


def test_deterministic(h):
    w = I.SINGLE_PLANAR
    pg, _ = _params(w.n_beads, dt=w.dt, kappa=w.kappa, seed=w.seed)
    outs = []
    for _ in range(2):
        xg = _to_dev(w.initial())
        for s in range(3):
            h.step(pg, s, xg, B.PREC_MIXED)
        outs.append(xg.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def test_param_errors_are_synchronous(h):
    pg = B.make_params(10, hstar=0.9, a=0.5)
    x = torch.zeros(30, dtype=torch.float64, device=DEV)
    with pytest.raises(B.BdError) as e:
        h.step(pg, 0, x)
    assert e.value.status == B.ERR_PARAM
