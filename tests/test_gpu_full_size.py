"""The bench's workload at full size: one chain of N = 4096 beads
(n = 3N = 12288), uniaxial flow Wi = 5, through the C ABI in the launch
configuration `bench.py` times (the library's defaults: four-panel steps
while more than 4096 rows remain, lookahead, matrix-core diagonal blocks).

At this size the oracle cannot factor the matrix inside a test, so the
checks are outputs the oracle computes one by one and properties that hold
at any size:

* assembly (Eqs. 7-9): sampled entries of D against the oracle's 3 x 3
  blocks, at the FP64 rounding level;
* Cholesky (Eq. 10): (L L^T)_ij at sampled (i, j) against the oracle's
  D_ij.  FP64: |(L L^T - D)_ij| <= 2 (n + 1) u (|L| |L^T|)_ij: the backward
  error bound (n + 1) u |L||L^T| of the Cholesky factorisation plus as
  much again for the test's own length-n dot product (u = 2^-53;
  |L||L^T| <= 1 entrywise here since D_ii = 1).  Mixed: every entry of
  L L^T - D is at most its Frobenius norm, so the bound
  ||L L^T - D||_F <= 1e-6 ||D||_F caps each sampled entry at
  1e-6 ||D||_F; the full residual is also formed with an FP64 GEMM;
* two whole steps (Eq. 6 with the rigid-rod solve), each against the
  oracle's step from the same state and seeds: FP64 within 1e-10 b, mixed
  within 1e-6 b, rod lengths within 1e-10 b.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as o
from paper_2208_06559_amd import binding as B
from paper_2208_06559_amd import inputs as I

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
W = I.LONG_UNIAXIAL
N = W.n_beads
n = 3 * N
SAMPLES = 3000


@pytest.fixture(scope="module")
def h():
    torch.cuda.set_device(0)
    hh = B.Handle(0)
    yield hh
    hh.close()


def _params():
    kw = dict(dt=W.dt, kappa=W.kappa, seed=W.seed, hstar=W.hstar, a=W.a, b=W.b)
    return B.make_params(N, **kw), o.make_params(N, **kw)


def _pairs(seed):
    """Sampled lower-triangle positions (i >= j): random ones, the diagonal
    and the corners of the matrix (first and last panels)."""
    rng = np.random.default_rng(seed)
    i = rng.integers(0, n, SAMPLES)
    j = rng.integers(0, n, SAMPLES)
    d = rng.integers(0, n, 200)
    edge = np.array([0, 1, 127, 128, n - 129, n - 128, n - 2, n - 1])
    ii = np.concatenate([np.maximum(i, j), d, np.repeat(edge, len(edge))])
    jj = np.concatenate([np.minimum(i, j), d, np.tile(edge, len(edge))])
    keep = ii >= jj
    return ii[keep], jj[keep]


def _oracle_D(x, ii, jj):
    """D_ij one entry at a time from the oracle's 3 x 3 RPY block."""
    out = np.empty(len(ii))
    for e, (i, j) in enumerate(zip(ii, jj)):
        bi, bj = i // 3, j // 3
        if bi == bj:
            out[e] = 1.0 if i == j else 0.0
        else:
            out[e] = o.rpy_block(W.hstar, W.a, x[bi] - x[bj])[i % 3, j % 3]
    return out


def _assemble(h, pg, x):
    """D (lower triangle) in a zeroed column-major (n, n) buffer: buf[c, r] = D(r, c)."""
    buf = torch.zeros((n, n), dtype=torch.float64, device=DEV)
    h.rpy_assemble(pg, torch.tensor(x, dtype=torch.float64, device=DEV), buf, n, B.FILL_LOWER)
    return buf


def test_rpy_assemble_full_size_sampled(h):
    pg, _ = _params()
    x = W.initial()
    buf = _assemble(h, pg, x)
    ii, jj = _pairs(1)
    got = buf[torch.as_tensor(jj, device=DEV), torch.as_tensor(ii, device=DEV)].cpu().numpy()
    ref = _oracle_D(x, ii, jj)
    np.testing.assert_allclose(got, ref, rtol=1e-14, atol=1e-15)
    up = torch.triu(buf[:2048, :2048].t(), 1)  # strict upper part of a corner block
    assert torch.count_nonzero(up).item() == 0


@pytest.mark.parametrize("prec", [B.PREC_FP64, B.PREC_MIXED])
def test_cholesky_full_size(h, prec):
    pg, _ = _params()
    x = W.initial()
    buf = _assemble(h, pg, x)
    D = buf.t().clone()          # D(r, c) for r >= c, zero above
    D = D + torch.tril(D, -1).t()  # full symmetric D
    h.cholesky(buf, n, n, prec)
    st = h.info()
    assert st["status"] == B.OK and st["potrf_info"] == 0, st
    L = buf.t()                  # L(r, c), zero above the diagonal
    assert torch.count_nonzero(torch.triu(L[:2048, :2048], 1)).item() == 0
    diag = torch.diagonal(L)
    assert bool(torch.all(diag > 0).item())
    ii, jj = _pairs(2)
    ti, tj = torch.as_tensor(ii, device=DEV), torch.as_tensor(jj, device=DEV)
    llt = (L[ti, :] * L[tj, :]).sum(dim=1).cpu().numpy()  # (L L^T)_ij one by one
    ref = _oracle_D(x, ii, jj)
    r = np.abs(llt - ref)
    dnorm = torch.linalg.norm(D).item()
    if prec == B.PREC_FP64:
        bound = 2 * (n + 1) * 2.0**-53
        assert r.max() <= bound, (r.max(), bound)
    else:
        assert r.max() <= 1e-6 * dnorm, (r.max(), 1e-6 * dnorm)
        res = torch.linalg.norm(L @ L.t() - D).item() / dnorm
        assert res <= 1e-6, res


def test_step_full_size(h):
    """The first two steps of the workload, each from the oracle's state
    (step 0 from the start, step 1 from the oracle's step-0 result)."""
    pg, po = _params()
    x = W.initial()
    for s in range(2):
        xo, io = o.step(po, s, x)
        assert io["status"] == o.OK
        for prec, tol in ((B.PREC_FP64, 1e-10), (B.PREC_MIXED, 1e-6)):
            xg = torch.tensor(x, dtype=torch.float64, device=DEV)
            h.step(pg, s, xg, prec)
            st = h.info()
            assert st["status"] == B.OK, (s, prec, st)
            xn = xg.cpu().numpy()
            err = np.abs(xn - xo).max() / W.b
            print(f"N = {N} step {s} prec {prec}: max |dr|/b vs oracle {err:.3e}", flush=True)
            assert err <= tol, (s, prec, err)
            rods = np.linalg.norm(np.diff(xn, axis=0), axis=1)
            assert np.abs(rods - W.b).max() <= 1e-10, (s, prec)
        x = xo


@pytest.mark.parametrize("Nb", [6400, 4101])
def test_step_longest_chain(h, Nb):
    """Chains beyond 4097 beads (the tridiagonal system of the tension solve
    in global memory): N = 6400 beads, n = 19200, the paper's longest chain
    (6399 rods, Section 4's largest matrix order), and N = 4101, just past
    the in-LDS solve; uniaxial extension at Wi = 5, one step of each
    precision from the oracle's start."""
    rate = 5.0 / I.relaxation_time(Nb)
    kw = dict(dt=W.dt, kappa=I.kappa_for("uniaxial", rate), seed=W.seed, hstar=W.hstar, a=W.a,
              b=W.b)
    pg, po = B.make_params(Nb, **kw), o.make_params(Nb, **kw)
    x = I.random_walk(Nb, W.b, W.seed)
    xo, io = o.step(po, 0, x)
    assert io["status"] == o.OK
    for prec, tol in ((B.PREC_FP64, 1e-10), (B.PREC_MIXED, 1e-6)):
        xg = torch.tensor(x, dtype=torch.float64, device=DEV)
        h.step(pg, 0, xg, prec)
        st = h.info()
        assert st["status"] == B.OK, (prec, st)
        xn = xg.cpu().numpy()
        err = np.abs(xn - xo).max() / W.b
        print(f"N = {Nb} prec {prec}: max |dr|/b vs oracle {err:.3e}, newton "
              f"{st['newton_iters']}, krylov {st['krylov_iters']}", flush=True)
        assert err <= tol, (prec, err)
        rods = np.linalg.norm(np.diff(xn, axis=0), axis=1)
        assert np.abs(rods - W.b).max() <= 1e-10, prec
