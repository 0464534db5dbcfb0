"""The stiff-spring step (the paper's own Fraenkel springs, Eq. 3, with the
semi-implicit link update of Eqs. 13-17) through the C ABI against the
oracle's step from the same state and seeds: FP64 within 1e-10 b, mixed
within 1e-6 b (the factor's residual bound carried through one step), at
small sizes with a ragged tail and at the bench's full size N = 4096."""
import ctypes as C

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


@pytest.mark.parametrize("prec,tol", [(B.PREC_FP64, 1e-10), (B.PREC_MIXED, 1e-6)])
@pytest.mark.parametrize("K", [1e3, 1e4])
@pytest.mark.parametrize("N,noise", [(2, 0), (3, 1), (32, 0), (300, 1), (1001, 0)])
def test_fraenkel_step_vs_oracle(h, prec, tol, K, N, noise):
    kw = dict(dt=1e-4, kappa=I.kappa_for("shear", 2.0), seed=5, chain_id=N, noise=noise)
    pg, po = _params(N, **kw)
    x0 = I.random_walk(N, seed=5, chain=N) * 1.01
    xo, io = o.step_fraenkel(po, K, 9, x0)
    assert io["status"] == o.OK
    xg = torch.tensor(x0, dtype=torch.float64, device=DEV)
    h.step_fraenkel(pg, K, 9, xg, prec)
    st = h.info()
    assert st["status"] == B.OK, st
    xn = xg.cpu().numpy()
    assert np.abs(xn - xo).max() / pg.b <= tol, np.abs(xn - xo).max()
    assert abs(st["max_rod_err"] - io["max_rod_err"]) <= 10 * tol


def test_fraenkel_several_steps(h):
    N, K = 64, 1e4
    kw = dict(dt=1e-4, kappa=I.kappa_for("planar", 1.0), seed=6)
    pg, po = _params(N, **kw)
    xo = I.random_walk(N, seed=6)
    xg = torch.tensor(xo, dtype=torch.float64, device=DEV)
    for s in range(5):
        xo, io = o.step_fraenkel(po, K, s, xo)
        h.step_fraenkel(pg, K, s, xg, B.PREC_FP64)
    assert h.info()["status"] == B.OK
    assert np.abs(xg.cpu().numpy() - xo).max() <= 1e-10


def test_fraenkel_full_size(h):
    W = I.LONG_UNIAXIAL
    kw = dict(dt=W.dt, kappa=W.kappa, seed=W.seed, hstar=W.hstar, a=W.a, b=W.b)
    pg, po = _params(W.n_beads, **kw)
    x0 = W.initial()
    xo, io = o.step_fraenkel(po, 1e4, 0, x0)
    assert io["status"] == o.OK
    for prec, tol in ((B.PREC_FP64, 1e-10), (B.PREC_MIXED, 1e-6)):
        xg = torch.tensor(x0, dtype=torch.float64, device=DEV)
        h.step_fraenkel(pg, 1e4, 0, xg, prec)
        assert h.info()["status"] == B.OK
        assert np.abs(xg.cpu().numpy() - xo).max() / W.b <= tol, prec


def test_fraenkel_argument_errors(h):
    L = B.lib()
    pg = B.make_params(8)
    x = torch.zeros(8 * 3, dtype=torch.float64, device=DEV)
    ws = h.workspace(B.OP_STEP, 24)
    for K in (0.0, -1.0, float("inf")):
        assert L.bd_step_fraenkel(h._h, C.byref(pg), K, 0, x.data_ptr(), 0, ws.data_ptr(),
                                  ws.numel()) == B.ERR_PARAM
    big = B.make_params(8194)
    assert L.bd_step_fraenkel(h._h, C.byref(big), 1e3, 0, x.data_ptr(), 0, ws.data_ptr(),
                              ws.numel()) == B.ERR_UNSUPPORTED
