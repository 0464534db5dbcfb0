"""The adjoint of the noise product through the C ABI against the oracle's
adjoint (pinned by central differences and the adjoint identities): Lbar
on the lower triangle (the strict upper part untouched) and xibar."""
import numpy as np
import pytest
import torch

from oracle import oracle as o
from paper_2208_06559_amd import binding as B

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def h():
    torch.cuda.set_device(0)
    hh = B.Handle(0)
    yield hh
    hh.close()


def _cm(M, ld, fill=0.0):
    n = M.shape[0]
    buf = np.full((n, ld), fill)
    buf[:, :n] = M.T
    return torch.tensor(buf, dtype=torch.float64, device=DEV)


@pytest.mark.parametrize("N,noise", [(2, 0), (33, 1), (400, 0)])
def test_brownian_adjoint_vs_oracle(h, N, noise):
    n = 3 * N
    kw = dict(dt=1e-4, noise=noise)
    pg, po = B.make_params(N, **kw), o.make_params(N, **kw)
    rng = np.random.default_rng(N)
    L = np.tril(rng.normal(size=(n, n))) + 2 * np.eye(n)
    xi, ybar = rng.normal(size=n), rng.normal(size=n)
    ld, ldb = n + 1, n + 2
    Lbar = torch.full((n, ldb), 7.0, dtype=torch.float64, device=DEV)  # sentinel everywhere
    xibar = torch.empty(n, dtype=torch.float64, device=DEV)
    h.brownian_adjoint(pg, _cm(L, ld), ld, torch.tensor(xi, device=DEV),
                       torch.tensor(ybar, device=DEV), Lbar, ldb, xibar)
    torch.cuda.synchronize()
    Lr, xr = o.brownian_adjoint(po, L, xi, ybar)
    got = Lbar.cpu().numpy()[:, :n].T  # (row, col)
    low = np.tril(np.ones((n, n), dtype=bool))
    np.testing.assert_allclose(got[low], Lr[low], rtol=1e-14, atol=1e-300)
    assert np.all(got[~low] == 7.0)
    np.testing.assert_allclose(xibar.cpu().numpy(), xr, rtol=1e-12, atol=1e-12 * np.abs(xr).max())
