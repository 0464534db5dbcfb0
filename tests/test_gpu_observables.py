"""Chain observables (end-to-end vector, R_g^2) through the C ABI against
the oracle's definitions, for packed chains of uneven size (one bead up to
a few thousand) and for the ensemble workload's 256 chains."""
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


def _check(h, xs):
    counts = [len(x) for x in xs]
    xp = torch.tensor(np.concatenate(xs), dtype=torch.float64, device=DEV)
    got = h.observables(xp, counts).cpu().numpy()
    for c, x in enumerate(xs):
        ref = o.observables(x)
        scale = max(1.0, float(np.abs(x).max()))
        np.testing.assert_allclose(got[c], ref, rtol=1e-12, atol=1e-13 * scale * scale)


def test_observables_uneven_chains(h):
    sizes = [1, 2, 3, 64, 65, 257, 1000, 4097]
    _check(h, [I.random_walk(n, seed=n) + 3.0 for n in sizes])


def test_observables_ensemble_workload(h):
    w = I.ENSEMBLE_SHEAR
    spec = I.ensemble_chains(w, I.ensemble_sizes(w.chains, seed=w.seed))
    _check(h, [d["x"] for d in spec])


def test_observables_argument_errors(h):
    L = B.lib()
    x = torch.zeros(6, dtype=torch.float64, device=DEV)
    assert L.bd_observables(h._h, 0, x.data_ptr(), x.data_ptr(), x.data_ptr()) == B.ERR_PARAM
    assert L.bd_observables(h._h, 1, None, x.data_ptr(), x.data_ptr()) == B.ERR_PARAM
