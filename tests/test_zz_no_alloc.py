"""bd_brownian_noalloc (the noise product with the library's fixed scratch
array) against bd_brownian (the same product with a caller workspace),
through the C ABI: two calls in a row, the second with a smaller matrix,
each bitwise equal to bd_brownian on the same input (the two share their
kernels and reduction order); sizes beyond the array are refused."""
import ctypes as C

import pytest
import torch

from paper_2208_06559_amd import binding as B

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _lower_buffer(n, ld, seed):
    """(n, ld) column-major buffer: a seeded random lower triangle, NaN above
    the diagonal and in the padding (the product must not read them)."""
    g = torch.Generator(device=DEV)
    g.manual_seed(seed)
    buf = torch.rand((n, ld), generator=g, dtype=torch.float64, device=DEV) - 0.5
    rows = torch.arange(n, device=DEV).view(n, 1)   # column c of the matrix
    cols = torch.arange(ld, device=DEV).view(1, ld)  # row index within it
    buf[(cols < rows) | (cols >= n)] = float("nan")
    return buf


@pytest.fixture(scope="module")
def h():
    torch.cuda.set_device(0)
    hh = B.Handle(0)
    yield hh
    hh.close()


@pytest.mark.parametrize("sizes", [((4096, 0), (301, 1)), ((1000, 1), (2, 0))])
def test_noalloc_matches_workspace_call(h, sizes):
    for call, (N, noise) in enumerate(sizes):
        n = 3 * N
        ld = n + 7
        p = B.make_params(N, dt=5e-5, seed=11 + call, chain_id=call, noise=noise)
        L = _lower_buffer(n, ld, 100 + N)
        y_ref = torch.full((n,), float("nan"), dtype=torch.float64, device=DEV)
        xi_ref = torch.full((n,), float("nan"), dtype=torch.float64, device=DEV)
        h.brownian(p, 7, L, ld, y_ref, xi_ref)
        y = torch.full((n,), float("nan"), dtype=torch.float64, device=DEV)
        xi = torch.full((n,), float("nan"), dtype=torch.float64, device=DEV)
        h.brownian_noalloc(p, 7, L, ld, y, xi)
        torch.cuda.synchronize()
        assert h.info()["status"] == B.OK
        assert torch.isfinite(y).all() and torch.isfinite(xi).all()
        assert torch.equal(xi, xi_ref), f"call {call} (N={N}): xi differs"
        assert torch.equal(y, y_ref), f"call {call} (N={N}): y differs"


def test_noalloc_refuses_sizes_beyond_the_array(h):
    N = 4097  # n = 12291 > 12288
    n = 3 * N
    p = B.make_params(N)
    L = torch.zeros((1, 1), dtype=torch.float64, device=DEV)
    y = torch.zeros((n,), dtype=torch.float64, device=DEV)
    st = B.lib().bd_brownian_noalloc(h._h, C.byref(p), 0, C.c_void_p(L.data_ptr()), n,
                                     C.c_void_p(y.data_ptr()), None)
    assert st == B.ERR_UNSUPPORTED
    st = B.lib().bd_brownian_noalloc(h._h, C.byref(B.make_params(10)), 0,
                                     C.c_void_p(L.data_ptr()), 29, C.c_void_p(y.data_ptr()), None)
    assert st == B.ERR_PARAM  # ld < n
