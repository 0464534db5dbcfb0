"""Kramers stress and N1 (Section 5, Eqs. 28-29) through the C ABI against
the oracle's definition, for springs and rigid rods, packed chains of
uneven size; and the paper's low-h* check (Section 5) on the stiff-spring
step: with fixed noise, the departure from the run without HI is linear
in h*, and the GPU follows the oracle at each h*."""
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


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _stretched(N, seed):
    """random-walk chain whose bonds are stretched or compressed by up to 3 %"""
    x = I.random_walk(N, seed=seed)
    q = np.diff(x, axis=0) * (1.0 + 0.03 * np.random.default_rng(seed).uniform(-1, 1, (N - 1, 1)))
    return np.vstack([x[:1], x[0] + np.cumsum(q, axis=0)]) + 2.0


SIZES = [2, 3, 65, 300, 1000, 4097]


def _tol(ref):
    return 1e-12 * max(1.0, float(np.abs(ref).max()))


def test_stress_springs_uneven_chains(h):
    K = 1e4
    xs = [_stretched(n, n) for n in SIZES]
    got = h.stress(_dev(np.concatenate(xs)), SIZES, k_spring=K).cpu().numpy()
    for c, x in enumerate(xs):
        ref = o.kramers_stress(x, 1.0, k_spring=K)
        np.testing.assert_allclose(got[c], ref, rtol=1e-12, atol=_tol(ref))


def test_stress_rigid_given_tensions(h):
    rng = np.random.default_rng(7)
    xs = [I.random_walk(n, seed=3 * n) for n in SIZES]
    Ts = [rng.normal(scale=50.0, size=n - 1) for n in SIZES]
    got = h.stress(_dev(np.concatenate(xs)), SIZES, tensions=_dev(np.concatenate(Ts)),
                   b=1.0).cpu().numpy()
    for c, (x, T) in enumerate(zip(xs, Ts)):
        ref = o.kramers_stress(x, 1.0, tensions=T)
        np.testing.assert_allclose(got[c], ref, rtol=1e-12, atol=_tol(ref))


@pytest.mark.parametrize("N", [2, 40, 513])
def test_stress_from_gpu_tensions(h, N):
    # tensions of one constraint solve (bd_constrain's T_out) against the
    # oracle's solve of the same step, then the stress of both
    pg = B.make_params(N, dt=1e-3)
    po = o.make_params(N, dt=1e-3)
    x = I.random_walk(N, seed=N)
    xs = x + 0.03 * np.random.default_rng(N).normal(size=x.shape)
    _, Tref, iref = o.constrain(po, x, xs)
    assert iref["status"] == o.OK
    T = torch.zeros(N - 1, dtype=torch.float64, device=DEV)
    h.constrain(pg, _dev(x), _dev(xs), T)
    assert h.info()["status"] == B.OK
    Tg = T.cpu().numpy()
    np.testing.assert_allclose(Tg, Tref, rtol=0, atol=1e-8 * max(1.0, np.abs(Tref).max()))
    got = h.stress(_dev(x), [N], tensions=T).cpu().numpy()[0]
    ref = o.kramers_stress(x, 1.0, tensions=Tref)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-8 * max(1.0, np.abs(ref).max()))


def test_stress_argument_errors(h):
    L = B.lib()
    x = torch.zeros(6, dtype=torch.float64, device=DEV)
    p = x.data_ptr()
    assert L.bd_stress(h._h, 0, p, p, None, 1.0, 1.0, p) == B.ERR_PARAM
    assert L.bd_stress(h._h, 1, p, p, None, 0.0, 1.0, p) == B.ERR_PARAM  # springs need K > 0
    assert L.bd_stress(h._h, 1, p, p, p, 0.0, -1.0, p) == B.ERR_PARAM


def test_low_hstar_stiff_springs(h):
    # The paper checks its HI code by a run at negligible h* (Section 5,
    # chain of 100 Kuhn steps in uniaxial extension at Wi = 3): it must
    # reproduce the run without HI.  With the noise fixed the check is
    # pathwise: x(h*) - x(0) is linear in h* for small h*.
    N, K, steps = 101, 1e4, 10
    kap = I.kappa_for("uniaxial", 3.0 / I.relaxation_time(N))
    x0 = I.random_walk(N, seed=21)
    runs, oracle = {}, {}
    for hs in (0.0, 1e-5, 1e-4, 1e-3):
        kw = dict(dt=1e-4, kappa=kap, seed=21, hstar=hs, noise=B.NOISE_UNIFORM_PAPER)
        pg, po = B.make_params(N, **kw), o.make_params(N, **kw)
        xg = _dev(x0)
        xo = x0.copy()
        for s in range(steps):
            h.step_fraenkel(pg, K, s, xg, B.PREC_FP64)
            xo, io = o.step_fraenkel(po, K, s, xo)
            assert io["status"] == o.OK
        assert h.info()["status"] == B.OK
        runs[hs] = xg.cpu().numpy()
        oracle[hs] = xo
        assert np.abs(runs[hs] - xo).max() <= 1e-10
    d = {hs: np.abs(runs[hs] - runs[0.0]).max() for hs in (1e-5, 1e-4, 1e-3)}
    assert d[1e-5] > 0.0
    for lo, hi in ((1e-5, 1e-4), (1e-4, 1e-3)):
        assert abs(d[hi] / d[lo] / 10.0 - 1.0) < 0.05, d
    # the stress of the low-h* run matches the run without HI to O(h*)
    sg = h.stress(_dev(np.concatenate([runs[0.0], runs[1e-5]])), [N, N], k_spring=K).cpu().numpy()
    n1 = sg[:, 6]
    assert abs(n1[1] - n1[0]) <= 2e-3 * max(1.0, abs(n1[0]))
    print(f"low h*: departures {d}; N1 without HI {n1[0]:.6g}, at h*=1e-5 {n1[1]:.6g}")
