"""Pathwise gradients of the ensemble-mean fractional stretch through a
differentiable trajectory (torch.autograd.Function over bd_step, backward by
bd_step_adjoint with checkpoints): the differentiation workload (64 chains
of 256 beads, planar extension at Wi = 1, dt = 1e-4, 200 steps, fixed Philox
seeds, checkpoints every 20 steps), gradients in h* and the strain rate
against central differences of the same GPU trajectories; a reduced version
against the oracle's gradient; and checkpoint intervals that must not
change the result."""
import numpy as np
import pytest
import torch

from oracle import oracle as o
from paper_2208_06559_amd import autograd as AG
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


def _t(v, grad=False):
    return torch.tensor(v, dtype=torch.float64, device=DEV, requires_grad=grad)


def _stretch(X, b=1.0):
    """ensemble-mean |r_{N-1} - r_0| / ((N - 1) b)"""
    N = X.shape[1]
    return torch.linalg.norm(X[:, -1] - X[:, 0], dim=1).mean() / ((N - 1) * b)


def _setup(w, chains):
    X0 = _t(np.stack([w.initial(c) for c in range(chains)]))
    base = dict(dt=w.dt, seed=w.seed, b=w.b, a=w.a)
    K0 = _t(I.kappa_for(w.flow, 1.0))
    return X0, base, K0


def _grad(h, X0, base, K0, hs, rate, steps, every, chains):
    hstar, erate = _t(hs, True), _t(rate, True)
    X = AG.trajectory(X0, hstar, erate * K0, h, base, range(chains), 0, steps, every)
    J = _stretch(X)
    J.backward()
    return J.item(), hstar.grad.item(), erate.grad.item()


def _J(h, X0, base, K0, hs, rate, steps, chains):
    with torch.no_grad():
        X = AG.trajectory(X0, _t(hs), _t(rate) * K0, h, base, range(chains), 0, steps, steps)
    return _stretch(X).item()


def test_differentiation_workload_vs_central_differences(h):
    w = I.GRAD_PLANAR
    X0, base, K0 = _setup(w, w.chains)
    J, gh, ge = _grad(h, X0, base, K0, w.hstar, w.rate, w.steps, 20, w.chains)
    d = 1e-6
    fh = (_J(h, X0, base, K0, w.hstar + d, w.rate, w.steps, w.chains)
          - _J(h, X0, base, K0, w.hstar - d, w.rate, w.steps, w.chains)) / (2 * d)
    fe = (_J(h, X0, base, K0, w.hstar, w.rate + d, w.steps, w.chains)
          - _J(h, X0, base, K0, w.hstar, w.rate - d, w.steps, w.chains)) / (2 * d)
    print(f"J = {J:.12g}; dJ/dh* adjoint {gh:.10e} central {fh:.10e}; "
          f"dJ/de adjoint {ge:.10e} central {fe:.10e}", flush=True)
    assert abs(gh - fh) <= 1e-5 * abs(fh)
    assert abs(ge - fe) <= 1e-5 * abs(fe)


def test_reduced_workload_vs_oracle_gradient(h):
    # two chains of the differentiation workload over its first 20 steps
    w = I.GRAD_PLANAR
    chains, steps = 2, 20
    X0, base, K0 = _setup(w, chains)
    J, gh, ge = _grad(h, X0, base, K0, w.hstar, w.rate, steps, 20, chains)
    ps = [o.make_params(w.n_beads, dt=w.dt, hstar=w.hstar, kappa=w.rate * I.kappa_for(w.flow, 1.0),
                        seed=w.seed, chain_id=c, b=w.b, a=w.a) for c in range(chains)]
    Jo, gho, geo = o.stretch_gradient(ps, X0.cpu().numpy(), steps, I.kappa_for(w.flow, 1.0))
    print(f"J {J:.15g} oracle {Jo:.15g}; dJ/dh* {gh:.12e} oracle {gho:.12e}; "
          f"dJ/de {ge:.12e} oracle {geo:.12e}", flush=True)
    assert abs(J - Jo) <= 1e-12 * abs(Jo)
    assert abs(gh - gho) <= 1e-9 * abs(gho)
    assert abs(ge - geo) <= 1e-9 * abs(geo)


def test_checkpoint_interval_does_not_change_the_gradient(h):
    w = I.GRAD_PLANAR
    chains, steps, N = 3, 23, 32
    X0 = _t(np.stack([I.random_walk(N, seed=9, chain=c) for c in range(chains)]))
    base = dict(dt=w.dt, seed=9, b=1.0, a=0.5)
    K0 = _t(I.kappa_for("planar", 1.0))
    ref = _grad(h, X0, base, K0, 0.25, 30.0, steps, 1, chains)
    for every in (7, 20, 23, 100):
        assert _grad(h, X0, base, K0, 0.25, 30.0, steps, every, chains) == ref
