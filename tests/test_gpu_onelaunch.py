"""The one-launch tension solve (BDRPY_CONSTRAIN=onelaunch: the whole
Newton-GMRES iteration in one launch with grid barriers, no host round
trip): every step bitwise equal to the default host-polled launches, and a
step captured in a HIP graph replaying to the same positions as the eager
step, replay after replay with eager work in between."""
import os

import numpy as np
import pytest
import torch

from paper_2208_06559_amd import binding as B
from paper_2208_06559_amd import inputs as I

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def handles():
    torch.cuda.set_device(0)
    h0 = B.Handle(0)
    old = os.environ.get("BDRPY_CONSTRAIN")
    os.environ["BDRPY_CONSTRAIN"] = "onelaunch"
    try:
        h1 = B.Handle(0)
    finally:
        if old is None:
            del os.environ["BDRPY_CONSTRAIN"]
        else:
            os.environ["BDRPY_CONSTRAIN"] = old
    yield h0, h1
    h1.close()
    h0.close()


@pytest.mark.parametrize("N,prec", [(2, B.PREC_FP64), (33, B.PREC_FP64), (300, B.PREC_MIXED),
                                    (1025, B.PREC_FP64), (4096, B.PREC_MIXED),
                                    (5000, B.PREC_FP64)])
def test_onelaunch_equals_polled_bitwise(handles, N, prec):
    h0, h1 = handles
    w = I.LONG_UNIAXIAL
    p = B.make_params(N, dt=w.dt, kappa=I.kappa_for("uniaxial", 5.0 / I.relaxation_time(N)),
                      seed=7, chain_id=N)
    x0 = torch.tensor(I.random_walk(N, seed=7, chain=N), dtype=torch.float64, device=DEV)
    xa, xb = x0.clone(), x0.clone()
    for s in range(2):
        h0.step(p, s, xa, prec)
        ia = h0.info()
        h1.step(p, s, xb, prec)
        ib = h1.info()
        assert ia["status"] == B.OK and ib == ia, (s, ia, ib)
        assert torch.equal(xa, xb), (N, s, (xa - xb).abs().max().item())


def test_onelaunch_step_replays_from_a_graph(handles):
    h0, h1 = handles
    N, S = 300, 5
    p = B.make_params(N, dt=1e-4, kappa=I.kappa_for("planar", 1e-3), seed=11)
    n = 3 * N
    ws = h1.workspace(B.OP_STEP, n, B.PREC_FP64)
    starts = [torch.tensor(I.random_walk(N, seed=11, chain=c), dtype=torch.float64, device=DEV)
              for c in range(3)]
    xg = starts[0].clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        h1.step(p, S, xg.clone(), B.PREC_FP64, ws)  # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        h1.step(p, S, xg, B.PREC_FP64, ws)
    torch.cuda.synchronize()
    for rep in range(3):
        for c, x0 in enumerate(starts):
            xg.copy_(x0)
            g.replay()
            torch.cuda.synchronize()
            ref = x0.clone()
            h0.step(p, S, ref, B.PREC_FP64)  # eager, between the replays
            assert h0.info()["status"] == B.OK
            torch.cuda.synchronize()
            assert torch.equal(xg, ref), (rep, c, (xg - ref).abs().max().item())
            rods = torch.linalg.norm(xg[1:] - xg[:-1], dim=1)
            assert (rods - 1.0).abs().max().item() <= 1e-10
