"""Ensembles through the C ABI: many independent chains advanced by shared
launches (the chain is the third grid dimension of every kernel).

* Every chain of an ensemble step equals bd_step on that chain alone,
  bitwise: the same kernels, arithmetic and reduction orders and the same
  factorisation schedule (four-panel steps: bd_step on a handle created
  with BDRPY_WIDE_ROWS=0; two-panel steps: BDRPY_ENS_PANELS=2 against the
  default handle, n <= 4096).
* Against the oracle's step from the same state and seeds, each chain is
  within the single-chain tolerances: FP64 1e-10 b, mixed 1e-6 b, every rod
  length within 1e-10 b.
* The ensemble of uneven chains the bench times (256 chains, N from 64 to
  1024, shear at Wi = 10 on each chain's own relaxation time): every chain
  converges with exact rod lengths, and sampled chains (the smallest, the
  largest and two more) equal bd_step bitwise and the oracle within the
  same tolerances.
"""
import ctypes as C
import os

import numpy as np
import pytest
import torch

from oracle import oracle as o
from paper_2208_06559_amd import binding as B
from paper_2208_06559_amd import inputs as I

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
FLOWS = ("none", "shear", "planar", "uniaxial")
# n = 6 .. 600: less than one panel, ragged last panels, several two-panel steps
SIZES = [2, 3, 17, 45, 86, 130, 200, 43, 128]


@pytest.fixture(scope="module")
def h():
    torch.cuda.set_device(0)
    hh = B.Handle(0)
    yield hh
    hh.close()


def _chains(sizes, seed=3, dt=1e-4, wi=2.0):
    """(gpu params, oracle params, initial positions) per chain: mixed flows,
    one chain with the paper's uniform noise."""
    out = []
    for c, nb in enumerate(sizes):
        flow = FLOWS[c % len(FLOWS)]
        rate = 0.0 if flow == "none" else wi / I.relaxation_time(max(nb, 2))
        kw = dict(dt=dt, kappa=I.kappa_for(flow, rate), seed=seed, chain_id=c,
                  noise=B.NOISE_UNIFORM_PAPER if c == 5 else B.NOISE_GAUSSIAN)
        out.append((B.make_params(nb, **kw), o.make_params(nb, **kw), I.random_walk(nb, seed=seed, chain=c)))
    return out


def _packed(chains):
    return torch.tensor(np.concatenate([x for _, _, x in chains]), dtype=torch.float64, device=DEV)


def _split(xp, chains):
    out, r = [], 0
    for pg, _, _ in chains:
        out.append(xp[r:r + pg.n_beads])
        r += pg.n_beads
    return out


@pytest.fixture(scope="module")
def h_wide():
    """A handle whose single-chain factorisations take four-panel steps
    throughout (the ensembles' default schedule)."""
    old = os.environ.get("BDRPY_WIDE_ROWS")
    os.environ["BDRPY_WIDE_ROWS"] = "0"
    try:
        hh = B.Handle(0)
    finally:
        if old is None:
            del os.environ["BDRPY_WIDE_ROWS"]
        else:
            os.environ["BDRPY_WIDE_ROWS"] = old
    yield hh
    hh.close()


def _ensemble_with_panels(h, params, xp, prec, panels):
    old = os.environ.get("BDRPY_ENS_PANELS")
    os.environ["BDRPY_ENS_PANELS"] = str(panels)
    try:
        return B.Ensemble(h, params, xp, prec)
    finally:
        if old is None:
            del os.environ["BDRPY_ENS_PANELS"]
        else:
            os.environ["BDRPY_ENS_PANELS"] = old


@pytest.mark.parametrize("panels", [4, 2])
@pytest.mark.parametrize("prec", [B.PREC_FP64, B.PREC_MIXED])
def test_ensemble_equals_single_chain_bitwise(h, h_wide, prec, panels):
    chains = _chains(SIZES)
    xp = _packed(chains)
    ens = _ensemble_with_panels(h, [pg for pg, _, _ in chains], xp, prec, panels)
    hs = h_wide if panels == 4 else h
    singles = [torch.tensor(x, dtype=torch.float64, device=DEV) for _, _, x in chains]
    for s in range(3):
        ens.step(s)
        infos = ens.info()
        for c, (pg, _, _) in enumerate(chains):
            hs.step(pg, s, singles[c], prec)
            st = hs.info()
            assert st == infos[c], (s, c, st, infos[c])
            assert st["status"] == B.OK
        for c, xg in enumerate(_split(xp, chains)):
            assert torch.equal(xg, singles[c]), (prec, s, c)
    ens.close()


@pytest.mark.parametrize("prec", [B.PREC_FP64, B.PREC_MIXED])
def test_ensemble_long_chain_bitwise(h, h_wide, prec):
    """A chain of more than 1024 beads (the ensemble's matrix-free product
    then stages its beads j in two LDS rounds where the single-chain kernel
    uses one; the same summation order) and more than 4096 rows (four-panel
    steps to the end), beside short chains."""
    chains = _chains([1500, 40, 700], seed=11)
    xp = _packed(chains)
    ens = B.Ensemble(h, [pg for pg, _, _ in chains], xp, prec)
    singles = [torch.tensor(x, dtype=torch.float64, device=DEV) for _, _, x in chains]
    for s in range(2):
        ens.step(s)
        infos = ens.info()
        for c, (pg, _, _) in enumerate(chains):
            h_wide.step(pg, s, singles[c], prec)
            assert h_wide.info() == infos[c], (s, c)
    for c, xg in enumerate(_split(xp, chains)):
        assert torch.equal(xg, singles[c]), (prec, c)
    ens.close()


@pytest.mark.parametrize("sizes", [[300], [50, 50, 50, 50], [2, 2]])
def test_ensemble_edge_shapes_bitwise(h, h_wide, sizes):
    """One chain; equal sizes (ties in the size order); only two-bead
    chains (less than one panel)."""
    chains = _chains(sizes, seed=13)
    xp = _packed(chains)
    ens = B.Ensemble(h, [pg for pg, _, _ in chains], xp, B.PREC_MIXED)
    ens.step(4)
    infos = ens.info()
    for c, (xg, (pg, _, x0)) in enumerate(zip(_split(xp, chains), chains)):
        single = torch.tensor(x0, dtype=torch.float64, device=DEV)
        h_wide.step(pg, 4, single, B.PREC_MIXED)
        assert h_wide.info() == infos[c], c
        assert torch.equal(xg, single), c
    ens.close()


@pytest.mark.parametrize("prec,tol", [(B.PREC_FP64, 1e-10), (B.PREC_MIXED, 1e-6)])
def test_ensemble_vs_oracle(h, prec, tol):
    chains = _chains(SIZES, seed=7)
    xp = _packed(chains)
    ens = B.Ensemble(h, [pg for pg, _, _ in chains], xp, prec)
    ens.step(11)
    infos = ens.info()
    for c, (xg, (pg, po, x0)) in enumerate(zip(_split(xp, chains), chains)):
        xo, io = o.step(po, 11, x0)
        assert io["status"] == o.OK and infos[c]["status"] == B.OK, (c, io, infos[c])
        xn = xg.cpu().numpy()
        assert np.abs(xn - xo).max() / pg.b <= tol, (c, np.abs(xn - xo).max())
        rods = np.linalg.norm(np.diff(xn, axis=0), axis=1)
        assert np.abs(rods - pg.b).max() <= 1e-10, c
    ens.close()


def test_ensemble_argument_errors(h):
    L = B.lib()
    chains = _chains([4, 5])
    arr = (B.Params * 2)(*[pg for pg, _, _ in chains])
    nbytes = B.ensemble_workspace_size([pg for pg, _, _ in chains])
    ws = torch.empty(nbytes, dtype=torch.uint8, device=DEV)
    x = _packed(chains)
    e = C.c_void_p()
    assert L.bd_ensemble_create(h._h, 0, arr, 0, x.data_ptr(), ws.data_ptr(), nbytes, C.byref(e)) == B.ERR_PARAM
    assert L.bd_ensemble_create(h._h, 2, arr, 0, x.data_ptr(), ws.data_ptr(), nbytes - 1, C.byref(e)) == B.ERR_PARAM
    assert L.bd_ensemble_create(h._h, 2, arr, 7, x.data_ptr(), ws.data_ptr(), nbytes, C.byref(e)) == B.ERR_PARAM
    assert not e.value
    big = (B.Params * 1)(B.make_params(4098))
    out = C.c_size_t(0)
    assert L.bd_ensemble_workspace_size(1, big, 0, C.byref(out)) == B.ERR_UNSUPPORTED
    assert L.bd_ensemble_step(None, 0) == B.ERR_PARAM


W = I.ENSEMBLE_SHEAR


@pytest.mark.parametrize("prec,tol", [(B.PREC_FP64, 1e-10), (B.PREC_MIXED, 1e-6)])
def test_ensemble_full_size(h, h_wide, prec, tol):
    """Three steps of the 256-chain workload: after each, every chain's rods
    within 1e-10 b; sampled chains (the smallest, the largest and two more)
    bitwise equal to bd_step from the same state, and within the
    single-chain tolerance of the oracle's step from that state."""
    sizes = I.ensemble_sizes(W.chains, seed=W.seed)
    spec = I.ensemble_chains(W, sizes)
    pgs = [B.make_params(d["n_beads"], dt=W.dt, kappa=d["kappa"], seed=d["seed"],
                         chain_id=d["chain_id"], hstar=W.hstar, a=W.a, b=W.b) for d in spec]
    xp = torch.tensor(np.concatenate([d["x"] for d in spec]), dtype=torch.float64, device=DEV)
    ens = B.Ensemble(h, pgs, xp, prec)
    xs = _split(xp, [(p, None, None) for p in pgs])
    order = np.argsort(sizes, kind="stable")
    sampled = sorted({int(order[0]), int(order[-1]), 17, 200})
    worst = 0.0
    for s in range(3):
        before = {c: xs[c].cpu().numpy().copy() for c in sampled}
        ens.step(s)
        infos = ens.info()
        assert all(i["status"] == B.OK for i in infos), s
        for c in range(len(spec)):
            rods = torch.linalg.norm(xs[c][1:] - xs[c][:-1], dim=1)
            assert (rods - W.b).abs().max().item() <= 1e-10, (s, c)
        for c in sampled:
            d = spec[c]
            single = torch.tensor(before[c], dtype=torch.float64, device=DEV)
            h_wide.step(pgs[c], s, single, prec)
            assert h_wide.info() == infos[c], (s, c)
            assert torch.equal(single, xs[c]), (s, c)
            po = o.make_params(d["n_beads"], dt=W.dt, kappa=d["kappa"], seed=d["seed"],
                               chain_id=d["chain_id"], hstar=W.hstar, a=W.a, b=W.b)
            xo, io = o.step(po, s, before[c])
            assert io["status"] == o.OK
            err = np.abs(xs[c].cpu().numpy() - xo).max() / W.b
            assert err <= tol, (s, c, err)
            worst = max(worst, err)
    print(f"ensemble prec {prec}: 3 steps, sampled chains {sampled}, worst |dr|/b vs oracle "
          f"{worst:.3e}", flush=True)
    ens.close()


@pytest.mark.parametrize("prec", [B.PREC_FP64, B.PREC_MIXED])
def test_captured_ensemble_step_replays_bitwise(h, prec):
    # one step captured in a HIP graph (bd_ensemble_capture), replayed step
    # after step, against a second plan of the same chains stepping with
    # plain launches in between; a jump of the step counter resets the
    # device counter
    chains = _chains(SIZES)
    xa, xb = _packed(chains), _packed(chains)
    params = [pg for pg, _, _ in chains]
    plain = B.Ensemble(h, params, xa, prec)
    graph = B.Ensemble(h, params, xb, prec)
    plain.step(0)
    graph.step(0)  # a plain step first: its product count sizes the budget
    graph.capture()
    for s in (1, 2, 3, 7, 8):
        plain.step(s)
        graph.step(s)
        ia, ib = plain.info(), graph.info()
        assert all(i["status"] == B.OK for i in ib), (s, ib)
        assert ia == ib, s
        assert torch.equal(xa, xb), (prec, s, (xa - xb).abs().max().item())
    plain.close()
    graph.close()
