"""Differentiable rigid-rod trajectories: a ``torch.autograd.Function`` over
``bd_step`` whose backward runs ``bd_step_adjoint`` (the hand-written
adjoints of the tension solve, the noise product, the Cholesky
factorisation and the RPY assembly, Eqs. 6-10 and the rigid limit of Eqs.
13-17) backwards through the steps, with checkpoints.

The noise is fixed by each chain's Philox key (seed, chain_id), so the
gradients are pathwise.  Every step runs in the library's kernels through
the C ABI; this module only orders the calls and keeps the checkpoints.
"""
from __future__ import annotations

import torch

from . import binding as B


def _chain_params(base: dict, chain_id: int, n_beads: int, hstar: float, kappa) -> B.Params:
    kw = dict(base)
    kw["chain_id"] = chain_id
    kw["hstar"] = hstar
    kw["kappa"] = kappa
    return B.make_params(n_beads, **kw)


def _run(handle: B.Handle, p: B.Params, x: torch.Tensor, step0: int, nsteps: int,
         keep_every: int | None = None):
    """Advances x in place by nsteps FP64 steps; returns the states at
    steps 0, keep_every, 2 keep_every, ... (before stepping) if asked."""
    kept = []
    for s in range(nsteps):
        if keep_every and s % keep_every == 0:
            kept.append(x.clone())
        handle.step(p, step0 + s, x, B.PREC_FP64)
        _status(handle, f"bd_step (step {step0 + s})")
    return kept


def _status(handle: B.Handle, where: str):
    st = handle.info()
    if st["status"] != B.OK:
        raise B.BdError(st["status"], where)


class Trajectory(torch.autograd.Function):
    """X = Trajectory.apply(X0, hstar, kappa, handle, base, chain_ids, step0,
    nsteps, every): nsteps rigid-rod FP64 steps (bd_step) of the chains X0
    (C x N x 3, float64, on the handle's device), chain c with Philox key
    (base['seed'], chain_ids[c]), all with the HI strength hstar (0-d
    tensor) and the flow kappa (3 x 3 tensor, v = kappa . r); returns the
    final positions.  Differentiable in X0, hstar and kappa.  The forward
    keeps every `every`-th state per chain; the backward recomputes each
    segment from its checkpoint and runs bd_step_adjoint over it in reverse,
    accumulating the h* and kappa gradients on the device."""

    @staticmethod
    def forward(ctx, X0, hstar, kappa, handle, base, chain_ids, step0, nsteps, every):
        hs = float(hstar.detach().cpu())
        kap = kappa.detach().cpu().double().numpy().reshape(9)
        C_, N = X0.shape[0], X0.shape[1]
        out = torch.empty_like(X0)
        ckpts = []
        for c in range(C_):
            p = _chain_params(base, int(chain_ids[c]), N, hs, kap)
            x = X0[c].detach().clone().contiguous()
            ckpts.append(_run(handle, p, x, step0, nsteps, keep_every=every))
            out[c] = x
        ctx.handle, ctx.base, ctx.chain_ids = handle, base, list(chain_ids)
        ctx.step0, ctx.nsteps, ctx.every = step0, nsteps, every
        ctx.hs, ctx.kap = hs, kap
        ctx.ckpts = ckpts
        return out

    @staticmethod
    def backward(ctx, gX):
        handle, every, nsteps = ctx.handle, ctx.every, ctx.nsteps
        C_, N = gX.shape[0], gX.shape[1]
        dev = gX.device
        hbar = torch.zeros(1, dtype=torch.float64, device=dev)
        kbar = torch.zeros(9, dtype=torch.float64, device=dev)
        gX0 = torch.empty_like(gX)
        for c in range(C_):
            p = _chain_params(ctx.base, ctx.chain_ids[c], N, ctx.hs, ctx.kap)
            xbar = gX[c].detach().clone().contiguous()
            for k in range(len(ctx.ckpts[c]) - 1, -1, -1):
                s0 = k * every
                s1 = min(s0 + every, nsteps)
                # recompute the segment's states from its checkpoint
                states = [ctx.ckpts[c][k]]
                for s in range(s0, s1 - 1):
                    x = states[-1].clone()
                    handle.step(p, ctx.step0 + s, x, B.PREC_FP64)
                    _status(handle, f"bd_step (chain {c}, step {ctx.step0 + s})")
                    states.append(x)
                for s in range(s1 - 1, s0 - 1, -1):
                    handle.step_adjoint(p, ctx.step0 + s, states[s - s0], xbar, hbar, kbar)
                    _status(handle, f"bd_step_adjoint (chain {c}, step {ctx.step0 + s})")
            gX0[c] = xbar
        return gX0, hbar[0].to(dtype=torch.float64), kbar.view(3, 3), None, None, None, None, None, None


def trajectory(X0: torch.Tensor, hstar: torch.Tensor, kappa: torch.Tensor, handle: B.Handle,
               base: dict, chain_ids, step0: int, nsteps: int, every: int = 20) -> torch.Tensor:
    """Final positions of nsteps differentiable rigid-rod steps (see
    Trajectory); ``every``: the checkpoint interval."""
    return Trajectory.apply(X0, hstar, kappa, handle, base, list(chain_ids), step0, nsteps,
                            every)
