"""Autotuner of the factorisation schedule on this GPU.

The blocked Cholesky (Eq. 10) updates the trailing matrix by one, two or
four 128-column panels per pass; four panels divide the HBM traffic of the
trailing matrix per flop but lengthen the chain of diagonal blocks and
panel solves that the update cannot hide, so the best width depends on the
matrix order, the precision and the GPU.  This script times the library's
factorisation (bd_cholesky, HIP events) for every candidate schedule at a
ladder of matrix orders and both precisions, and the 256-chain ensemble
step for both ensemble step widths, and writes the fastest choices with
every timing to tuning.json beside it.  Handle(tuned=True) and bench.py
apply that table through bd_set_schedules / bd_set_ensemble_panels.

Run on the GPU:  python -m paper_2208_06559_amd.tune  [--out PATH]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
if os.path.dirname(HERE) not in sys.path:
    sys.path.insert(0, os.path.dirname(HERE))

from paper_2208_06559_amd import binding as B  # noqa: E402
from paper_2208_06559_amd import inputs as I  # noqa: E402

SIZES = [768, 1536, 3072, 6144, 12288, 19200]
PRECS = {"fp64": B.PREC_FP64, "mixed": B.PREC_MIXED}
BIG = 1 << 62


def candidates(n: int):
    """(step_panels, wide_rows): one or two panels throughout, or four while
    more than wide_rows rows remain."""
    out = [(1, 0), (2, 0)]
    for w in (0, 2048, 4096, 8192):
        if w < n:
            out.append((4, w))
    return out


def time_cholesky(h, n: int, prec: int, D0: torch.Tensor, reps: int) -> float:
    A = torch.empty_like(D0)
    ws = h.workspace(B.OP_CHOLESKY, n, prec)
    A.copy_(D0)
    h.cholesky(A, n, n, prec, ws)  # warm-up
    times = []
    for _ in range(reps):
        A.copy_(D0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        h.cholesky(A, n, n, prec, ws)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    if h.info()["status"] != B.OK:
        raise RuntimeError(f"factorisation failed at n = {n}")
    return float(np.median(times))


def tune_cholesky(h, log):
    table, rows = {}, []
    for i, n in enumerate(SIZES):
        N = n // 3
        p = B.make_params(N)
        x = torch.tensor(I.random_walk(N, seed=4), dtype=torch.float64, device="cuda:0")
        D0 = torch.empty((n, n), dtype=torch.float64, device="cuda:0")
        h.rpy_assemble(p, x, D0, n, B.FILL_LOWER)
        reps = 5 if n <= 6144 else 3
        n_max = int(math.sqrt(n * SIZES[i + 1])) if i + 1 < len(SIZES) else BIG
        for name, prec in PRECS.items():
            res = {}
            for sp, wr in candidates(n):
                h.set_schedules([dict(n_max=BIG, prec=prec, step_panels=sp, wide_rows=wr)])
                res[f"{sp}x{wr}"] = time_cholesky(h, n, prec, D0, reps)
            best = min(res, key=res.get)
            sp, wr = (int(v) for v in best.split("x"))
            table.setdefault(name, {})[str(n)] = {"ms": res, "best": best}
            rows.append(dict(n_max=n_max, prec=prec, step_panels=sp,
                             wide_rows=wr if wr > 0 else 0))
            log(f"n = {n} {name}: " + ", ".join(f"{k} {v:.3f} ms" for k, v in res.items())
                + f" -> {best}")
        del D0
        torch.cuda.empty_cache()
    h.set_schedules([])
    return table, rows


def tune_ensemble(h, rows, log, steps: int = 6):
    w = I.ENSEMBLE_SHEAR
    sizes = I.ensemble_sizes(w.chains, seed=w.seed)
    spec = I.ensemble_chains(w, sizes)
    pgs = [B.make_params(d["n_beads"], dt=w.dt, kappa=d["kappa"], seed=d["seed"],
                         chain_id=d["chain_id"], hstar=w.hstar, a=w.a, b=w.b) for d in spec]
    x0 = torch.tensor(np.concatenate([d["x"] for d in spec]), dtype=torch.float64,
                      device="cuda:0")
    out, choice = {}, {}
    for name, prec in PRECS.items():
        res = {}
        for panels in (2, 4):
            h.set_ensemble_panels(prec, panels)
            xp = x0.clone()
            ens = B.Ensemble(h, pgs, xp, prec)
            for s in range(2):
                ens.step(s)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for s in range(steps):
                ens.step(2 + s)
            torch.cuda.synchronize()
            res[str(panels)] = 1e3 * (time.perf_counter() - t0) / steps
            if any(i["status"] != B.OK for i in ens.info()):
                raise RuntimeError("ensemble step failed")
            ens.close()
        best = min(res, key=res.get)
        out[name] = {"ms_per_step": res, "best": int(best)}
        choice[name] = int(best)
        log(f"ensemble {name}: " + ", ".join(f"{k} panels {v:.3f} ms" for k, v in res.items())
            + f" -> {best}")
    h.set_ensemble_panels(B.PREC_FP64, 0)
    h.set_ensemble_panels(B.PREC_MIXED, 0)
    return out, choice


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=B.TUNING_PATH)
    args = ap.parse_args()

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    h = B.Handle(0)
    chol, rows = tune_cholesky(h, log)
    ens, choice = tune_ensemble(h, rows, log)
    rec = {"gpu": torch.cuda.get_device_name(0),
           "command": "python -m paper_2208_06559_amd.tune",
           "sizes": SIZES,
           "cholesky_ms": chol,
           "schedules": rows,
           "ensemble": ens,
           "ensemble_panels": choice}
    with open(args.out, "w") as f:
        json.dump(rec, f, indent=1)
    h.close()
    print(json.dumps({"schedules": rows, "ensemble_panels": choice}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
