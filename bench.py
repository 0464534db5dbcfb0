#!/usr/bin/env python3
"""Benchmark of the bead-rod BD + RPY hot path on one MI355X.

Workload: one chain of N = 4096 beads (3N = 12288), b = 1, h* = 0.25,
a = 0.5, uniaxial extension at Wi = 5, dt = 5e-5, seeded random-walk start
(synthetic; the paper uses no dataset).  A step is one full pass of the hot
path: RPY assembly, Cholesky, correlated noise, predictor and rod-tension
solve.  Reports BD steps/s for the mixed-precision form (headline) and for
FP64, the Cholesky TFLOP/s of both, the roofline of the dominant kernel and
the CPU oracle on a bounded sample.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6   # TFLOP/s, MI355X dense FP64 (vector = matrix)
PEAK_FP32 = 157.3  # TFLOP/s, MI355X dense FP32 matrix
PEAK_HBM = 8000.0  # GB/s
METRIC = "BD steps/s + Cholesky TFLOP/s at 3N=12288, mixed vs FP64 on 1 MI355X"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def chol_flops(n: int) -> float:
    return n**3 / 3.0 + n**2 / 2.0 + n / 6.0


def step_width(n: int, k0: int, nb: int, max_panels: int, wide_rows: int) -> int:
    """Columns of the factorisation step starting at column k0: up to
    max_panels panels while more than wide_rows rows remain, two after."""
    panels = max_panels if n - k0 > wide_rows else min(max_panels, 2)
    return min(panels * nb, n - k0)


def syrk_launches(n: int, nb: int = 128, max_panels: int = 4, wide_rows: int = 4096,
                  lookahead: bool = True) -> list[tuple]:
    """Every trailing-update launch of one factorisation in the library's
    schedule (steps of up to `max_panels` panels, see step_width, with
    lookahead): per launch (flops, lower elements updated, operand rows,
    kdim, kind) with flops = 2 per multiply-add over the lower elements of
    the tiles it updates; kind "next" for the columns of the next step (the
    lookahead chain, kernel syrk_next_*), "bulk" for the rest (kernel
    syrk_update_*)."""
    out = []

    def trailing(r0, kdim, tiles, nnext):
        m = n - r0
        mt = -(-m // nb)
        nnext = min(nnext, mt)
        if tiles == "next":
            nt = sum(mt - q for q in range(nnext))
            elems = 0
            for q in range(nnext):
                wq = min(nb, m - nb * q)
                elems += (m - nb * q) * wq - wq * (wq - 1) // 2
            rows = m
        elif tiles == "rest":
            nt = (mt - nnext) * (mt - nnext + 1) // 2
            m2 = m - nb * nnext
            elems, rows = m2 * (m2 + 1) // 2, m2
        else:
            nt = mt * (mt + 1) // 2
            elems, rows = m * (m + 1) // 2, m
        if nt > 0:
            out.append((2.0 * elems * kdim, float(elems), rows, kdim,
                        "next" if tiles == "next" else "bulk"))

    def width(k0):
        return step_width(n, k0, nb, max_panels, wide_rows)

    def factor_step(k0):
        kp, end = k0, k0 + width(k0)
        while kp < end:
            if kp > k0:
                trailing(kp, kp - k0, "next", 1)
            kp += nb
        return end - k0

    if not lookahead:
        k = 0
        while k < n:
            w = factor_step(k)
            if k + w < n:
                trailing(k + w, w, "all", 0)
            k += w
        return out
    w, k = factor_step(0), 0
    while k + w < n:
        r0 = k + w
        nnext = -(-width(r0) // nb)
        trailing(r0, w, "next", nnext)
        wn = factor_step(r0)
        trailing(r0, w, "rest", nnext)
        k, w = r0, wn
    return out


def schedule_in_use(tuning: dict | None, n: int, prec: int) -> tuple[int, int]:
    """(step panels, wide rows) that the library applies to an order-n
    factorisation: the first row of the handle's schedule table with this
    precision and n <= n_max, else the handle's defaults (environment)."""
    for r in (tuning or {}).get("schedules", []):
        if r["prec"] == prec and n <= r["n_max"]:
            return int(r["step_panels"]), int(r["wide_rows"])
    sp = os.environ.get("BDRPY_STEP_PANELS", "")
    mp = 1 if sp.startswith("1") else 2 if sp.startswith("2") else 4
    return mp, int(os.environ.get("BDRPY_WIDE_ROWS", "4096"))


def syrk_per_launch(n: int, esize: int, kind: str = "bulk",
                    schedule: tuple[int, int] | None = None) -> tuple[float, float, int]:
    """Average algorithmic flops and HBM bytes per trailing-update launch of
    one kind, and the launch count, of one factorisation in the schedule
    (step panels, wide rows).  Bytes: each updated lower element of C read
    and written once in FP64 (16 B) plus each operand row of L read once
    (kdim values of `esize` bytes)."""
    mp, wide = schedule if schedule is not None else schedule_in_use(None, n, -1)
    la = not os.environ.get("BDRPY_LOOKAHEAD", "").startswith("0")
    ls = [x for x in syrk_launches(n, max_panels=mp, wide_rows=wide, lookahead=la)
          if x[4] == kind]
    fl = sum(x[0] for x in ls)
    by = sum(16.0 * x[1] + x[2] * x[3] * esize for x in ls)
    return fl / len(ls), by / len(ls), len(ls)


COPY_PROBE_BYTES = 1 << 30
PROFILES = os.path.join(ROOT, "profiles")
MFMA_RECORD = os.path.join(PROFILES, "cholesky_mfma_counters_n12288.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2208_06559_amd", "csrc", "cholesky.hip")


def copy_probe(torch) -> int:
    """Three device-to-device copies of COPY_PROBE_BYTES each: every copy
    reads and writes that many bytes of HBM exactly once."""
    src = torch.ones(COPY_PROBE_BYTES // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": COPY_PROBE_BYTES, "copies": 3}), flush=True)
    return 0


def _records(prefix: str, paths):
    """The JSON records after `prefix` in the committed summaries whose
    kernel source still has the hash they were measured with."""
    import hashlib
    try:
        with open(KERNEL_SOURCE, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return []
    out = []
    for path in paths:
        try:
            with open(path) as f:
                for line in f:
                    if line.startswith(prefix):
                        rec = json.loads(line[len(prefix):])
                        if rec.get("source_sha256") == sha:
                            out.append(rec)
        except (OSError, ValueError):
            continue
    return out


def measured_traffic(kernel: str, schedule: tuple[int, int]):
    """HBM bytes per launch of `kernel` from the committed counter summaries
    (profiles/*_traffic.md), or None when there is none, the kernel source
    changed since or it was measured under another factorisation schedule
    (step panels, wide rows): the average launch depends on it."""
    import glob
    for rec in _records("traffic_record: ", sorted(glob.glob(os.path.join(PROFILES, "*_traffic.md")))):
        if rec.get("kernel") == kernel and rec.get("schedule") == list(schedule):
            return float(rec["hbm_bytes_per_launch"])
    return None


def measured_mfma(kernel: str, schedule: tuple[int, int]):
    """Matrix-core counters of `kernel` (syrk_update_f32 / _f64) from the
    committed summary, or None (as for measured_traffic)."""
    name = {"syrk_update_f32": "syrk_update_kernel<float, 128, true>",
            "syrk_update_f64": "syrk_update_kernel<double, 128, true>"}.get(kernel)
    prec = "mixed" if kernel.endswith("f32") else "fp64"
    for rec in _records("mfma_record: ", [MFMA_RECORD]):
        k = rec.get("kernels", {}).get(name)
        if k and rec.get("schedules", {}).get(prec) == list(schedule):
            return {"mfma_busy_frac": k["mfma_busy_frac"],
                    "mfma_flops_per_dispatch": k["mfma_flops_per_dispatch"],
                    "source": "profiles/cholesky_mfma_counters_n12288.md"}
    return None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def error_series(B, torch, np, h, p, x0, n, w, args) -> dict:
    """Mixed-precision error along the workload's trajectory: the mixed and
    FP64 steps run side by side from the same start and noise for
    `series_steps` steps; after every step the largest bead-position
    difference in units of b, and every `series_every` steps (and at the
    start) the relative residual ||B B^T - D||_F / ||D||_F of the mixed
    factor of D at the mixed trajectory's configuration, the product formed
    by an FP64 GEMM (validation only)."""
    xm, xd = x0.clone(), x0.clone()
    wsm = h.workspace(B.OP_STEP, n, B.PREC_MIXED)
    wsd = h.workspace(B.OP_STEP, n, B.PREC_FP64)
    wsc = h.workspace(B.OP_CHOLESKY, n, B.PREC_MIXED)
    D = torch.empty((n, n), dtype=torch.float64, device=x0.device)
    pos, res_steps, res = [], [], []

    def residual(x):
        h.rpy_assemble(p, x, D, n, B.FILL_FULL)
        Dm = B.matrix_view(D, n).clone()
        h.cholesky(D, n, n, B.PREC_MIXED, wsc)
        if h.info()["status"] != B.OK:
            raise RuntimeError("series: mixed factorisation failed")
        L = torch.tril(B.matrix_view(D, n))
        r = (torch.linalg.norm(L @ L.T - Dm) / torch.linalg.norm(Dm)).item()
        del L, Dm
        return r

    for s in range(args.series_steps):
        if s % args.series_every == 0:
            res_steps.append(s)
            res.append(residual(xm))
        h.step(p, s, xm, B.PREC_MIXED, wsm)
        h.step(p, s, xd, B.PREC_FP64, wsd)
        st = h.info()
        if st["status"] != B.OK:
            raise RuntimeError(f"series step {s}: {st}")
        pos.append(((xm - xd).abs().max() / w.b).item())
    res_steps.append(args.series_steps)
    res.append(residual(xm))
    del D
    torch.cuda.empty_cache()
    out = {"steps": args.series_steps, "position_error_per_step": pos,
           "position_error_max": max(pos), "residual_steps": res_steps,
           "residual_mixed": res, "residual_mixed_max": max(res)}
    log(f"series: position error max {out['position_error_max']:.3e} b, "
        f"residual max {out['residual_mixed_max']:.3e}")
    return out


def ensemble_leg(B, I, torch, np, precs, args, dev) -> dict:
    """The uneven ensemble (256 chains, N from 64 to 1024, shear at Wi = 10
    on each chain's relaxation time) advanced by bd_ensemble_step: ensemble
    steps per second and chain steps per second, plus the Cholesky-equivalent
    rate sum_c n_c^3/3 flop per step / step time (a lower bound on what the
    factorisations alone reach, since the step time includes everything)."""
    w = I.ENSEMBLE_SHEAR
    sizes = I.ensemble_sizes(w.chains, seed=w.seed)
    spec = I.ensemble_chains(w, sizes)
    pgs = [B.make_params(d["n_beads"], dt=w.dt, kappa=d["kappa"], seed=d["seed"],
                         chain_id=d["chain_id"], hstar=w.hstar, a=w.a, b=w.b) for d in spec]
    x0 = torch.tensor(np.concatenate([d["x"] for d in spec]), dtype=torch.float64, device=dev)
    flops = float(sum(chol_flops(3 * int(v)) for v in sizes))
    out = {"workload": w.name, "chains": int(w.chains), "n_beads_min": int(sizes.min()),
           "n_beads_max": int(sizes.max()), "sum_n3_over_3": flops}
    h = B.Handle(0, tuned=True)
    warm = 2
    for name, prec in precs.items():
        xp = x0.clone()
        ens = B.Ensemble(h, pgs, xp, prec)
        for s in range(warm):
            ens.step(s)
        infos = ens.info()
        if any(i["status"] != B.OK for i in infos):
            raise RuntimeError(f"ensemble {name} warmup failed")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(args.ensemble_steps):
            ens.step(warm + s)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        infos = ens.info()
        if any(i["status"] != B.OK for i in infos):
            raise RuntimeError(f"ensemble {name} timed steps failed")
        h.profile_begin()
        ens.step(warm + args.ensemble_steps)
        prof = h.profile_end()
        # the same steps replayed from a captured HIP graph
        ens.capture()
        s0 = warm + args.ensemble_steps + 1
        ens.step(s0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(args.ensemble_steps):
            ens.step(s0 + 1 + s)
        torch.cuda.synchronize()
        gwall = time.perf_counter() - t0
        ginfos = ens.info()
        if any(i["status"] != B.OK for i in ginfos):
            raise RuntimeError(f"ensemble {name} captured steps failed")
        ms = 1e3 * wall / args.ensemble_steps
        chol = {k: v for k, v in prof.items()
                if k.startswith(("potrf", "panel_solve", "syrk"))}
        out[name] = {
            "ensemble_steps_per_s": args.ensemble_steps / wall,
            "chain_steps_per_s": w.chains * args.ensemble_steps / wall,
            "ms_per_step": ms,
            "cholesky_equiv_tflops": flops / (ms * 1e-3) / 1e12,
            "kernel_ms_per_step": {k: v[1] for k, v in sorted(prof.items(), key=lambda kv: -kv[1][1])},
            "kernel_launches_per_step": {k: v[0] for k, v in prof.items()},
            "cholesky_kernels_ms_per_step": sum(v[1] for v in chol.values()),
            "max_newton_iters": max(i["newton_iters"] for i in infos),
            "max_rod_err": max(i["max_rod_err"] for i in infos),
            "graph_ensemble_steps_per_s": args.ensemble_steps / gwall,
            "graph_ms_per_step": 1e3 * gwall / args.ensemble_steps,
        }
        log(f"ensemble {name}: {out[name]['ensemble_steps_per_s']:.2f} steps/s "
            f"({ms:.3f} ms/step, {out[name]['chain_steps_per_s']:.0f} chain-steps/s); "
            f"captured graph {out[name]['graph_ms_per_step']:.3f} ms/step")
        ens.close()
        del ens, xp
        torch.cuda.empty_cache()
    h.close()
    if not args.no_cpu:
        # the oracle on every 8th chain by size (32 chains), scaled to the
        # whole ensemble by sum n^3 (the factorisation dominates its time)
        from oracle import oracle as o
        order = np.argsort(sizes, kind="stable")[::8]
        t_sample, n3_sample = 0.0, 0.0
        for c in order:
            d = spec[int(c)]
            po = o.make_params(d["n_beads"], dt=w.dt, kappa=d["kappa"], seed=d["seed"],
                               chain_id=d["chain_id"], hstar=w.hstar, a=w.a, b=w.b)
            t0 = time.perf_counter()
            o.step(po, 0, d["x"])
            t_sample += time.perf_counter() - t0
            n3_sample += float(3 * d["n_beads"]) ** 3
        n3_all = float(sum(float(3 * int(v)) ** 3 for v in sizes))
        est = t_sample * n3_all / n3_sample
        out["cpu_baseline"] = {"value": 1.0 / est, "unit": "ensemble steps/s",
                               "chain_steps_per_s": w.chains / est, "cores": o.num_threads(),
                               "kind": "oracle",
                               "sample": f"1 oracle FP64 step of {len(order)} chains (every 8th "
                                         f"by size), {t_sample:.2f} s, scaled by sum n^3 "
                                         f"({n3_all / n3_sample:.2f}x) to the {w.chains} chains"}
        log(f"ensemble cpu oracle: {out['cpu_baseline']}")
    return out


def fraenkel_leg(B, torch, h, p, x0, n, w, precs, args) -> dict:
    """bd_step_fraenkel (stiff springs, K = 1e4) on the single-chain workload."""
    K = 1e4
    fraenkel = {"k_spring": K, "workload": w.name}
    for name, prec in precs.items():
        ws = h.workspace(B.OP_STEP, n, prec)
        xx = x0.clone()
        for s in range(3):
            h.step_fraenkel(p, K, s, xx, prec, ws)
        if h.info()["status"] != B.OK:
            raise RuntimeError(f"fraenkel {name} warmup failed")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(args.fraenkel_steps):
            h.step_fraenkel(p, K, 3 + s, xx, prec, ws)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = h.info()
        if st["status"] != B.OK:
            raise RuntimeError(f"fraenkel {name} timed steps failed")
        fraenkel[name] = {"steps_per_s": args.fraenkel_steps / wall,
                          "ms_per_step": 1e3 * wall / args.fraenkel_steps,
                          "max_spring_extension_last": st["max_rod_err"]}
        log(f"fraenkel {name}: {fraenkel[name]['steps_per_s']:.2f} steps/s")
    return fraenkel


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--chol-reps", type=int, default=10)
    ap.add_argument("--profile-steps", type=int, default=5)
    ap.add_argument("--cpu-beads", type=int, default=4096,
                    help="chain length of the CPU oracle sample (scaled to N=4096 by n^3)")
    ap.add_argument("--cpu-beads-single", type=int, default=1024,
                    help="chain length of the single-thread oracle sample (scaled by n^3)")
    ap.add_argument("--series-steps", type=int, default=200,
                    help="steps of the mixed-vs-FP64 error series (0: skip it)")
    ap.add_argument("--series-every", type=int, default=20,
                    help="residual of the mixed factor every this many steps of the series")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--ensemble-steps", type=int, default=20,
                    help="timed steps of the 256-chain ensemble leg (0: skip it)")
    ap.add_argument("--fraenkel-steps", type=int, default=50,
                    help="timed steps of the stiff-spring leg at N = 4096 (0: skip it)")
    ap.add_argument("--fraenkel-only", action="store_true",
                    help="run only the stiff-spring leg and print its record")
    ap.add_argument("--ensemble-only", action="store_true",
                    help="run only the ensemble leg and print its record")
    ap.add_argument("--only", choices=["all", "mixed", "fp64"], default="all",
                    help="restrict the timed steps to one precision (for profiler runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of known size (calibrates the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs one chain on one GPU; --gpus must be 1 "
              "(independent chains shard across GPUs with no communication)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    if args.copy_probe:
        return copy_probe(torch)

    from paper_2208_06559_amd import binding as B
    from paper_2208_06559_amd import inputs as I

    w = I.LONG_UNIAXIAL
    N, n = w.n_beads, w.n
    dev = "cuda:0"
    torch.cuda.set_device(0)
    kw = dict(dt=w.dt, kappa=w.kappa, seed=w.seed, hstar=w.hstar, a=w.a, b=w.b)
    p = B.make_params(N, **kw)
    x0_np = w.initial()
    x0 = torch.tensor(x0_np, dtype=torch.float64, device=dev)
    h = B.Handle(0, tuned=True)  # the autotuner's schedules, if tuning.json exists
    precs = {"mixed": B.PREC_MIXED, "fp64": B.PREC_FP64}
    if args.only != "all":
        precs = {args.only: precs[args.only]}

    if args.ensemble_only:
        print(json.dumps({"ensemble": ensemble_leg(B, I, torch, np, precs, args, dev)}), flush=True)
        h.close()
        return 0
    if args.fraenkel_only:
        print(json.dumps({"fraenkel": fraenkel_leg(B, torch, h, p, x0, n, w, precs, args)}),
              flush=True)
        h.close()
        return 0

    # ---------------------------------------------------------- step rate
    result = {}
    finals = {}
    for name, prec in precs.items():
        ws = h.workspace(B.OP_STEP, n, prec)
        x = x0.clone()
        for s in range(args.warmup):
            h.step(p, s, x, prec, ws)
        info = h.info()
        if info["status"] != B.OK:
            raise RuntimeError(f"{name} warmup failed: {info}")
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record()
        for s in range(args.steps):
            h.step(p, args.warmup + s, x, prec, ws)
        ev1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        gpu_ms = ev0.elapsed_time(ev1)
        info = h.info()
        if info["status"] != B.OK:
            raise RuntimeError(f"{name} timed steps failed: {info}")
        xf = x.cpu().numpy()
        rods = np.linalg.norm(np.diff(xf, axis=0), axis=1)
        ms = 1e3 * wall / args.steps
        result[name] = {
            "steps_per_s": args.steps / wall,
            "ms_per_step": ms,
            "gpu_event_ms_per_step": gpu_ms / args.steps,
            "newton_iters_last": info["newton_iters"],
            "krylov_iters_last": info["krylov_iters"],
            "max_rod_err_final": float(np.abs(rods - w.b).max()),
        }
        finals[name] = xf
        log(f"{name}: {result[name]['steps_per_s']:.2f} steps/s ({ms:.3f} ms/step)")

    # ------------------------------------------------ Cholesky TFLOP/s
    ld = n
    D = torch.empty((n, ld), dtype=torch.float64, device=dev)
    for name, prec in precs.items():
        ws = h.workspace(B.OP_CHOLESKY, n, prec)
        times = []
        for r in range(args.chol_reps):
            h.rpy_assemble(p, x0, D, ld, B.FILL_LOWER)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            h.cholesky(D, n, ld, prec, ws)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        if h.info()["status"] != B.OK:
            raise RuntimeError(f"{name} cholesky failed")
        med = float(np.median(times))
        tf = chol_flops(n) / (med * 1e-3) / 1e12
        peak = PEAK_FP32 if prec == B.PREC_MIXED else PEAK_FP64
        result[name].update({"cholesky_ms": med, "cholesky_tflops": tf,
                             "cholesky_frac_of_peak": tf / peak, "peak_tflops": peak})
        log(f"{name}: cholesky {med:.3f} ms = {tf:.2f} TFLOP/s ({100 * tf / peak:.1f}% of {peak})")

    # ------------------------------------ residual and position error
    extra = {}
    Dfull = torch.empty((n, ld), dtype=torch.float64, device=dev)
    h.rpy_assemble(p, x0, Dfull, ld, B.FILL_FULL)
    Dm = B.matrix_view(Dfull, n)
    dn = torch.linalg.norm(Dm).item()
    for name, prec in precs.items():
        A = Dfull.clone()
        h.cholesky(A, n, ld, prec, h.workspace(B.OP_CHOLESKY, n, prec))
        L = torch.tril(B.matrix_view(A, n))
        res = torch.linalg.norm(L @ L.T - Dm).item() / dn
        result[name]["residual_LLT_minus_D_over_D"] = res
        del A, L
        torch.cuda.empty_cache()
    if len(precs) == 2:
        xs = {}
        for name, prec in precs.items():
            xx = x0.clone()
            h.step(p, 0, xx, prec, h.workspace(B.OP_STEP, n, prec))
            xs[name] = xx.cpu().numpy()
        extra["position_error_1step"] = float(np.abs(xs["mixed"] - xs["fp64"]).max() / w.b)
        extra["position_error_after_run"] = float(
            np.abs(finals["mixed"] - finals["fp64"]).max() / w.b)
    del Dfull, Dm, D
    torch.cuda.empty_cache()

    # ------------------------------------------- dominant-kernel roofline
    def isolated_bulk(kern, pr, sched, f32):
        """The same kernel with the lookahead stream off (every launch of
        the factorisation in order on one stream, nothing beside it): its
        average launch time over one step's factorisation, and the fraction
        of peak that gives, beside the in-stream figure above (where the
        diagonal blocks and panel solves of the next step share the GPU)."""
        old = os.environ.get("BDRPY_LOOKAHEAD")
        os.environ["BDRPY_LOOKAHEAD"] = "0"
        try:
            hs = B.Handle(0, tuned=True)
        finally:
            if old is None:
                del os.environ["BDRPY_LOOKAHEAD"]
            else:
                os.environ["BDRPY_LOOKAHEAD"] = old
        try:
            xx = x0.clone()
            wsp = hs.workspace(B.OP_STEP, n, pr)
            hs.step(p, 0, xx, pr, wsp)
            torch.cuda.synchronize()
            hs.profile_begin()
            hs.step(p, 1, xx, pr, wsp)
            st = hs.profile_end()
            if hs.info()["status"] != B.OK or kern not in st:
                return None
            launches, kms = st[kern]
            ls = [x for x in syrk_launches(n, max_panels=sched[0], wide_rows=sched[1],
                                           lookahead=False) if x[4] == "bulk"]
            if launches != len(ls):
                return None
            fl = sum(x[0] for x in ls) / launches
            peak_fl = PEAK_FP32 if f32 else PEAK_FP64
            avg_s = kms * 1e-3 / launches
            return {"avg_launch_ms": kms / launches, "launches": launches,
                    "achieved": fl / avg_s / 1e12, "frac": fl / avg_s / 1e12 / peak_fl,
                    "note": "lookahead off: the kernel alone on the GPU"}
        finally:
            hs.close()

    def profile(prec_name):
        pr = precs[prec_name]
        xx = x0.clone()
        wsp = h.workspace(B.OP_STEP, n, pr)
        h.step(p, 0, xx, pr, wsp)
        torch.cuda.synchronize()
        h.profile_begin()
        for s in range(args.profile_steps):
            h.step(p, 1 + s, xx, pr, wsp)
        stats = h.profile_end()
        tot = sum(v[1] for v in stats.values())
        kern = max(stats, key=lambda k: stats[k][1])
        launches, kms = stats[kern]
        brk = {k: {"launches_per_step": v[0] / args.profile_steps,
                   "ms_per_step": v[1] / args.profile_steps,
                   "share": v[1] / tot}
               for k, v in sorted(stats.items(), key=lambda kv: -kv[1][1])}
        if "rpy_assemble" in brk:
            # the assembly writes the lower triangle once: n(n+1)/2 doubles
            ab = brk["rpy_assemble"]
            a_s = ab["ms_per_step"] / ab["launches_per_step"] * 1e-3
            a_by = n * (n + 1) / 2 * 8
            ab["hbm"] = {"bytes_per_launch": a_by, "achieved_GBps": a_by / a_s / 1e9,
                         "peak_GBps": PEAK_HBM, "frac": a_by / a_s / 1e9 / PEAK_HBM}
        if kern.startswith("syrk_update"):
            f32 = kern.endswith("f32")
            sched = schedule_in_use(h.tuning, n, pr)
            fl, by, cnt = syrk_per_launch(n, 4 if f32 else 8, schedule=sched)
            assert launches == cnt * args.profile_steps, (launches, cnt, sched)
            avg_s = kms * 1e-3 / launches
            peak_fl = PEAK_FP32 if f32 else PEAK_FP64
            # roofline: HBM-bound when the intensity is below the ridge point
            if fl / by < peak_fl * 1e12 / (PEAK_HBM * 1e9):
                achieved, peak, unit, bound = by / avg_s / 1e9, PEAK_HBM, "GB/s", "hbm"
            else:
                achieved, peak, unit, bound = fl / avg_s / 1e12, peak_fl, "TFLOP/s", "mfma"
            rf = {"bound": bound, "kernel": kern, "achieved": achieved, "peak": peak,
                  "unit": unit, "frac": achieved / peak,
                  "isolated": isolated_bulk(kern, pr, sched, f32),
                  "traffic": measured_traffic(kern, sched),
                  "mfma_counters": measured_mfma(kern, sched),
                  "schedule": {"step_panels": sched[0], "wide_rows": sched[1]},
                  "cholesky_frac_of_peak": result[prec_name].get("cholesky_frac_of_peak"),
                  "algorithmic_flops_per_launch": fl, "algorithmic_bytes_per_launch": by,
                  "intensity_flop_per_byte": fl / by,
                  "tflops_per_launch_avg": fl / avg_s / 1e12,
                  "avg_launch_ms": kms / launches, "launches": launches}
        else:
            rf = {"bound": "latency", "kernel": kern, "achieved": None, "peak": None,
                  "unit": None, "frac": None, "traffic": None,
                  "avg_launch_ms": kms / launches, "launches": launches}
        log(f"{prec_name}: dominant kernel {kern}: {rf}")
        return rf, brk

    head = "mixed" if "mixed" in precs else next(iter(precs))
    roof, breakdown = profile(head)
    other = {}
    for name in precs:
        if name != head:
            other[name] = dict(zip(("roofline", "kernel_breakdown"), profile(name)))

    # ------------------------------------------------ library context
    try:
        Dt = torch.empty((n, n), dtype=torch.float64, device=dev)
        Dbuf = torch.empty((n, ld), dtype=torch.float64, device=dev)
        h.rpy_assemble(p, x0, Dbuf, ld, B.FILL_FULL)
        Dt.copy_(B.matrix_view(Dbuf, n))
        del Dbuf
        torch.linalg.cholesky(Dt)
        torch.cuda.synchronize()
        tt = []
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            torch.linalg.cholesky(Dt)
            e1.record()
            torch.cuda.synchronize()
            tt.append(e0.elapsed_time(e1))
        lib_ms = float(np.median(tt))
        extra["torch_linalg_cholesky_fp64"] = {"ms": lib_ms,
                                               "tflops": chol_flops(n) / (lib_ms * 1e-3) / 1e12}
        del Dt
        torch.cuda.empty_cache()
    except Exception as e:  # context only
        extra["torch_linalg_cholesky_fp64"] = {"error": str(e)[:200]}

    # ------------------------------------------------ CPU oracle sample
    cpu = None
    if not args.no_cpu:
        from oracle import oracle as o
        Ns = min(args.cpu_beads, N)
        po = o.make_params(Ns, **kw)
        xs0 = x0_np[:Ns].copy()
        t0 = time.perf_counter()
        _, io = o.step(po, 0, xs0)
        dt_s = time.perf_counter() - t0
        scale = (Ns / N) ** 3
        threads = o.num_threads()
        # one thread, on a shorter piece of the same chain (the unblocked
        # factorisation, n^3/3 flop, dominates the oracle's step)
        N1 = min(args.cpu_beads_single, N)
        o.set_num_threads(1)
        t0 = time.perf_counter()
        _, io1 = o.step(o.make_params(N1, **kw), 0, x0_np[:N1].copy())
        dt_1 = time.perf_counter() - t0
        o.set_num_threads(threads)
        s1 = (N1 / N) ** 3
        cpu = {"value": scale / dt_s, "unit": "steps/s", "cores": threads, "kind": "oracle",
               "sample": f"1 oracle FP64 step of the same chain truncated to N={Ns} "
                         f"(n={3 * Ns}), {dt_s:.2f} s measured on {threads} threads, scaled by "
                         f"(n_s/n)^3 = {scale:.4g} to n={n}",
               "measured_s_per_step": dt_s, "status": io["status"],
               "cpu_model": cpu_model(),
               "single_thread": {"value": s1 / dt_1, "unit": "steps/s", "cores": 1,
                                 "sample": f"1 oracle FP64 step of the chain truncated to N={N1} "
                                           f"(n={3 * N1}), {dt_1:.2f} s on 1 thread, scaled "
                                           f"by (n_s/n)^3 = {s1:.4g} to n={n}",
                                 "measured_s_per_step": dt_1, "status": io1["status"]}}
        log(f"cpu oracle: {cpu}")

    series = (error_series(B, torch, np, h, p, x0, n, w, args)
              if args.series_steps > 0 and len(precs) == 2 else None)
    ens = ensemble_leg(B, I, torch, np, precs, args, dev) if args.ensemble_steps > 0 else None
    fraenkel = fraenkel_leg(B, torch, h, p, x0, n, w, precs, args) if args.fraenkel_steps > 0 else None


    mixed = result.get("mixed")
    fp64 = result.get("fp64")
    headrec = result[head]
    out = {
        "metric": METRIC,
        "value": headrec["steps_per_s"],
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": headrec["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-mfma+f64" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n_beads": N, "n": n, "b": w.b, "hstar": w.hstar,
                   "a": w.a, "dt": w.dt, "flow": w.flow, "wi": w.wi, "rate": w.rate,
                   "precision": head, "chains": 1},
        "mixed": mixed,
        "fp64": fp64,
        "mixed_vs_fp64_steps": (mixed["steps_per_s"] / fp64["steps_per_s"]) if mixed and fp64 else None,
        "roofline": roof,
        "kernel_breakdown": breakdown,
        "other_precision_profile": other,
        "cpu_baseline": cpu,
        "mixed_error_series": series,
        "ensemble": ens,
        "fraenkel": fraenkel,
        "context": extra,
        "tuning": ({"schedules": h.tuning["schedules"], "ensemble_panels": h.tuning["ensemble_panels"],
                    "source": "paper_2208_06559_amd/tuning.json"} if h.tuning else None),
    }
    print(json.dumps(out), flush=True)
    h.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
