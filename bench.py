#!/usr/bin/env python3
"""Throughput of the fused LSE sweeps of Dual (O-)BDRS on one MI355X.

Workload: two seeded 128x128 grid histograms (16384 points per side, 2.68e8
implicit cost entries per sweep), squared Euclidean cost scaled to max 1.
One step = one block of 50 iterations of Algorithm 1 (row sweep + column
sweep each) whose last column sweep carries the fused certificate of
Prop. 3 / Algorithm 2, followed by the float64 certificate reductions and
the host readback -- the whole hot path once.  The timed region holds K such
steps with the inputs resident in HBM.  Printed: one JSON line.

Also reported: the dominant kernel's roofline fraction (sweep durations from
HIP events recorded by the library on its own stream), the time to a 1%
relative duality gap for plain BDRS (lambda = 1) and O-BDRS (lambda = 1.99),
and the FP64 oracle timed on the host on a bounded sample of the same sweeps.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gentries/s of fused LSE sweeps + time-to-1% rel. gap; p50/p99 serve latency"
ETA = 1.0            # initial temperature of the 128x128 workload
CERT_EVERY = 50
CU, LANES, CLK = 256, 64, 2.4e9
EXP_SLOTS = 2        # v_exp_f32 issues at half the FMA rate on gfx950


def sweep_peak_gentries(dim: int) -> float:
    """FP32 exp/VALU roofline of one sweep entry: d FMAs + 1 add (weight) +
    1 add (accumulate) + one exp2 at half rate, on 256 CUs x 64 lanes x 2.4 GHz."""
    return CU * LANES * CLK / (dim + 2 + EXP_SLOTS) / 1e9


def cpu_baseline(prob, seconds: float = 12.0) -> dict:
    """The FP64 oracle's LSE sweep on sampled output rows, timed on the host."""
    import numpy as np
    from oracle import lse
    rng = np.random.default_rng(0)
    w = rng.normal(0, 10, prob.n)
    rows_per_call = 256
    done = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        rows = rng.choice(prob.m, rows_per_call, replace=False)
        lse.implicit_lse(prob.x, prob.y, prob.cost_scale, 0.01, w, rows=rows)
        done += rows_per_call
    dt = time.perf_counter() - t0
    entries = done * prob.n
    return {"value": entries / dt / 1e9, "unit": "Gentries/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} random output rows x {prob.n} columns of the row sweep "
                      f"({entries:.3g} entries, {dt:.1f} s, numpy FP64, one thread)"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--lam", type=float, default=1.0)
    ap.add_argument("--no-ttg", action="store_true", help="skip the time-to-1%% runs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--ttg-cap", type=int, default=20000)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 256 MiB device-to-device copy (known bytes) so that "
                         "HBM traffic counters can be scaled")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the solver is "
              "single-GPU and no multi-GPU path is built.", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_2609_33814_amd import bdrs, inputs

    dev = torch.device("cuda:0")
    prob = inputs.c2_problem()
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    X, Y = t(prob.x, torch.float32), t(prob.y, torch.float32)
    R, C = t(prob.r, torch.float64), t(prob.c, torch.float64)
    print(f"[bench] workload grid128x128 m=n={prob.m} eta={ETA} lambda={args.lam}", flush=True)

    sv = bdrs.Solver(X, Y, R, C, prob.cost_scale, eta=ETA, lam=args.lam)
    for _ in range(args.warmup):
        sv.solve(0.0, CERT_EVERY, CERT_EVERY)
    torch.cuda.synchronize()
    sv.profile(True)
    t0 = time.perf_counter()
    last = None
    for _ in range(args.steps):
        _, last = sv.solve(0.0, CERT_EVERY, CERT_EVERY)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = sv.profile_read()
    sv.profile(False)
    sweeps = args.steps * CERT_EVERY * 2
    entries = sweeps * prob.m * prob.n
    value = entries / wall / 1e9
    per_sweep_ms = prof["ms"] / max(prof["sweeps"], 1)
    achieved = prob.m * prob.n / (per_sweep_ms * 1e-3) / 1e9
    peak = sweep_peak_gentries(prob.dim)
    print(f"[bench] timed {args.steps} steps: {wall*1e3:.1f} ms, {value:.1f} Gentries/s; "
          f"sweep kernel {per_sweep_ms*1e3:.1f} us avg over {prof['sweeps']} launches "
          f"({achieved:.1f} Gentries/s, {achieved/peak:.3f} of {peak:.0f})", flush=True)

    ttg = {}
    if not args.no_ttg:
        for lam in (1.0, 1.99):
            s2 = bdrs.Solver(X, Y, R, C, prob.cost_scale, eta=ETA, lam=lam)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ok, ce = s2.solve(0.01, args.ttg_cap, CERT_EVERY)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            ttg[f"lambda={lam}"] = {"reached": bool(ok), "seconds": round(dt, 4),
                                    "iterations": int(ce["k"]) + 1,
                                    "rel_gap_best": ce["rel_gap_best"],
                                    "U_best": ce["U_best"], "L_best": ce["L_best"]}
            print(f"[bench] time-to-1% lambda={lam}: {ttg[f'lambda={lam}']}", flush=True)
            s2.close()

    if args.calib_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)   # 256 MiB
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print("[bench] calibration copy: 268435456 bytes read, 268435456 bytes written", flush=True)
        del src, dst

    cpu = None if args.no_cpu else cpu_baseline(prob)
    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "Gentries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall * 1e3 / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "grid128x128 Gaussian-mixture histograms (seeds 21, 22), "
                               "n=m=16384, d=2, sq. Euclidean cost scaled to max 1",
                   "eta": ETA, "lambda": args.lam, "cert_every": CERT_EVERY,
                   "step": "50 iterations (100 sweeps) + fused certificate",
                   "last_rel_gap": last["rel_gap"] if last else None},
        "roofline": {"bound": "alu", "achieved": round(achieved, 2), "peak": round(peak, 2),
                     "unit": "Gentries/s", "frac": round(achieved / peak, 4), "traffic": None,
                     "kernel": "k_sweep<2,false>", "per_launch_us": round(per_sweep_ms * 1e3, 3)},
        "cpu_baseline": cpu,
        "time_to_1pct": ttg,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
