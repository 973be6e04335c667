"""Writes the split-count table for the workload shapes (bdrs_autotune).

Usage: python -m paper_2609_33814_amd.autotune [--out PATH] [--rounds N]

Shapes: square grids of side 32, 64, 128, 256 and 512 (d = 2, the grid
histogram workloads and the batch / serve size menus) and the 1024x1024-point
colour-transfer clouds (d = 3).  Each shape is tuned on its own seeded
instance at eta = 0.1; the table is saved as JSON and is loaded by the
binding when the library is first loaded.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None, help="output JSON (default: the package's table)")
    ap.add_argument("--rounds", type=int, default=30)
    ap.add_argument("--sides", default="32,64,128,256,512")
    ap.add_argument("--no-colour", action="store_true")
    args = ap.parse_args()
    os.environ["BDRS_TUNING"] = "none"  # tune from the heuristic, not from an older table
    import numpy as np
    import torch
    from paper_2609_33814_amd import bdrs, inputs
    out = args.out or bdrs.TUNING_PATH
    dev = torch.device("cuda:0")
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    jobs = [(f"grid{s}", lambda s=s: inputs.grid_problem(s, 7001, 7002), args.rounds)
            for s in (int(v) for v in args.sides.split(","))]
    if not args.no_colour:
        jobs.append(("colour1M", inputs.c3_problem, max(3, args.rounds // 6)))
    for name, make, rounds in jobs:
        prob = make()
        t0 = time.perf_counter()
        e = bdrs.autotune(t(prob.x, torch.float32), t(prob.y, torch.float32), t(prob.r, torch.float64),
                          t(prob.c, torch.float64), prob.cost_scale, eta=0.1, rounds=rounds)
        print(f"[autotune] {name}: {json.dumps(e)} ({time.perf_counter() - t0:.1f} s)", flush=True)
    bdrs.save_tuning(out)
    print(f"[autotune] wrote {out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
