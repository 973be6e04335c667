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
relative duality gap for plain BDRS (lambda = 1) and O-BDRS (lambda = 1.2,
1.5, 1.99) from inputs resident (solver creation included), the 64-problem
batch's makespan against sequential solves, the serve latencies (p50/p99)
of Poisson requests against one-at-a-time FIFO, and the FP64 oracle timed
on the host on a bounded sample of the same sweeps.
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
ETA = 0.1            # initial temperature of the grid workloads (chosen from the oracle's gap curves)
CERT_EVERY = 50
# Serving: requests above this many implicit entries per sweep (a 256x256 grid
# problem has 4.3e9; the GPU is saturated well below that) run one at a time.
BIG_WORK = 1e9
CU, LANES, CLK = 256, 64, 2.4e9
EXP_SLOTS = 1        # issue slots of one v_exp_f32: the colour sweep's counters show 6.80 VALU
                     # instructions per entry (one of them the exp) issued at 98% of the
                     # 64 lane-ops/CU/cycle ceiling, which a 2-slot exp would put above 100%


# HBM traffic of one k_sweep<2,0> launch on the 128x128 grids (16 row and 16
# column splits), averaged over the row and column sweeps of the profiled
# replay of the default run (k = 150 ... 1149): rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE per dispatch, each scaled by what the counter reads for a 256 MiB
# device copy (x2.000 and x1.000).  It holds for the kernel sources with this
# sha256 (of bdrs_kernels.hip followed by bdrs_internal.h) and those split
# counts only; otherwise it is reported as null.
TRAFFIC_KERNEL_SHA256 = "633d46953d215f376c287b60b5ff776a06218199df7e69343cad1dca31ba95eb"
TRAFFIC_SPLITS = (16, 16)
TRAFFIC_BYTES_PER_LAUNCH = 6.41e6
# Counters of the same profile (per dispatch of k_sweep<2,0> in the replay):
# VALU lane instructions and v_exp_f32 per evaluated entry (x 64 / evaluated
# entries), VALU issue utilisation (lane instructions / duration / (256 x 64 x
# 2.4 GHz)) and rocprof's VALUBusy.
PROFILE_COUNTERS = {"valu_instr_per_evaluated_entry": 10.98, "exp_per_evaluated_entry": 1.023,
                    "valu_issue_frac": 0.426, "VALUBusy": 26.3,
                    "source": "profiles/k_sweep_grid128x128.md"}


def profiled_counters(splits):
    return PROFILE_COUNTERS if measured_traffic(splits) is not None else None


def measured_traffic(splits):
    import hashlib
    m = hashlib.sha256()
    try:
        for name in ("bdrs_kernels.hip", "bdrs_internal.h"):
            m.update(open(os.path.join(ROOT, "paper_2609_33814_amd", "csrc", name), "rb").read())
    except OSError:
        return None
    sha = m.hexdigest()
    if sha != TRAFFIC_KERNEL_SHA256 or splits != TRAFFIC_SPLITS:
        return None
    return TRAFFIC_BYTES_PER_LAUNCH


def sweep_peak_gentries(dim: int) -> float:
    """FP32 exp/VALU roofline of one sweep entry, in Gentries/s: the fewest
    VALU issue slots an entry can take in the tile-expanded form (d FMAs,
    1 add of the weight, the exp2, 1 add into the sum) on 256 CUs x 64 lanes
    x 2.4 GHz."""
    return CU * LANES * CLK / (dim + 2 + EXP_SLOTS) / 1e9


def _oracle_rows(task):
    """One block of sampled output rows of the oracle's row sweep (pool worker)."""
    from oracle import lse
    x, y, scale, w, rows = task
    lse.implicit_lse(x, y, scale, 0.01, w, rows=rows)
    return rows.size


def cpu_baseline(prob, seconds: float = 12.0) -> dict:
    """The FP64 oracle's LSE sweep on sampled output rows, timed on the host:
    first in this process (one thread), then with a fork pool of worker
    processes over blocks of rows, one per core of this process's CPU share
    (at most 16).  Runs before the GPU is touched, so forking is safe."""
    import multiprocessing as mp
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
    one = entries / dt / 1e9
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    tasks = [(prob.x, prob.y, prob.cost_scale, w, rng.choice(prob.m, rows_per_call, replace=False))
             for _ in range(int(one * 1e9 * seconds * cores / (rows_per_call * prob.n)) + cores)]
    with mp.get_context("fork").Pool(cores) as pool:
        t1 = time.perf_counter()
        done_all = sum(pool.imap_unordered(_oracle_rows, tasks))
        dt_all = time.perf_counter() - t1
    entries_all = done_all * prob.n
    return {"value": entries_all / dt_all / 1e9, "unit": "Gentries/s", "cores": cores, "kind": "oracle",
            "sample": f"{done_all} random output rows x {prob.n} columns of the row sweep "
                      f"({entries_all:.3g} entries, {dt_all:.1f} s, numpy FP64, {cores} worker processes)",
            "single_thread": {"value": one, "cores": 1,
                              "sample": f"{done} rows x {prob.n} columns ({entries:.3g} entries, {dt:.1f} s)"}}


def run_batch(log=True) -> dict:
    """64 grid problems with sides drawn from {32, 64, 128, 256} (seed 41), each
    solved to a 1% relative gap: one after another with bdrs_solve, then all at
    once with bdrs_batch_solve (captured 50-iteration blocks).  Solver set-up
    is outside both timed regions; results must agree bit for bit."""
    import numpy as np
    import torch
    from paper_2609_33814_amd import bdrs, inputs
    dev = torch.device("cuda:0")
    sides = inputs.batch_sides()
    probs = [inputs.batch_problem(p, s) for p, s in enumerate(sides)]
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    data = [(t(p.x, torch.float32), t(p.y, torch.float32), t(p.r, torch.float64), t(p.c, torch.float64),
             p.cost_scale) for p in probs]
    cap, tau = 40000, 0.01
    if log:
        print(f"[bench] batch of {len(probs)} grids, sides {sorted(set(sides))}, eta={ETA}", flush=True)
    # warm-up of every kernel variant
    w = bdrs.Solver(*data[0][:4], data[0][4], eta=ETA)
    w.solve(tau, 100, CERT_EVERY)
    bdrs.batch_solve([w], tau, 100, CERT_EVERY)
    w.close()
    seq_t, seq = 0.0, []
    for i, d in enumerate(data):
        sv = bdrs.Solver(*d[:4], d[4], eta=ETA)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ok, ce = sv.solve(tau, cap, CERT_EVERY)
        torch.cuda.synchronize()
        seq_t += time.perf_counter() - t0
        seq.append((ok, ce))
        sv.close()
        if log and (i + 1) % 16 == 0:
            print(f"[bench] batch workload, sequential: {i + 1} solved, {seq_t:.2f} s", flush=True)
    svs = [bdrs.Solver(*d[:4], d[4], eta=ETA) for d in data]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, certs, sts = bdrs.batch_solve(svs, tau, cap, CERT_EVERY, use_graph=True)
    torch.cuda.synchronize()
    bat_t = time.perf_counter() - t0
    for sv in svs:
        sv.close()
    same = all(c["k"] == s[1]["k"] and c["U"] == s[1]["U"] and c["L"] == s[1]["L"] for c, s in zip(certs, seq))
    reached = sum(1 for x in sts if x == bdrs.OK)
    entries = sum(2.0 * p.m * p.n * (c["k"] + 1) for p, c in zip(probs, certs))
    out = {"makespan_s": round(bat_t, 3), "sequential_s": round(seq_t, 3),
           "speedup_vs_sequential": round(seq_t / bat_t, 4),
           "batched_gentries_per_s": round(entries / bat_t / 1e9, 1),
           "sequential_gentries_per_s": round(entries / seq_t / 1e9, 1),
           "reached": reached, "problems": len(probs), "bitwise_equal_alone_vs_batched": bool(same),
           "workload": "64 grid histogram pairs, sides from {32,64,128,256} (seed 41), seeds (4100+2p, 4101+2p), "
                       f"eta {ETA}, 1% relative gap, cap {cap}",
           "iterations": {str(s): sorted(set(c["k"] + 1 for c, sd in zip(certs, sides) if sd == s))
                          for s in sorted(set(sides))}}
    if log:
        print(f"[bench] batch: {out['makespan_s']} s batched vs {out['sequential_s']} s sequential "
              f"({out['speedup_vs_sequential']}x), {reached}/{len(probs)} reached, bitwise {same}", flush=True)
    return out


def batch_mode(args) -> int:
    out = run_batch()
    line = {
        "metric": "makespan of 64 uneven grid OT solves to 1% relative gap", "value": out["makespan_s"],
        "unit": "s", "n_gpus": 1, "higher_is_better": False, "dtype": "f32", "data": "synthetic",
        "config": {"workload": out["workload"], "eta": ETA, "lambda": 1.0, "cert_every": CERT_EVERY},
        **{k: v for k, v in out.items() if k not in ("makespan_s", "workload")},
    }
    print(json.dumps(line), flush=True)
    return 0


def run_serve(n_req: int, menu: list, load: float, plain: bool = False, log=True) -> dict:
    """Poisson arrivals of grid OT requests (sides from `menu`, drawn with seed
    52; inter-arrival gaps with seed 51; request q seeds (5100+2q, 5101+2q)),
    each stopped at a 1% relative gap.  The arrival rate is `load` times the
    sequential capacity measured on a sample.  The same arrival schedule is
    served twice: one request at a time (FIFO) and with continuous batching
    (up to 32 running requests in a 1 GiB pool, requests above BIG_WORK
    entries per sweep one at a time).  Latency = completion - submission,
    including the host preparation of the request and its upload."""
    import threading
    import numpy as np
    from paper_2609_33814_amd import bdrs, inputs
    sides = [menu[i] for i in np.random.default_rng(52).integers(0, len(menu), n_req)]
    probs = [inputs.grid_problem(s, 5100 + 2 * q, 5101 + 2 * q) for q, s in enumerate(sides)]
    tau, cap, block, pool = 0.01, 20000, CERT_EVERY, 1 << 30
    if log:
        print(f"[bench] serve: {n_req} requests, sides {menu}, eta={ETA}, pool {pool >> 20} MiB", flush=True)

    # sequential capacity from a sample of requests served alone
    calib = bdrs.Server(pool, 1, block)
    sample = probs[: min(16, n_req)]
    t0 = time.perf_counter()
    for q, p in enumerate(sample):
        calib.wait(calib.submit(p, eta=ETA, tau=tau, max_iters=cap))
        if log and (q + 1) % 4 == 0:
            print(f"[bench] serve calibration: {q + 1} of {len(sample)} alone, {time.perf_counter() - t0:.1f} s",
                  flush=True)
    mean_s = (time.perf_counter() - t0) / len(sample)
    calib.close()
    rate = load / mean_s
    gaps = np.random.default_rng(51).exponential(1.0 / rate, n_req)
    arrivals = np.cumsum(gaps) - gaps[0]
    if log:
        print(f"[bench] serve: sequential capacity {1 / mean_s:.2f} solves/s; arrival rate {rate:.2f}/s", flush=True)

    def run(max_slots, big_work=0.0):
        srv = bdrs.Server(pool, max_slots, block)
        srv.set_policy(big_work)
        tickets = [None] * n_req
        start = time.perf_counter()

        def feeder():
            for q in range(n_req):
                delay = arrivals[q] - (time.perf_counter() - start)
                if delay > 0:
                    time.sleep(delay)
                tickets[q] = srv.submit(probs[q], eta=ETA, tau=tau, max_iters=cap)

        th = threading.Thread(target=feeder)
        th.start()
        th.join()
        res = []
        for q, tk in enumerate(tickets):
            res.append(srv.wait(tk))
            if log and (q + 1) % 8 == 0:
                print(f"[bench] serve, max_slots={max_slots}: {q + 1} of {n_req} done at "
                      f"{time.perf_counter() - start:.1f} s", flush=True)
        srv.close()
        lat = np.array([r["t_done"] - r["t_submit"] for r in res])
        span = max(r["t_done"] for r in res) - min(r["t_submit"] for r in res)
        ok = sum(1 for r in res if r["status"] == bdrs.OK)
        out = dict(p50_s=round(float(np.percentile(lat, 50)), 4), p99_s=round(float(np.percentile(lat, 99)), 4),
                   mean_s=round(float(lat.mean()), 4), solves_per_s=round(n_req / span, 3), reached=ok)
        if log:
            print(f"[bench] serve, max_slots={max_slots}: {out}", flush=True)
        return out, res

    fifo, res_f = run(1)
    cont, res_c = run(32, BIG_WORK)
    same = all(a["cert"]["k"] == b["cert"]["k"] and a["cert"]["U"] == b["cert"]["U"] and
               a["cert"]["L"] == b["cert"]["L"] for a, b in zip(res_f, res_c))
    plain_out = run(32, 0.0)[0] if plain else None
    return {"continuous_batching": cont, "fifo_sequential": fifo, "continuous_batching_arrival_order": plain_out,
            "p99_speedup": round(fifo["p99_s"] / cont["p99_s"], 3),
            "p50_speedup": round(fifo["p50_s"] / cont["p50_s"], 3),
            "results_equal_fifo_vs_batched": bool(same), "requests": n_req,
            "workload": f"{n_req} grid requests, sides from {menu} (seed 52), arrivals Exp (seed 51) at "
                        f"{load} x sequential capacity, eta {ETA}, 1% relative gap",
            "block_iters": block, "pool_MiB": pool >> 20, "max_slots": 32, "big_work": BIG_WORK}


def serve_mode(args) -> int:
    menu = [int(v) for v in args.serve_sides.split(",")]
    out = run_serve(args.requests, menu, args.load, plain=args.serve_plain)
    line = {
        "metric": "p50/p99 latency of OT solve requests to 1% relative gap (Poisson arrivals)",
        "value": out["continuous_batching"]["p99_s"], "unit": "s", "n_gpus": 1, "higher_is_better": False,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": out["workload"], "eta": ETA, "lambda": 1.0, "block_iters": out["block_iters"],
                   "pool_MiB": out["pool_MiB"], "max_slots": 32, "big_work": BIG_WORK},
        **{k: v for k, v in out.items() if k not in ("workload", "block_iters", "pool_MiB", "max_slots", "big_work")},
    }
    print(json.dumps(line), flush=True)
    return 0


def colour_mode(args) -> int:
    """Colour transfer, 1024x1024 RGB points per side (1.1e12 implicit entries
    per sweep), eta = 0.1, lambda = 1, certificate every 20 iterations, a fixed
    budget of `colour_iters` iterations; reports Gentries/s, the per-launch
    sweep time and the gap trajectory."""
    import numpy as np
    import torch
    from paper_2609_33814_amd import bdrs, inputs
    dev = torch.device("cuda:0")
    prob = inputs.c3_problem()
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    eta, every, iters = 0.1, 20, args.colour_iters
    print(f"[bench] colour m=n={prob.m} d=3 eta={eta} cert every {every}, {iters} iterations", flush=True)
    sv = bdrs.Solver(t(prob.x, torch.float32), t(prob.y, torch.float32), t(prob.r, torch.float64),
                     t(prob.c, torch.float64), prob.cost_scale, eta=eta)
    sv.step(1)            # warm-up: one iteration, then restart from zero
    torch.cuda.synchronize()
    sv.close()
    sv = bdrs.Solver(t(prob.x, torch.float32), t(prob.y, torch.float32), t(prob.r, torch.float64),
                     t(prob.c, torch.float64), prob.cost_scale, eta=eta)
    traj = []
    sv.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, reached_at = 0, None
    while done < iters:
        _, ce = sv.solve(0.0, every, every)
        done += every
        el = time.perf_counter() - t0
        traj.append({"k": int(ce["k"]), "rel_gap": ce["rel_gap"], "rel_gap_best": ce["rel_gap_best"],
                     "s": round(el, 3)})
        if reached_at is None and ce["rel_gap_best"] <= 0.01:
            reached_at = {"iterations": int(ce["k"]) + 1, "seconds": round(el, 3)}
        print(f"[bench] k={ce['k']} rel_gap={ce['rel_gap']:.5f} best={ce['rel_gap_best']:.5f} t={el:.1f}s",
              flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = sv.profile_read()
    sv.profile(False)
    per_sweep_ms = prof["ms"] / max(prof["sweeps"], 1)
    implicit_rate = prob.m * prob.n / (per_sweep_ms * 1e-3) / 1e9
    evaluated_frac = prof["evaluated"] / max(prof["entries"], 1.0)
    achieved = implicit_rate * evaluated_frac
    peak = sweep_peak_gentries(prob.dim)
    value = 2.0 * prob.m * prob.n * iters / wall / 1e9
    # the state plan of the last iterate: marginal errors and barycentric projection
    t1 = time.perf_counter()
    pl = sv.plan()
    plan_s = time.perf_counter() - t1
    print(f"[bench] state plan: {plan_s:.2f} s, {pl['stats']}", flush=True)
    line = {
        "metric": "Gentries/s of fused LSE sweeps (colour transfer)", "value": round(value, 2),
        "unit": "Gentries/s", "n_gpus": 1, "steps": iters, "higher_is_better": True, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "colour transfer, 1048576 RGB points per side from 8-component Gaussian "
                               "mixtures (seeds 31, 32), uniform weights, sq. Euclidean cost scaled to max 1",
                   "eta": eta, "lambda": 1.0, "cert_every": every},
        "s_per_iteration": round(wall / iters, 4),
        "roofline": {"bound": "alu", "achieved": round(achieved, 2), "peak": round(peak, 2),
                     "unit": "Gentries/s", "frac": round(achieved / peak, 4), "traffic": None,
                     "kernel": "k_sweep<3,0> (plain mode)", "per_launch_us": round(per_sweep_ms * 1e3, 3),
                     "implicit_gentries_per_s": round(implicit_rate, 2),
                     "evaluated_fraction": round(evaluated_frac, 4)},
        "time_to_1pct": reached_at, "trajectory": traj,
        "state_plan": {"seconds": round(plan_s, 3), **pl["stats"]},
    }
    print(json.dumps(line), flush=True)
    return 0


def colour10m_mode(args) -> int:
    """Colour transfer at 4238x2365 = 10,022,870 RGB points per side (1.0e14
    implicit entries per sweep), eta = 0.01: three timed iterations and one
    certificate; reports the median seconds per iteration."""
    import numpy as np
    import torch
    from paper_2609_33814_amd import bdrs, inputs
    dev = torch.device("cuda:0")
    prob = inputs.c3b_problem()
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    eta = 0.01
    print(f"[bench] colour m=n={prob.m} d=3 eta={eta}", flush=True)
    sv = bdrs.Solver(t(prob.x, torch.float32), t(prob.y, torch.float32), t(prob.r, torch.float64),
                     t(prob.c, torch.float64), prob.cost_scale, eta=eta)
    secs = []
    for it in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sv.step(1)
        torch.cuda.synchronize()
        secs.append(time.perf_counter() - t0)
        print(f"[bench] iteration {it}: {secs[-1]:.2f} s", flush=True)
    t0 = time.perf_counter()
    ce = sv.certificate()
    cert_s = time.perf_counter() - t0
    print(f"[bench] certificate: {cert_s:.2f} s rel_gap={ce['rel_gap']:.4f}", flush=True)
    med = float(np.median(secs))
    value = 2.0 * prob.m * prob.n / med / 1e9
    peak = sweep_peak_gentries(prob.dim)
    line = {
        "metric": "seconds per iteration (colour transfer, 10M points per side)", "value": round(med, 3),
        "unit": "s/iteration", "n_gpus": 1, "steps": 3, "higher_is_better": False, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "colour transfer, 10022870 RGB points per side (seeds 33, 34), uniform "
                               "weights, sq. Euclidean cost scaled to max 1", "eta": eta, "lambda": 1.0},
        "gentries_per_s": round(value, 1), "frac_of_sweep_roofline": round(value / peak, 4),
        "iteration_s": [round(x, 3) for x in secs], "certificate_s": round(cert_s, 3),
        "rel_gap_after_3": ce["rel_gap"],
    }
    print(json.dumps(line), flush=True)
    return 0


def export_mode(args) -> int:
    """Feasible plan export on the 128x128 grids (eta = 0.1, after 300
    iterations): the factors of the rounded and of the repaired plan
    (bdrs_export_plan, host-timed with the sweeps it runs) and the dense
    16384 x 16384 float64 plan from them (bdrs_plan_entries, HIP events on
    the solver's stream).  The dense kernel writes 8 bytes per entry and
    reads O(m + n): its roofline is HBM bandwidth."""
    import numpy as np
    import torch
    from paper_2609_33814_amd import bdrs, inputs
    dev = torch.device("cuda:0")
    prob = inputs.c2_problem()
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    sv = bdrs.Solver(t(prob.x, torch.float32), t(prob.y, torch.float32), t(prob.r, torch.float64),
                     t(prob.c, torch.float64), prob.cost_scale, eta=ETA)
    sv.step(300)
    torch.cuda.synchronize()
    L = bdrs.lib()
    P = torch.empty((prob.m, prob.n), dtype=torch.float64, device=dev)
    out = {}
    for kind in ("rounded", "repaired"):
        ts = []
        for _ in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ex = sv.export_plan(kind)
            ts.append(time.perf_counter() - t0)
        f = lambda k: ex[k].data_ptr()
        call = lambda: bdrs.check(L.bdrs_plan_entries(sv.handle, f("log_u"), f("log_v"), f("a"), f("b"),
                                                      ex["info"]["eps"], 0, prob.m, P.data_ptr()))
        call()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        for a, b in ev:
            a.record()
            call()
            b.record()
        torch.cuda.synchronize()
        ms = sorted(a.elapsed_time(b) for a, b in ev)
        med = ms[len(ms) // 2]
        row, col = P.sum(dim=1), P.sum(dim=0)
        r, c = t(prob.r, torch.float64), t(prob.c, torch.float64)
        out[kind] = {"export_ms": round(1e3 * sorted(ts)[2], 3), "entries_ms": round(med, 4),
                     "entries_gb_per_s": round(P.numel() * 8 / (med * 1e-3) / 1e9, 1),
                     "cost": ex["info"]["cost"], "mass": ex["info"]["mass"],
                     "max_rel_row_error": float(((row - r).abs() / r).max()),
                     "max_rel_col_error": float(((col - c).abs() / c).max())}
        print(f"[bench] {kind}: {out[kind]}", flush=True)
    sv.close()
    gbs = out["rounded"]["entries_gb_per_s"]
    line = {
        "metric": "dense feasible-plan export, GB/s written (16384 x 16384 float64)", "value": gbs,
        "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "higher_is_better": True, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "grid128x128 Gaussian-mixture histograms (seeds 21, 22), n=m=16384, "
                               "after 300 iterations at eta 0.1", "eta": ETA, "lambda": 1.0},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s",
                     "frac": round(gbs / 8000.0, 4), "traffic": None, "kernel": "k_plan_entries<2>",
                     "bytes_per_launch": prob.m * prob.n * 8},
        "plans": out,
    }
    print(json.dumps(line), flush=True)
    return 0


def ablation_mode(args) -> int:
    """Momentum / kernel ablation on the 128x128 grids (seeds 21, 22), eta =
    0.1: every row-update variant at lambda = 1 and O-BDRS at lambda = 1.2,
    1.5 and 1.99, each run to a 1% certified relative gap (cap 20000
    iterations, certificate every 50); the last iterate's
    state plan is also rounded onto Pi(r, c), the feasible cost the ablation
    compares.  With --round-curve a second run of each variant rounds its
    state plan after every iteration (outside any timing, as in the
    ablation) and reports the feasible cost f_k at log-spaced k, its minimum
    and (f_k - L) / f_k against the largest certified lower bound L of all
    variants (which bounds the gap to the optimum from above)."""
    import numpy as np
    import torch
    from paper_2609_33814_amd import bdrs, inputs
    dev = torch.device("cuda:0")
    prob = inputs.c2_problem()
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    X, Y, R, C = t(prob.x, torch.float32), t(prob.y, torch.float32), t(prob.r, torch.float64), t(prob.c, torch.float64)
    cap = args.ttg_cap
    out = {}
    # the four row-update variants and the debiased one at lambda = 1, then
    # O-BDRS at the paper's overrelaxations: the ablation's eight methods
    methods = [(name, name, 1.0) for name in bdrs.VARIANTS]
    methods += [(f"o_bdrs_{lam}", "dual_bdrs", lam) for lam in (1.2, 1.5, 1.99)]
    for name, variant, lam in methods:
        sv = bdrs.Solver(X, Y, R, C, prob.cost_scale, eta=ETA, lam=lam, variant=variant)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ok, ce = sv.solve(0.01, cap, CERT_EVERY)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rd = sv.round()   # feasible plan of the last iterate (two-sided rounding), outside the timing
        out[name] = {"reached": bool(ok), "iterations": int(ce["k"]) + 1, "seconds": round(dt, 4),
                     "rel_gap_best": ce["rel_gap_best"], "U_best": ce["U_best"], "L_best": ce["L_best"],
                     "rounded_cost": rd["cost"], "rounded_rel_gap": (rd["cost"] - ce["L_best"]) / rd["cost"]}
        print(f"[bench] {name}: {out[name]}", flush=True)
        sv.close()
        if args.round_curve:
            K = out[name]["iterations"]
            sv = bdrs.Solver(X, Y, R, C, prob.cost_scale, eta=ETA, lam=lam, variant=variant)
            f = np.empty(K)
            for k in range(K):
                sv.step(1)
                f[k] = sv.round()["cost"]
            sv.close()
            out[name]["_f"] = f
            print(f"[bench] {name}: rounded after each of {K} iterations, min f {f.min():.6g} "
                  f"at k = {int(f.argmin()) + 1}", flush=True)
    if args.round_curve:
        L = max(v["L_best"] for v in out.values())
        for name, v in out.items():
            f = v.pop("_f")
            ks = sorted({min(int(round(10 ** (e / 4))), len(f)) for e in range(0, 4 * 5)} | {len(f)})
            v["rounded_curve"] = {"k": ks, "f": [float(f[k - 1]) for k in ks],
                                  "gap_vs_L": [float((f[k - 1] - L) / f[k - 1]) for k in ks]}
            v["rounded_min"] = float(f.min())
            v["rounded_min_gap_vs_L"] = float((f.min() - L) / f.min())
        print(f"[bench] largest certified lower bound over the variants: L = {L:.9g}", flush=True)
    line = {
        "metric": "iterations and seconds to a 1% certified relative gap per row-update variant",
        "value": out["dual_bdrs"]["seconds"], "unit": "s", "n_gpus": 1, "higher_is_better": False,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "grid128x128 Gaussian-mixture histograms (seeds 21, 22)", "eta": ETA,
                   "lambda": "1 for the row-update variants; 1.2, 1.5, 1.99 for O-BDRS",
                   "cert_every": CERT_EVERY, "cap": cap},
        "variants": out,
    }
    print(json.dumps(line), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--lam", type=float, default=1.0)
    ap.add_argument("--no-ttg", action="store_true", help="skip the time-to-1%% runs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-problem batch (makespan vs sequential)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serve run (p50/p99 vs FIFO)")
    ap.add_argument("--serve-requests", type=int, default=48,
                    help="requests of the default run's serve measurement (sides 32, 64, 128)")
    ap.add_argument("--ttg-cap", type=int, default=20000)
    ap.add_argument("--mode", choices=("sweep", "batch", "serve", "colour", "colour10m", "ablation", "export"),
                    default="sweep",
                    help="sweep: the headline line (default); batch: 64 uneven grid problems, "
                         "sequential solves vs one batched solve, to a 1%% gap; serve: Poisson "
                         "arrivals, FIFO one-at-a-time vs continuous batching; colour: 1M-point "
                         "colour transfer; colour10m: 10M points, per-iteration time; ablation: "
                         "row-update variants to a 1%% gap; export: dense feasible-plan export")
    ap.add_argument("--colour-iters", type=int, default=100)
    ap.add_argument("--round-curve", action="store_true",
                    help="ablation: also round each variant's state plan after every iteration")
    ap.add_argument("--serve-sides", default="32,64,128", help="grid sides of the serve requests")
    ap.add_argument("--serve-plain", action="store_true",
                    help="also serve with arrival-order admission (no size-aware policy)")
    ap.add_argument("--requests", type=int, default=96)
    ap.add_argument("--load", type=float, default=0.8, help="arrival rate / sequential capacity")
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

    if args.mode == "sweep" and not args.no_cpu:
        cpu = cpu_baseline(inputs.c2_problem())   # before the GPU is first used
        print(f"[bench] oracle on the host: {cpu['value']:.3f} Gentries/s on {cpu['cores']} cores, "
              f"{cpu['single_thread']['value']:.3f} on one", flush=True)
    else:
        cpu = None
    dev = torch.device("cuda:0")
    if args.mode == "batch":
        return batch_mode(args)
    if args.mode == "serve":
        return serve_mode(args)
    if args.mode == "colour":
        return colour_mode(args)
    if args.mode == "colour10m":
        return colour10m_mode(args)
    if args.mode == "ablation":
        return ablation_mode(args)
    if args.mode == "export":
        return export_mode(args)
    prob = inputs.c2_problem()
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    X, Y = t(prob.x, torch.float32), t(prob.y, torch.float32)
    R, C = t(prob.r, torch.float64), t(prob.c, torch.float64)
    print(f"[bench] workload grid128x128 m=n={prob.m} eta={ETA} lambda={args.lam}", flush=True)

    sv = bdrs.Solver(X, Y, R, C, prob.cost_scale, eta=ETA, lam=args.lam)
    tuned = [e for e in bdrs.tune_table() if (e["dim"], e["m"], e["n"]) == (prob.dim, prob.m, prob.n)]
    splits = (tuned[0]["splits_row"], tuned[0]["splits_col"]) if tuned else None
    for _ in range(args.warmup):
        sv.solve(0.0, CERT_EVERY, CERT_EVERY)
    torch.cuda.synchronize()
    start_state, start_hints = sv.get_state(), sv.get_hints()
    t0 = time.perf_counter()
    last = None
    for _ in range(args.steps):
        _, last = sv.solve(0.0, CERT_EVERY, CERT_EVERY)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # the same steps again from the same state, each sweep bracketed by HIP
    # events (kernel time) and followed by its evaluated-tile count
    sv.set_state(start_state)
    sv.set_hints(start_hints)
    sv.profile(True)
    last_prof = None
    for _ in range(args.steps):
        _, last_prof = sv.solve(0.0, CERT_EVERY, CERT_EVERY)
    prof = sv.profile_read()
    sv.profile(False)
    if last is not None and last_prof["rel_gap"] != last["rel_gap"]:
        raise RuntimeError("the profiled replay diverged from the timed steps")
    sweeps = args.steps * CERT_EVERY * 2
    entries = sweeps * prob.m * prob.n
    value = entries / wall / 1e9
    per_sweep_ms = prof["ms"] / max(prof["sweeps"], 1)
    implicit_rate = prob.m * prob.n / (per_sweep_ms * 1e-3) / 1e9
    # the roofline counts the entries the sweeps evaluated: tiles whose bound
    # puts every term below 2^-64 of the running maximum are skipped
    evaluated_frac = prof["evaluated"] / max(prof["entries"], 1.0)
    achieved = implicit_rate * evaluated_frac
    peak = sweep_peak_gentries(prob.dim)
    print(f"[bench] timed {args.steps} steps: {wall*1e3:.1f} ms, {value:.1f} Gentries/s; "
          f"sweep kernel {per_sweep_ms*1e3:.1f} us avg over {prof['sweeps']} launches "
          f"({implicit_rate:.1f} implicit Gentries/s; {evaluated_frac:.3f} of the entries evaluated at "
          f"{achieved:.1f} Gentries/s, {achieved/peak:.3f} of {peak:.0f})", flush=True)

    ttg = {}
    if not args.no_ttg:
        for lam in (1.0, 1.2, 1.5, 1.99):
            # the clock starts with the inputs resident: solver creation (workspace,
            # validation, tile order, upload) is inside, data generation outside
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s2 = bdrs.Solver(X, Y, R, C, prob.cost_scale, eta=ETA, lam=lam)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ok, ce = s2.solve(0.01, args.ttg_cap, CERT_EVERY)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            iters = int(ce["k"]) + 1
            ttg[f"lambda={lam}"] = {"reached": bool(ok), "seconds": round(t2 - t0, 4),
                                    "seconds_create": round(t1 - t0, 4), "seconds_solve": round(t2 - t1, 4),
                                    "iterations": iters,
                                    "whole_solve_gentries_per_s": round(2.0 * prob.m * prob.n * iters / (t2 - t0) / 1e9,
                                                                         1),
                                    "rel_gap_best": ce["rel_gap_best"],
                                    "U_best": ce["U_best"], "L_best": ce["L_best"]}
            print(f"[bench] time-to-1% lambda={lam}: {ttg[f'lambda={lam}']}", flush=True)
            s2.close()

    batch = None if args.no_batch else run_batch()
    serve = None
    if not args.no_serve:
        serve = run_serve(args.serve_requests, [32, 64, 128], 0.8)

    if args.calib_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)   # 256 MiB
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print("[bench] calibration copy: 268435456 bytes read, 268435456 bytes written", flush=True)
        del src, dst

    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "Gentries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall * 1e3 / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "grid128x128 Gaussian-mixture histograms (seeds 21, 22), "
                               "n=m=16384, d=2, sq. Euclidean cost scaled to max 1",
                   "eta": ETA, "lambda": args.lam, "cert_every": CERT_EVERY,
                   "step": "50 iterations (100 sweeps) + fused certificate",
                   "timed_window": {"k_first": args.warmup * CERT_EVERY,
                                    "k_last": (args.warmup + args.steps) * CERT_EVERY - 1,
                                    "evaluated_fraction": round(evaluated_frac, 4),
                                    "note": "value counts implicit entries m n per sweep; the sweeps "
                                            "evaluate the fraction above (the rest lies below 2^-T of "
                                            "each output's maximum and is skipped)"},
                   "last_rel_gap": last["rel_gap"] if last else None},
        "roofline": {"bound": "alu", "achieved": round(achieved, 2), "peak": round(peak, 2),
                     "unit": "Gentries/s", "frac": round(achieved / peak, 4),
                     "traffic": measured_traffic(splits), "traffic_unit": "HBM bytes per launch",
                     "kernel": "k_sweep<2,0> (plain mode)", "per_launch_us": round(per_sweep_ms * 1e3, 3),
                     "splits": list(splits) if splits else None,
                     "implicit_gentries_per_s": round(implicit_rate, 2),
                     "evaluated_fraction": round(evaluated_frac, 4),
                     "exp_per_s": round(achieved * 1e9, 0),  # one v_exp_f32 per evaluated entry
                     "counters": profiled_counters(splits)},
        "cpu_baseline": cpu,
        "time_to_1pct": ttg,
        "batch": batch,
        "serve": serve,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
