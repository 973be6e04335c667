"""Oracle trajectories for the GPU tests of the batched and served paths.

Runs ``oracle.alg1.run`` for several problems at once in a thread pool
(NumPy releases the interpreter lock inside its array operations, and no
process is forked from a test process that has initialised the GPU) and
compares a GPU certificate sequence's end with the oracle's.
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor

import numpy as np

from oracle import alg1

# the bars of the 500-iteration 32x32 trajectory test (Algorithm 1 run by both
# sides from the same inputs, each on its own): relative gap within 1e-3
# relative, U and L within 1e-4 relative
GAP_TOL, BOUND_TOL = 1e-3, 1e-4


def _f32(v):
    return v.astype(np.float32).astype(np.float64)


def run_many(cases, workers: int = 16):
    """cases: (problem, eta, lam, iters, cert_every, tau_rel) tuples; returns,
    per case in order, the oracle's certificate list and that of the same run
    with every LSE result rounded to float32 (the oracle's own sensitivity to
    float32 sweeps)."""
    def one(c):
        prob, eta, lam, iters, every, tau = c
        return alg1.run(prob, eta, lam, iters, cert_every=every, tau_rel=tau)[1]

    def one32(c):
        prob, eta, lam, iters, every, tau = c
        return alg1.run(prob, eta, lam, iters, cert_every=every, tau_rel=tau, perturb=_f32)[1]
    with ThreadPoolExecutor(max(1, min(workers, 2 * len(cases)))) as ex:
        plain = [ex.submit(one, c) for c in cases]
        r32 = [ex.submit(one32, c) for c in cases]
        return [(a.result(), b.result()) for a, b in zip(plain, r32)]


def compare_final(gpu_cert: dict, runs, tau=None) -> str:
    """Checks a GPU run's last certificate against the oracle's run of the
    same problem (runs = one item of run_many): the same stopping iteration
    (the oracle stops at its first certificate whose best relative gap meets
    tau, or at the cap), the relative gap at that certificate within 1e-3
    relative, and U and L within 1e-4 relative, or, where the oracle's own
    float32-rounded run moves them further, within that.  Returns a one-line
    summary; raises AssertionError otherwise."""
    certs, certs32 = runs
    ref = certs[-1]
    assert gpu_cert["k"] == ref["k"], (gpu_cert["k"], ref["k"])
    if tau is not None:
        # the stop is decided at the same certificate: earlier ones miss tau on both sides
        assert all(c["rel_best"] > tau for c in certs[:-1])
    d_gap = abs(gpu_cert["rel_gap"] - ref["rel"]) / abs(ref["rel"])
    d_u = abs(gpu_cert["U"] - ref["U"]) / abs(ref["U"])
    d_l = abs(gpu_cert["L"] - ref["L"]) / abs(ref["L"])
    r32 = {c["k"]: c for c in certs32}.get(ref["k"])
    s_u = abs(r32["U"] - ref["U"]) / abs(ref["U"]) if r32 else 0.0
    s_l = abs(r32["L"] - ref["L"]) / abs(ref["L"]) if r32 else 0.0
    assert d_gap <= GAP_TOL, ("gap", d_gap, gpu_cert["rel_gap"], ref["rel"])
    assert d_u <= max(BOUND_TOL, s_u) and d_l <= max(BOUND_TOL, s_l), ("bounds", d_u, d_l, s_u, s_l)
    return (f"k={ref['k']} gap {gpu_cert['rel_gap']:.6f} vs {ref['rel']:.6f} (rel err {d_gap:.1e}; "
            f"U {d_u:.1e}, L {d_l:.1e}; float32-rounded oracle U {s_u:.1e}, L {s_l:.1e})")
