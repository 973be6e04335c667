"""Oracle trajectories for the GPU tests of the batched and served paths.

Runs ``oracle.alg1.run`` for several problems at once in a thread pool
(NumPy releases the interpreter lock inside its array operations, and no
process is forked from a test process that has initialised the GPU) and
compares a GPU certificate sequence's end with the oracle's.
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor

from oracle import alg1

# the bars of the 500-iteration 32x32 trajectory test (Algorithm 1 run by both
# sides from the same inputs, each on its own): relative gap within 1e-3
# relative, U and L within 1e-4 relative
GAP_TOL, BOUND_TOL = 1e-3, 1e-4


def run_many(cases, workers: int = 16):
    """cases: (problem, eta, lam, iters, cert_every, tau_rel) tuples; returns
    the oracle's certificate list of each run, in order."""
    def one(c):
        prob, eta, lam, iters, every, tau = c
        return alg1.run(prob, eta, lam, iters, cert_every=every, tau_rel=tau)[1]
    with ThreadPoolExecutor(max(1, min(workers, len(cases)))) as ex:
        return list(ex.map(one, cases))


def compare_final(gpu_cert: dict, certs: list, tau=None) -> str:
    """Checks a GPU run's last certificate against the oracle's run of the
    same problem: the same stopping iteration (the oracle stops at its first
    certificate whose best relative gap meets tau, or at the cap), and the
    relative gap, U and L at that certificate within the trajectory bars.
    Returns a one-line summary; raises AssertionError otherwise."""
    ref = certs[-1]
    assert gpu_cert["k"] == ref["k"], (gpu_cert["k"], ref["k"])
    if tau is not None:
        # the stop is decided at the same certificate: earlier ones miss tau on both sides
        assert all(c["rel_best"] > tau for c in certs[:-1])
    d_gap = abs(gpu_cert["rel_gap"] - ref["rel"]) / abs(ref["rel"])
    d_u = abs(gpu_cert["U"] - ref["U"]) / abs(ref["U"])
    d_l = abs(gpu_cert["L"] - ref["L"]) / abs(ref["L"])
    assert d_gap <= GAP_TOL, ("gap", d_gap, gpu_cert["rel_gap"], ref["rel"])
    assert d_u <= BOUND_TOL and d_l <= BOUND_TOL, ("bounds", d_u, d_l)
    return f"k={ref['k']} gap {gpu_cert['rel_gap']:.6f} vs {ref['rel']:.6f} (rel err {d_gap:.1e}; U {d_u:.1e}, L {d_l:.1e})"
