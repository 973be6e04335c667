"""Solve server: a request's result in a mix of concurrent requests equals its
result alone (bdrs_solve with cert_every = block_iters), bit for bit;
admission respects the memory budget; invalid requests fail alone."""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2609_33814_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu


def alone(prob, eta, tau, cap, block):
    from paper_2609_33814_amd import bdrs
    d = torch.device("cuda:0")
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=d)
    sv = bdrs.Solver(t(prob.x, torch.float32), t(prob.y, torch.float32), t(prob.r, torch.float64),
                     t(prob.c, torch.float64), prob.cost_scale, eta=eta)
    ok, ce = sv.solve(tau, cap, block)
    sv.close()
    return ok, ce


def test_server_results_equal_alone_and_budget_is_respected():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_33814_amd import bdrs
    sides = [16, 32, 24, 40, 16, 32, 48, 20]
    probs = [inputs.grid_problem(s, 800 + 2 * i, 801 + 2 * i) for i, s in enumerate(sides)]
    eta, tau, cap, block = 0.3, 0.02, 3000, 50
    ref = [alone(p, eta, tau, cap, block) for p in probs]
    # a pool that holds only a few requests at once forces queueing
    need = max(bdrs.workspace_size(p.m, p.n, 2) for p in probs)
    srv = bdrs.Server(pool_bytes=3 * need + (1 << 20), max_slots=4, block_iters=block)
    tickets = []
    peak = 0
    for i, p in enumerate(probs):
        tickets.append(srv.submit(p, eta=eta, tau=tau, max_iters=cap))
        if i % 3 == 2:
            time.sleep(0.01)                      # staggered arrivals
        peak = max(peak, srv.stats()["running"])
    res = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    assert st["running"] == 0 and st["queued"] == 0
    assert peak <= 4
    for (ok, ce), r in zip(ref, res):
        assert r["state"] == 2
        assert (r["status"] == bdrs.OK) == ok
        for key in ("k", "L", "U", "L_best", "U_best", "rel_gap_best"):
            assert r["cert"][key] == ce[key], key
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]


def test_server_rejects_and_isolates_bad_requests():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_33814_amd import bdrs
    srv = bdrs.Server(pool_bytes=64 << 20, max_slots=2, block_iters=50)
    big = inputs.random_problem(1 << 20, 1 << 20, 2, 1)
    assert bdrs.workspace_size(big.m, big.n, 2) > (64 << 20)
    with pytest.raises(bdrs.BdrsError) as ei:          # can never fit the pool
        srv.submit(big, max_iters=100)
    assert ei.value.status == bdrs.E_NOMEM
    good = inputs.grid_problem(16, 3, 4)
    with pytest.raises(bdrs.BdrsError) as ei:          # max_iters not a block multiple
        srv.submit(good, max_iters=75)
    assert ei.value.status == bdrs.E_INVALID
    bad = inputs.grid_problem(16, 5, 6)
    bad.r = bad.r.copy()
    bad.r[3] = -1.0                                     # contents are checked at submit
    tg = srv.submit(good, eta=0.3, tau=0.05, max_iters=2000)
    with pytest.raises(bdrs.BdrsError) as ei:
        srv.submit(bad, max_iters=100)
    assert ei.value.status == bdrs.E_INVALID and "r[3]" in str(ei.value)
    with pytest.raises(bdrs.BdrsError) as ei:          # omega must be > 0
        srv.submit(good, omega=0.0, max_iters=100)
    assert ei.value.status == bdrs.E_INVALID
    rg = srv.wait(tg)
    srv.close()
    assert rg["status"] in (bdrs.OK, bdrs.NOT_CONVERGED) and rg["cert"]["k"] >= 49


def test_size_aware_policy_runs_large_requests_one_at_a_time():
    """With big_work set, two large requests never overlap and a small request
    that arrived after the second large one is admitted before it; every
    result still equals the request solved alone."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_33814_amd import bdrs
    big1, big2 = inputs.grid_problem(24, 900, 901), inputs.grid_problem(24, 902, 903)  # 331776 entries
    small = inputs.grid_problem(8, 904, 905)                                              # 4096 entries
    eta, block = 0.3, 50
    srv = bdrs.Server(pool_bytes=64 << 20, max_slots=8, block_iters=block)
    srv.set_policy(1e5)
    t1 = srv.submit(big1, eta=eta, tau=0.0, max_iters=300)
    t2 = srv.submit(big2, eta=eta, tau=0.0, max_iters=300)
    t3 = srv.submit(small, eta=eta, tau=0.0, max_iters=100)
    r1, r2, r3 = srv.wait(t1), srv.wait(t2), srv.wait(t3)
    srv.close()
    assert r2["t_admit"] >= r1["t_done"]          # large requests do not overlap
    assert r3["t_admit"] <= r2["t_admit"]         # the small one passed the waiting large one
    for prob, r, cap in ((big1, r1, 300), (big2, r2, 300), (small, r3, 100)):
        _, ce = alone(prob, eta, 0.0, cap, block)
        assert r["cert"]["U"] == ce["U"] and r["cert"]["L"] == ce["L"] and r["cert"]["k"] == ce["k"]


def test_served_results_match_the_oracle():
    """Requests of grids 16x16 to 32x32 (eta = 1, stop at a 10% certified
    relative gap or after 600 iterations) served concurrently in a pool that
    holds a few at a time, each against the FP64 oracle's own run of
    Algorithm 1 with the certificate of Prop. 3 every block: the same
    stopping iteration, and the relative gap, U and L at that certificate
    within the trajectory bars (kappa2 r^2 <= 24 at these temperatures)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_33814_amd import bdrs
    import oracle_runs
    sides = [16, 24, 20, 32, 16, 24, 20, 28]
    probs = [inputs.grid_problem(s, 800 + 2 * i, 801 + 2 * i) for i, s in enumerate(sides)]
    eta, tau, cap, block = 1.0, 0.1, 600, 50
    refs = oracle_runs.run_many([(p, eta, 1.0, cap, block, tau) for p in probs])
    need = max(bdrs.workspace_size(p.m, p.n, 2) for p in probs)
    srv = bdrs.Server(pool_bytes=4 * need + (1 << 20), max_slots=4, block_iters=block)
    tickets = [srv.submit(p, eta=eta, tau=tau, max_iters=cap) for p in probs]
    res = [srv.wait(t) for t in tickets]
    srv.close()
    assert len({r["cert"]["k"] for r in res}) > 1
    for i, (r, ref) in enumerate(zip(res, refs)):
        reached = ref[0][-1]["rel_best"] <= tau
        assert r["status"] == (bdrs.OK if reached else bdrs.NOT_CONVERGED), (i, r["status"])
        print(f"served request {i} (side {sides[i]}):", oracle_runs.compare_final(r["cert"], ref, tau))


def test_set_policy_validates():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_33814_amd import bdrs
    srv = bdrs.Server(pool_bytes=1 << 20, max_slots=1, block_iters=10)
    with pytest.raises(bdrs.BdrsError):
        srv.set_policy(float("inf"))
    srv.set_policy(-1.0)   # back to arrival order
    srv.close()
