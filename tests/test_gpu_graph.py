"""Captured iteration blocks: bdrs_step enqueues only kernels and keeps the
iteration counter on the device, so a captured block of iterations can be
replayed; every replay must equal the eager run bit for bit."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2609_33814_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu


def make(prob, stream):
    from paper_2609_33814_amd import bdrs
    d = torch.device("cuda:0")
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=d)
    return bdrs.Solver(t(prob.x, torch.float32), t(prob.y, torch.float32), t(prob.r, torch.float64),
                       t(prob.c, torch.float64), prob.cost_scale, eta=0.5, lam=1.5, stream=stream)


def test_graph_replays_match_eager_iterations():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    prob = inputs.grid_problem(40, 5, 6)
    s = torch.cuda.Stream()
    g_sv = make(prob, s)
    e_sv = make(prob, s)
    block = 10
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        g_sv.step(block)           # warm-up outside the capture
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=s):
        g_sv.step(block)           # captured, not executed
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        e_sv.step(block)
    for rep in range(4):
        graph.replay()
        with torch.cuda.stream(s):
            e_sv.step(block)       # eager work between the replays
            junk = torch.randn(1000, device="cuda").sum()  # unrelated eager kernels
        torch.cuda.synchronize()
        a, b = g_sv.get_state(), e_sv.get_state()
        assert a["k"] == b["k"] == block * (rep + 2)
        for key in ("la", "lb", "lb_prev", "lah", "lbh", "lt"):
            assert torch.equal(a[key], b[key]), (rep, key)
        del junk
    ca, cb = g_sv.certificate(), e_sv.certificate()
    assert ca["U"] == cb["U"] and ca["L"] == cb["L"]


def _solver(prob, graph, lam=1.0):
    from paper_2609_33814_amd import bdrs
    d = torch.device("cuda:0")
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=d)
    return bdrs.Solver(t(prob.x, torch.float32), t(prob.y, torch.float32), t(prob.r, torch.float64),
                       t(prob.c, torch.float64), prob.cost_scale, eta=0.1, lam=lam, graph=graph)


@pytest.mark.parametrize("lam,every", [(1.0, 50), (1.5, 50), (1.0, 20)])
def test_solve_block_graphs_match_eager_solve(lam, every):
    """bdrs_solve replays a captured graph for aligned blocks of cert_every
    iterations (50 and 20 here); with graphs off it launches every kernel
    itself.
    Both must agree bit for bit: aligned blocks, a first block that starts off
    the block grid (7 eager steps first) and a last block cut short by
    max_iters."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    prob = inputs.grid_problem(32, 11, 12)
    runs = []
    cap = 2 * every + 30
    for graph in (True, False):
        sv = _solver(prob, graph, lam)
        sv.step(7)
        ok1, ce1 = sv.solve(0.0, cap, every)   # eager to the grid, a block as graphs, eager tail
        ok2, ce2 = sv.solve(0.005, 2000, every)
        runs.append((ok1, ce1, ok2, ce2, sv.get_state(), sv.get_hints()))
    a, b = runs
    assert a[0] == b[0] and a[2] == b[2]
    for ca, cb in ((a[1], b[1]), (a[3], b[3])):
        for key in ca:   # bitwise: equal, or both NaN (fields a plain solve leaves unset)
            assert ca[key] == cb[key] or (ca[key] != ca[key] and cb[key] != cb[key]), (key, ca, cb)
    assert a[1]["k"] == 7 + cap - 1
    for key in ("la", "lb", "lb_prev", "lah", "lbh", "lt"):
        assert torch.equal(a[4][key], b[4][key]), key
    assert a[4]["k"] == b[4]["k"]
    for key in ("row", "col"):
        assert torch.equal(a[5][key], b[5][key]), key


def test_solve_logged_records_every_certificate(tmp_path):
    """solve_logged writes one JSON line per certificate and ends where one
    solve call ends, bit for bit."""
    import json
    from paper_2609_33814_amd import bdrs, inputs
    prob = inputs.grid_problem(32, 11, 12)
    d = torch.device("cuda:0")
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=d)
    mk = lambda: bdrs.Solver(t(prob.x, torch.float32), t(prob.y, torch.float32), t(prob.r, torch.float64),
                             t(prob.c, torch.float64), prob.cost_scale, eta=0.1)
    a, b = mk(), mk()
    path = str(tmp_path / "certs.jsonl")
    ok_a, ce_a = a.solve_logged(0.01, 5000, 50, path)
    ok_b, ce_b = b.solve(0.01, 5000, 50)
    assert ok_a and ok_b
    recs = [json.loads(line) for line in open(path)]
    assert [r["k"] for r in recs] == list(range(49, ce_b["k"] + 1, 50))
    assert all(x["rel_gap_best"] >= y["rel_gap_best"] for x, y in zip(recs, recs[1:]))
    assert all(x["t_wall"] <= y["t_wall"] for x, y in zip(recs, recs[1:]))
    for key in ("k", "L", "U", "rel_gap", "L_best", "U_best", "rel_gap_best", "delta"):
        assert ce_a[key] == ce_b[key] == recs[-1][key], key
    sa, sb = a.get_state(), b.get_state()
    for key in ("la", "lb", "lah"):
        assert torch.equal(sa[key], sb[key]), key
    a.close()
    b.close()


def test_solve_logged_from_a_misaligned_start(tmp_path):
    """After step(7) the first logged block runs to the next multiple of
    cert_every (k = 49), so the logged run certifies exactly where one
    solve call from k = 7 does and stops at the same iteration, bit for bit;
    a cap that is not a multiple of cert_every ends with the remainder."""
    import json
    from paper_2609_33814_amd import bdrs, inputs
    prob = inputs.grid_problem(32, 11, 12)
    d = torch.device("cuda:0")
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=d)
    mk = lambda: bdrs.Solver(t(prob.x, torch.float32), t(prob.y, torch.float32), t(prob.r, torch.float64),
                             t(prob.c, torch.float64), prob.cost_scale, eta=0.1)
    for tau, cap in ((0.01, 5000), (0.0, 180)):
        a, b = mk(), mk()
        a.step(7)
        b.step(7)
        path = str(tmp_path / f"certs_{cap}.jsonl")
        ok_a, ce_a = a.solve_logged(tau, cap, 50, path)
        ok_b, ce_b = b.solve(tau, cap, 50)
        assert ok_a == ok_b
        recs = [json.loads(line) for line in open(path)]
        ks = [r["k"] for r in recs]
        assert ks[0] == 49 and all(k % 50 == 49 for k in ks[:-1]), ks
        assert ks[-1] == ce_b["k"]
        if not ok_b:
            assert ce_b["k"] == 7 + cap - 1
        for key in ("k", "L", "U", "rel_gap", "L_best", "U_best", "rel_gap_best", "delta"):
            assert ce_a[key] == ce_b[key] == recs[-1][key], key
        assert a.iterations() == b.iterations() == ce_b["k"] + 1
        a.close()
        b.close()
