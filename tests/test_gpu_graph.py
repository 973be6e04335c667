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
