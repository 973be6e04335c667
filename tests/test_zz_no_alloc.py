"""bdrs_batch_solve_static (the batched solve whose work lists live in the
library's static device array, for callers that cannot allocate) against
bdrs_batch_solve with a caller workspace: bitwise the same certificates,
statuses and final states on two calls in a row, the second with fewer and
smaller problems; a batch whose work lists exceed the array is refused on the
host before any device work."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2609_33814_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu


def make(prob, eta=0.5):
    from paper_2609_33814_amd import bdrs
    d = torch.device("cuda:0")
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=d)
    return bdrs.Solver(t(prob.x, torch.float32), t(prob.y, torch.float32), t(prob.r, torch.float64),
                       t(prob.c, torch.float64), prob.cost_scale, eta=eta)


def static_call(solvers, tau, cap, every):
    """bdrs_batch_solve_static through the C ABI; returns (status, certs, statuses)."""
    from paper_2609_33814_amd import bdrs
    n = len(solvers)
    arr = (ctypes.c_void_p * n)(*[s.handle.value for s in solvers])
    outs = (bdrs.Cert * n)()
    sts = (ctypes.c_int32 * n)()
    st = bdrs.lib().bdrs_batch_solve_static(arr, n, float(tau), 1, int(cap), int(every), outs, sts)
    return st, [o.as_dict() for o in outs], list(sts)


def test_static_batch_equals_workspace_batch_twice():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_33814_amd import bdrs
    tau, cap, every = 0.05, 2000, 50
    calls = [([16, 32, 24, 48, 20, 32], 900), ([12, 16, 8], 960)]   # the second smaller
    for sides, seed in calls:
        probs = [inputs.grid_problem(s, seed + 2 * i, seed + 1 + 2 * i) for i, s in enumerate(sides)]
        a = [make(p) for p in probs]
        b = [make(p) for p in probs]
        st_a, certs_a, sts_a = bdrs.batch_solve(a, tau, cap, every, use_graph=False)
        st_b, certs_b, sts_b = static_call(b, tau, cap, every)
        assert st_b == st_a and sts_b == sts_a, (st_a, st_b, sts_a, sts_b)
        assert len({c["k"] for c in certs_b}) > 1          # members retired at different certificates
        for i, (ca, cb) in enumerate(zip(certs_a, certs_b)):
            for key in ("k", "L", "U", "L_best", "U_best", "rel_gap_best", "delta", "cost_Z", "n_nonfinite",
                        "negative_gap"):
                assert ca[key] == cb[key], (sides, i, key, ca[key], cb[key])
            sa, sb = a[i].get_state(), b[i].get_state()
            assert sa["k"] == sb["k"] == ca["k"] + 1
            for key in ("la", "lb", "lb_prev", "lah", "lbh", "lt"):
                assert torch.equal(sa[key], sb[key]), (sides, i, key)
        for s in a + b:
            s.close()


def test_static_batch_refuses_work_lists_beyond_the_array():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_33814_amd import bdrs
    prob = inputs.grid_problem(512, 970, 971)
    solvers = []
    size = ctypes.c_size_t()
    while True:
        solvers.append(make(prob))
        arr = (ctypes.c_void_p * len(solvers))(*[s.handle.value for s in solvers])
        assert bdrs.lib().bdrs_batch_workspace_size(arr, len(solvers), ctypes.byref(size)) == bdrs.OK
        if size.value > bdrs.BATCH_STATIC_BYTES:
            break
        assert len(solvers) < 200
    st, _, _ = static_call(solvers, 0.01, 100, 50)
    assert st == bdrs.E_NOMEM
    assert "static array" in bdrs.last_error()
    assert all(s.iterations() == 0 for s in solvers)     # nothing ran
    for s in solvers:
        s.close()
