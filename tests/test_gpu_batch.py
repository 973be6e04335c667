"""Batched solving: each problem's result in a batch equals its result alone,
bit for bit (same kernels' arithmetic, same splits), with and without a
captured iteration block; problems retire at their own certificates."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2609_33814_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu


def make(prob, eta=1.0, lam=1.0):
    from paper_2609_33814_amd import bdrs
    d = torch.device("cuda:0")
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=d)
    return bdrs.Solver(t(prob.x, torch.float32), t(prob.y, torch.float32), t(prob.r, torch.float64),
                       t(prob.c, torch.float64), prob.cost_scale, eta=eta, lam=lam)


def problems():
    sides = [16, 32, 24, 48, 20, 32]
    return [inputs.grid_problem(s, 700 + 2 * i, 701 + 2 * i) for i, s in enumerate(sides)]


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_equals_alone_bitwise(use_graph):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_33814_amd import bdrs
    probs = problems()
    tau, cap, ce_every = 0.05, 2000, 50
    alone = []
    for p in probs:
        sv = make(p, eta=0.5)
        ok, ce = sv.solve(tau, cap, ce_every)
        alone.append((ok, ce, sv.get_state()))
    batch = [make(p, eta=0.5) for p in probs]
    st, certs, sts = bdrs.batch_solve(batch, tau, cap, ce_every, use_graph=use_graph)
    ks = set()
    for i, (ok, ce, state) in enumerate(alone):
        assert (sts[i] == bdrs.OK) == ok, i
        b = certs[i]
        ks.add(b["k"])
        for key in ("k", "L", "U", "L_best", "U_best", "rel_gap_best", "delta"):
            assert b[key] == ce[key], (i, key, b[key], ce[key])
        bs = batch[i].get_state()
        assert bs["k"] == state["k"]
        for key in ("la", "lb", "lb_prev", "lah", "lbh", "lt"):
            assert torch.equal(bs[key], state[key]), (i, key)
    assert len(ks) > 1          # problems retired at different certificates


def test_batch_rejects_misaligned_and_mixed_dims():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_33814_amd import bdrs
    a = make(inputs.grid_problem(16, 1, 2))
    b = make(inputs.random_problem(50, 60, 3, 3))
    with pytest.raises(bdrs.BdrsError) as ei:
        bdrs.batch_solve([a, b], 0.01, 100, 50)
    assert ei.value.status == bdrs.E_INVALID
    a.step(7)
    c = make(inputs.grid_problem(16, 3, 4))
    with pytest.raises(bdrs.BdrsError) as ei:
        bdrs.batch_solve([a, c], 0.01, 100, 50)
    assert ei.value.status == bdrs.E_STATE


def test_batched_results_match_the_oracle():
    """Every problem of a mixed batch (grids 16x16 to 32x32, eta = 1,
    captured 50-iteration blocks, stop at a 5% certified relative gap or
    after 600 iterations) against the FP64 oracle's own run of Algorithm 1
    with the certificate of Prop. 3 every 50 iterations: the same stopping
    iteration, and the relative gap, U and L at that certificate within the
    trajectory bars.  At these temperatures kappa2 r^2 <= 24 (r the tile
    radius), where the float32 trajectories stay within the bars (the eta =
    0.1 stop parity test covers the low-temperature end)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_33814_amd import bdrs
    import oracle_runs
    sides = [16, 20, 24, 32, 16, 24]
    probs = [inputs.grid_problem(s, 700 + 2 * i, 701 + 2 * i) for i, s in enumerate(sides)]
    eta, tau, cap, every = 1.0, 0.05, 600, 50
    refs = oracle_runs.run_many([(p, eta, 1.0, cap, every, tau) for p in probs])
    batch = [make(p, eta=eta) for p in probs]
    st, certs, sts = bdrs.batch_solve(batch, tau, cap, every, use_graph=True)
    assert st == bdrs.NOT_CONVERGED and sts.count(bdrs.OK) >= 1
    assert len({c["k"] for c in certs}) > 1          # problems retired at different certificates
    for i, (ce, ref) in enumerate(zip(certs, refs)):
        print(f"batch member {i} (side {sides[i]}):", oracle_runs.compare_final(ce, ref, tau))
        assert ce["negative_gap"] == 0
        assert (sts[i] == bdrs.OK) == (ref[0][-1]["rel_best"] <= tau)


def test_batched_256_member_certificate_matches_the_oracle():
    """A batch with a 256x256 member (65536 points per side, 4.3e9 implicit
    entries per sweep) next to 64x64 and 128x128 ones, eta = 0.1, 300
    iterations in captured 50-iteration blocks: each member's fused
    certificate at k = 299 against Prop. 3 / Algorithm 2 evaluated by the
    oracle over all entries from the member's own state (the bars of a
    certificate from an identical state)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_33814_amd import bdrs
    from oracle import alg1, certificate
    probs = [inputs.grid_problem(s, 4100 + 2 * i, 4101 + 2 * i) for i, s in enumerate([256, 64, 128])]
    eta, iters, every = 0.1, 300, 50
    batch = [make(p, eta=eta) for p in probs]
    st, certs, sts = bdrs.batch_solve(batch, 0.0, iters, every, use_graph=True)
    eps = alg1.schedule(eta, 1.0, iters - 1)
    for p, sv, ce in zip(probs, batch, certs):
        gs = sv.get_state()
        assert ce["k"] == iters - 1 and gs["k"] == iters
        npy = lambda key: gs[key].cpu().numpy()
        ref = certificate.certificate(p.x, p.y, p.cost_scale, p.r, p.c, npy("lah"), npy("lbh"), npy("lt"), eps,
                                      workers=16)
        dU = abs(ce["U"] - ref["U"]) / ref["U"]
        print(f"batched {p.m} points: dL {abs(ce['L'] - ref['L']) / abs(ref['L']):.1e} dU {dU:.1e} "
              f"ddelta {abs(ce['delta'] - ref['delta']):.1e} gap {ce['rel_gap']:.6f} vs {ref['rel']:.6f}")
        assert abs(ce["L"] - ref["L"]) <= 1e-9 * abs(ref["L"])
        assert dU <= 1e-6
        assert abs(ce["delta"] - ref["delta"]) <= 1e-4 * ref["delta"] + 2e-6
        assert abs(ce["rel_gap"] - ref["rel"]) <= 1e-3 * abs(ref["rel"])
        assert ce["n_nonfinite"] == 0 and ce["negative_gap"] == 0
