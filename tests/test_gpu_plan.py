"""State-plan outputs (row / column sums, marginal-error statistics,
barycentric projection) of the HIP path against the oracle, evaluated on the
GPU's own dual state so that only the plan evaluation is compared.

Tolerances: the sums are exp(log alpha + LSE), so a float32 sweep's LSE
error (<= 1e-5 relative to max(1, |LSE|), the per-sweep bar) becomes the
same relative error of each sum; the barycentre is a convex combination of
target points, and its float32 accumulation (coordinates below 2^8, relative
rounding ~1e-7 per term and the tile-relative weights) keeps the error below
1e-5 of the coordinate span.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import plan  # noqa: E402
from paper_2609_33814_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def solver_for(prob, eta, lam=1.0):
    from paper_2609_33814_amd import bdrs
    d = dev()
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=d)
    return bdrs.Solver(t(prob.x, torch.float32), t(prob.y, torch.float32), t(prob.r, torch.float64),
                       t(prob.c, torch.float64), prob.cost_scale, eta=eta, lam=lam)


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


CASES = [
    ("grid32", lambda: inputs.c1_problem(), 1.0, 1.0, 60),
    ("grid24_obdrs", lambda: inputs.grid_problem(24, 7, 8), 0.3, 1.99, 40),
    ("rand_ragged_d3", lambda: inputs.random_problem(700, 333, 3, 9), 0.5, 1.5, 25),
    ("rand_d1", lambda: inputs.random_problem(130, 200, 1, 10), 0.2, 1.0, 30),
]


@pytest.mark.parametrize("name,make,eta,lam,iters", CASES, ids=[c[0] for c in CASES])
def test_plan_matches_oracle(name, make, eta, lam, iters):
    prob = make()
    sv = solver_for(prob, eta, lam)
    sv.step(iters)
    st = sv.get_state()
    la, lb = st["la"].cpu().numpy(), st["lb"].cpu().numpy()
    out = sv.plan()
    eps = plan.plan_temperature(eta, lam, iters)
    assert out["stats"]["k"] == iters and abs(out["stats"]["eps"] - eps) <= 1e-15 * eps
    row = plan.row_marginal(prob.x, prob.y, prob.cost_scale, eps, la, lb)
    col = plan.col_marginal(prob.x, prob.y, prob.cost_scale, eps, la, lb)
    bary = plan.barycentric(prob.x, prob.y, prob.cost_scale, eps, lb)
    lse_scale = max(1.0, float(np.max(np.abs(np.log(row) - la))), float(np.max(np.abs(np.log(col) - lb))))
    tol = 1e-5 * lse_scale
    assert rel(out["row"].cpu().numpy(), row) <= tol
    assert rel(out["col"].cpu().numpy(), col) <= tol
    span = float(np.ptp(prob.y.astype(np.float64), axis=0).max())
    assert np.max(np.abs(out["bary"].cpu().numpy() - bary)) <= 1e-5 * span
    ref = plan.marginal_stats(row, col, prob.r, prob.c)
    got = out["stats"]
    assert abs(got["mass"] - ref["mass"]) <= tol * ref["mass"]
    # each sum is accurate to `tol` relative, so an error statistic moves by
    # at most tol times the same statistic of the sums themselves
    bound = dict(row_l1=row.sum(), col_l1=col.sum(), row_max_abs=row.max(), col_max_abs=col.max(),
                 row_max_rel=(row / prob.r).max(), col_max_rel=(col / prob.c).max())
    for key, b in bound.items():
        assert abs(got[key] - ref[key]) <= tol * float(b) + 1e-15, key
    sv.close()


def test_bdrs_plan_column_sums_are_c_and_iteration_unchanged():
    """lambda = 1: the plan's column sums are c (Sec. 2); evaluating the plan
    leaves the following iterations bit for bit as without it."""
    prob = inputs.grid_problem(40, 3, 4)
    a = solver_for(prob, 0.1)
    b = solver_for(prob, 0.1)
    a.step(100)
    b.step(100)
    out = a.plan()
    c = prob.c
    assert np.max(np.abs(out["col"].cpu().numpy() - c) / c) <= 1e-4
    assert out["stats"]["col_max_rel"] <= 1e-4
    a.step(50)
    b.step(50)
    sa, sb = a.get_state(), b.get_state()
    for key in ("la", "lb", "lb_prev", "lah", "lbh", "lt"):
        assert torch.equal(sa[key], sb[key]), key
    assert a.certificate()["U"] == b.certificate()["U"]


def test_plan_needs_an_iteration():
    from paper_2609_33814_amd import bdrs
    prob = inputs.grid_problem(8, 1, 2)
    sv = solver_for(prob, 1.0)
    with pytest.raises(bdrs.BdrsError) as ei:
        sv.plan()
    assert ei.value.status == bdrs.E_STATE


def test_full_size_colour_barycentre_sampled_rows():
    """1024x1024 colour clouds after a few iterations: barycentres of sampled
    source points against the oracle."""
    prob = inputs.c3_problem()
    sv = solver_for(prob, 0.1)
    sv.step(3)
    st = sv.get_state()
    lb = st["lb"].cpu().numpy()
    out = sv.plan(marginals=False)
    eps = plan.plan_temperature(0.1, 1.0, 3)
    rows = np.random.default_rng(4).choice(prob.m, 48, replace=False)
    ref = np.concatenate([plan.barycentric(prob.x, prob.y, prob.cost_scale, eps, lb, rows=rows[a:a + 16])
                          for a in range(0, rows.size, 16)])
    got = out["bary"].cpu().numpy()[rows]
    assert np.max(np.abs(got - ref)) <= 1e-5
    assert np.isfinite(out["stats"]["row_l1"]) and out["stats"]["mass"] > 0
