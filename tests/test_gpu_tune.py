"""Autotuner and tuned layouts: the split count changes only how the input
tiles are grouped into work items, so every count must give the oracle's
sweep (within the per-sweep tolerance), and bdrs_autotune must enter one of
its candidates into the table."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import lse  # noqa: E402
from paper_2609_33814_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def tensors(prob):
    d = dev()
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=d)
    return t(prob.x, torch.float32), t(prob.y, torch.float32), t(prob.r, torch.float64), t(prob.c, torch.float64)


@pytest.fixture
def table():
    from paper_2609_33814_amd import bdrs
    keep = bdrs.tune_table()
    yield bdrs
    bdrs.tune_clear()
    for e in keep:
        bdrs.tune_set(e)


@pytest.mark.parametrize("splits", [(1, 1), (3, 7), (25, 2), (64, 64)])
def test_every_split_count_matches_oracle(table, splits):
    bdrs = table
    prob = inputs.random_problem(1600, 1000, 2, 17)   # 25 and 16 tiles, ragged tail
    bdrs.tune_set(dict(dim=2, m=1600, n=1000, splits_row=splits[0], splits_col=splits[1]))
    x, y, r, c = tensors(prob)
    sv = bdrs.Solver(x, y, r, c, prob.cost_scale, eta=0.1)
    rng = np.random.default_rng(5)
    for transpose in (False, True):
        src, dst = (prob.y, prob.x) if transpose else (prob.x, prob.y)
        for eps in (1.0, 1e-3):
            w = rng.normal(0, 20, dst.shape[0])
            got = sv.lse(torch.as_tensor(w, device=dev()), eps, transpose=transpose).cpu().numpy()
            ref = lse.implicit_lse(src, dst, prob.cost_scale, eps, w)
            err = np.max(np.abs(got - ref)) / max(1.0, np.max(np.abs(ref)))
            assert err <= 1e-5, (splits, transpose, eps, err)
    sv.close()


def test_solves_agree_across_split_counts(table):
    bdrs = table
    prob = inputs.grid_problem(40, 3, 4)
    x, y, r, c = tensors(prob)
    certs = []
    for splits in ((1, 1), (5, 9)):
        bdrs.tune_set(dict(dim=2, m=1600, n=1600, splits_row=splits[0], splits_col=splits[1]))
        sv = bdrs.Solver(x, y, r, c, prob.cost_scale, eta=0.1)
        _, ce = sv.solve(0.0, 200, 50)
        certs.append(ce)
        sv.close()
    a, b = certs
    assert abs(a["U"] - b["U"]) <= 1e-5 * abs(b["U"])
    assert abs(a["L"] - b["L"]) <= 1e-5 * abs(b["L"])


def test_autotune_enters_a_candidate(table):
    bdrs = table
    prob = inputs.grid_problem(64, 9, 10)
    x, y, r, c = tensors(prob)
    e = bdrs.autotune(x, y, r, c, prob.cost_scale, eta=0.1, rounds=5)
    assert e["dim"] == 2 and e["m"] == e["n"] == 4096
    assert e["candidates"] >= 2
    assert 0 < e["us_row"] <= e["us_row_default"] + 1e-9
    assert 0 < e["us_col"] <= e["us_col_default"] + 1e-9
    assert 1 <= e["splits_row"] <= 64 and 1 <= e["splits_col"] <= 64
    tab = [t for t in bdrs.tune_table() if (t["dim"], t["m"], t["n"]) == (2, 4096, 4096)]
    assert len(tab) == 1 and tab[0]["splits_row"] == e["splits_row"]
    # a solver made afterwards runs with the tuned layout and certifies
    sv = bdrs.Solver(x, y, r, c, prob.cost_scale, eta=0.1)
    _, ce = sv.solve(0.0, 100, 50)
    assert np.isfinite(ce["U"]) and ce["L"] <= ce["U"] * (1 + 1e-9)
    sv.close()
