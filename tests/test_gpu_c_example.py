"""The C ABI driven from plain C (paper_2609_33814_amd/examples/solve_grid.c,
built by paper_2609_33814_amd/build.py): a separate process with its own HIP
allocations solves a 32x32 grid problem to a 1% certified gap, rounds the
state plan and exports the repaired plan densely in strips of rows; both
feasible costs must lie above the certified lower bound, and the dense
plan's row and column sums must match r and c."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

BIN = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2609_33814_amd", "examples", "solve_grid")


def test_c_example_solves_and_rounds():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert os.path.exists(BIN), "build the library first (python -m paper_2609_33814_amd.build)"
    res = subprocess.run([BIN, "32", "0.1", "1.0", "0.01"], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
    k, L, U, rel, rounded, secs, repaired, err = res.stdout.split()
    k, L, U, rel, rounded, repaired, err = int(k), float(L), float(U), float(rel), float(rounded), \
        float(repaired), float(err)
    assert (k + 1) % 50 == 0 and rel <= 0.01 and 0 < L <= U
    assert L <= rounded * (1 + 1e-9) and L <= repaired * (1 + 1e-9)
    assert err <= 1e-4
