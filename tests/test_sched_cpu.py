"""The solve server's scheduling pieces on the host (no GPU): the pool
allocator, the admission choice and the admission / block / retire loop
with a fake executor (tests/sched_driver.cpp, compiled here with g++ against
paper_2609_33814_amd/csrc/bdrs_sched.h, the header the server uses)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_scheduler_with_fake_executor(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "sched_driver")
    src = os.path.join(ROOT, "tests", "sched_driver.cpp")
    inc = os.path.join(ROOT, "paper_2609_33814_amd", "csrc")
    subprocess.run([cxx, "-std=c++17", "-O1", "-Wall", "-Werror", "-I", inc, src, "-o", exe],
                   check=True, capture_output=True, text=True)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0 and res.stdout.strip().endswith("ok"), res.stdout + res.stderr
