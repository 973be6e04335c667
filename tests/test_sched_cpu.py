"""The solve server's scheduling pieces on the host (no GPU): the pool
allocator, the admission choice and the admission / block / retire loop
with a fake executor (tests/sched_driver.cpp, compiled here with g++ against
paper_2609_33814_amd/csrc/bdrs_sched.h, the header the server uses)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


# plain, then with the address and undefined-behaviour sanitizers (host code only)
@pytest.mark.parametrize("flags", [[], ["-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                                        "-fno-sanitize-recover=undefined"]], ids=["plain", "asan_ubsan"])
def test_scheduler_with_fake_executor(tmp_path, flags):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "sched_driver")
    src = os.path.join(ROOT, "tests", "sched_driver.cpp")
    inc = os.path.join(ROOT, "paper_2609_33814_amd", "csrc")
    build = subprocess.run([cxx, "-std=c++17", "-O1", "-Wall", "-Werror", *flags, "-I", inc, src, "-o", exe],
                           capture_output=True, text=True)
    if build.returncode != 0 and flags:
        pytest.skip("sanitizer runtime not available: " + build.stderr[-200:])
    assert build.returncode == 0, build.stderr
    res = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0 and res.stdout.strip().endswith("ok"), res.stdout + res.stderr
