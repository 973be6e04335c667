"""Builds the gfx950 shared library libbdrs.so in-tree with hipcc.

Usage: python -m paper_2609_33814_amd.build  (or call build()).
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libbdrs.so")
SOURCES = ["bdrs_kernels.hip", "bdrs_api.hip", "bdrs_server.hip", "bdrs_tune.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    "--offload-arch=gfx950",
    # no packed FP32 (v_pk_*_f32) anywhere: the compiler must not form them
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"),
]


EXAMPLE_SRC = os.path.join(PKG, "examples", "solve_grid.c")
EXAMPLE_BIN = os.path.join(PKG, "examples", "solve_grid")


def build_example(verbose: bool = False) -> str:
    """The plain-C example against the C ABI (host compiler, links libbdrs.so)."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    tmp = EXAMPLE_BIN + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(rocm, "include"),
           EXAMPLE_SRC, "-L", PKG, "-lbdrs", "-L", os.path.join(rocm, "lib"), "-lamdhip64", "-lm",
           "-Wl,-rpath,$ORIGIN/..", "-Wl,-rpath," + os.path.join(rocm, "lib"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("gcc failed building the C example")
    os.replace(tmp, EXAMPLE_BIN)
    return EXAMPLE_BIN


def build(verbose: bool = False) -> str:
    """Compiles every HIP source into libbdrs.so (and the C example); returns the library path."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libbdrs.so")
    os.replace(tmp, LIB)
    build_example(verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
