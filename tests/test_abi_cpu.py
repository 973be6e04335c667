"""C-ABI boundary checks that need no GPU: symbols, sizes, host-side validation."""
import ctypes
import os
import re

import pytest

from paper_2609_33814_amd import bdrs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            names |= set(re.findall(r"^\s*(?:BDRS_API\s+)?(?:bdrs_status|const char\s*\*)\s*(bdrs_\w+)\s*\(", src, re.M))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = bdrs.lib()
    declared = header_functions()
    assert len(declared) >= 10
    for name in declared:
        assert hasattr(L, name), name
    assert set(declared) >= set(bdrs.EXPORTS)
    assert bdrs.lib().bdrs_version().decode().startswith("bdrs")


def test_workspace_is_linear_in_points():
    a = bdrs.workspace_size(1024, 1024, 2)
    b = bdrs.workspace_size(16384, 16384, 2)
    c = bdrs.workspace_size(1 << 20, 1 << 20, 3)
    assert 0 < a < b < c
    # O(m + n): well under 200 bytes per point at 1M points per side
    assert c / (2 << 20) < 200


@pytest.mark.parametrize("m,n,dim", [(0, 4, 2), (4, 0, 2), (4, 4, 0), (4, 4, 4), (-3, 4, 2)])
def test_workspace_size_rejects_bad_sizes(m, n, dim):
    out = ctypes.c_size_t()
    p = bdrs.make_params(m, n, dim)
    assert bdrs.lib().bdrs_workspace_size(ctypes.byref(p), ctypes.byref(out)) == bdrs.E_INVALID
    assert bdrs.last_error()


def _good(**kw):
    ws = bdrs.workspace_size(8, 9, 2)
    base = dict(m=8, n=9, dim=2, x=0x1000, y=0x2000, r=0x3000, c=0x4000, cost_scale=1.0,
                eta=1.0, lam=1.0, omega=1.0, workspace=0x10000, workspace_bytes=ws)
    base.update(kw)
    return bdrs.make_params(**base)


@pytest.mark.parametrize("field,value,code,word", [
    ("x", 0, bdrs.E_INVALID, "x"), ("y", 0, bdrs.E_INVALID, "y"),
    ("r", 0, bdrs.E_INVALID, "r"), ("c", 0, bdrs.E_INVALID, "c"),
    ("cost_scale", 0.0, bdrs.E_INVALID, "cost_scale"),
    ("cost_scale", float("nan"), bdrs.E_INVALID, "cost_scale"),
    ("eta", -1.0, bdrs.E_INVALID, "eta"), ("eta", float("inf"), bdrs.E_INVALID, "eta"),
    ("lam", 0.99, bdrs.E_INVALID, "lambda"), ("lam", 2.0, bdrs.E_INVALID, "lambda"),
    ("omega", -1.0, bdrs.E_INVALID, "omega"),
    ("workspace", 0, bdrs.E_INVALID, "workspace"),
    ("workspace", 0x10010, bdrs.E_INVALID, "aligned"),
    ("workspace_bytes", 100, bdrs.E_NOMEM, "workspace"),
    ("flags", 0x80, bdrs.E_INVALID, "flags"),
])
def test_create_validates_before_any_device_call(field, value, code, word):
    p = _good(**{field: value})
    h = ctypes.c_void_p(1)
    st = bdrs.lib().bdrs_create(ctypes.byref(p), ctypes.byref(h))
    assert st == code
    assert word in bdrs.last_error()
    assert not h.value


def test_create_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    p = _good()
    h = ctypes.c_void_p()
    assert bdrs.lib().bdrs_create(ctypes.byref(p), ctypes.byref(h)) == bdrs.E_DEVICE
    assert "device" in bdrs.last_error()


def test_null_handles_are_rejected():
    L = bdrs.lib()
    ce = bdrs.Cert()
    assert L.bdrs_step(None, 1) == bdrs.E_INVALID
    assert L.bdrs_certificate(None, ctypes.byref(ce)) == bdrs.E_INVALID
    assert L.bdrs_solve(None, 0.01, 1, 10, 5, ctypes.byref(ce)) == bdrs.E_INVALID
    assert L.bdrs_destroy(None) == bdrs.OK
    assert L.bdrs_create(None, None) == bdrs.E_INVALID
