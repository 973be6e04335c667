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


def test_workspace_is_linear_in_points(saved_table):
    # heuristic split counts (the tuning table is emptied by the fixture)
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
    ("omega", -1.0, bdrs.E_INVALID, "omega"), ("omega", 0.0, bdrs.E_INVALID, "omega"),
    ("omega", float("inf"), bdrs.E_INVALID, "omega"),
    ("workspace", 0, bdrs.E_INVALID, "workspace"),
    ("workspace", 0x10010, bdrs.E_INVALID, "aligned"),
    ("workspace_bytes", 100, bdrs.E_NOMEM, "workspace"),
    ("flags", 0x80, bdrs.E_INVALID, "flags"),
    ("flags", 8, bdrs.E_INVALID, "DEBIASED"),
    ("flags", 8 | 2, bdrs.E_INVALID, "DEBIASED"),
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


# ----------------------------------------------------------------------------
# batch / server argument checks (host only)
# ----------------------------------------------------------------------------
def test_batch_rejects_bad_arguments_on_host():
    L = bdrs.lib()
    out = ctypes.c_size_t()
    assert L.bdrs_batch_workspace_size(None, 1, ctypes.byref(out)) == bdrs.E_INVALID
    arr = (ctypes.c_void_p * 2)(None, None)
    assert L.bdrs_batch_workspace_size(arr, 0, ctypes.byref(out)) == bdrs.E_INVALID
    assert "count" in bdrs.last_error()
    assert L.bdrs_batch_workspace_size(arr, 2, ctypes.byref(out)) == bdrs.E_INVALID
    assert "NULL" in bdrs.last_error()
    ce = (bdrs.Cert * 2)()
    sts = (ctypes.c_int32 * 2)()
    assert L.bdrs_batch_solve(arr, 2, None, 0, 0.01, 1, 100, 50, 1, ce, sts) == bdrs.E_INVALID


@pytest.mark.parametrize("pool,nbytes,slots,block,word", [
    (0, 1 << 20, 4, 50, "pool"), (0x10010, 1 << 20, 4, 50, "pool"), (0x10000, 16, 4, 50, "pool_bytes"),
    (0x10000, 1 << 20, 0, 50, "max_slots"), (0x10000, 1 << 20, 4, 0, "block_iters"),
])
def test_server_create_validates_on_host(pool, nbytes, slots, block, word):
    h = ctypes.c_void_p()
    assert bdrs.lib().bdrs_server_create(pool, nbytes, slots, block, ctypes.byref(h)) == bdrs.E_INVALID
    assert word in bdrs.last_error()
    assert not h.value


def test_server_calls_reject_null_server():
    L = bdrs.lib()
    t = ctypes.c_uint64()
    res = bdrs.Result()
    assert L.bdrs_server_submit(None, None, ctypes.byref(t)) == bdrs.E_INVALID
    assert L.bdrs_server_poll(None, 1, ctypes.byref(res)) == bdrs.E_INVALID
    assert L.bdrs_server_wait(None, 1, ctypes.byref(res)) == bdrs.E_INVALID
    assert L.bdrs_server_destroy(None) in (bdrs.OK, bdrs.E_INVALID)
    assert L.bdrs_server_set_policy(None, 1e9) == bdrs.E_INVALID


def test_plan_and_round_reject_null_solver():
    L = bdrs.lib()
    st = bdrs.RoundStats()
    assert L.bdrs_round(None, ctypes.byref(st)) == bdrs.E_INVALID
    ps = bdrs.PlanStats()
    assert L.bdrs_plan(None, None, None, None, ctypes.byref(ps)) == bdrs.E_INVALID


# ----------------------------------------------------------------------------
# tuning table (host only)
# ----------------------------------------------------------------------------
@pytest.fixture
def saved_table():
    keep = bdrs.tune_table()
    bdrs.tune_clear()
    yield
    bdrs.tune_clear()
    for e in keep:
        bdrs.tune_set(e)


def test_tune_table_roundtrip_and_layout(saved_table, tmp_path):
    base = bdrs.workspace_size(16384, 16384, 2)
    bdrs.tune_set(dict(dim=2, m=16384, n=16384, splits_row=256, splits_col=2))
    tab = bdrs.tune_table()
    assert len(tab) == 1 and tab[0]["splits_row"] == 256 and tab[0]["splits_col"] == 2
    # 256 splits x 16384 outputs of 24-byte partial records dominate the workspace
    assert bdrs.workspace_size(16384, 16384, 2) >= 256 * 16384 * 24 > base
    # other shapes are untouched
    assert bdrs.workspace_size(16384, 16385, 2) < 256 * 16384 * 24
    # replace, not append
    bdrs.tune_set(dict(dim=2, m=16384, n=16384, splits_row=3, splits_col=3))
    assert len(bdrs.tune_table()) == 1 and bdrs.tune_table()[0]["splits_row"] == 3
    path = str(tmp_path / "t.json")
    bdrs.save_tuning(path)
    bdrs.tune_clear()
    assert bdrs.tune_table() == []
    assert bdrs.load_tuning(path) == 1
    assert bdrs.tune_table()[0]["splits_col"] == 3


def test_tune_set_normalises_split_counts(saved_table):
    # 100 points -> 2 input tiles: at most 2 splits own a tile
    bdrs.tune_set(dict(dim=3, m=100, n=100, splits_row=50, splits_col=1))
    e = bdrs.tune_table()[0]
    assert e["splits_row"] == 2 and e["splits_col"] == 1
    # 20 tiles and 7 asked: ceil(20/7) = 3 tiles per split -> 7 splits own a tile
    bdrs.tune_set(dict(dim=2, m=1280, n=1280, splits_row=7, splits_col=6))
    e = bdrs.tune_table()[1]
    assert e["splits_row"] == 7 and e["splits_col"] == 5  # 6 asked: 4 tiles per split -> 5


@pytest.mark.parametrize("field,value", [("dim", 0), ("dim", 4), ("m", 0), ("n", -1),
                                         ("splits_row", 0), ("splits_col", -2)])
def test_tune_set_rejects_bad_entries(saved_table, field, value):
    e = dict(dim=2, m=64, n=64, splits_row=1, splits_col=1)
    e[field] = value
    with pytest.raises(bdrs.BdrsError):
        bdrs.tune_set(e)
    assert bdrs.tune_table() == []


def test_tune_get_index_out_of_range(saved_table):
    e = bdrs.TuneEntry()
    n = ctypes.c_int32()
    assert bdrs.lib().bdrs_tune_get(0, ctypes.byref(e), ctypes.byref(n)) == bdrs.E_INVALID
    assert n.value == 0


def test_autotune_validates_on_host(saved_table):
    L = bdrs.lib()
    need = ctypes.c_size_t()
    p = _good()
    assert L.bdrs_autotune_workspace_size(ctypes.byref(p), ctypes.byref(need)) == bdrs.OK
    assert need.value >= bdrs.workspace_size(8, 9, 2)
    e = bdrs.TuneEntry()
    p = _good(workspace_bytes=need.value)
    assert L.bdrs_autotune(ctypes.byref(p), 0, ctypes.byref(e)) == bdrs.E_INVALID
    assert "rounds" in bdrs.last_error()
    big = ctypes.c_size_t()
    pb = bdrs.make_params(1 << 20, 1 << 20, 3)
    assert L.bdrs_autotune_workspace_size(ctypes.byref(pb), ctypes.byref(big)) == bdrs.OK
    pb = bdrs.make_params(1 << 20, 1 << 20, 3, 0x1000, 0x2000, 0x3000, 0x4000, 1.0, 0.1, 1.0, 1.0,
                          0x10000, bdrs.workspace_size(1 << 20, 1 << 20, 3))
    if big.value > bdrs.workspace_size(1 << 20, 1 << 20, 3):
        assert L.bdrs_autotune(ctypes.byref(pb), 5, ctypes.byref(e)) == bdrs.E_NOMEM
    import torch
    if not torch.cuda.is_available():
        assert L.bdrs_autotune(ctypes.byref(p), 5, ctypes.byref(e)) == bdrs.E_DEVICE
    assert bdrs.tune_table() == []


def test_variant_flags_need_lambda_one():
    p = _good(flags=2, lam=1.5)
    h = ctypes.c_void_p()
    assert bdrs.lib().bdrs_create(ctypes.byref(p), ctypes.byref(h)) == bdrs.E_INVALID
    assert "lambda" in bdrs.last_error()


def test_keep_best_state_adds_a_linear_region(saved_table):
    m, n = 1000, 1200
    a = bdrs.workspace_size(m, n, 2)
    b = bdrs.workspace_size(m, n, 2, bdrs.F_KEEP_BEST_STATE)
    # 7 float64 state vectors and 2 int32 hint vectors (padded), 256-byte aligned
    assert a < b <= a + (7 * 8 + 2 * 4) * (m + n + 2 * 256) + 9 * 256


def test_restore_best_rejects_null_solver():
    assert bdrs.lib().bdrs_restore_best(None, None) == bdrs.E_INVALID
    assert bdrs.last_error()


def test_export_plan_rejects_null_solver_and_bad_kind():
    L = bdrs.lib()
    assert L.bdrs_export_plan(None, bdrs.PLAN_ROUNDED, None, None, None, None, None) == bdrs.E_INVALID
    assert "NULL" in bdrs.last_error()
    assert L.bdrs_plan_entries(None, None, None, None, None, 1.0, 0, 0, None) == bdrs.E_INVALID
    assert bdrs.last_error()


def test_static_batch_rejects_bad_arguments_on_host():
    L = bdrs.lib()
    ce = (bdrs.Cert * 2)()
    sts = (ctypes.c_int32 * 2)()
    assert L.bdrs_batch_solve_static(None, 1, 0.01, 1, 100, 50, ce, sts) == bdrs.E_INVALID
    arr = (ctypes.c_void_p * 2)(None, None)
    assert L.bdrs_batch_solve_static(arr, 0, 0.01, 1, 100, 50, ce, sts) == bdrs.E_INVALID
    assert "count" in bdrs.last_error()
    assert L.bdrs_batch_solve_static(arr, 2, 0.01, 1, 100, 50, ce, sts) == bdrs.E_INVALID
    assert "NULL" in bdrs.last_error()
