"""CPU checks of the C-ABI library: it loads, exports every entry point the
header declares, and rejects bad arguments on the host before touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_2606_11390_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gs.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_five_path_calls():
    names = _declared()
    for n in ("gs_project", "gs_bin_sort", "gs_rasterize_fwd", "gs_rasterize_bwd", "gs_project_bwd"):
        assert n in names


def test_library_loads_and_exports_every_declared_symbol():
    L = B.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert set(_declared()) == set(B.exported_symbols())
    assert L.gs_abi_version() == B.GS_ABI_VERSION
    assert L.gs_strerror(0) == b"ok"
    assert L.gs_strerror(-4) == b"workspace too small"


def _sizes(*wh):
    import numpy as np
    a = np.asarray(wh, np.int32).reshape(-1)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def test_host_side_argument_checks():
    L = B.lib()
    p = ctypes.c_void_p(16)          # never dereferenced: every call below fails its checks
    sz, szp = _sizes(64, 48)
    # gs_project: negative N, bad degree, bad tile, bad view size, bad near/far
    args = lambda **kw: [kw.get("means", p), p, p, p, p, kw.get("n", 10), kw.get("deg", 0), p, p,
                         kw.get("sizes", szp), kw.get("V", 1), kw.get("near", 0.01), kw.get("far", 1e10),
                         0.3, kw.get("tile", 16), kw.get("mode", 0), p, p, p, p, p, p, None, None]
    assert L.gs_project(*args(n=-1)) == -1
    assert L.gs_project(*args(deg=4)) == -1
    assert L.gs_project(*args(tile=12)) == -1
    assert L.gs_project(*args(mode=3)) == -1 and L.gs_project(*args(mode=-1)) == -1
    assert L.gs_project(*args(V=0)) == -1
    assert L.gs_project(*args(V=65)) == -1
    assert L.gs_project(*args(near=0.0)) == -1
    assert L.gs_project(*args(far=0.001)) == -1
    assert L.gs_project(*args(means=None)) == -1
    bad, badp = _sizes(0, 48)
    assert L.gs_project(*args(sizes=badp)) == -1
    # gs_bin_sort: workspace too small, capacity out of range, misaligned workspace
    ws = B.bin_sort_workspace_size(10, 1, 100, 12)
    assert ws > 0
    aligned = ctypes.c_void_p(256)
    assert L.gs_bin_sort(p, p, 10, 1, szp, 16, 100, aligned, ws - 1, p, p, p, p, None) == -4
    assert L.gs_bin_sort(p, p, 10, 1, szp, 16, 0, aligned, ws, p, p, p, p, None) == -1
    assert L.gs_bin_sort(p, p, 10, 1, szp, 16, 100, ctypes.c_void_p(260), ws, p, p, p, p, None) == -1
    # rasterisers: bad tile, missing outputs, a queue without a schedule
    bg = (ctypes.c_float * 3)(0, 0, 0)
    assert L.gs_rasterize_fwd(p, p, p, 10, 1, szp, 24, 0, 0, bg, None, None, p, p, p, None) == -1
    assert L.gs_rasterize_fwd(p, p, p, 10, 1, szp, 16, 0, 0, bg, None, None, None, p, p, None) == -1
    assert L.gs_rasterize_fwd(p, p, p, 10, 1, szp, 16, 0, 0, bg, None, p, p, p, p, None) == -1
    assert L.gs_rasterize_fwd(p, p, p, 10, 1, szp, 16, 32, 4, bg, None, None, p, p, p, None) == -1
    assert L.gs_rasterize_fwd(p, p, p, 10, 1, szp, 8, 16, 4, bg, None, None, p, p, p, None) == -1
    nan = (ctypes.c_float * 3)(float("nan"), 0, 0)
    assert L.gs_rasterize_fwd(p, p, p, 10, 1, szp, 16, 0, 0, nan, None, None, p, p, p, None) == -1
    assert L.gs_rasterize_bwd(p, p, p, 10, 1, szp, 16, 0, 0, bg, None, None, p, p, None, None, p, 0, None) == -1
    assert L.gs_rasterize_bwd(p, p, p, 10, 1, szp, 16, 8, 4, bg, None, None, p, p, p, None, p, 0, None) == -1
    assert L.gs_project_bwd(p, p, p, p, p, 10, 5, p, p, szp, 1, 0.3, p, p, p, p, p, p, p, None) == -1
    # gs_project_bwd_part: unknown part; the seen part needs the parameters,
    # the unseen part only flags and outputs
    assert L.gs_project_bwd_part(p, p, p, p, p, 10, 3, p, p, szp, 1, 0.3, p, p, p, p, p, p, p, 3, None) == -1
    assert L.gs_project_bwd_part(None, p, p, p, p, 10, 3, p, p, szp, 1, 0.3, p, p, p, p, p, p, p, 1, None) == -1
    assert L.gs_project_bwd_part(None, None, None, None, None, 10, 3, None, None, szp, 1, 0.0, p, None, None, p, p,
                                 p, p, 2, None) == -1
    assert L.gs_project_bwd_part(None, None, None, None, None, 0, 3, None, None, szp, 1, float("nan"), None, None,
                                 None, None, None, None, None, 2, None) == 0
    # gs_project_bwd_adam: N above 2^30, bad betas / eps / rate, a missing moment
    five = (ctypes.c_void_p * 5)(*([16] * 5))
    hole = (ctypes.c_void_p * 5)(16, 16, None, 16, 16)
    rates = (ctypes.c_float * 5)(1e-3, 1e-3, 1e-3, 1e-3, 1e-3)
    bad_rate = (ctypes.c_float * 5)(1e-3, float("inf"), 1e-3, 1e-3, 1e-3)
    fused = lambda **kw: [p, p, p, p, p, kw.get("n", 10), 3, p, p, szp, 1, 0.3, p, p, kw.get("m", five), five,
                          kw.get("lr", rates), kw.get("b1", 0.9), 0.999, kw.get("eps", 1e-15), p, None]
    assert L.gs_project_bwd_adam(*fused(n=(1 << 30) + 1)) == -1
    assert L.gs_project_bwd_adam(*fused(b1=1.0)) == -1
    assert L.gs_project_bwd_adam(*fused(eps=0.0)) == -1
    assert L.gs_project_bwd_adam(*fused(lr=bad_rate)) == -1
    assert L.gs_project_bwd_adam(*fused(m=hole)) == -1
    assert L.gs_loss_l2(p, p, 10, p, p, p, 0, None) == -4
    assert L.gs_loss_l2_noalloc(p, p, -1, p, p, None) == -1
    assert L.gs_loss_l2_noalloc(p, p, 10, None, p, None) == -1
    assert L.gs_loss_l2_noalloc(None, p, 10, p, p, None) == -1
    assert L.gs_tile_schedule(p, 0, p, 0, None) == -1
    assert L.gs_tile_order_xcd(100, 0, aligned, 4096, None) == -1
    assert L.gs_tile_order_xcd(100, 8, aligned, 8, None) == -4
    assert L.gs_tile_schedule_size(0) == 0


def test_workspace_sizes_grow_with_problem():
    a = B.bin_sort_workspace_size(1000, 1, 5000, 64)
    b = B.bin_sort_workspace_size(1000, 2, 5000, 128)
    c = B.bin_sort_workspace_size(1000, 1, 50000, 64)
    assert 0 < a < b and a < c
    assert B.loss_workspace_size(10) >= 8
    assert B.tile_schedule_size(100) >= 400
