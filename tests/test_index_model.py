"""Host-side index model of every kernel launch of one training step, at the
shapes of the large workloads (20M Gaussians in 16 views of mixed size, 60M
Gaussians in eight 4K views) and of the 4K workload, for every tile edge and a
range of intersection capacities.

For each launch the model restates, from the launch code, the grid, the
element count each block walks and the largest index every kernel can read or
write, and checks them against the size of the buffer it touches: 32-bit
index arithmetic that could wrap, grids beyond the hardware limits, workspace
regions smaller than their largest index.  The workspace layouts are
recomputed here and their totals compared with the library's own size
functions (host code, callable without a GPU), and the tunable constants are
read from the kernel sources, so the model follows them.  It checks bounds,
not values: the GPU parity tests check values.
"""
import math
import os
import re

import numpy as np
import pytest

from paper_2606_11390_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_11390_amd", "csrc")

U32 = 1 << 32
I32 = 1 << 31
GRID_X_MAX = (1 << 31) - 1


def _const(src, name):
    text = open(os.path.join(CSRC, src)).read()
    m = re.search(r"constexpr int %s = (\d+);" % name, text)
    assert m, (src, name)
    return int(m.group(1))


RS_THREADS = _const("binsort.hip", "RS_THREADS")
RS_ITEMS = _const("binsort.hip", "RS_ITEMS")
RS_CHUNK = RS_THREADS * RS_ITEMS
RS_MAX_BLOCKS = _const("binsort.hip", "RS_MAX_BLOCKS")
RS_MAX_BITS = _const("binsort.hip", "RS_MAX_BITS")
SC_THREADS = _const("binsort.hip", "SC_THREADS")
SC_ITEMS = _const("binsort.hip", "SC_ITEMS")
EMIT_SPAN = _const("binsort.hip", "EMIT_SPAN")
EMIT_THREADS = _const("binsort.hip", "EMIT_THREADS")
SPLAT, GRAD = 12, 9


def align256(x):
    return (x + 255) // 256 * 256


def sort_blocks(n):
    return max(1, min(RS_MAX_BLOCKS, (n + 2 * RS_CHUNK - 1) // (2 * RS_CHUNK)))


def block_span(n, nb, b):
    per = (n + nb - 1) // nb
    per = (per + RS_CHUNK - 1) // RS_CHUNK * RS_CHUNK
    return min(n, per * b), min(n, per * b + per)


def plan_passes(total):
    npass = (total + RS_MAX_BITS - 1) // RS_MAX_BITS
    return [total // npass + (1 if p < total % npass else 0) for p in range(npass)]


def bits_for(n):
    b = 1
    while b < 32 and (1 << b) < n:
        b += 1
    return b


def bin_layout(vn, cap):
    """Regions of the binning workspace in the library's order, with sizes."""
    regions = [("dk0", 4 * vn), ("dv0", 4 * vn), ("dk1", 4 * vn), ("dv1", 4 * vn), ("offs", 4 * vn),
               ("tk", 4 * cap), ("tv", 4 * cap), ("hist", 4 * (1 << RS_MAX_BITS) * RS_MAX_BLOCKS),
               ("dtot", 4 * (1 << RS_MAX_BITS)), ("part", 8 * RS_MAX_BLOCKS), ("srect", 8 * vn),
               ("cnt", 4 * 16),
               ("bsrc", 4 * ((cap + EMIT_SPAN - 1) // EMIT_SPAN + 1))]
    return {k: v for k, v in regions}, sum(align256(v) for _, v in regions)


def grid_ok(blocks, threads):
    assert 1 <= blocks <= GRID_X_MAX, blocks
    assert blocks * threads < U32, (blocks, threads)


def check_radix_pass(n, nb, bits, hist_bytes, key_bytes_in, key_bytes_out, gather_bytes=None):
    """k_rs_hist / k_rs_spine / k_rs_scatter over n elements in nb blocks."""
    assert 1 <= nb <= RS_MAX_BLOCKS and bits <= RS_MAX_BITS
    grid_ok(nb, RS_THREADS)
    grid_ok(1 << bits, 1024)
    # the histogram is [digit][block]
    assert ((1 << bits) - 1) * nb + nb - 1 < hist_bytes // 4
    if n == 0:
        return
    # every block's span, in 32-bit arithmetic as the kernels form it
    per = (n + nb - 1) // nb
    per = (per + RS_CHUNK - 1) // RS_CHUNK * RS_CHUNK
    assert per * nb >= n
    last_beg, last_end = block_span(n, nb, nb - 1)
    assert last_end == n
    # largest element index a chunk forms: base + RS_CHUNK - 1 with base < end
    assert n - 1 + RS_CHUNK - 1 < U32
    # loads past the end read element end - 1 (in range); scatter writes
    # below the element count (destinations are ranks of counted elements)
    assert n <= key_bytes_in // 4
    assert n <= key_bytes_out // 4
    if gather_bytes is not None:
        assert n <= gather_bytes // 8


def check_zero_share(n, V, n_waves):
    """Wave w of n_waves zeroes chunks [w C / n, (w + 1) C / n) of the C
    64-Gaussian chunks: the ranges tile [0, C) exactly once, the products stay
    in 64 bits, flag loads are clamped to [V][N] and stores (lanes g < N
    only) land inside their [planes][N] tensor."""
    chunks = (n + 63) // 64
    assert (n_waves - 1 + 1) * chunks < (1 << 63)
    w = np.arange(n_waves, dtype=np.int64)
    lo = (w * chunks + n_waves - 1) // n_waves
    hi = ((w + 1) * chunks + n_waves - 1) // n_waves
    assert lo[0] == 0 and hi[-1] == chunks
    assert (lo[1:] == hi[:-1]).all() and (hi >= lo).all()
    last_g = min((chunks - 1) * 64 + 63, n - 1)
    assert (V - 1) * n + last_g < V * n
    assert (48 - 1) * n + last_g < 48 * n


def model_step(sizes, n, tile, cap):
    """Every launch of project -> bin_sort -> tile schedule -> raster fwd ->
    loss -> raster bwd -> project bwd for one workload, capacity cap."""
    V = len(sizes)
    vn = n * V
    assert vn < U32                       # pair indices are 32-bit
    tiles_x = [(w + tile - 1) // tile for w, h in sizes]
    tiles_y = [(h + tile - 1) // tile for w, h in sizes]
    total_tiles = sum(a * b for a, b in zip(tiles_x, tiles_y))
    assert total_tiles <= 0x3FFFFFFF      # the view table's tile offsets are int32
    pixels = sum(w * h for w, h in sizes)

    # projection: one thread per Gaussian, record [V][N][12] with 64-bit offsets
    grid_ok((n + 255) // 256, 256)
    assert (vn - 1) * SPLAT + SPLAT - 1 < (1 << 63)

    # binning workspace: the library's total equals the regions recomputed here
    regions, total = bin_layout(vn, cap)
    assert B.lib().gs_bin_sort_workspace_size(n, V, cap, total_tiles) == total

    # 1. depth passes over the visible pairs (at most vn of them)
    nb_d = sort_blocks(vn)
    dw = plan_passes(32)
    for p, bits in enumerate(dw):
        check_radix_pass(vn, nb_d, bits, regions["hist"], regions["dk0"], regions["dk1"],
                         regions["srect"] if p == len(dw) - 1 else None)
    # 2. scan: partial sums per block (the first kernel also zeroes the 2 T
    # range ints, grid-stride), then offsets and emission sources, every block
    # reading all nb_d partial sums
    grid_ok(nb_d, SC_THREADS)
    assert nb_d <= regions["part"] // 8
    assert vn - 1 + SC_THREADS * SC_ITEMS - 1 < U32
    last = (cap + EMIT_SPAN - 1) // EMIT_SPAN
    # bsrc[k] for k * EMIT_SPAN < min(offset + count, cap), and bsrc[last]
    assert last < regions["bsrc"] // 4
    assert ((cap - 1) // EMIT_SPAN) < regions["bsrc"] // 4
    # 64-bit running sums: a pair covers at most total_tiles tiles
    assert vn * total_tiles < (1 << 64)
    # 3. emission: one workgroup per EMIT_SPAN slots below the capacity
    emit_blocks = (cap + EMIT_SPAN - 1) // EMIT_SPAN
    grid_ok(emit_blocks, EMIT_THREADS)
    assert (emit_blocks - 1) * EMIT_SPAN + EMIT_SPAN - 1 < U32      # slot index, 32-bit
    assert emit_blocks - 1 + 1 <= last                              # bsrc[blockIdx.x + 1]
    # at most EMIT_SPAN + 1 sources per workgroup, read from s0 <= s1 < visible pairs
    fused = emit_blocks <= RS_MAX_BLOCKS
    tbits = bits_for(total_tiles)
    tw = plan_passes(tbits)
    if fused:
        assert ((1 << tw[0]) - 1) * emit_blocks + emit_blocks - 1 < regions["hist"] // 4
    # keys are global tile ids below 2^tbits, values Gaussian indices below N
    assert total_tiles <= (1 << tbits) and sum(tw) == tbits
    # 4. tile passes over the (at most cap) intersections
    nb_t = sort_blocks(cap)
    for p, bits in enumerate(tw):
        nb = emit_blocks if (fused and p == 0) else nb_t
        check_radix_pass(cap, nb, bits, regions["hist"], 4 * cap, 4 * cap)
        if fused and p == 0:
            # the emission's histogram columns are the scatter's blocks: one
            # EMIT_SPAN-slot chunk each
            assert block_span(cap, nb, 0)[1] <= EMIT_SPAN or cap <= EMIT_SPAN
    # 5. ranges: 4 keys per thread over the capacity
    grid_ok((cap + 1023) // 1024, 256)
    assert 4 * ((cap + 1023) // 1024 * 256) < U32
    # tile schedule: one 8-bit pass over the tiles
    nb_s = min(RS_MAX_BLOCKS, max(1, (total_tiles + RS_CHUNK - 1) // RS_CHUNK))
    sched = align256(4 * total_tiles) + align256(4 * 256 * RS_MAX_BLOCKS) + align256(4 * 256)
    assert B.lib().gs_tile_schedule_size(total_tiles) == sched
    check_radix_pass(total_tiles, nb_s, 8, 4 * 256 * RS_MAX_BLOCKS, 8 * total_tiles, 4 * total_tiles)
    # rasterisers: one workgroup per tile; a tile's list is a range of the
    # intersections; records at (view * N + Gaussian) * 12 + 11, 64-bit
    grid_ok(total_tiles, 64 * 8)
    assert (V - 1) * n * SPLAT + (n - 1) * SPLAT + SPLAT - 1 == vn * SPLAT - 1
    # images [3][H][W] per view at 3 * pixel offset; T and n_contrib per pixel
    assert 3 * pixels < (1 << 63)
    # backward: the 2-D gradient record zeroed by a 16-byte fill of V N 9 floats
    nfill = vn * GRAD
    nv = nfill // 4
    grid_ok((max(nv, 4) + 255) // 256, 256)
    # gradient atomics at (view * N + Gaussian) * 9 + j, 64-bit
    assert (vn - 1) * GRAD + GRAD - 1 < (1 << 63)
    # loss over 3 * pixels elements
    grid_ok(max(1, (3 * pixels + 1023) // 1024), 256)
    # the fused L2 backward's zeroing of unseen Gaussians' parameter
    # gradients, for every waves-per-tile count a tile edge allows
    for wpt in (1, 2, 4, 8, 16):
        if wpt * 64 <= tile * tile:
            check_zero_share(n, V, (total_tiles + 1) // 2 * wpt)
    # projection backward: one thread per Gaussian; SH planes at j * 3 N + g
    grid_ok((n + 255) // 256, 256)
    assert (16 * 3 - 1) * n + n - 1 < (1 << 63)
    return {"total_tiles": total_tiles, "emit_blocks": emit_blocks, "fused": fused, "depth_blocks": nb_d,
            "tile_passes": tw}


def _multiview_sizes():
    """The 16 view sizes of the 20M-Gaussian workload (same draw as the scene
    generator, without building the scene)."""
    from paper_2606_11390_amd import scenes
    rng = np.random.default_rng(4 + 1000)
    picks = rng.integers(0, len(scenes.VIEW_SIZES), size=16)
    return [scenes.VIEW_SIZES[i] for i in picks]


WORKLOADS = {
    "uhd": ([(3840, 2160)], 5_000_000),
    "multiview": (None, 20_000_000),
    "city": ([(3840, 2160)] * 8, 60_000_000),
}


@pytest.mark.parametrize("name", list(WORKLOADS))
@pytest.mark.parametrize("tile", [8, 16, 32])
def test_every_launch_in_bounds(name, tile):
    sizes, n = WORKLOADS[name]
    sizes = sizes or _multiview_sizes()
    # capacities from the renderer's first guess up to the ABI's limit, through
    # the fused / unfused emission boundary and the capped block counts
    caps = sorted({1 << 20, RS_MAX_BLOCKS * EMIT_SPAN, RS_MAX_BLOCKS * EMIT_SPAN + 1,
                   2 * RS_CHUNK * RS_MAX_BLOCKS + 1, 1 << 28, (1 << 31) - 1})
    seen = set()
    for cap in caps:
        out = model_step(sizes, n, tile, cap)
        seen.add(out["fused"])
    assert seen == {True, False}


def test_view_table_limits():
    # the 16-view workload at 8-pixel tiles: tile ids need 20 bits, three passes
    sizes = _multiview_sizes()
    tiles = sum(((w + 7) // 8) * ((h + 7) // 8) for w, h in sizes)
    assert bits_for(tiles) <= 21 and len(plan_passes(bits_for(tiles))) == 3
    # pair counts: 16 x 20M and 8 x 60M stay below 2^32 (the ABI rejects more)
    assert 16 * 20_000_000 < U32 and 8 * 60_000_000 < U32


def test_block_spans_cover_every_element_once():
    # the spans of the nb blocks tile [0, n) exactly, for counts around the
    # capped block count and the chunk size
    for n in [1, RS_CHUNK - 1, RS_CHUNK, 2 * RS_CHUNK * RS_MAX_BLOCKS - 1, 2 * RS_CHUNK * RS_MAX_BLOCKS + 7,
              320_000_000, (1 << 31) - 1]:
        nb = sort_blocks(n)
        end_prev = 0
        for b in range(nb):
            beg, end = block_span(n, nb, b)
            assert beg == end_prev or beg == end == n
            assert beg % RS_CHUNK == 0 or beg == n
            end_prev = end
        assert end_prev == n


@pytest.mark.parametrize("n", [5_000_000, 20_000_000, 60_000_000])
def test_morton_order_and_gather_in_bounds(n):
    """The Morton reordering run before the benchmarks (gs_morton_order, then
    gs_gather_columns per parameter tensor) at the 4K, 16-view and city
    Gaussian counts: the workspace layout recomputed here matches the
    library's size, every radix pass (8, 8, 8 and 6 bits over n keys, the
    first computing the codes from the means) stays inside its regions, and
    the gather's grid and largest plane offset fit."""
    t = n
    keys = align256(4 * t)
    hist = align256(4 * 256 * RS_MAX_BLOCKS)
    assert B.lib().gs_morton_workspace_size(n) == 3 * keys + hist + align256(4 * 256)
    nb = sort_blocks(t)
    for bits in (8, 8, 8, 6):
        check_radix_pass(t, nb, bits, 4 * 256 * RS_MAX_BLOCKS, 4 * t, 4 * t)
    # the index plane (values) is the caller's int32 order[n] or the third
    # key-sized region; the 30-bit codes fit the four passes
    assert 8 + 8 + 8 + 6 == 30
    # gather: one thread per destination column, 64-bit plane offsets, up to
    # 48 SH planes per tensor
    grid_ok((t + 255) // 256, 256)
    assert (48 - 1) * t + t - 1 < (1 << 63)

