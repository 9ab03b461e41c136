"""Helpers for the GPU parity tests: run one C-ABI stage on numpy inputs.

Inputs of a stage come from the seeded scene generators or from the oracle
(rounded to the ABI's float32 layout); nothing computed by the GPU is ever fed
to the oracle.
"""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle
from tests import records as RC
from paper_2606_11390_amd import binding as B

F32 = np.float32


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=None):
    a = np.ascontiguousarray(a if dtype is None else np.asarray(a, dtype))
    return torch.from_numpy(a).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


# ---------------------------------------------------------------- oracle side
def oracle_views(scene, tile, near=0.01, far=1e10, eps2d=0.3, P=None, radius_mode=0):
    """Oracle projection of every view, plus the ABI arrays built from it."""
    P = P or oracle.Params.of(scene)
    V, N = scene.n_views, scene.n
    projs = []
    rec = np.zeros((V, N, 12), F32)
    depth = np.zeros((V, N), F32)
    radii = np.zeros((V, N, 2), np.int32)
    tiles = np.zeros((V, N), np.int32)
    rects = np.zeros((V, N, 2), np.int32)
    flags = np.zeros((V, N), np.uint8)
    for v in range(V):
        W, H = (int(x) for x in scene.sizes[v])
        pr = oracle.project(P, scene.viewmats[v], scene.intrinsics[v], W, H, near, far, eps2d, tile, radius_mode)
        projs.append(pr)
        rec[v] = RC.to_record(pr)
        depth[v] = pr["depth"].astype(F32)
        radii[v] = pr["radii"].T
        tiles[v] = pr["tiles"]
        rects[v] = pack_rects(oracle.tile_rects(rec[v, :, 0], rec[v, :, 1], pr["radii"], tile, W, H))
        flags[v] = pr["visible"] | (pr["clamp"] << 1)
    return P, projs, dict(splats=rec, depths=depth, radii=radii, tiles=tiles, rects=rects, flags=flags)


def pack_rects(r):
    """(x0, y0, x1, y1) rows -> the ABI's packed pair x0 | y0 << 16, x1 | y1 << 16."""
    r = np.asarray(r, np.int64)
    return np.stack([r[:, 0] | (r[:, 1] << 16), r[:, 2] | (r[:, 3] << 16)], axis=1).astype(np.int32)


def oracle_binning(arrs, sizes, tile):
    views = [(arrs["splats"][v, :, 0], arrs["splats"][v, :, 1], arrs["depths"][v], arrs["radii"][v].T.copy())
             for v in range(len(sizes))]
    return oracle.bin_views(views, sizes, tile)


# ------------------------------------------------------------------- GPU side
def gpu_project(scene, tile, near=0.01, far=1e10, eps2d=0.3, radius_mode=0, clear=None):
    """``clear``: an initial [V][N][9] 2-D gradient buffer handed to the
    projection as grad2d_clear; its contents after the call are returned as
    ``grad2d``."""
    V, N = scene.n_views, scene.n
    out = dict(splats=torch.zeros(V * N * 12, device="cuda"), depths=torch.zeros(V * N, device="cuda"),
               radii=torch.zeros(V * N * 2, dtype=torch.int32, device="cuda"),
               tiles=torch.zeros(V * N, dtype=torch.int32, device="cuda"),
               rects=torch.zeros(V * N * 2, dtype=torch.int32, device="cuda"),
               flags=torch.zeros(V * N, dtype=torch.uint8, device="cuda"))
    g2 = None if clear is None else dev(np.asarray(clear, np.float32).reshape(-1))
    B.project(dev(scene.means), dev(scene.log_scales), dev(scene.quats), dev(scene.opacity_logits),
              dev(scene.sh), scene.sh_degree, dev(scene.viewmats), dev(scene.intrinsics), scene.sizes, near,
              far, eps2d, tile, out["splats"], out["depths"], out["radii"], out["tiles"], out["rects"],
              out["flags"], radius_mode, grad2d_clear=g2)
    h = {k: host(v) for k, v in out.items()}
    res = dict(splats=h["splats"].reshape(V, N, 12), depths=h["depths"].reshape(V, N),
               radii=h["radii"].reshape(V, N, 2), tiles=h["tiles"].reshape(V, N),
               rects=h["rects"].reshape(V, N, 2), flags=h["flags"].reshape(V, N))
    if g2 is not None:
        res["grad2d"] = host(g2).reshape(V, N, 9)
    return res


def gpu_bin_sort(arrs, sizes, tile, capacity):
    V, N = arrs["depths"].shape
    _, toff, _ = B.tile_grid(sizes, tile)
    T = int(toff[-1])
    ws = torch.empty(B.bin_sort_workspace_size(N, V, capacity, T), dtype=torch.uint8, device="cuda")
    it = torch.full((capacity,), -7, dtype=torch.int32, device="cuda")
    ig = torch.full((capacity,), -7, dtype=torch.int32, device="cuda")
    rg = torch.full((2 * T,), -7, dtype=torch.int32, device="cuda")
    info = torch.full((4,), -7, dtype=torch.int32, device="cuda")
    B.bin_sort(dev(arrs["rects"].reshape(-1)), dev(arrs["depths"].reshape(-1)), N, sizes, tile, capacity, ws, it,
               ig, rg, info)
    return host(it), host(ig), host(rg).reshape(T, 2), host(info)


def _order(order, rg, T):
    """Schedule buffer and queue of a rasteriser tile order (see render.py):
    False / "tile", "xcd", "heavy", True / "queue"."""
    order = {False: "tile", True: "queue"}.get(order, order)
    if order == "tile":
        return None, None
    sched = torch.empty(B.tile_schedule_size(T), dtype=torch.uint8, device="cuda")
    if order == "xcd":
        B.tile_order_xcd(T, 8, sched)
        return sched, None
    B.tile_schedule(rg, T, sched)
    return sched, (torch.zeros(1, dtype=torch.int32, device="cuda") if order == "queue" else None)


def gpu_raster_fwd(splats, gids, ranges, sizes, tile, bg=(0, 0, 0), persistent=False, block=(0, 0)):
    V, N = splats.shape[:2]
    _, toff, poff = B.tile_grid(sizes, tile)
    P = int(poff[-1])
    img = torch.full((3 * P,), float("nan"), device="cuda")
    T = torch.full((P,), float("nan"), device="cuda")
    last = torch.full((P,), -7, dtype=torch.int32, device="cuda")
    rg = dev(np.asarray(ranges, np.int32).reshape(-1))
    sched, q = _order(persistent, rg, int(toff[-1]))
    B.rasterize_fwd(dev(splats.reshape(-1)), dev(np.asarray(gids, np.int32)), rg, N, sizes, tile, bg, sched, q,
                    img, T, last, block=block)
    return host(img), host(T), host(last)


def gpu_raster_bwd(splats, gids, ranges, sizes, tile, T_final, last, d_img, d_alpha=None, bg=(0, 0, 0),
                   persistent=False, block=(0, 0)):
    V, N = splats.shape[:2]
    _, toff, poff = B.tile_grid(sizes, tile)
    g = torch.zeros(V * N * 9, device="cuda")
    rg = dev(np.asarray(ranges, np.int32).reshape(-1))
    sched, q = _order(persistent, rg, int(toff[-1]))
    B.rasterize_bwd(dev(splats.reshape(-1)), dev(np.asarray(gids, np.int32)), rg, N, sizes, tile, bg, sched, q,
                    dev(T_final, F32), dev(last, np.int32), dev(d_img, F32),
                    None if d_alpha is None else dev(d_alpha, F32), g, block=block)
    return host(g).reshape(V, N, 9)


def gpu_project_bwd(scene, flags, grad2d, eps2d=0.3, parts=(B.GRADS_ALL,), fill=0.0):
    """gs_project_bwd (or the parts of gs_project_bwd_part in the order
    given) into gradient buffers filled with ``fill`` beforehand."""
    N, K = scene.n, (scene.sh_degree + 1) ** 2
    d = dict(means=torch.full((3, N), fill, device="cuda"), log_scales=torch.full((3, N), fill, device="cuda"),
             quats=torch.full((4, N), fill, device="cuda"), opacity_logits=torch.full((N,), fill, device="cuda"),
             sh=torch.full((K, 3, N), fill, device="cuda"))
    fl, g2 = dev(flags.reshape(-1)), dev(grad2d.reshape(-1), F32)
    for part in parts:
        inputs = part != B.GRADS_UNSEEN
        pick = (lambda t: t) if inputs else (lambda t: None)
        B.project_bwd(pick(dev(scene.means)), pick(dev(scene.log_scales)), pick(dev(scene.quats)),
                      pick(dev(scene.opacity_logits)), pick(dev(scene.sh)), scene.sh_degree,
                      pick(dev(scene.viewmats)), pick(dev(scene.intrinsics)), scene.sizes, eps2d, fl, pick(g2),
                      d["means"], d["log_scales"], d["quats"], d["opacity_logits"], d["sh"], part=part)
    return {k: host(v) for k, v in d.items()}


# --------------------------------------------------------------- comparisons
def rel_max(x, y):
    """max |x - y| / max |y|"""
    y = np.asarray(y, np.float64)
    s = np.max(np.abs(y)) if y.size else 0.0
    return float(np.max(np.abs(np.asarray(x, np.float64) - y)) / s) if s > 0 else float(np.max(np.abs(x)) if np.size(x) else 0.0)


def rel_l2(x, y):
    """||x - y||_2 / ||y||_2"""
    y = np.asarray(y, np.float64)
    s = np.linalg.norm(y)
    d = np.linalg.norm(np.asarray(x, np.float64) - y)
    return float(d / s) if s > 0 else float(d)


def unpack(flat, sizes, ch):
    out, o = [], 0
    for w, h in np.asarray(sizes).reshape(-1, 2):
        n = ch * int(w) * int(h)
        out.append(flat[o:o + n].reshape((ch, int(h), int(w)) if ch > 1 else (int(h), int(w))))
        o += n
    return out


def ambiguity(scene, o, tile, proj_margin=2e-6, pix_margin=1e-4, depth_ulps=4):
    """Where float32 evaluation may legitimately take another discrete decision
    than the FP64 oracle, from the oracle's own outputs only (nothing from the
    GPU): pixels whose compositing decisions (alpha skip, 0.99 clamp, stop) lie
    within ``pix_margin`` relative of their thresholds; the pixels where two
    Gaussians adjacent in a tile's sorted list and within ``depth_ulps``
    float32 ulps of depth (their order may swap) are both composited; the
    pixels, in its tile rectangle widened by one tile, where a Gaussian whose
    image-changing projection decisions (cull tests, radii, tile rectangle)
    lie within ``proj_margin`` reaches (nearly) alpha 1/255.  Returns per-view boolean pixel
    masks [H][W] and a boolean mask over the Gaussians: those an ambiguous
    pixel composites (or nearly), or with any projection decision within
    ``proj_margin``, in any view."""
    N = scene.n
    gmask = np.zeros(N, bool)
    pmasks = []
    for v, (W, H) in enumerate(np.asarray(scene.sizes).reshape(-1, 2)):
        W, H = int(W), int(H)
        TX, TY = (W + tile - 1) // tile, (H + tile - 1) // tile
        pr = o["projs"][v]
        rng = o["ranges"][o["offsets"][v]:o["offsets"][v + 1]]
        vals = o["vals"]
        tmask = np.zeros((TY, TX), bool)
        # projection decisions near a threshold: every one of them for the
        # gradients (the clamps of the Jacobian and of the colour put kinks in
        # them), those that can change an image discontinuously (visibility,
        # radii, tile rectangle) for the pixels
        gmask |= pr["margin"] < proj_margin
        # the pixels such a Gaussian can change: inside its tile rectangle
        # widened by one tile, where its alpha is (nearly) 1/255 or more
        A, Bc, C = pr["conic"]
        thr = (1.0 / 255.0) * (1.0 - 1e-3)

        def alpha_at(g, xs, ys):
            dx, dy = pr["u"][g] - (xs + 0.5), pr["v"][g] - (ys + 0.5)
            with np.errstate(over="ignore", invalid="ignore"):
                return pr["sigma"][g] * np.exp(-0.5 * (A[g] * dx * dx + C[g] * dy * dy) - Bc[g] * dx * dy)

        pm = o["fwds"][v]["margin"] < pix_margin
        for g in np.nonzero(pr["margin_img"] < proj_margin)[0]:
            with np.errstate(invalid="ignore"):
                r = 3.0 * np.sqrt(max(pr["cov"][0][g], pr["cov"][2][g], 0.0)) + 1.0
            u, vv = pr["u"][g], pr["v"][g]
            if not (np.isfinite(r) and np.isfinite(u) and np.isfinite(vv)) or pr["sigma"][g] <= 0:
                # no projection to go by (culled before it): the whole view
                tmask[:] = True
                continue
            x0 = int(np.clip(np.floor((u - r) / tile) - 1, 0, TX)) * tile
            x1 = min(W, int(np.clip(np.floor((u + r) / tile) + 2, 0, TX)) * tile)
            y0 = int(np.clip(np.floor((vv - r) / tile) - 1, 0, TY)) * tile
            y1 = min(H, int(np.clip(np.floor((vv + r) / tile) + 2, 0, TY)) * tile)
            if x1 <= x0 or y1 <= y0:
                continue
            ys, xs = np.mgrid[y0:y1, x0:x1]
            near = ~(alpha_at(g, xs, ys) < thr)
            pm[ys[near], xs[near]] = True
        pm |= np.repeat(np.repeat(tmask, tile, axis=0), tile, axis=1)[:H, :W]
        # near depth ties inside a tile's sorted list: the pixels of the tile
        # where both Gaussians of the pair are (nearly) composited

        z32 = pr["depth"].astype(np.float32)
        for t in range(TX * TY):
            s, e = int(rng[t][0]), int(rng[t][1])
            if e - s < 2:
                continue
            gl = vals[s:e]
            z = z32[gl].astype(np.float64)
            close = np.abs(np.diff(z)) <= depth_ulps * np.spacing(np.abs(z[1:]).astype(np.float32))
            if not np.any(close):
                continue
            ty, tx = divmod(t, TX)
            ys, xs = np.mgrid[ty * tile:min(H, ty * tile + tile), tx * tile:min(W, tx * tile + tile)]
            for k in np.nonzero(close)[0]:
                both = ~(alpha_at(gl[k], xs, ys) < thr) & ~(alpha_at(gl[k + 1], xs, ys) < thr)
                pm[ys[both], xs[both]] = True
        pmasks.append(pm)
        # Gaussians an ambiguous pixel composites, or nearly (alpha within
        # 0.1 % of 1/255), in its list up to one entry past the oracle's stop:
        # their gradient terms from that pixel may differ
        visits = o["fwds"][v]["visits"]
        ys, xs = np.nonzero(pm)
        for y, x in zip(ys, xs):
            t = (y // tile) * TX + x // tile
            s, e = int(rng[t][0]), int(rng[t][1])
            g = vals[s:min(e, s + int(visits[y, x]) + 1)]
            dx, dy = pr["u"][g] - (x + 0.5), pr["v"][g] - (y + 0.5)
            with np.errstate(over="ignore", invalid="ignore"):
                a = pr["sigma"][g] * np.exp(-0.5 * (A[g] * dx * dx + C[g] * dy * dy) - Bc[g] * dx * dy)
            gmask[g[~(a < (1.0 / 255.0) * (1.0 - 1e-3))]] = True
    return pmasks, gmask
