"""ctypes binding of the C ABI in ``include/gs.h`` (argument marshalling only).

Every function here checks tensor dtypes, devices and shapes, passes
``data_ptr()`` values and torch's current HIP stream to the library, and
returns.  All computation happens in the HIP kernels of ``libgs.so``; there is
no fallback: if the library is missing or the tensors are not on a GPU the
call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgs.so")

GS_ABI_VERSION = 5
GS_MAX_VIEWS = 64
SPLAT_FLOATS = 12
GRAD_FLOATS = 9
FLAG_VISIBLE = 1
INFO_VISIBLE, INFO_ISECT, INFO_OVERFLOW = 0, 1, 2
RADIUS_3SIGMA, RADIUS_OPACITY, RADIUS_EIGEN = 0, 1, 2

_lib = None

_p = ctypes.c_void_p
_i64 = ctypes.c_int64
_int = ctypes.c_int
_f = ctypes.c_float
_sz = ctypes.c_size_t

# name -> (restype, argtypes), mirroring include/gs.h
_SIGS = {
    "gs_abi_version": (_int, []),
    "gs_strerror": (ctypes.c_char_p, [_int]),
    "gs_project": (_int, [_p, _p, _p, _p, _p, _i64, _int, _p, _p, _p, _int, _f, _f, _f, _int, _int,
                          _p, _p, _p, _p, _p, _p, _p, _p]),
    "gs_densify_stats": (_int, [_p, _p, _p, _i64, _int, _p, _p, _p, _p, _p]),
    "gs_bin_sort_workspace_size": (_sz, [_i64, _int, _i64, _i64]),
    "gs_bin_sort": (_int, [_p, _p, _i64, _int, _p, _int, _i64, _p, _sz, _p, _p, _p, _p, _p]),
    "gs_tile_schedule_size": (_sz, [_i64]),
    "gs_tile_schedule": (_int, [_p, _i64, _p, _sz, _p]),
    "gs_tile_order_xcd": (_int, [_i64, _int, _p, _sz, _p]),
    "gs_rasterize_fwd": (_int, [_p, _p, _p, _i64, _int, _p, _int, _int, _int, _p, _p, _p, _p, _p, _p, _p]),
    "gs_rasterize_bwd": (_int, [_p, _p, _p, _i64, _int, _p, _int, _int, _int, _p, _p, _p, _p, _p, _p, _p, _p,
                                _int, _p]),
    "gs_rasterize_bwd_l2_workspace_size": (_sz, [_int, _p, _int]),
    "gs_rasterize_bwd_l2": (_int, [_p, _p, _p, _i64, _int, _p, _int, _int, _int, _p, _p, _p, _p, _p, _p, _p,
                                   _p, _int, _p, _sz, _p, _int, _p, _p]),
    "gs_project_bwd": (_int, [_p, _p, _p, _p, _p, _i64, _int, _p, _p, _p, _int, _f, _p, _p, _p, _p,
                              _p, _p, _p, _p]),
    "gs_project_bwd_part": (_int, [_p, _p, _p, _p, _p, _i64, _int, _p, _p, _p, _int, _f, _p, _p, _p, _p,
                                   _p, _p, _p, _int, _p]),
    "gs_project_bwd_adam": (_int, [_p, _p, _p, _p, _p, _i64, _int, _p, _p, _p, _int, _f, _p, _p, _p, _p, _p,
                                   _f, _f, _f, _p, _p]),
    "gs_raster_visits": (_int, [_p, _p, _p, _i64, _int, _p, _int, _p, _p, _p, _p, _p]),
    "gs_adam": (_int, [_int, _p, _p, _p, _p, _p, _p, _f, _f, _f, _p, _p]),
    "gs_morton_workspace_size": (_sz, [_i64]),
    "gs_morton_order": (_int, [_p, _i64, _p, _p, _p, _sz, _p, _p]),
    "gs_gather_columns": (_int, [_p, _int, _i64, _p, _p, _p]),
    "gs_ssim_workspace_size": (_sz, [_int, _p]),
    "gs_loss_ssim_l1": (_int, [_p, _p, _int, _p, _f, _p, _p, _p, _sz, _p]),
    "gs_loss_workspace_size": (_sz, [_i64]),
    "gs_loss_l2": (_int, [_p, _p, _i64, _p, _p, _p, _sz, _p]),
    "gs_loss_l2_noalloc": (_int, [_p, _p, _i64, _p, _p, _p]),
}


class GSError(RuntimeError):
    pass


def lib():
    """The loaded ``libgs.so`` (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise GSError(f"{LIB_PATH} not built; run __graft_entry__.build() or "
                          "python -m paper_2606_11390_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        if L.gs_abi_version() != GS_ABI_VERSION:
            raise GSError("libgs.so ABI version mismatch")
        _lib = L
    return _lib


def exported_symbols():
    return tuple(_SIGS)


def _check(rc, what):
    if rc != 0:
        raise GSError(f"{what}: {lib().gs_strerror(rc).decode()} ({rc})")


def _ptr(t, dtype=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise GSError(f"{name} must live on the GPU (got {t.device})")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise GSError(f"{name} must be contiguous")
    return t.data_ptr()


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _host_i32(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
    return a, a.ctypes.data_as(ctypes.c_void_p)


def _host_f32(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    return a, a.ctypes.data_as(ctypes.c_void_p)


def tile_grid(sizes, tile):
    """Per-view tiles_x, tile offsets (length V+1) and pixel offsets (length V+1)."""
    sizes = np.asarray(sizes, np.int64).reshape(-1, 2)
    tx = (sizes[:, 0] + tile - 1) // tile
    ty = (sizes[:, 1] + tile - 1) // tile
    toff = np.concatenate([[0], np.cumsum(tx * ty)])
    poff = np.concatenate([[0], np.cumsum(sizes[:, 0] * sizes[:, 1])])
    return tx, toff, poff


F32, I32, U8 = torch.float32, torch.int32, torch.uint8


def project(means, log_scales, quats, opacity_logits, sh, sh_degree, viewmats, intrinsics, sizes,
            near, far, eps2d, tile, splats, depths, radii, tiles_touched, tile_rects, flags, radius_mode=0,
            grad2d_clear=None):
    n = means.shape[1]
    sz, szp = _host_i32(sizes)
    rc = lib().gs_project(_ptr(means, F32, "means"), _ptr(log_scales, F32, "log_scales"),
                          _ptr(quats, F32, "quats"), _ptr(opacity_logits, F32, "opacity_logits"),
                          _ptr(sh, F32, "sh"), n, int(sh_degree), _ptr(viewmats, F32, "viewmats"),
                          _ptr(intrinsics, F32, "intrinsics"), szp, sz.shape[0], float(near), float(far),
                          float(eps2d), int(tile), int(radius_mode), _ptr(splats, F32, "splats"), _ptr(depths, F32, "depths"),
                          _ptr(radii, I32, "radii"), _ptr(tiles_touched, I32, "tiles_touched"),
                          _ptr(tile_rects, I32, "tile_rects"), _ptr(flags, U8, "flags"),
                          _ptr(grad2d_clear, F32, "grad2d_clear"), _stream())
    _check(rc, "gs_project")


def bin_sort_workspace_size(n, n_views, capacity, total_tiles):
    return int(lib().gs_bin_sort_workspace_size(n, n_views, capacity, total_tiles))


def bin_sort(tile_rects, depths, n, sizes, tile, capacity, workspace, isect_tile, isect_gid, tile_ranges, info):
    sz, szp = _host_i32(sizes)
    rc = lib().gs_bin_sort(_ptr(tile_rects, I32, "tile_rects"), _ptr(depths, F32, "depths"), n,
                           sz.shape[0], szp, int(tile), int(capacity), _ptr(workspace, U8, "workspace"),
                           workspace.numel(), _ptr(isect_tile, I32, "isect_tile"),
                           _ptr(isect_gid, I32, "isect_gid"), _ptr(tile_ranges, I32, "tile_ranges"),
                           _ptr(info, I32, "info"), _stream())
    _check(rc, "gs_bin_sort")


def tile_schedule_size(total_tiles):
    return int(lib().gs_tile_schedule_size(total_tiles))


def tile_schedule(tile_ranges, total_tiles, schedule):
    rc = lib().gs_tile_schedule(_ptr(tile_ranges, I32, "tile_ranges"), int(total_tiles),
                                _ptr(schedule, U8, "schedule"), schedule.numel(), _stream())
    _check(rc, "gs_tile_schedule")


def tile_order_xcd(total_tiles, n_xcd, schedule):
    rc = lib().gs_tile_order_xcd(int(total_tiles), int(n_xcd), _ptr(schedule, U8, "schedule"), schedule.numel(),
                                 _stream())
    _check(rc, "gs_tile_order_xcd")


def rasterize_fwd(splats, isect_gid, tile_ranges, n, sizes, tile, background, schedule, queue, images,
                  T_final, n_contrib, block=(0, 0)):
    sz, szp = _host_i32(sizes)
    bg, bgp = _host_f32(background)
    rc = lib().gs_rasterize_fwd(_ptr(splats, F32, "splats"), _ptr(isect_gid, I32, "isect_gid"),
                                _ptr(tile_ranges, I32, "tile_ranges"), n, sz.shape[0], szp, int(tile),
                                int(block[0]), int(block[1]), bgp,
                                _ptr(schedule, U8, "schedule"), _ptr(queue, I32, "queue"),
                                _ptr(images, F32, "images"), _ptr(T_final, F32, "T_final"),
                                _ptr(n_contrib, I32, "n_contrib"), _stream())
    _check(rc, "gs_rasterize_fwd")


def rasterize_bwd(splats, isect_gid, tile_ranges, n, sizes, tile, background, schedule, queue, T_final,
                  n_contrib, d_images, d_alpha, grad2d, accumulate=False, block=(0, 0)):
    sz, szp = _host_i32(sizes)
    bg, bgp = _host_f32(background)
    rc = lib().gs_rasterize_bwd(_ptr(splats, F32, "splats"), _ptr(isect_gid, I32, "isect_gid"),
                                _ptr(tile_ranges, I32, "tile_ranges"), n, sz.shape[0], szp, int(tile),
                                int(block[0]), int(block[1]), bgp,
                                _ptr(schedule, U8, "schedule"), _ptr(queue, I32, "queue"),
                                _ptr(T_final, F32, "T_final"), _ptr(n_contrib, I32, "n_contrib"),
                                _ptr(d_images, F32, "d_images"), _ptr(d_alpha, F32, "d_alpha"),
                                _ptr(grad2d, F32, "grad2d"), int(bool(accumulate)), _stream())
    _check(rc, "gs_rasterize_bwd")


def rasterize_bwd_l2_workspace_size(sizes, tile):
    sz, szp = _host_i32(sizes)
    return int(lib().gs_rasterize_bwd_l2_workspace_size(sz.shape[0], szp, int(tile)))


def rasterize_bwd_l2(splats, isect_gid, tile_ranges, n, sizes, tile, background, schedule, T_final, n_contrib,
                     images, targets, loss, grad2d, workspace, accumulate=False, block=(0, 0), unseen=None):
    """gs_loss_l2 and gs_rasterize_bwd in one pass (d_images is not stored).
    ``unseen``: (flags, sh_degree, [d_means, d_log_scales, d_quats,
    d_opacity_logits, d_sh]) to also write the zero gradients of the
    Gaussians no view sees."""
    sz, szp = _host_i32(sizes)
    bg, bgp = _host_f32(background)
    fl, deg, planes = None, 0, None
    if unseen is not None:
        flags, deg, grads = unseen
        fl = _ptr(flags, U8, "flags")
        names = ("d_means", "d_log_scales", "d_quats", "d_opacity_logits", "d_sh")
        planes = (ctypes.c_void_p * 5)(*[_ptr(t, F32, nm) for t, nm in zip(grads, names)])
    rc = lib().gs_rasterize_bwd_l2(_ptr(splats, F32, "splats"), _ptr(isect_gid, I32, "isect_gid"),
                                   _ptr(tile_ranges, I32, "tile_ranges"), n, sz.shape[0], szp, int(tile),
                                   int(block[0]), int(block[1]), bgp, _ptr(schedule, U8, "schedule"),
                                   _ptr(T_final, F32, "T_final"), _ptr(n_contrib, I32, "n_contrib"),
                                   _ptr(images, F32, "images"), _ptr(targets, F32, "targets"),
                                   _ptr(loss, F32, "loss"), _ptr(grad2d, F32, "grad2d"), int(bool(accumulate)),
                                   _ptr(workspace, U8, "workspace"), workspace.numel(), fl, int(deg), planes,
                                   _stream())
    _check(rc, "gs_rasterize_bwd_l2")


GRADS_ALL, GRADS_SEEN, GRADS_UNSEEN = 0, 1, 2


def project_bwd(means, log_scales, quats, opacity_logits, sh, sh_degree, viewmats, intrinsics, sizes,
                eps2d, flags, grad2d, d_means, d_log_scales, d_quats, d_opacity_logits, d_sh, part=GRADS_ALL):
    """gs_project_bwd, or with ``part`` GRADS_SEEN / GRADS_UNSEEN the half of
    it gs_project_bwd_part names (with GRADS_UNSEEN the parameters, cameras
    and grad2d may be None)."""
    n = d_means.shape[1]
    sz, szp = _host_i32(sizes)
    args = (_ptr(means, F32, "means"), _ptr(log_scales, F32, "log_scales"),
            _ptr(quats, F32, "quats"), _ptr(opacity_logits, F32, "opacity_logits"),
            _ptr(sh, F32, "sh"), n, int(sh_degree), _ptr(viewmats, F32, "viewmats"),
            _ptr(intrinsics, F32, "intrinsics"), szp, sz.shape[0], float(eps2d),
            _ptr(flags, U8, "flags"), _ptr(grad2d, F32, "grad2d"),
            _ptr(d_means, F32, "d_means"), _ptr(d_log_scales, F32, "d_log_scales"),
            _ptr(d_quats, F32, "d_quats"), _ptr(d_opacity_logits, F32, "d_opacity_logits"),
            _ptr(d_sh, F32, "d_sh"))
    if part == GRADS_ALL:
        _check(lib().gs_project_bwd(*args, _stream()), "gs_project_bwd")
    else:
        _check(lib().gs_project_bwd_part(*args, int(part), _stream()), "gs_project_bwd_part")


def project_bwd_adam(means, log_scales, quats, opacity_logits, sh, sh_degree, viewmats, intrinsics, sizes, eps2d,
                     flags, grad2d, exp_avg, exp_avg_sq, lrs, beta1, beta2, eps, step):
    """gs_project_bwd and gs_adam in one pass: updates the five parameter
    tensors and their moments (lists in the order means, log_scales, quats,
    opacity_logits, sh) in place and advances ``step``."""
    if len(exp_avg) != 5 or len(exp_avg_sq) != 5 or len(lrs) != 5:
        raise GSError("project_bwd_adam takes five moments and rates (means, log_scales, quats, "
                      "opacity_logits, sh)")
    n = means.shape[1]
    sz, szp = _host_i32(sizes)
    M = (ctypes.c_void_p * 5)(*[_ptr(t, F32, "exp_avg") for t in exp_avg])
    V = (ctypes.c_void_p * 5)(*[_ptr(t, F32, "exp_avg_sq") for t in exp_avg_sq])
    lr = (ctypes.c_float * 5)(*[float(x) for x in lrs])
    rc = lib().gs_project_bwd_adam(_ptr(means, F32, "means"), _ptr(log_scales, F32, "log_scales"),
                                   _ptr(quats, F32, "quats"), _ptr(opacity_logits, F32, "opacity_logits"),
                                   _ptr(sh, F32, "sh"), n, int(sh_degree), _ptr(viewmats, F32, "viewmats"),
                                   _ptr(intrinsics, F32, "intrinsics"), szp, sz.shape[0], float(eps2d),
                                   _ptr(flags, U8, "flags"), _ptr(grad2d, F32, "grad2d"), M, V, lr, float(beta1),
                                   float(beta2), float(eps), _ptr(step, I32, "step"), _stream())
    _check(rc, "gs_project_bwd_adam")


def loss_workspace_size(n_elems):
    return int(lib().gs_loss_workspace_size(n_elems))


def loss_l2(images, targets, loss, d_images, workspace):
    rc = lib().gs_loss_l2(_ptr(images, F32, "images"), _ptr(targets, F32, "targets"), images.numel(),
                          _ptr(loss, F32, "loss"), _ptr(d_images, F32, "d_images"),
                          _ptr(workspace, U8, "workspace"), workspace.numel(), _stream())
    _check(rc, "gs_loss_l2")


def loss_l2_noalloc(images, targets, loss, d_images):
    """gs_loss_l2 with the library's own per-GPU partial-sum array (no
    workspace; allocates nothing)."""
    rc = lib().gs_loss_l2_noalloc(_ptr(images, F32, "images"), _ptr(targets, F32, "targets"), images.numel(),
                                  _ptr(loss, F32, "loss"), _ptr(d_images, F32, "d_images"), _stream())
    _check(rc, "gs_loss_l2_noalloc")


def raster_visits(splats, isect_gid, tile_ranges, n, sizes, tile, images, T_final, n_contrib, visits):
    sz, szp = _host_i32(sizes)
    rc = lib().gs_raster_visits(_ptr(splats, F32, "splats"), _ptr(isect_gid, I32, "isect_gid"),
                                _ptr(tile_ranges, I32, "tile_ranges"), n, sz.shape[0], szp, int(tile),
                                _ptr(images, F32, "images"), _ptr(T_final, F32, "T_final"),
                                _ptr(n_contrib, I32, "n_contrib"), _ptr(visits, I32, "visits"), _stream())
    _check(rc, "gs_raster_visits")


def adam(params, grads, exp_avg, exp_avg_sq, lrs, beta1, beta2, eps, step):
    """Fused Adam over matching lists of tensors (one launch)."""
    k = len(params)
    P = (ctypes.c_void_p * k)(*[_ptr(t, F32, "param") for t in params])
    G = (ctypes.c_void_p * k)(*[_ptr(t, F32, "grad") for t in grads])
    M = (ctypes.c_void_p * k)(*[_ptr(t, F32, "exp_avg") for t in exp_avg])
    V = (ctypes.c_void_p * k)(*[_ptr(t, F32, "exp_avg_sq") for t in exp_avg_sq])
    n = (ctypes.c_int64 * k)(*[t.numel() for t in params])
    lr = (ctypes.c_float * k)(*[float(x) for x in lrs])
    rc = lib().gs_adam(k, P, G, M, V, n, lr, float(beta1), float(beta2), float(eps), _ptr(step, I32, "step"),
                       _stream())
    _check(rc, "gs_adam")


def morton_order(means, origin, inv_cell, workspace, order):
    n = means.shape[1]
    o, op = _host_f32(origin)
    c, cp = _host_f32(inv_cell)
    rc = lib().gs_morton_order(_ptr(means, F32, "means"), n, op, cp, _ptr(workspace, U8, "workspace"),
                               workspace.numel(), _ptr(order, I32, "order"), _stream())
    _check(rc, "gs_morton_order")


def morton_workspace_size(n):
    return int(lib().gs_morton_workspace_size(n))


def gather_columns(src, order, dst):
    """dst[..., i] = src[..., order[i]] for planar [C][N] (or [N]) tensors."""
    n = src.shape[-1]
    C = src.numel() // max(n, 1)
    rc = lib().gs_gather_columns(_ptr(src, F32, "src"), C, n, _ptr(order, I32, "order"), _ptr(dst, F32, "dst"),
                                 _stream())
    _check(rc, "gs_gather_columns")


def ssim_workspace_size(sizes):
    sz, szp = _host_i32(np.asarray(sizes).reshape(-1, 2))
    return int(lib().gs_ssim_workspace_size(sz.shape[0], szp))


def loss_ssim_l1(images, targets, sizes, lam, loss, d_images, workspace):
    sz, szp = _host_i32(np.asarray(sizes).reshape(-1, 2))
    rc = lib().gs_loss_ssim_l1(_ptr(images, F32, "images"), _ptr(targets, F32, "targets"), sz.shape[0], szp,
                               float(lam), _ptr(loss, F32, "loss"), _ptr(d_images, F32, "d_images"),
                               _ptr(workspace, U8, "workspace"), workspace.numel(), _stream())
    _check(rc, "gs_loss_ssim_l1")


def densify_stats(grad2d, flags, radii, n, sizes, grad_accum, count, max_radius):
    sz, szp = _host_i32(np.asarray(sizes).reshape(-1, 2))
    rc = lib().gs_densify_stats(_ptr(grad2d, F32, "grad2d"), _ptr(flags, U8, "flags"), _ptr(radii, I32, "radii"),
                                int(n), sz.shape[0], szp, _ptr(grad_accum, F32, "grad_accum"),
                                _ptr(count, I32, "count"), _ptr(max_radius, I32, "max_radius"), _stream())
    _check(rc, "gs_densify_stats")
