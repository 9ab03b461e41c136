"""FP64 CPU oracle of the Gaussian-splatting hot path.

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the CPU
baseline of ``bench.py`` import this package; the product path
(``paper_2606_11390_amd``) never does, and nothing here is computed by, read
from or shared with the HIP path.  The arithmetic lives in ``gs_oracle.c``
(plain double-precision loops); this module marshals numpy arrays to it and
adds the one piece that is a plain definition over numpy arrays, the L2 loss.
The conversion between the oracle's quantities and the 12-float splat record
that the C ABI exchanges between stages is test glue and lives in
``tests/records.py``.

Each function follows the operator list of the paper's Section 4 (projection
and SH colour per Gaussian, then per camera depth sort / binning,
rasterisation and image-space loss, and their backward passes); the formulas
are those of 3D Gaussian Splatting, which the paper cites for the method.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "_gs_oracle.so")
_lib = None

ALPHA_MIN = float(np.float32(1.0 / 255.0))
ALPHA_MAX = float(np.float32(0.99))
T_MIN = float(np.float32(1e-4))

_D = ctypes.POINTER(ctypes.c_double)
_F = ctypes.POINTER(ctypes.c_float)
_I = ctypes.POINTER(ctypes.c_int32)
_U8 = ctypes.POINTER(ctypes.c_uint8)
_U64 = ctypes.POINTER(ctypes.c_uint64)
_i64 = ctypes.c_int64
_int = ctypes.c_int
_dbl = ctypes.c_double


def lib():
    """Load (building with gcc if needed) the C oracle."""
    global _lib
    if _lib is None:
        src = os.path.join(HERE, "gs_oracle.c")
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        L.or_project.argtypes = [_i64, _int, _D, _D, _D, _D, _D, _D, _D, _int, _int, _dbl, _dbl, _dbl,
                                 _int, _int, _D, _D, _D, _D, _D, _D, _D, _I, _I, _U8, _U8, _D, _D]
        L.or_bin_emit.argtypes = [_i64, _F, _F, _F, _I, _int, _int, _int, _i64, _U64, _I, _i64]
        L.or_bin_emit.restype = _i64
        L.or_sort_pairs.argtypes = [_i64, _U64, _I]
        L.or_tile_ranges.argtypes = [_i64, _U64, _i64, _I]
        L.or_raster_fwd.argtypes = [_int, _int, _int, _I, _I, _i64, _D, _D, _D, _D, _D, _D, _D, _D,
                                    _D, _D, _I, _I, _D]
        L.or_raster_bwd.argtypes = [_int, _int, _int, _I, _I, _i64, _D, _D, _D, _D, _D, _D, _D, _D,
                                    _D, _D, _D, _D, _D, _D, _D, _D, _D]
        L.or_project_bwd.argtypes = [_i64, _int, _D, _D, _D, _D, _D, _D, _D, _int, _int, _dbl, _dbl,
                                     _dbl, _int, _int, _D, _D, _D, _D, _D, _D, _D, _D, _D]
        L.or_sh_basis.argtypes = [_int, _D, _D]
        L.or_quat_rot.argtypes = [_D, _D]
        L.or_tile_rect.argtypes = [ctypes.c_float, ctypes.c_float, _int, _int, _int, _int, _int, _I]
        L.or_tile_rects.argtypes = [_i64, _F, _F, _I, _int, _int, _int, _I]
        L.or_raster_fwd_rect.argtypes = [_int, _int, _int, _I, _I, _i64, _D, _D, _D, _D, _D, _D, _D, _D,
                                         _int, _int, _int, _int, _D, _U64]
        L.or_set_threads.argtypes = [_int]
        L.or_num_procs.restype = _int
        _lib = L
    return _lib


def set_threads(n):
    """Threads of the oracle's parallel loops (1 = serial, the default; see
    the note on threads in gs_oracle.c)."""
    lib().or_set_threads(int(n))


def num_procs():
    return int(lib().or_num_procs())


def _p(a, t):
    return a.ctypes.data_as(t)


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# small pieces exposed for the pins
# --------------------------------------------------------------------------
def sh_basis(d, K=16):
    d = _d(d)
    y = np.zeros(K)
    lib().or_sh_basis(K, _p(d, _D), _p(y, _D))
    return y


def quat_rot(q):
    q = _d(q)
    r = np.zeros(9)
    lib().or_quat_rot(_p(q, _D), _p(r, _D))
    return r.reshape(3, 3)


def tile_rect(u, v, rx, ry, tile, W, H):
    r = np.zeros(4, np.int32)
    lib().or_tile_rect(float(u), float(v), int(rx), int(ry), tile, W, H, _p(r, _I))
    return tuple(int(x) for x in r)


def tile_rects(u32, v32, radii, tile, W, H):
    """Tile rectangles [n][4] = (x0, y0, x1, y1) of n Gaussians from their
    float32 means and radii [2][n] (reading R8); zero rows where culled."""
    u32 = np.ascontiguousarray(u32, np.float32)
    v32 = np.ascontiguousarray(v32, np.float32)
    radii = np.ascontiguousarray(radii, np.int32)
    n = u32.shape[0]
    out = np.zeros((n, 4), np.int32)
    lib().or_tile_rects(n, _p(u32, _F), _p(v32, _F), _p(radii, _I), int(tile), int(W), int(H), _p(out, _I))
    return out


# --------------------------------------------------------------------------
# projection
# --------------------------------------------------------------------------
class Params:
    """FP64 copies of a scene's Gaussian parameters (planar [C][N])."""

    def __init__(self, means, log_scales, quats, opacity_logits, sh, sh_degree):
        self.means = _d(means)
        self.log_scales = _d(log_scales)
        self.quats = _d(quats)
        self.opac = _d(opacity_logits)
        self.sh = _d(sh)
        self.deg = int(sh_degree)

    @classmethod
    def of(cls, scene):
        return cls(scene.means, scene.log_scales, scene.quats, scene.opacity_logits, scene.sh,
                   scene.sh_degree)

    @property
    def n(self):
        return self.means.shape[1]

    def copy(self):
        return Params(self.means.copy(), self.log_scales.copy(), self.quats.copy(),
                      self.opac.copy(), self.sh.copy(), self.deg)


RADIUS_3SIGMA, RADIUS_OPACITY, RADIUS_EIGEN = 0, 1, 2


def project(P, viewmat, intr, W, H, near=0.01, far=1e10, eps2d=0.3, tile=16, radius_mode=RADIUS_3SIGMA):
    """Projection + SH colour of all Gaussians into one view (FP64).
    ``radius_mode`` picks the screen box that selects tiles: the per-axis
    3-sigma box, the opacity-aware box (3-sigma box clipped to the region
    alpha >= 1/255) or the square of the largest eigenvalue."""
    N = P.n
    vm, it = _d(viewmat).reshape(12), _d(intr).reshape(4)
    out = dict(u=np.zeros(N), v=np.zeros(N), depth=np.zeros(N), cov=np.zeros((3, N)),
               conic=np.zeros((3, N)), sigma=np.zeros(N), rgb=np.zeros((3, N)),
               radii=np.zeros((2, N), np.int32), tiles=np.zeros(N, np.int32),
               clamp=np.zeros(N, np.uint8), visible=np.zeros(N, np.uint8), margin=np.zeros(N),
               margin_img=np.zeros(N))
    rc = lib().or_project(N, P.deg, _p(P.means, _D), _p(P.log_scales, _D), _p(P.quats, _D),
                          _p(P.opac, _D), _p(P.sh, _D), _p(vm, _D), _p(it, _D), int(W), int(H),
                          float(near), float(far), float(eps2d), int(tile), int(radius_mode),
                          *[_p(out[k], _D) for k in ("u", "v", "depth", "cov", "conic", "sigma", "rgb")],
                          _p(out["radii"], _I), _p(out["tiles"], _I), _p(out["clamp"], _U8),
                          _p(out["visible"], _U8), _p(out["margin"], _D), _p(out["margin_img"], _D))
    assert rc == 0
    return out


# --------------------------------------------------------------------------
# binning
# --------------------------------------------------------------------------
def tile_grid(W, H, tile):
    return (W + tile - 1) // tile, (H + tile - 1) // tile


def bin_view(u32, v32, depth32, radii, W, H, tile, tile_offset=0):
    """Unsorted intersection keys/values of one view (float32 inputs)."""
    u32 = np.ascontiguousarray(u32, np.float32)
    v32 = np.ascontiguousarray(v32, np.float32)
    z32 = np.ascontiguousarray(depth32, np.float32)
    radii = np.ascontiguousarray(radii, np.int32)
    N = u32.shape[0]
    L = lib()
    m = L.or_bin_emit(N, _p(u32, _F), _p(v32, _F), _p(z32, _F), _p(radii, _I), W, H, tile,
                      tile_offset, None, None, 0)
    keys = np.zeros(max(m, 1), np.uint64)
    vals = np.zeros(max(m, 1), np.int32)
    L.or_bin_emit(N, _p(u32, _F), _p(v32, _F), _p(z32, _F), _p(radii, _I), W, H, tile, tile_offset,
                  _p(keys, _U64), _p(vals, _I), m)
    return keys[:m], vals[:m]


def sort_pairs(keys, vals):
    keys = np.ascontiguousarray(keys, np.uint64).copy()
    vals = np.ascontiguousarray(vals, np.int32).copy()
    assert lib().or_sort_pairs(keys.shape[0], _p(keys, _U64), _p(vals, _I)) == 0
    return keys, vals


def tile_ranges(keys, n_tiles):
    keys = np.ascontiguousarray(keys, np.uint64)
    r = np.zeros(2 * n_tiles, np.int32)
    assert lib().or_tile_ranges(keys.shape[0], _p(keys, _U64), n_tiles, _p(r, _I)) == 0
    return r.reshape(n_tiles, 2)


def bin_views(views, sizes, tile):
    """Binning of several views into one global tile space.

    ``views`` holds per view (u32, v32, depth32, radii[2][N]).  Returns sorted
    keys, values, ranges [T_total][2] and the per-view tile offsets."""
    keys, vals, offs = [], [], [0]
    for (u, v, z, r), (W, H) in zip(views, sizes):
        k, x = bin_view(u, v, z, r, int(W), int(H), tile, offs[-1])
        keys.append(k)
        vals.append(x)
        tx, ty = tile_grid(int(W), int(H), tile)
        offs.append(offs[-1] + tx * ty)
    keys = np.concatenate(keys) if keys else np.zeros(0, np.uint64)
    vals = np.concatenate(vals) if vals else np.zeros(0, np.int32)
    keys, vals = sort_pairs(keys, vals)
    return keys, vals, tile_ranges(keys, offs[-1]), np.asarray(offs, np.int64)


# --------------------------------------------------------------------------
# compositing
# --------------------------------------------------------------------------
def raster_fwd(W, H, tile, ranges, vals, sp, bg=(0.0, 0.0, 0.0)):
    """Forward compositing of one view.  ``ranges`` [tiles][2] index ``vals``;
    ``sp`` holds FP64 u, v, conic [3][N], sigma, rgb [3][N]."""
    N = sp["u"].shape[0]
    ranges = np.ascontiguousarray(ranges, np.int32)
    vals = np.ascontiguousarray(vals, np.int32)
    u, v, cA, cB, cC = _d(sp["u"]), _d(sp["v"]), _d(sp["conic"][0]), _d(sp["conic"][1]), _d(sp["conic"][2])
    sig, rgb, bg = _d(sp["sigma"]), _d(sp["rgb"]), _d(bg)
    img = np.zeros((3, H, W))
    T = np.zeros((H, W))
    last = np.zeros((H, W), np.int32)
    visits = np.zeros((H, W), np.int32)
    margin = np.zeros((H, W))
    rc = lib().or_raster_fwd(W, H, tile, _p(ranges, _I), _p(vals, _I), N, _p(u, _D), _p(v, _D),
                             _p(cA, _D), _p(cB, _D), _p(cC, _D), _p(sig, _D), _p(rgb, _D),
                             _p(bg, _D), _p(img, _D), _p(T, _D), _p(last, _I), _p(visits, _I),
                             _p(margin, _D))
    assert rc == 0
    return dict(img=img, T=T, last=last, visits=visits, margin=margin)


def raster_fwd_rect(W, H, tile, ranges, vals, sp, x0, y0, x1, y1, bg=(0.0, 0.0, 0.0)):
    """Forward compositing of the pixel rectangle [x0, x1) x [y0, y1) of one
    view (as ``raster_fwd``): image [3][h][w] and per-pixel decision
    signatures [h][w] (uint64)."""
    N = sp["u"].shape[0]
    ranges = np.ascontiguousarray(ranges, np.int32)
    vals = np.ascontiguousarray(vals, np.int32)
    u, v, cA, cB, cC = _d(sp["u"]), _d(sp["v"]), _d(sp["conic"][0]), _d(sp["conic"][1]), _d(sp["conic"][2])
    sig, rgb, bg = _d(sp["sigma"]), _d(sp["rgb"]), _d(bg)
    h, w = y1 - y0, x1 - x0
    img = np.zeros((3, h, w))
    sg = np.zeros((h, w), np.uint64)
    rc = lib().or_raster_fwd_rect(W, H, tile, _p(ranges, _I), _p(vals, _I), N, _p(u, _D), _p(v, _D), _p(cA, _D),
                                  _p(cB, _D), _p(cC, _D), _p(sig, _D), _p(rgb, _D), _p(bg, _D), int(x0), int(y0),
                                  int(x1), int(y1), _p(img, _D), _p(sg, _U64))
    assert rc == 0
    return img, sg


def raster_bwd(W, H, tile, ranges, vals, sp, d_img, d_alpha=None, bg=(0.0, 0.0, 0.0)):
    """Backward compositing of one view.  Returns FP64 gradients with respect
    to u, v, conic (A, B, C), sigma and rgb ([3][N])."""
    N = sp["u"].shape[0]
    ranges = np.ascontiguousarray(ranges, np.int32)
    vals = np.ascontiguousarray(vals, np.int32)
    u, v, cA, cB, cC = _d(sp["u"]), _d(sp["v"]), _d(sp["conic"][0]), _d(sp["conic"][1]), _d(sp["conic"][2])
    sig, rgb, bg = _d(sp["sigma"]), _d(sp["rgb"]), _d(bg)
    d_img = _d(d_img)
    da = _d(d_alpha) if d_alpha is not None else None
    g = dict(u=np.zeros(N), v=np.zeros(N), conic=np.zeros((3, N)), sigma=np.zeros(N),
             rgb=np.zeros((3, N)))
    gc = g["conic"]
    gA, gB, gC = np.zeros(N), np.zeros(N), np.zeros(N)
    rc = lib().or_raster_bwd(W, H, tile, _p(ranges, _I), _p(vals, _I), N, _p(u, _D), _p(v, _D),
                             _p(cA, _D), _p(cB, _D), _p(cC, _D), _p(sig, _D), _p(rgb, _D),
                             _p(bg, _D), _p(d_img, _D), _p(da, _D) if da is not None else None,
                             _p(g["u"], _D), _p(g["v"], _D), _p(gA, _D), _p(gB, _D), _p(gC, _D),
                             _p(g["sigma"], _D), _p(g["rgb"], _D))
    assert rc == 0
    gc[0], gc[1], gc[2] = gA, gB, gC
    return g


def project_bwd(P, viewmat, intr, W, H, g, near=0.01, far=1e10, eps2d=0.3, tile=16, acc=None,
                radius_mode=RADIUS_3SIGMA):
    """Backward of :func:`project` for one view.  ``g`` holds upstream
    gradients u, v, conic [3][N], sigma, rgb [3][N].  Accumulates into ``acc``
    (dict of means, log_scales, quats, opac, sh) and returns it."""
    N = P.n
    K = (P.deg + 1) ** 2
    if acc is None:
        acc = dict(means=np.zeros((3, N)), log_scales=np.zeros((3, N)), quats=np.zeros((4, N)),
                   opac=np.zeros(N), sh=np.zeros((K, 3, N)))
    vm, it = _d(viewmat).reshape(12), _d(intr).reshape(4)
    guv = _d(np.stack([g["u"], g["v"]]))
    gcon, gsig, grgb = _d(g["conic"]), _d(g["sigma"]), _d(g["rgb"])
    rc = lib().or_project_bwd(N, P.deg, _p(P.means, _D), _p(P.log_scales, _D), _p(P.quats, _D),
                              _p(P.opac, _D), _p(P.sh, _D), _p(vm, _D), _p(it, _D), int(W), int(H),
                              float(near), float(far), float(eps2d), int(tile), int(radius_mode), _p(guv, _D),
                              _p(gcon, _D), _p(gsig, _D), _p(grgb, _D), _p(acc["means"], _D),
                              _p(acc["log_scales"], _D), _p(acc["quats"], _D), _p(acc["opac"], _D),
                              _p(acc["sh"], _D))
    assert rc == 0
    return acc


# --------------------------------------------------------------------------
# loss
# --------------------------------------------------------------------------
def l2_loss(imgs, targets):
    """L = mean over all views, channels and pixels of (img - target)^2 and
    dL/dimg = 2 (img - target) / count (the image-space loss of Section 4;
    mean rather than sum is a reading)."""
    count = sum(int(np.asarray(t).size) for t in targets)
    loss = sum(float(np.sum((_d(i) - _d(t)) ** 2)) for i, t in zip(imgs, targets)) / count
    grads = [2.0 * (_d(i) - _d(t)) / count for i, t in zip(imgs, targets)]
    return loss, grads


# --------------------------------------------------------------------------
# whole step (FP64 end to end)
# --------------------------------------------------------------------------
def step(scene, P=None, tile=16, near=0.01, far=1e10, eps2d=0.3, bg=(0.0, 0.0, 0.0), backward=True,
         radius_mode=RADIUS_3SIGMA):
    """One forward (+ backward) pass of the whole path in FP64.

    Binning takes its decisions on the FP32-rounded mean, radius and depth
    (reading R8/R10), exactly as the method stores them; everything else is
    FP64.  Returns images, loss, per-view projections, lists and, if
    requested, parameter gradients."""
    if P is None:
        P = Params.of(scene)
    projs, views = [], []
    for v in range(scene.n_views):
        W, H = (int(x) for x in scene.sizes[v])
        pr = project(P, scene.viewmats[v], scene.intrinsics[v], W, H, near, far, eps2d, tile, radius_mode)
        projs.append(pr)
        views.append((pr["u"].astype(np.float32), pr["v"].astype(np.float32),
                      pr["depth"].astype(np.float32), pr["radii"]))
    keys, vals, ranges, offs = bin_views(views, scene.sizes, tile)
    imgs, fwds = [], []
    for v in range(scene.n_views):
        W, H = (int(x) for x in scene.sizes[v])
        pr = projs[v]
        f = raster_fwd(W, H, tile, ranges[offs[v]:offs[v + 1]], vals, pr, bg)
        fwds.append(f)
        imgs.append(f["img"])
    loss, dimgs = l2_loss(imgs, scene.targets)
    out = dict(imgs=imgs, loss=loss, projs=projs, keys=keys, vals=vals, ranges=ranges,
               offsets=offs, fwds=fwds, d_imgs=dimgs)
    if backward:
        acc = None
        for v in range(scene.n_views):
            W, H = (int(x) for x in scene.sizes[v])
            g2 = raster_bwd(W, H, tile, ranges[offs[v]:offs[v + 1]], vals, projs[v], dimgs[v], None, bg)
            acc = project_bwd(P, scene.viewmats[v], scene.intrinsics[v], W, H, g2, near, far, eps2d,
                              tile, acc, radius_mode)
        out["grads"] = acc
    return out


# --------------------------------------------------------------------------
# adaptive density control statistics (3D Gaussian Splatting, Kerbl et al.
# 2023; the paper densifies with it, Section 5)
# --------------------------------------------------------------------------
def densify_stats(g_uv, visible, radii, sizes, acc=None):
    """Running sums over the views that see each Gaussian: the norm of the
    gradient with respect to the projected mean in normalised device
    coordinates (u = ((x_ndc + 1) W - 1) / 2, so d/dx_ndc = W / 2 d/du), the
    number of such views, and the largest screen radius.  ``g_uv[v]`` is
    [2][N] (dL/du, dL/dv), ``visible[v]`` [N], ``radii[v]`` [2][N]."""
    N = np.asarray(visible[0]).shape[0]
    if acc is None:
        acc = dict(grad=np.zeros(N), count=np.zeros(N, np.int64), max_radius=np.zeros(N, np.int64))
    for v, (W, H) in enumerate(np.asarray(sizes).reshape(-1, 2)):
        vis = np.asarray(visible[v]).astype(bool)
        gx = _d(g_uv[v][0]) * (W / 2.0)
        gy = _d(g_uv[v][1]) * (H / 2.0)
        acc["grad"][vis] += np.hypot(gx, gy)[vis]
        acc["count"][vis] += 1
        r = np.max(np.asarray(radii[v]), axis=0)
        acc["max_radius"][vis] = np.maximum(acc["max_radius"][vis], r[vis])
    return acc


# --------------------------------------------------------------------------
# optimiser (the paper's Section 3.2 fused Adam; Kingma and Ba 2015)
# --------------------------------------------------------------------------
def adam(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-15):
    """One Adam step at step number t (1-based), FP64, bias-corrected:
    returns the new (p, m, v)."""
    p, g, m, v = _d(p), _d(g), _d(m), _d(v)
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


# --------------------------------------------------------------------------
# 3-D Morton order (the paper's Section 5.2 locality pass)
# --------------------------------------------------------------------------
def morton_cells(means, origin, inv_cell):
    """10-bit cell per axis: clamp(floor((mu - origin) * inv_cell), 0, 1023),
    float32 subtraction then multiplication (non-finite -> 0)."""
    m = np.asarray(means, np.float32)
    o = np.asarray(origin, np.float32)[:, None]
    c = np.asarray(inv_cell, np.float32)[:, None]
    with np.errstate(invalid="ignore", over="ignore"):
        t = np.floor((m - o) * c)
    t = np.where(np.isfinite(t), t, 0.0)
    return np.clip(t, 0, 1023).astype(np.int64)


def morton_codes(means, origin, inv_cell):
    """30-bit codes: bit 3b + k is bit b of axis k's cell (plain bit loop)."""
    cells = morton_cells(means, origin, inv_cell)
    code = np.zeros(cells.shape[1], np.int64)
    for b in range(10):
        for k in range(3):
            code |= ((cells[k] >> b) & 1) << (3 * b + k)
    return code


def morton_order(means, origin, inv_cell):
    return np.argsort(morton_codes(means, origin, inv_cell), kind="stable").astype(np.int32)


# --------------------------------------------------------------------------
# SSIM + L1 image loss (the paper's per-camera fused SSIM loss operator,
# Section 4; SSIM of Wang et al. 2004 with the 3D Gaussian Splatting
# settings: 11x11 Gaussian window, sigma 1.5, zero padding, C1 = 0.01^2,
# C2 = 0.03^2, loss = (1 - lam) mean|x - y| + lam (1 - mean SSIM))
# --------------------------------------------------------------------------
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2


def ssim_window(size=11, sigma=1.5):
    x = np.arange(size) - size // 2
    w = np.exp(-(x * x) / (2.0 * sigma * sigma))
    return w / w.sum()


def _blur(img, w):
    """Separable 'same' convolution with zero padding (rows, then columns).
    The padding is explicit so that axes shorter than the window keep their
    length."""
    r = len(w) // 2
    a = np.apply_along_axis(lambda q: np.convolve(np.pad(q, r), w, mode="valid"), -1, _d(img))
    return np.apply_along_axis(lambda q: np.convolve(np.pad(q, r), w, mode="valid"), -2, a)


def ssim_map(x, y):
    w = ssim_window()
    mx, my = _blur(x, w), _blur(y, w)
    exx, eyy, exy = _blur(_d(x) * x, w), _blur(_d(y) * y, w), _blur(_d(x) * y, w)
    A = 2 * mx * my + SSIM_C1
    Bv = 2 * (exy - mx * my) + SSIM_C2
    C = mx * mx + my * my + SSIM_C1
    D = (exx - mx * mx) + (eyy - my * my) + SSIM_C2
    return A * Bv / (C * D), (mx, my, exx, exy, A, Bv, C, D)


def ssim_l1_loss(imgs, targets, lam=0.2):
    """Loss over all views (each [3][H][W]) and d loss / d img per view.
    Means are over every element of every view."""
    count = sum(int(np.asarray(t).size) for t in targets)
    w = ssim_window()
    loss, grads = 0.0, []
    for x, y in zip(imgs, targets):
        x, y = _d(x), _d(y)
        S, (mx, my, exx, exy, A, Bv, C, D) = ssim_map(x, y)
        loss += (1 - lam) * np.abs(x - y).sum() / count + lam * (1.0 - S).sum() / count
        gS = -lam / count
        # S = A B / (C D) as a function of (mx, exx, exy) per pixel
        d_mx = gS * ((2 * my * Bv - 2 * my * A) / (C * D) - S * (2 * mx / C - 2 * mx / D))
        d_exx = gS * (-S / D)
        d_exy = gS * (2 * A / (C * D))
        g = _blur(d_mx, w) + 2 * x * _blur(d_exx, w) + y * _blur(d_exy, w)
        g += (1 - lam) * np.sign(x - y) / count
        grads.append(g)
    return loss, grads
