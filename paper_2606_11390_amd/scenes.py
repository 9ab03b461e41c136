"""Seeded synthetic Gaussian scenes, cameras and target images.

This module only *draws inputs*.  It holds no step of the splatting method
(no projection, colour, binning or compositing arithmetic), so the GPU path and
the CPU oracle can both take their inputs from it without sharing any of the
method's code.

Every array comes from ``numpy.random.default_rng(seed)`` (PCG64) in a fixed
draw order, is generated in float64 (SH coefficients in float32, to bound host
memory at tens of millions of Gaussians) and is cast once to float32.

Layouts (planar structure-of-arrays, the layout the C ABI takes):

* ``means[3][N]``, ``log_scales[3][N]``, ``quats[4][N]`` (w, x, y, z, need not
  be unit), ``opacity_logits[N]``, ``sh[K][3][N]`` with ``K = (deg+1)**2`` and
  coefficient index ``l*l + l + m``;
* cameras: ``viewmats[V][12]`` (world-to-camera ``[R|t]``, row-major, OpenCV
  axes: +x right, +y down, +z forward), ``intrinsics[V][4]`` (fx, fy, cx, cy),
  ``sizes[V][2]`` (width, height);
* targets: one ``[3][H][W]`` float32 image per view, uniform in [0, 1).

The five workloads are those the benchmark configurations name (scene sizes,
value distributions, camera rigs); ``n_gaussians`` may shrink a scene for
tests while keeping its distributions.
"""
from __future__ import annotations

import dataclasses
import numpy as np

VIEW_SIZES = ((640, 480), (1280, 720), (1920, 1080), (2560, 1440), (3840, 2160))


@dataclasses.dataclass
class Scene:
    means: np.ndarray          # [3][N] f32
    log_scales: np.ndarray     # [3][N] f32
    quats: np.ndarray          # [4][N] f32 (w, x, y, z)
    opacity_logits: np.ndarray  # [N] f32
    sh: np.ndarray             # [K][3][N] f32
    sh_degree: int
    viewmats: np.ndarray       # [V][12] f32
    intrinsics: np.ndarray     # [V][4] f32
    sizes: np.ndarray          # [V][2] i32 (W, H)
    targets: list              # V arrays [3][H][W] f32
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.means.shape[1])

    @property
    def n_views(self) -> int:
        return int(self.sizes.shape[0])

    @property
    def pixels(self) -> int:
        return int(sum(int(w) * int(h) for w, h in self.sizes))


def _look_at(eye, target, world_up=(0.0, 0.0, 1.0)):
    """World-to-camera [R|t] for a camera at ``eye`` looking at ``target``."""
    eye = np.asarray(eye, np.float64)
    fwd = np.asarray(target, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    up = np.asarray(world_up, np.float64)
    if abs(float(fwd @ up)) > 0.99:
        up = np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    rot = np.stack([right, down, fwd])          # rows: camera axes in world
    t = -rot @ eye
    return np.concatenate([rot, t[:, None]], axis=1).reshape(12)


def _cube_surface_point(rng, half):
    face = int(rng.integers(0, 6))
    axis, sign = face // 2, (1.0 if face % 2 else -1.0)
    p = rng.uniform(-half, half, size=3)
    p[axis] = sign * half
    return p


def _haar_rotation(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _unit_quats(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def _sh(rng, n, degree, dc_std, rest_std, chunk=1 << 20):
    k = (degree + 1) ** 2
    sh = np.empty((k, 3, n), np.float32)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        block = rng.standard_normal((k, 3, e - s), dtype=np.float32)
        block[0] *= np.float32(dc_std)
        if k > 1:
            block[1:] *= np.float32(rest_std)
        sh[:, :, s:e] = block
    return sh


def _blob_means(rng, n, n_blobs, half):
    centres = rng.uniform(-half, half, size=(n_blobs, 3))
    stds = rng.uniform(0.5, 3.0, size=(n_blobs, 3))
    rots = np.stack([_haar_rotation(rng) for _ in range(n_blobs)])
    which = rng.integers(0, n_blobs, size=n)
    local = rng.standard_normal((n, 3)) * stds[which]
    pts = centres[which] + np.einsum("nij,nj->ni", rots[which], local)
    return pts.T


def _targets(rng, sizes):
    return [rng.uniform(0.0, 1.0, size=(3, int(h), int(w))).astype(np.float32)
            for w, h in sizes]


def _finish(means, log_scales, quats, opac, sh, degree, viewmats, intr, sizes, rng, name):
    sizes = np.asarray(sizes, np.int32).reshape(-1, 2)
    return Scene(means=np.ascontiguousarray(means, np.float32),
                 log_scales=np.ascontiguousarray(log_scales, np.float32),
                 quats=np.ascontiguousarray(quats, np.float32),
                 opacity_logits=np.ascontiguousarray(opac, np.float32),
                 sh=np.ascontiguousarray(sh, np.float32), sh_degree=degree,
                 viewmats=np.ascontiguousarray(np.asarray(viewmats, np.float64).reshape(-1, 12), np.float32),
                 intrinsics=np.ascontiguousarray(np.asarray(intr, np.float64).reshape(-1, 4), np.float32),
                 sizes=sizes, targets=_targets(rng, sizes), name=name)


def tiny(seed=1, n_gaussians=2000, width=128, height=128, focal=120.0):
    """2,000 Gaussians, SH degree 0, one 128x128 pinhole camera at the origin."""
    rng = np.random.default_rng(seed)
    n = n_gaussians
    means = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(2, 6, n)])
    log_scales = rng.normal(-3.0, 0.5, size=(3, n))
    quats = _unit_quats(rng, n)
    opac = rng.normal(0.0, 1.0, size=n)
    sh = _sh(rng, n, 0, 0.3, 0.0)
    viewmat = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1).reshape(12)
    intr = [focal, focal, width / 2.0, height / 2.0]
    return _finish(means, log_scales, quats, opac, sh, 0, viewmat, intr, [(width, height)], rng, "tiny")


def blobs(seed, n_gaussians, n_blobs, half, views, sh_degree=3, log_scale=(-4.0, 0.7),
          opacity_std=1.5, name="blobs"):
    """Blob-mixture scene: Gaussians drawn from ``n_blobs`` anisotropic 3-D
    normal blobs (centres uniform in a cube of half-size ``half``, per-axis std
    uniform in [0.5, 3] m, Haar-random orientation); each camera sits on the
    cube surface looking at the origin.  ``views`` is a list of
    (width, height, fx) triples."""
    rng = np.random.default_rng(seed)
    n = n_gaussians
    means = _blob_means(rng, n, n_blobs, half)
    log_scales = rng.normal(log_scale[0], log_scale[1], size=(3, n))
    quats = _unit_quats(rng, n)
    opac = rng.normal(0.0, opacity_std, size=n)
    sh = _sh(rng, n, sh_degree, 0.3, 0.05)
    viewmats, intr, sizes = [], [], []
    for (w, h, f) in views:
        viewmats.append(_look_at(_cube_surface_point(rng, half), (0.0, 0.0, 0.0)))
        intr.append([f, f, w / 2.0, h / 2.0])
        sizes.append((w, h))
    return _finish(means, log_scales, quats, opac, sh, sh_degree, viewmats, intr, sizes, rng, name)


def hd(seed=2, n_gaussians=200_000):
    """200k Gaussians (32 blobs, 20 m cube), SH degree 3, one 1920x1080 view, f=1500."""
    return blobs(seed, n_gaussians, 32, 10.0, [(1920, 1080, 1500.0)], name="hd")


def uhd(seed=3, n_gaussians=5_000_000, width=3840, height=2160, focal=3000.0):
    """5M Gaussians (512 blobs, 200 m cube), SH degree 3, one 3840x2160 view, f=3000."""
    return blobs(seed, n_gaussians, 512, 100.0, [(width, height, focal)], name="uhd")


def multiview(seed=4, n_gaussians=20_000_000, n_views=16):
    """20M Gaussians (2,048 blobs, 500 m cube), SH degree 3, 16 views of sizes
    drawn uniformly from 640x480 ... 3840x2160, fx = 0.78125 W (the same
    horizontal field of view as the 1080p and 4K rigs)."""
    rng = np.random.default_rng(seed + 1000)
    picks = rng.integers(0, len(VIEW_SIZES), size=n_views)
    views = [(VIEW_SIZES[i][0], VIEW_SIZES[i][1], 0.78125 * VIEW_SIZES[i][0]) for i in picks]
    return blobs(seed, n_gaussians, 2048, 250.0, views, name="multiview")


def city(seed=5, n_gaussians=60_000_000, n_views=8, n_boxes=5000, width=3840, height=2160,
         focal=3000.0):
    """City-like scene: 40 % of the Gaussians on a 2 km x 2 km ground plane
    (z ~ N(0, 0.05)), 60 % on the walls and roofs of ``n_boxes`` axis-aligned
    boxes (footprint sides U(10, 60) m, heights U(5, 120) m, faces picked in
    proportion to area); log-scales N(-5, 0.8).  Cameras stand 2 m above the
    ground outside every box, pitch 0, heading uniform."""
    rng = np.random.default_rng(seed)
    n = n_gaussians
    n_ground = int(round(0.4 * n))
    n_box = n - n_ground
    ground = np.stack([rng.uniform(-1000, 1000, n_ground), rng.uniform(-1000, 1000, n_ground),
                       rng.normal(0.0, 0.05, n_ground)])
    cx = rng.uniform(-1000, 1000, n_boxes)
    cy = rng.uniform(-1000, 1000, n_boxes)
    sx = rng.uniform(10, 60, n_boxes)
    sy = rng.uniform(10, 60, n_boxes)
    hz = rng.uniform(5, 120, n_boxes)
    # faces: 0/1 walls normal to x, 2/3 walls normal to y, 4 roof
    areas = np.stack([sy * hz, sy * hz, sx * hz, sx * hz, sx * sy], axis=1)
    flat = (areas / areas.sum()).reshape(-1)
    pick = rng.choice(flat.size, size=n_box, p=flat)
    b, f = pick // 5, pick % 5
    a1 = rng.uniform(-0.5, 0.5, n_box)
    a2 = rng.uniform(0.0, 1.0, n_box)
    x = cx[b] + np.where(f == 0, -0.5, np.where(f == 1, 0.5, a1)) * sx[b]
    y = cy[b] + np.where(f == 2, -0.5, np.where(f == 3, 0.5, np.where(f == 4, a2 - 0.5, a1))) * sy[b]
    z = np.where(f == 4, hz[b], a2 * hz[b])
    x = np.where(f == 4, cx[b] + a1 * sx[b], x)
    means = np.concatenate([ground, np.stack([x, y, z])], axis=1)
    log_scales = rng.normal(-5.0, 0.8, size=(3, n))
    quats = _unit_quats(rng, n)
    opac = rng.normal(0.0, 1.5, size=n)
    sh = _sh(rng, n, 3, 0.3, 0.05)
    viewmats, intr, sizes = [], [], []
    while len(viewmats) < n_views:
        px, py = rng.uniform(-1000, 1000, 2)
        inside = (np.abs(px - cx) < 0.5 * sx) & (np.abs(py - cy) < 0.5 * sy)
        if inside.any():
            continue
        head = rng.uniform(0, 2 * np.pi)
        eye = np.array([px, py, 2.0])
        viewmats.append(_look_at(eye, eye + np.array([np.cos(head), np.sin(head), 0.0])))
        intr.append([focal, focal, width / 2.0, height / 2.0])
        sizes.append((width, height))
    return _finish(means, log_scales, quats, opac, sh, 3, viewmats, intr, sizes, rng, "city")


def random_upstream(seed, shape, dtype=np.float32):
    """Seeded N(0, 1) cotangent used to drive backward passes in tests."""
    return np.random.default_rng(seed).standard_normal(shape).astype(dtype)
