"""Splatting step on one GPU: buffers, autograd wrapper and a capturable step.

``Renderer`` owns every device buffer of the path for a fixed Gaussian count,
SH degree and set of view sizes, and runs the C-ABI calls in order on torch's
current stream:

    gs_project (also zeroing the visible pairs' 2-D gradient records)
    -> gs_bin_sort -> [gs_tile_schedule] -> gs_rasterize_fwd
    -> gs_rasterize_bwd_l2 (the L2 loss and the rasteriser backward in one
       pass, accumulating into those records; gs_loss_l2 -> gs_rasterize_bwd
       when ``fuse_l2`` is off or the backward runs on the work queue)
    -> gs_project_bwd

The rasterisers' tile order is chosen per pass (``order``, ``order_bwd``):
"tile" (one workgroup per tile in tile order), "xcd" (a static order giving
each XCD one band of neighbouring tiles), "heavy" (longest lists dispatched
first, recomputed every step) or "queue" (persistent waves pulling the heavy-
first order from a global counter).  None of them changes a result bit.

``render()`` exposes the differentiable part as a ``torch.autograd.Function``;
``Renderer.step()`` runs forward + L2 loss + backward without autograd and
without any host synchronisation, so it can be captured in a HIP graph
(``Renderer.capture()``).  Intersection capacity is fixed per renderer; the
overflow word of ``gs_bin_sort`` tells the caller to grow it
(``Renderer.fit_capacity()``).
"""
from __future__ import annotations

import gc

import numpy as np
import torch

from . import binding as B


ORDERS = ("tile", "xcd", "heavy", "queue")
# dies with private L2 caches that a grid launch is spread over round-robin
N_XCD = 8


class Renderer:
    def __init__(self, n, sh_degree, sizes, tile=16, capacity=1 << 20, near=0.01, far=1e10, eps2d=0.3,
                 background=(0.0, 0.0, 0.0), persistent=False, block=(0, 0), block_bwd=None, device="cuda",
                 radius_mode=0, order=None, order_bwd=None, fuse_l2=True, loss="l2", ssim_lambda=0.2,
                 unseen_in_bwd=True):
        # screen box rule of the projection (GS_RADIUS_*)
        self.radius_mode = int(radius_mode)
        # step(): L2 loss formed inside the rasteriser backward (d_images not stored)
        self.fuse_l2 = bool(fuse_l2)
        # the step's image loss: "l2" (mean squared error) or "ssim_l1" (the 3D
        # Gaussian Splatting training loss, (1 - lambda) L1 + lambda (1 - SSIM))
        if loss not in ("l2", "ssim_l1"):
            raise ValueError(f"unknown loss {loss!r}")
        self.loss_kind = loss
        self.ssim_lambda = float(ssim_lambda)
        # step() with the fused L2 backward: the zero gradients of the
        # Gaussians no view sees are written by the compositing backward's
        # waves (they need only the projection's flags), and the projection
        # backward writes the seen Gaussians' gradients alone
        self.unseen_in_bwd = bool(unseen_in_bwd)
        # wave pixel blocks (width, pixels per lane) of the forward and backward rasterisers
        self.block = tuple(int(x) for x in block)
        self.block_bwd = self.block if block_bwd is None else tuple(int(x) for x in block_bwd)
        self.n = int(n)
        self.deg = int(sh_degree)
        self.sizes = np.asarray(sizes, np.int32).reshape(-1, 2)
        self.V = int(self.sizes.shape[0])
        if not 1 <= self.V <= B.GS_MAX_VIEWS:
            raise ValueError("view count out of range")
        self.tile = int(tile)
        self.near, self.far, self.eps2d = float(near), float(far), float(eps2d)
        self.background = np.asarray(background, np.float32)
        # tile order of each rasteriser pass; persistent=True selects the queue
        self.order = order if order is not None else ("queue" if persistent else "tile")
        self.order_bwd = order_bwd if order_bwd is not None else self.order
        for o in (self.order, self.order_bwd):
            if o not in ORDERS:
                raise ValueError(f"unknown tile order {o!r}")
        self.device = torch.device(device)
        self.tiles_x, self.tile_off, self.pix_off = B.tile_grid(self.sizes, self.tile)
        self.total_tiles = int(self.tile_off[-1])
        self.pixels = int(self.pix_off[-1])
        V, N, dev = self.V, self.n, self.device
        e = lambda *s, dt=torch.float32: torch.empty(*s, dtype=dt, device=dev)
        self.splats = e(V * N * B.SPLAT_FLOATS)
        self.depths = e(V * N)
        self.radii = e(V * N * 2, dt=torch.int32)
        self.tiles_touched = e(V * N, dt=torch.int32)
        self.tile_rects = e(V * N * 2, dt=torch.int32)
        self.flags = e(V * N, dt=torch.uint8)
        self.ranges = e(self.total_tiles * 2, dt=torch.int32)
        self.info = torch.zeros(4, dtype=torch.int32, device=dev)
        self.images = e(3 * self.pixels)
        self.T_final = e(self.pixels)
        self.n_contrib = e(self.pixels, dt=torch.int32)
        self.grad2d = torch.zeros(V * N * B.GRAD_FLOATS, dtype=torch.float32, device=dev)
        self.d_images = e(3 * self.pixels)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.loss_ws = e(max(1, B.loss_workspace_size(3 * self.pixels)), dt=torch.uint8)
        self.l2_ws = e(max(8, B.rasterize_bwd_l2_workspace_size(self.sizes, self.tile)), dt=torch.uint8)
        self.ssim_ws = (e(max(8, B.ssim_workspace_size(self.sizes)), dt=torch.uint8) if loss == "ssim_l1"
                        else None)
        self.queue = torch.zeros(1, dtype=torch.int32, device=dev)
        self.schedule = e(max(1, B.tile_schedule_size(self.total_tiles)), dt=torch.uint8)
        self.schedule_xcd = e(max(1, B.tile_schedule_size(self.total_tiles)), dt=torch.uint8)
        B.tile_order_xcd(self.total_tiles, N_XCD, self.schedule_xcd)
        self.capacity = 0
        self.set_capacity(capacity)
        self.graph = None

    # ---------------------------------------------------------------- buffers
    def set_capacity(self, capacity):
        capacity = int(max(1, min(capacity, 0x7FFFFFFF)))
        if capacity == self.capacity:
            return
        self.capacity = capacity
        self.isect_tile = torch.empty(capacity, dtype=torch.int32, device=self.device)
        self.isect_gid = torch.empty(capacity, dtype=torch.int32, device=self.device)
        ws = B.bin_sort_workspace_size(self.n, self.V, capacity, self.total_tiles)
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=self.device)
        self.graph = None

    def memory_bytes(self):
        return sum(t.numel() * t.element_size() for t in self.__dict__.values() if isinstance(t, torch.Tensor))

    # ------------------------------------------------------------ the stages
    def project(self, P, cams, clear_grad2d=False):
        """``clear_grad2d``: also zero the visible pairs' 2-D gradient records,
        so that the backward of this step may accumulate into them."""
        B.project(P["means"], P["log_scales"], P["quats"], P["opacity_logits"], P["sh"], self.deg,
                  cams["viewmats"], cams["intrinsics"], self.sizes, self.near, self.far, self.eps2d,
                  self.tile, self.splats, self.depths, self.radii, self.tiles_touched, self.tile_rects,
                  self.flags, self.radius_mode, grad2d_clear=self.grad2d if clear_grad2d else None)

    def bin_sort(self):
        B.bin_sort(self.tile_rects, self.depths, self.n, self.sizes, self.tile, self.capacity, self.workspace,
                   self.isect_tile, self.isect_gid, self.ranges, self.info)
        if "heavy" in (self.order, self.order_bwd) or "queue" in (self.order, self.order_bwd):
            B.tile_schedule(self.ranges, self.total_tiles, self.schedule)

    @property
    def persistent(self):
        return self.order == "queue"

    def _sched(self, order=None):
        order = order or self.order
        if order == "tile":
            return None, None
        if order == "xcd":
            return self.schedule_xcd, None
        if order == "heavy":
            return self.schedule, None
        return self.schedule, self.queue

    def raster_fwd(self, images=None):
        s, q = self._sched()
        B.rasterize_fwd(self.splats, self.isect_gid, self.ranges, self.n, self.sizes, self.tile,
                        self.background, s, q, self.images if images is None else images, self.T_final,
                        self.n_contrib, block=self.block)

    def raster_bwd(self, d_images, d_alpha=None, accumulate=False):
        s, q = self._sched(self.order_bwd)
        B.rasterize_bwd(self.splats, self.isect_gid, self.ranges, self.n, self.sizes, self.tile,
                        self.background, s, q, self.T_final, self.n_contrib, d_images, d_alpha, self.grad2d,
                        accumulate=accumulate, block=self.block_bwd)

    def project_bwd(self, P, cams, grads, part=B.GRADS_ALL):
        B.project_bwd(P["means"], P["log_scales"], P["quats"], P["opacity_logits"], P["sh"], self.deg,
                      cams["viewmats"], cams["intrinsics"], self.sizes, self.eps2d, self.flags, self.grad2d,
                      grads["means"], grads["log_scales"], grads["quats"], grads["opacity_logits"],
                      grads["sh"], part=part)


    def loss_l2(self, targets):
        B.loss_l2(self.images, targets, self.loss, self.d_images, self.loss_ws)

    @property
    def fused_l2_active(self):
        return self.loss_kind == "l2" and self.fuse_l2 and self.order_bwd != "queue"

    def set_loss(self, loss, ssim_lambda=None):
        """Switch the step's image loss ("l2" or "ssim_l1"); graphs captured
        before keep the loss they were captured with."""
        if loss not in ("l2", "ssim_l1"):
            raise ValueError(f"unknown loss {loss!r}")
        self.loss_kind = loss
        if ssim_lambda is not None:
            self.ssim_lambda = float(ssim_lambda)
        if loss == "ssim_l1" and self.ssim_ws is None:
            self.ssim_ws = torch.empty(max(8, B.ssim_workspace_size(self.sizes)), dtype=torch.uint8,
                                       device=self.device)

    def loss_raster_bwd(self, targets, accumulate=False, unseen_grads=None):
        """L2 loss of ``images`` against ``targets`` and the rasteriser
        backward of its gradient in one pass (``self.d_images`` is not
        written); with ``unseen_grads`` (a gradient dict) it also writes the
        zero gradients of the Gaussians no view sees."""
        s, _ = self._sched(self.order_bwd)
        unseen = None
        if unseen_grads is not None:
            unseen = (self.flags, self.deg, [unseen_grads[k] for k in ("means", "log_scales", "quats",
                                                                         "opacity_logits", "sh")])
        B.rasterize_bwd_l2(self.splats, self.isect_gid, self.ranges, self.n, self.sizes, self.tile,
                           self.background, s, self.T_final, self.n_contrib, self.images, targets, self.loss,
                           self.grad2d, self.l2_ws, accumulate=accumulate, block=self.block_bwd, unseen=unseen)

    def loss_ssim_l1(self, targets):
        B.loss_ssim_l1(self.images, targets, self.sizes, self.ssim_lambda, self.loss, self.d_images,
                       self.ssim_ws)

    def loss_and_raster_bwd(self, targets, accumulate=False, unseen_grads=None):
        """The image loss and the rasteriser backward; returns True when the
        zero gradients of unseen Gaussians were written into ``unseen_grads``
        (the fused L2 path), so the projection backward may write only the
        seen ones."""
        if self.loss_kind == "ssim_l1":
            self.loss_ssim_l1(targets)
            self.raster_bwd(self.d_images, accumulate=accumulate)
        elif self.fused_l2_active:
            self.loss_raster_bwd(targets, accumulate, unseen_grads)
            return unseen_grads is not None
        else:
            self.loss_l2(targets)
            self.raster_bwd(self.d_images, accumulate=accumulate)
        return False

    def forward(self, P, cams, images=None, clear_grad2d=False):
        """Projection, binning and compositing of every view into ``images``
        (default: the renderer's own buffer).  T_final and n_contrib stay in
        the renderer for the backward."""
        self.project(P, cams, clear_grad2d)
        self.bin_sort()
        self.raster_fwd(images)
        return self.images if images is None else images

    def check_overflow(self):
        """One host read of the binning's device counters: raises if the last
        binning overflowed its intersection capacity (lists were truncated;
        grow it with ``fit_capacity`` and run again)."""
        info = self.info.cpu().numpy()
        if info[B.INFO_OVERFLOW]:
            raise B.GSError(f"intersection capacity {self.capacity} < {int(info[B.INFO_ISECT])}; "
                            "call Renderer.fit_capacity()")

    def backward(self, P, cams, d_images, grads, d_alpha=None):
        self.raster_bwd(d_images, d_alpha)
        self.project_bwd(P, cams, grads)
        return grads

    # ---------------------------------------------------------- whole step
    def step(self, P, cams, targets, grads):
        """Forward, the image loss (``loss``: L2, or SSIM + L1) against packed
        ``targets`` and backward into ``grads`` (dict of tensors shaped like
        the parameters)."""
        # the projection zeroes the 2-D gradient records the backward adds to
        self.forward(P, cams, clear_grad2d=True)
        split = self.loss_and_raster_bwd(targets, accumulate=True,
                                         unseen_grads=grads if self.unseen_in_bwd else None)
        self.project_bwd(P, cams, grads, part=B.GRADS_SEEN if split else B.GRADS_ALL)
        return grads

    def train_step(self, P, cams, targets, grads, optimizer, fused=False):
        """``step`` followed by the optimizer's fused update of ``P`` (the
        training step the paper's backend runs; capturable).  ``fused``: the
        projection backward applies the update itself (gs_project_bwd_adam)
        and ``grads`` is neither written nor read."""
        if not fused:
            self.step(P, cams, targets, grads)
            optimizer.update(grads)
            return
        self.forward(P, cams, clear_grad2d=True)
        self.loss_and_raster_bwd(targets, accumulate=True)
        optimizer.update_fused(self, P, cams)

    def fit_capacity(self, P, cams, headroom=1.25):
        """Run projection + binning eagerly and grow the intersection capacity
        until nothing overflows.  Returns the intersection count."""
        while True:
            self.project(P, cams)
            self.bin_sort()
            info = self.info.cpu().numpy()
            m = int(info[B.INFO_ISECT])
            if not info[B.INFO_OVERFLOW]:
                if m > self.capacity:
                    raise B.GSError("intersection count above capacity without overflow flag")
                return m
            self.set_capacity(int(m * headroom) + 1024)

    def capture(self, P, cams, targets, grads, warmup=2):
        """Capture ``step`` in a HIP graph (after eager warm-up) and return it;
        ``replay()`` then runs the whole step with one launch."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for _ in range(warmup):
                self.step(P, cams, targets, grads)
        torch.cuda.current_stream().wait_stream(s)
        # a graph held only by a reference cycle must not be destroyed by the
        # collector while this stream is capturing (HIP refuses that)
        gc.collect()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step(P, cams, targets, grads)
        # the captured launches read and write these tensors on every replay
        # and torch does not track them: the graph keeps them alive
        g.gs_tensors = (P, cams, targets, grads)
        self.graph = g
        return g

    def capture_train(self, P, cams, targets, grads, optimizer, warmup=2, fused=False):
        """Capture ``train_step`` (forward, loss, backward and the Adam update)
        in one HIP graph.  Warm-up steps update the parameters too."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for _ in range(warmup):
                self.train_step(P, cams, targets, grads, optimizer, fused=fused)
        torch.cuda.current_stream().wait_stream(s)
        gc.collect()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.train_step(P, cams, targets, grads, optimizer, fused=fused)
        g.gs_tensors = (P, cams, targets, grads, optimizer)
        return g

    def replay(self):
        self.graph.replay()


# per-parameter learning rates of 3D Gaussian Splatting's training recipe
# (means 1.6e-4 x scene extent, log-scales 5e-3, quaternions 1e-3, opacity
# logits 5e-2, SH DC 2.5e-3 and higher bands 2.5e-3 / 20); one rate per tensor
PARAM_KEYS = ("means", "log_scales", "quats", "opacity_logits", "sh")
DEFAULT_LRS = dict(means=1.6e-4, log_scales=5e-3, quats=1e-3, opacity_logits=5e-2, sh=2.5e-3)


class Adam:
    """Fused Adam (gs_adam) over a dict of planar parameter tensors: the first
    and second moments live beside the parameters in HBM and the step count
    in device memory, so an update can be replayed from a captured graph."""

    def __init__(self, P, lrs=None, betas=(0.9, 0.999), eps=1e-15):
        self.P = P
        self.keys = list(P)
        lrs = dict(DEFAULT_LRS, **(lrs or {}))
        self.lrs = [float(lrs[k]) for k in self.keys]
        self.b1, self.b2 = (float(b) for b in betas)
        self.eps = float(eps)
        self.m = {k: torch.zeros_like(v) for k, v in P.items()}
        self.v = {k: torch.zeros_like(v) for k, v in P.items()}
        self.t = torch.zeros(1, dtype=torch.int32, device=next(iter(P.values())).device)

    def update(self, grads):
        B.adam([self.P[k] for k in self.keys], [grads[k] for k in self.keys], [self.m[k] for k in self.keys],
               [self.v[k] for k in self.keys], self.lrs, self.b1, self.b2, self.eps, self.t)

    def update_fused(self, renderer, P, cams):
        """The renderer's projection backward (from its 2-D gradients of the
        last rasteriser backward) fused with this update: same result as
        ``renderer.project_bwd`` into gradient tensors, then ``update``."""
        if P is not self.P and any(P[k] is not self.P[k] for k in PARAM_KEYS):
            raise B.GSError("update_fused: P is not the optimizer's parameter set")
        lr = dict(zip(self.keys, self.lrs))
        r = renderer
        B.project_bwd_adam(*[self.P[k] for k in PARAM_KEYS], r.deg, cams["viewmats"], cams["intrinsics"], r.sizes,
                           r.eps2d, r.flags, r.grad2d, [self.m[k] for k in PARAM_KEYS],
                           [self.v[k] for k in PARAM_KEYS], [lr[k] for k in PARAM_KEYS], self.b1, self.b2, self.eps,
                           self.t)

    def state_bytes(self):
        return sum(2 * t.numel() * t.element_size() for t in self.P.values())


def params_to_device(scene, device="cuda"):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
    P = dict(means=t(scene.means), log_scales=t(scene.log_scales), quats=t(scene.quats),
             opacity_logits=t(scene.opacity_logits), sh=t(scene.sh))
    cams = dict(viewmats=t(scene.viewmats), intrinsics=t(scene.intrinsics))
    return P, cams


def morton_permute(P, bits=10):
    """The paper's locality pass (Section 5, run at densification time):
    reorder every parameter tensor by the 3-D Morton code of the means on a
    2^bits grid over their bounding box.  Returns the permuted copies and the
    order (new index i holds old Gaussian order[i])."""
    means = P["means"]
    n = means.shape[1]
    lo = means.min(dim=1).values.cpu().numpy().astype(np.float64)
    hi = means.max(dim=1).values.cpu().numpy().astype(np.float64)
    inv = (1 << bits) / np.maximum(hi - lo, 1e-30)
    ws = torch.empty(max(1, B.morton_workspace_size(n)), dtype=torch.uint8, device=means.device)
    order = torch.empty(n, dtype=torch.int32, device=means.device)
    B.morton_order(means, lo.astype(np.float32), inv.astype(np.float32), ws, order)
    out = {}
    for k, t in P.items():
        out[k] = torch.empty_like(t)
        B.gather_columns(t, order, out[k])
    return out, order


def packed_targets(scene, device="cuda"):
    return torch.from_numpy(np.concatenate([t.reshape(-1) for t in scene.targets])).to(device)


def zeros_like_params(P):
    return {k: torch.zeros_like(v) for k, v in P.items()}


def unpack_images(flat, sizes, channels=3):
    """Split a packed image buffer into per-view [C][H][W] views."""
    out, o = [], 0
    for w, h in np.asarray(sizes).reshape(-1, 2):
        n = channels * int(w) * int(h)
        out.append(flat[o:o + n].view(channels, int(h), int(w)) if channels > 1 else
                   flat[o:o + n].view(int(h), int(w)))
        o += n
    return out


class _Render(torch.autograd.Function):
    # The forward reads nothing back to the host: the binning's overflow flag
    # stays on the device, so size the capacity first (Renderer.fit_capacity)
    # or call Renderer.check_overflow() after the step.  The graph-captured
    # form of the step is Renderer.capture / capture_train.
    # The backward reuses the renderer's T_final and n_contrib, so it must run
    # before the renderer's next forward.
    @staticmethod
    def forward(ctx, renderer, viewmats, intrinsics, means, log_scales, quats, opacity_logits, sh):
        P = dict(means=means.detach().contiguous(), log_scales=log_scales.detach().contiguous(),
                 quats=quats.detach().contiguous(), opacity_logits=opacity_logits.detach().contiguous(),
                 sh=sh.detach().contiguous())
        cams = dict(viewmats=viewmats.contiguous(), intrinsics=intrinsics.contiguous())
        images = torch.empty(3 * renderer.pixels, dtype=torch.float32, device=renderer.device)
        renderer.forward(P, cams, images)
        ctx.renderer = renderer
        ctx.P, ctx.cams = P, cams
        return images

    @staticmethod
    def backward(ctx, d_images):
        r = ctx.renderer
        # gs_project_bwd overwrites every gradient element
        grads = {k: torch.empty_like(v) for k, v in ctx.P.items()}
        r.backward(ctx.P, ctx.cams, d_images.contiguous(), grads)
        return (None, None, None, grads["means"], grads["log_scales"], grads["quats"],
                grads["opacity_logits"], grads["sh"])


def render(renderer, P, cams):
    """Differentiable rendering of all views: packed images [sum 3 H W]."""
    return _Render.apply(renderer, cams["viewmats"], cams["intrinsics"], P["means"], P["log_scales"],
                         P["quats"], P["opacity_logits"], P["sh"])


class _L2Loss(torch.autograd.Function):
    # gs_loss_l2 computes the loss and its image gradient in one pass; the
    # backward scales that gradient by the incoming one (1 for loss.backward())
    @staticmethod
    def forward(ctx, renderer, images, targets):
        loss = torch.empty(1, dtype=torch.float32, device=images.device)
        d_images = torch.empty_like(images)
        B.loss_l2(images.detach().contiguous(), targets.contiguous(), loss, d_images, renderer.loss_ws)
        ctx.save_for_backward(d_images)
        return loss[0]

    @staticmethod
    def backward(ctx, g):
        (d_images,) = ctx.saved_tensors
        return None, d_images * g, None


def l2_loss(renderer, images, targets):
    """Differentiable mean squared error of packed images against packed targets
    (one gs_loss_l2 call; the renderer supplies its partial-sum workspace)."""
    return _L2Loss.apply(renderer, images, targets)


# ------------------------------------------------------------------ autotune
BLOCKS = {8: [(8, 1)], 16: [(8, 1), (16, 1), (16, 2), (16, 4)], 32: [(8, 1), (16, 2), (16, 4), (32, 4)]}


def _time_ms(fn, steps):
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / steps


def autotune(P, cams, targets, sh_degree, sizes, tiles=(8, 16, 32), steps=5, cache_path=None, log=None):
    """Pick the tile edge and wave block of the batched path by timing.

    For every tile edge the wave blocks of the compositing forward and of its
    backward are compared separately (they change no result bit), then the
    whole graph-captured step is timed once per tile edge with its best blocks.  The
    tile edge changes which Gaussians share a tile list and therefore the
    rendered image (as in any tile-based rasteriser); callers that need a
    fixed tile pass a single value in ``tiles``.  Returns a dict with the
    chosen ``tile``, ``block`` (forward), ``block_bwd`` and the measured
    milliseconds per candidate;
    with ``cache_path`` the result is stored in a JSON file keyed by the
    workload shape and reused."""
    import json
    import os
    n = int(P["means"].shape[1])
    # keyed by the workload shape only (a profiler can change what the device
    # reports as its name); keep one cache file per GPU model
    key = f"n={n}|deg={sh_degree}|sizes={np.asarray(sizes).tolist()}|tiles={list(tiles)}"
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return cache[key]
    grads = zeros_like_params(P)
    trials, best, per_tile = {}, None, {}
    for tile in tiles:
        r = Renderer(n, sh_degree, sizes, tile=tile, capacity=1 << 20, order="heavy", order_bwd="queue")
        r.fit_capacity(P, cams)
        r.step(P, cams, targets, grads)
        # three interleaved rounds over the candidates, median per candidate:
        # a drift of the clock during tuning then biases no candidate
        fwd_t, bwd_t = {}, {}
        for _ in range(3):
            for order in ORDERS:
                for blk in BLOCKS[tile]:
                    r.block = r.block_bwd = blk
                    r.order = r.order_bwd = order
                    r.raster_fwd()
                    fwd_t.setdefault((order, blk), []).append(_time_ms(r.raster_fwd, steps))
                    # the loss and the backward as the step runs them (in one
                    # pass unless the backward takes the work queue)
                    r.loss_and_raster_bwd(targets)
                    bwd_t.setdefault((order, blk), []).append(
                        _time_ms(lambda: r.loss_and_raster_bwd(targets), steps))
        fwd_ms = {k: float(np.median(v)) for k, v in fwd_t.items()}
        bwd_ms = {k: float(np.median(v)) for k, v in bwd_t.items()}
        # isolated launches see other cache states than the captured step: the
        # two best forward and backward candidates are decided inside it, each
        # combination captured once and timed in three interleaved rounds of
        # at least 10 replays (the first replays include the graph's upload)
        top_f = sorted(fwd_ms, key=fwd_ms.get)[:2]
        top_b = sorted(bwd_ms, key=bwd_ms.get)[:2]
        combos = [(f, b) for f in top_f for b in top_b]
        graphs = []
        for f, b in combos:
            (r.order, r.block), (r.order_bwd, r.block_bwd) = f, b
            r.raster_fwd()
            graphs.append(r.capture(P, cams, targets, grads, warmup=1))
            for _ in range(3):
                r.replay()
        step_t = [[] for _ in combos]
        for _ in range(3):
            for i, g in enumerate(graphs):
                step_t[i].append(_time_ms(g.replay, max(10, 2 * steps)))
        step_med = [float(np.median(v)) for v in step_t]
        i_best = int(np.argmin(step_med))
        (r.order, r.block), (r.order_bwd, r.block_bwd) = combos[i_best]
        ms = step_med[i_best]
        del graphs
        trials[f"tile{tile}"] = {"step_ms": ms,
                                 "in_step_ms": {f"{f[0]}/{f[1][0]}x{f[1][1]}+{b[0]}/{b[1][0]}x{b[1][1]}": v
                                                for (f, b), v in zip(combos, step_med)},
                                 "fwd_ms": {f"{o}/{b[0]}x{b[1]}": v for (o, b), v in fwd_ms.items()},
                                 "bwd_ms": {f"{o}/{b[0]}x{b[1]}": v for (o, b), v in bwd_ms.items()}}
        if log:
            log(f"autotune tile {tile}: fwd {r.order} {r.block} ({fwd_ms[(r.order, r.block)]:.3f} ms), bwd "
                f"{r.order_bwd} {r.block_bwd} ({bwd_ms[(r.order_bwd, r.block_bwd)]:.3f} ms), step {ms:.3f} ms; "
                "fwd " + ", ".join(f"{o}/{b[0]}x{b[1]}: {v:.3f}" for (o, b), v in fwd_ms.items()) + "; bwd " +
                ", ".join(f"{o}/{b[0]}x{b[1]}: {v:.3f}" for (o, b), v in bwd_ms.items()))
        cfg = {"tile": tile, "block": list(r.block), "block_bwd": list(r.block_bwd), "order": r.order,
               "order_bwd": r.order_bwd, "step_ms": ms}
        per_tile[str(tile)] = cfg
        if best is None or ms < best["step_ms"]:
            best = dict(cfg)
        del r
        torch.cuda.empty_cache()
    best["trials"] = trials
    best["per_tile"] = per_tile
    if cache_path:
        cache[key] = best
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return best
