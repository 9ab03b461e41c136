#!/usr/bin/env python
"""Forward+backward throughput of the splatting step on one MI355X.

Workload (default): 5,000,000 Gaussians from a 512-blob mixture in a 200 m
cube, SH degree 3, one 3840x2160 view (fx = fy = 3000) looking at the scene
centre from the cube surface; FP32 forward, L2 loss against a uniform target,
backward to every parameter.  Inputs are seeded and synthetic and resident in
HBM before timing starts.  The Gaussians are stored in 3-D Morton order, the
layout the paper's densification leaves them in (applied once, untimed); the
batched step is also reported on the generator's order.

Two paths are timed on the same inputs:
  plain   - one workgroup per tile in tile order, every call launched eagerly
            (per view, for several views);
  batched - all views in one launch per call, the rasterisers' tile order
            (band per XCD, heavy-first dispatch or a persistent heavy-first
            queue), tile edge and wave blocks autotuned, and the whole step
            replayed from one captured HIP graph.
The reported ``value`` is the batched path's megapixels/s; the plain path's
figure is reported beside it.  The roofline object covers the kernel with the
largest share of the step, timed with HIP events on the launch stream (and,
where a committed rocprofv3 summary of the workload exists, recomputed from
its average kernel duration).  The autograd path and the training step with
the fused Adam update are timed beside the headline.  The CPU baseline is the
FP64 oracle: the whole step on every available core, and a one-thread figure
from a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# HBM / VALU peaks of one MI355X (published)
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
# algorithmic FP32 operations per visit (one list entry examined by one
# pixel): the compositing forward ~20 vector operations and one exponential,
# the backward ~50 vector operations, one exponential and one division
FWD_OPS_PER_VISIT = 21
BWD_OPS_PER_VISIT = 52
# Adam: parameter, gradient and both moments read, parameter and moments written
ADAM_BYTES_PER_ELEMENT = 28


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_scene(cfg, n_override=None):
    from paper_2606_11390_amd import scenes
    kw = {} if n_override is None else {"n_gaussians": n_override}
    if cfg == "tiny":
        return scenes.tiny(**kw)
    if cfg == "hd":
        return scenes.hd(**kw)
    if cfg == "uhd":
        return scenes.uhd(**kw)
    if cfg == "multiview":
        return scenes.multiview(**kw)
    if cfg == "city":
        return scenes.city(**kw)
    raise SystemExit(f"unknown config {cfg}")


def per_step_ms(fn, steps, torch):
    """Duration of each of `steps` calls (events between consecutive calls)."""
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for i in range(steps):
        fn()
        ev[i + 1].record()
    ev[-1].synchronize()
    return [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]


def timed(fn, steps, torch):
    """Run fn `steps` times between two events on the current stream; ms per call."""
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / steps


def stage_times(r, P, cams, tg, grads, steps, torch):
    """Average duration of each call of the step inside whole steps: the calls
    of `steps` steps launched one after another on the launch stream, in the
    order of the captured step, with HIP events between them (the host stays
    ahead of the GPU, so an interval is the call's own GPU time).  As in the
    step, the projection zeroes the visible pairs' 2-D gradient records and
    the rasteriser backward accumulates into them."""
    from paper_2606_11390_amd import binding as B
    split = r.fused_l2_active and r.unseen_in_bwd
    part = B.GRADS_SEEN if split else B.GRADS_ALL
    if r.fused_l2_active:
        # the loss is formed inside the rasteriser backward: its call (the
        # backward kernel and the two small kernels that sum the loss
        # partials) is the "raster_bwd" stage; as in the step, it also
        # writes the zero gradients of unseen Gaussians, and the projection
        # backward the seen ones
        loss_bwd = [("raster_bwd", lambda: r.loss_raster_bwd(tg, accumulate=True,
                                                             unseen_grads=grads if split else None))]
    else:
        loss_bwd = [("loss", lambda: r.loss_l2(tg)),
                    ("raster_bwd", lambda: r.raster_bwd(r.d_images, accumulate=True))]
    calls = [
        ("project", lambda: r.project(P, cams, clear_grad2d=True)),
        ("bin_sort", r.bin_sort),
        ("raster_fwd", r.raster_fwd),
        *loss_bwd,
        ("project_bwd", lambda: r.project_bwd(P, cams, grads, part=part)),
    ]
    for _ in range(2):
        for _, fn in calls:
            fn()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(len(calls) + 1)] for _ in range(steps)]
    for i in range(steps):
        for k, (_, fn) in enumerate(calls):
            ev[i][k].record()
            fn()
        ev[i][-1].record()
    torch.cuda.synchronize()
    return {name: sum(ev[i][k].elapsed_time(ev[i][k + 1]) for i in range(steps)) / steps
            for k, (name, _) in enumerate(calls)}


# source files whose kernels a counter summary covers, per step call
KERNEL_SOURCES = {"raster_fwd": ["raster.hip", "gs_device.h"], "raster_bwd": ["raster.hip", "gs_device.h"],
                  "project": ["project.hip", "gs_device.h"], "project_bwd": ["project.hip", "gs_device.h"]}


def kernel_name(stage, r):
    """Name of the kernel one step call launches (as rocprofv3 reports it)."""
    if stage in ("raster_fwd", "raster_bwd"):
        fwd = stage == "raster_fwd"
        blk = r.block if fwd else r.block_bwd
        order = r.order if fwd else r.order_bwd
        if not fwd and r.fused_l2_active:
            return f"k_raster_bwd_l2<{r.tile}, {blk[0]}, {blk[1]}>"
        kind = "fwd" if fwd else "bwd"
        suffix = "_persistent" if order == "queue" else ""
        last = "" if (order == "queue" and kind == "fwd") else ", false"
        return f"k_raster_{kind}{suffix}<{r.tile}, {blk[0]}, {blk[1]}{last}>"
    return None


def trace_us(stage, r, workload):
    """(average, median) duration (us) of the stage's kernel in the committed
    rocprofv3 --kernel-trace --stats summary of this workload, or None."""
    name = kernel_name(stage, r)
    path = os.path.join(ROOT, "profiles", f"{workload}_step_kernel_stats.md")
    if name is None or not os.path.exists(path):
        return None
    for line in open(path):
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 4 and cells[0] == f"`{name}`":
            try:
                return float(cells[3]), (float(cells[5]) if len(cells) >= 6 and cells[5] else None)
            except ValueError:
                return None
    return None


def sources_sha1(stage):
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES.get(stage, []):
        with open(os.path.join(ROOT, "paper_2606_11390_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counted_traffic(stage, r, workload):
    """HBM bytes (read + written) per launch of the stage's kernel from the
    committed FETCH_SIZE / WRITE_SIZE summary of this workload, or None when
    there is none or it was taken on other kernel sources."""
    name = kernel_name(stage, r)
    path = os.path.join(ROOT, "profiles", f"{workload}_hbm_counters.md")
    if name is None or not os.path.exists(path):
        return None
    sha = sources_sha1(stage)
    for line in open(path):
        # traffic: kernel=<name> read_bytes=<int> write_bytes=<int> sources=<sha1 prefix>
        if not line.startswith("traffic: "):
            continue
        f = dict(kv.split("=", 1) for kv in line[len("traffic: "):].strip().split(" | "))
        if f.get("kernel") == name and f.get("sources") == sha:
            return int(f["read_bytes"]) + int(f["write_bytes"])
    return None


def counted_issue(stage, r, workload):
    """Executed vector work of the stage's kernel from the committed SQ
    counter summary of this workload: (vector instructions per launch, share
    of the SIMDs' busy quad-cycles that issued one), or None when there is
    none or it was taken on other kernel sources."""
    name = kernel_name(stage, r)
    path = os.path.join(ROOT, "profiles", f"{workload}_sq_counters.md")
    if name is None or not os.path.exists(path):
        return None
    sha = sources_sha1(stage)
    for line in open(path):
        # sq: kernel=<name> | valu_insts=<int> | valu_issue=<float> | waves=<int> | sources=<sha1 prefix>
        if not line.startswith("sq: "):
            continue
        f = dict(kv.split("=", 1) for kv in line[len("sq: "):].strip().split(" | "))
        if f.get("kernel") == name and f.get("sources") == sha:
            return int(f["valu_insts"]), float(f["valu_issue"])
    return None


def algorithmic_bytes(scene, visible, isect, total_tiles, split=False):
    """HBM bytes each HBM-bound call of the step must move at minimum, from
    the workload's counts (N Gaussians, V views, visible (view, Gaussian)
    pairs, M intersections, T tiles, P pixels).

    project      the means read for every Gaussian (12 B), the other
                 parameters (224 B at SH degree 3) for the Gaussians some view
                 sees (counted as min(N, visible pairs), exact for one view);
                 per pair depth, radii, tile count, tile rectangle and flags
                 written (25 B); the 48-byte splat record and the zeroed
                 36-byte 2-D gradient record per visible pair
    bin_sort     LSD radix sort, 16 B (key + value, read + write) per element
                 per pass: 4 depth passes over visible pairs (the first reads
                 depth and tile count, 8 B per pair), emission (24 B read per
                 visible pair, 8 B written per intersection), ceil(tile bits /
                 8) passes over the intersections, ranges (4 B read per
                 intersection, 8 B written per tile)
    loss         image and target read, image gradient written: 12 B per
                 element
    project_bwd  the gradients of every parameter written (236 B per
                 Gaussian, zero where no view sees it), the parameters read
                 for the Gaussians some view sees (min(N, visible pairs)),
                 flags read per pair, the 36-byte 2-D gradient per visible pair;
                 with ``split`` the zeros of unseen Gaussians are written by
                 the compositing backward instead, and only the seen
                 Gaussians' gradients count here
    """
    N, V = scene.n, scene.n_views
    K = (scene.sh_degree + 1) ** 2
    param = 4 * (3 + 3 + 4 + 1 + 3 * K)
    tbits = max(1, int(total_tiles - 1).bit_length())
    tpasses = (tbits + 7) // 8
    sort = (8 * V * N + 8 * visible + 3 * 16 * visible + 24 * visible + 8 * isect + tpasses * 16 * isect +
            4 * isect + 8 * total_tiles)
    seen = min(N, visible)
    return {"project": 12 * N + (param - 12) * seen + 25 * V * N + (48 + 36) * visible,
            "bin_sort": sort,
            "loss": 12 * 3 * scene.pixels,
            "project_bwd": (seen if split else N) * param + seen * param + V * N + 36 * visible}


def host_cpu():
    """CPU model (from /proc/cpuinfo), processors this process may run on, and
    the OpenMP thread count the environment sets."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = os.cpu_count() or 1
    omp = os.environ.get("OMP_NUM_THREADS")
    threads = min(avail, int(omp)) if omp and omp.isdigit() and int(omp) > 0 else avail
    return model, avail, threads


def cpu_one_core_sample(scene, tile, seed=0, frac=0.2, crop_frac=0.5):
    """FP64 oracle on one thread, on a bounded sample of the same step scaled
    to the frame: projection + its backward on a seeded `frac` of the
    Gaussians (scaled by 1/frac); binning, compositing forward and backward
    and loss on a centred crop of `crop_frac` of the width and height (all
    Gaussians projected into the crop camera, untimed), scaled by the pixel
    ratio.  Returns (estimated seconds per step, description)."""
    import oracle
    oracle.set_threads(1)
    rng = np.random.default_rng(seed)
    N = scene.n
    idx = np.sort(rng.choice(N, size=max(1, int(frac * N)), replace=False))
    P = oracle.Params(scene.means[:, idx], scene.log_scales[:, idx], scene.quats[:, idx],
                      scene.opacity_logits[idx], scene.sh[:, :, idx], scene.sh_degree)
    W, H = (int(x) for x in scene.sizes[0])
    vm, it = scene.viewmats[0], scene.intrinsics[0]
    t0 = time.perf_counter()
    oracle.project(P, vm, it, W, H, tile=tile)
    g = dict(u=np.ones(P.n), v=np.ones(P.n), conic=np.ones((3, P.n)), sigma=np.ones(P.n),
             rgb=np.ones((3, P.n)))
    oracle.project_bwd(P, vm, it, W, H, g, tile=tile)
    t_gauss = (time.perf_counter() - t0) * (N / P.n)
    cw, ch = max(tile, int(W * crop_frac)), max(tile, int(H * crop_frac))
    cit = np.array([it[0], it[1], it[2] - (W - cw) / 2.0, it[3] - (H - ch) / 2.0])
    Pall = oracle.Params.of(scene)
    prc = oracle.project(Pall, vm, cit, cw, ch, tile=tile)
    target = np.random.default_rng(seed + 1).uniform(0, 1, (3, ch, cw))
    t1 = time.perf_counter()
    keys, vals, ranges, offs = oracle.bin_views(
        [(prc["u"].astype(np.float32), prc["v"].astype(np.float32), prc["depth"].astype(np.float32),
          prc["radii"])], np.array([[cw, ch]]), tile)
    f = oracle.raster_fwd(cw, ch, tile, ranges, vals, prc)
    _, (dimg,) = oracle.l2_loss([f["img"]], [target])
    oracle.raster_bwd(cw, ch, tile, ranges, vals, prc, dimg)
    t_pix = (time.perf_counter() - t1) * (W * H) / (cw * ch)
    desc = (f"projection + projection backward of a seeded {frac:.0%} sample of the {N} Gaussians (scaled "
            f"x{N / P.n:.0f}); binning, compositing forward and backward and L2 loss of a centred {cw}x{ch} "
            f"crop (scaled x{W * H / (cw * ch):.0f})")
    return t_gauss + t_pix, desc


def cpu_full_step(scene, tile, threads):
    """Seconds of one whole FP64 oracle step (projection, binning,
    compositing, L2 loss and every backward pass) on `threads` threads."""
    import oracle
    oracle.set_threads(threads)
    try:
        t0 = time.perf_counter()
        oracle.step(scene, tile=tile)
        return time.perf_counter() - t0
    finally:
        oracle.set_threads(1)


def cpu_baseline(scene, tile):
    """The FP64 oracle as it stands, timed on this host: the whole step of the
    workload once on every available core (the reported value), plus a
    one-thread figure from a bounded sample of the same step."""
    model, avail, threads = host_cpu()
    t_all = cpu_full_step(scene, tile, threads)
    t_one, desc_one = cpu_one_core_sample(scene, tile)
    pix = scene.pixels
    return {"value": round(pix / t_all / 1e6, 6), "unit": "megapixels/s", "cores": threads, "kind": "oracle",
            "sample": (f"FP64 oracle, the whole step of this workload (projection, binning, compositing, L2 "
                       f"loss and all backward passes) once on {threads} OpenMP threads: {t_all:.2f} s"),
            "cpu_model": model, "cpus_available": avail, "seconds_measured": round(t_all, 3),
            "one_core": {"value": round(pix / t_one / 1e6, 6), "unit": "megapixels/s", "cores": 1,
                         "sample": f"FP64 oracle, 1 thread: {desc_one}; estimated full-step time {t_one:.1f} s"}}


def cpu_baseline_small_configs(tile):
    """Whole oracle steps of the 2,000-Gaussian 128x128 and the 200,000-Gaussian
    1920x1080 workloads, on one thread and on every available core."""
    from paper_2606_11390_amd import scenes
    _, _, threads = host_cpu()
    out = {}
    for name, sc in (("tiny", scenes.tiny()), ("hd", scenes.hd())):
        t1 = cpu_full_step(sc, tile, 1)
        tn = cpu_full_step(sc, tile, threads)
        out[name] = {"pixels": sc.pixels, "gaussians": sc.n, "seconds_1_thread": round(t1, 4),
                     f"seconds_{threads}_threads": round(tn, 4),
                     "mp_per_s_1_thread": round(sc.pixels / t1 / 1e6, 4),
                     f"mp_per_s_{threads}_threads": round(sc.pixels / tn / 1e6, 4)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="uhd", choices=["tiny", "hd", "uhd", "multiview", "city"])
    ap.add_argument("--n-gaussians", type=int, default=None)
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="batched path at --tile instead of the autotuned tile edge")
    ap.add_argument("--autotune-cache", default=None,
                    help="JSON file for the autotuner's choice: written on first use, reused after")
    ap.add_argument("--only", choices=["all", "batched", "plain"], default="all",
                    help="restrict to one path (for profiler runs)")
    ap.add_argument("--main-only", action="store_true",
                    help="time only the headline step (no radius / layout variants, no autograd or training "
                         "step): short runs under a profiler")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 256 MiB three times (reference for HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs one GPU's share of the step; --gpus must be 1"}))
        sys.exit(2)
    if args.copy_calibration:
        import torch
        src = torch.ones(64 << 20, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": src.numel() * 4, "dispatches": 3}))
        return

    import torch
    from paper_2606_11390_amd import binding as B
    from paper_2606_11390_amd import render as R

    t0 = time.time()
    scene = make_scene(args.config, args.n_gaussians)
    log(f"scene {scene.name}: N={scene.n} views={scene.n_views} pixels={scene.pixels} "
        f"({time.time() - t0:.1f} s)")
    P_gen, cams = R.params_to_device(scene)
    # the paper's locality pass: Gaussians stored in 3-D Morton order (it runs
    # at densification time, so it is applied once here, before any timing);
    # every path below runs on this layout, and the batched step is also
    # timed on the generator's order
    P, _ = R.morton_permute(P_gen)
    tg = R.packed_targets(scene)
    grads = R.zeros_like_params(P)
    pixels = scene.pixels
    gauss = scene.n * scene.n_views
    result = {}

    def run_path(cfg, graph, radius_mode=0):
        """cfg: None for the plain path (tile order, default wave block, tile
        edge --tile), else an autotuned configuration."""
        if cfg is None:
            r = R.Renderer(scene.n, scene.sh_degree, scene.sizes, tile=args.tile, capacity=1 << 22)
        else:
            r = R.Renderer(scene.n, scene.sh_degree, scene.sizes, tile=cfg["tile"], capacity=1 << 22,
                           block=tuple(cfg["block"]), block_bwd=tuple(cfg["block_bwd"]), order=cfg["order"],
                           order_bwd=cfg["order_bwd"], radius_mode=radius_mode)
        m = r.fit_capacity(P, cams)
        if graph:
            r.capture(P, cams, tg, grads, warmup=max(1, args.warmup))
            step = r.replay
        else:
            step = lambda: r.step(P, cams, tg, grads)
        # untimed warm-up of the step as it is timed (a graph's first replays
        # include its upload)
        for _ in range(max(1, args.warmup)):
            step()
        torch.cuda.synchronize()
        ms = timed(step, args.steps, torch)
        return r, m, ms, step

    def run_plain_per_view():
        """V single-view steps launched one after another (every call of the
        path once per view, parameters re-read and dense parameter gradients
        produced and summed per view): the baseline the batched path replaces."""
        rs, views = [], []
        for v in range(scene.n_views):
            r = R.Renderer(scene.n, scene.sh_degree, scene.sizes[v:v + 1], tile=args.tile, capacity=1 << 20)
            cv = {k: t[v:v + 1].contiguous() for k, t in cams.items()}
            o = int(np.sum(3 * scene.sizes[:v, 0].astype(np.int64) * scene.sizes[:v, 1]))
            n = 3 * int(scene.sizes[v, 0]) * int(scene.sizes[v, 1])
            r.fit_capacity(P, cv)
            rs.append(r)
            views.append((cv, tg[o:o + n]))
        gv = R.zeros_like_params(P)

        def step():
            for k in grads:
                grads[k].zero_()
            for r, (cv, t) in zip(rs, views):
                r.step(P, cv, t, gv)
                for k in grads:
                    grads[k].add_(gv[k])
        for _ in range(args.warmup):
            step()
        ms = timed(step, args.steps, torch)
        m = sum(int(r.info[B.INFO_ISECT]) for r in rs)
        return rs[0], m, ms

    if args.only in ("all", "plain"):
        if scene.n_views > 1:
            r_plain, m, ms_plain = run_plain_per_view()
        else:
            r_plain, m, ms_plain, _ = run_path(None, False)
        result["plain"] = {"ms_per_step": ms_plain, "mp_per_s": pixels / ms_plain / 1e3}
        log(f"plain: {ms_plain:.3f} ms/step, {pixels / ms_plain / 1e3:.1f} MP/s, M={m}")
        if args.only == "plain":
            r_main, ms_main = r_plain, ms_plain
        del_plain = args.only == "all"
    if args.only == "all" and del_plain:
        del r_plain
        torch.cuda.empty_cache()
    tuned = None
    if args.only in ("all", "batched"):
        tiles = (8, 16, 32) if args.autotune else (args.tile,)
        tuned = R.autotune(P, cams, tg, scene.sh_degree, scene.sizes, tiles=tiles, steps=max(3, args.steps // 4),
                           cache_path=args.autotune_cache, log=log)
        tuned = dict(tuned)
        tuned.pop("trials", None)
        per_tile = tuned.pop("per_tile", {})
        if str(args.tile) in per_tile and tuned["tile"] != args.tile:
            # like-for-like figure at the plain path's tile edge
            t16 = per_tile[str(args.tile)]
            r16, _, ms16, _ = run_path(t16, True)
            result["batched_same_tile"] = dict(t16, ms_per_step=ms16, mp_per_s=pixels / ms16 / 1e3)
            result["batched_same_tile"].pop("step_ms", None)
            del r16
            torch.cuda.empty_cache()
    if args.only in ("all", "batched") and not args.main_only:
        # the same step with the opacity-aware screen box: identical images and
        # gradients from fewer intersections (reported beside the headline)
        ro, mo, mso, _ = run_path(tuned, True, radius_mode=B.RADIUS_OPACITY)
        result["batched_opacity_radius"] = {"ms_per_step": mso, "mp_per_s": pixels / mso / 1e3,
                                            "intersections": int(mo)}
        log(f"batched, opacity-aware radius: {mso:.3f} ms/step, {pixels / mso / 1e3:.1f} MP/s, M={mo}")
        del ro
        torch.cuda.empty_cache()
        # the same step on the generator's order of the Gaussians
        P_m = P
        P = P_gen
        rg, mg, msg, _ = run_path(tuned, True)
        result["batched_generator_order"] = {"ms_per_step": msg, "mp_per_s": pixels / msg / 1e3}
        log(f"batched, generator order of the Gaussians: {msg:.3f} ms/step, {pixels / msg / 1e3:.1f} MP/s, M={mg}")
        P = P_m
        del rg
        torch.cuda.empty_cache()
    if args.only in ("all", "batched"):
        r_main, m, ms_main, step_main = run_path(tuned, True)
        # per-step spread of the same step (after the timed block)
        per = per_step_ms(step_main, args.steps, torch)
        result["per_step"] = {"median_ms": float(np.median(per)), "min_ms": float(np.min(per)),
                              "max_ms": float(np.max(per))}
        log(f"batched (tile {tuned['tile']}, orders {tuned['order']} / {tuned['order_bwd']}, blocks {tuned['block']} / "
            f"{tuned['block_bwd']}): {ms_main:.3f} ms/step, "
            f"{pixels / ms_main / 1e3:.1f} MP/s, M={m}")

    # per-call durations on the main path, HIP events on the launch stream
    st = stage_times(r_main, P, cams, tg, grads, args.steps, torch)
    log("stage ms (inside whole steps): " + ", ".join(f"{k} {v:.3f}" for k, v in st.items()))
    # algorithmic work of the compositing kernels
    vis = torch.empty(pixels, dtype=torch.int32, device="cuda")
    img2 = torch.empty(3 * pixels, device="cuda")
    T2 = torch.empty(pixels, device="cuda")
    c2 = torch.empty(pixels, dtype=torch.int32, device="cuda")
    B.raster_visits(r_main.splats, r_main.isect_gid, r_main.ranges, r_main.n, r_main.sizes, r_main.tile, img2,
                    T2, c2, vis)
    r_main.raster_fwd()
    fwd_visits = int(vis.to(torch.int64).sum())
    bwd_visits = int(r_main.n_contrib.to(torch.int64).sum())
    info = r_main.info.cpu().numpy()
    work = algorithmic_bytes(scene, int(info[B.INFO_VISIBLE]), int(info[B.INFO_ISECT]), r_main.total_tiles,
                             split=r_main.fused_l2_active and r_main.unseen_in_bwd)
    # algorithmic work per launch: bytes of the HBM-bound calls, FP32
    # operations of the compositing kernels (operations per visit x visits)
    alu_work = {"raster_fwd": (FWD_OPS_PER_VISIT, fwd_visits), "raster_bwd": (BWD_OPS_PER_VISIT, bwd_visits)}
    # in the step the compositing backward also writes the zero parameter
    # gradients of the groups of 64 Gaussians no view sees (236 B per
    # Gaussian at SH degree 3), work moved there from the projection backward
    side_bytes = {}
    if r_main.fused_l2_active and r_main.unseen_in_bwd:
        fl = r_main.flags.cpu().numpy().reshape(scene.n_views, scene.n)
        grp = np.arange(scene.n) // 64
        gseen = np.zeros(int(grp[-1]) + 1, bool)
        np.logical_or.at(gseen, grp, np.any(fl & B.FLAG_VISIBLE, axis=0))
        K = (scene.sh_degree + 1) ** 2
        side_bytes["raster_bwd"] = int((~gseen[grp]).sum()) * 4 * (11 + 3 * K)
    rooflines = {}
    for k, (opv, nv) in alu_work.items():
        ops = opv * nv
        ent = {"bound": "alu", "achieved": round(ops / (st[k] * 1e-3) / 1e12, 3), "peak": PEAK_FP32_TFLOPS,
               "unit": "TFLOP/s", "frac": round(ops / (st[k] * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4),
               "ops_per_visit": opv, "visits": nv, "work_per_launch": ops, "launch_us": round(st[k] * 1e3, 2)}
        if k in side_bytes:
            # the launch's two kinds of work, each at its own peak, as a share
            # of the launch time (a lower bound on what it could reach: the
            # stores could overlap the arithmetic entirely)
            t_ops = ops / (PEAK_FP32_TFLOPS * 1e12)
            t_bytes = side_bytes[k] / (PEAK_HBM_GBS * 1e9)
            ent["zero_grad_bytes"] = side_bytes[k]
            ent["frac_ops_plus_zero_bytes"] = round((t_ops + t_bytes) / (st[k] * 1e-3), 4)
        tr = trace_us(k, r_main, scene.name)
        if tr:
            ent["trace_avg_us"] = tr[0]
            ent["frac_from_trace"] = round(ops / (tr[0] * 1e-6) / 1e12 / PEAK_FP32_TFLOPS, 4)
            if tr[1]:
                ent["trace_median_us"] = tr[1]
                ent["frac_from_trace_median"] = round(ops / (tr[1] * 1e-6) / 1e12 / PEAK_FP32_TFLOPS, 4)
        ex = counted_issue(k, r_main, scene.name)
        if ex:
            # executed work: vector instructions per launch (SQ_INSTS_VALU) and
            # the share of busy SIMD quad-cycles that issued one
            ent["executed"] = {"valu_insts": ex[0], "valu_issue": ex[1],
                               "lane_valu_insts_per_visit": round(ex[0] * 64 / max(nv, 1), 2)}
        rooflines[k] = ent
    for k in ("project", "bin_sort", "loss", "project_bwd"):
        if k not in st:
            continue
        a = work[k] / (st[k] * 1e-3) / 1e9
        rooflines[k] = {"bound": "hbm", "achieved": round(a, 3), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": round(a / PEAK_HBM_GBS, 4), "work_per_launch": int(work[k]),
                        "launch_us": round(st[k] * 1e3, 2)}
    dom = max((k for k in st if k in rooflines), key=lambda k: st[k])
    roofline = dict({"kernel": dom}, **rooflines[dom])
    roofline["traffic"] = counted_traffic(dom, r_main, scene.name)

    # the autograd path (render -> l2_loss -> backward through the autograd
    # functions, launched eagerly) and the full training step (the fused step
    # plus the fused Adam update, replayed from one captured graph), on copies
    # of the parameters
    extra = {}
    if args.only != "plain" and not args.main_only:
        Pa = {k: v.clone().requires_grad_(True) for k, v in P.items()}

        def autograd_step():
            for t in Pa.values():
                t.grad = None
            R.l2_loss(r_main, R.render(r_main, Pa, cams), tg).backward()
        for _ in range(max(1, args.warmup)):
            autograd_step()
        ms_ag = timed(autograd_step, args.steps, torch)
        extra["autograd_step"] = {"ms_per_step": round(ms_ag, 4), "mp_per_s": round(pixels / ms_ag / 1e3, 3),
                                  "launch": "eager"}
        log(f"autograd step (eager): {ms_ag:.3f} ms/step")
        del Pa
        P_tr = {k: v.clone() for k, v in P.items()}
        opt = R.Adam(P_tr)
        g_tr = R.zeros_like_params(P_tr)
        gt = r_main.capture_train(P_tr, cams, tg, g_tr, opt, warmup=1)
        for _ in range(max(1, args.warmup)):
            gt.replay()
        ms_tr = timed(gt.replay, args.steps, torch)
        ms_adam = timed(lambda: opt.update(g_tr), args.steps, torch)
        adam_bytes = ADAM_BYTES_PER_ELEMENT * sum(t.numel() for t in P_tr.values())
        extra["train_step"] = {"ms_per_step": round(ms_tr, 4), "mp_per_s": round(pixels / ms_tr / 1e3, 3),
                               "adam_ms": round(ms_adam, 4),
                               "adam_gb_s": round(adam_bytes / (ms_adam * 1e-3) / 1e9, 1),
                               "adam_hbm_frac": round(adam_bytes / (ms_adam * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                               "adam_bytes": adam_bytes}
        log(f"training step with fused Adam (captured): {ms_tr:.3f} ms/step; Adam alone {ms_adam:.3f} ms "
            f"({adam_bytes / (ms_adam * 1e-3) / 1e9:.0f} GB/s)")
        ms_pb = timed(lambda: r_main.project_bwd(P_tr, cams, g_tr), args.steps, torch)
        del gt, opt, g_tr
        torch.cuda.empty_cache()
        # the same step with the update fused into the projection backward
        # (gs_project_bwd_adam): no gradient tensors are written or read
        opt_f = R.Adam(P_tr)
        gf = r_main.capture_train(P_tr, cams, tg, None, opt_f, warmup=1, fused=True)
        for _ in range(max(1, args.warmup)):
            gf.replay()
        ms_trf = timed(gf.replay, args.steps, torch)
        ms_pba = timed(lambda: opt_f.update_fused(r_main, P_tr, cams), args.steps, torch)
        # per element: parameter and both moments read and written (24 B);
        # per (view, Gaussian): flags, and the 2-D gradients where visible
        n_el = sum(t.numel() for t in P_tr.values())
        fused_bytes = 24 * n_el + scene.n_views * scene.n + 36 * int(r_main.info.cpu()[B.INFO_VISIBLE])
        extra["train_step"].update({
            "fused": {"ms_per_step": round(ms_trf, 4), "mp_per_s": round(pixels / ms_trf / 1e3, 3),
                      "project_bwd_adam_ms": round(ms_pba, 4),
                      "unfused_project_bwd_plus_adam_ms": round(ms_pb + ms_adam, 4),
                      "project_bwd_adam_gb_s": round(fused_bytes / (ms_pba * 1e-3) / 1e9, 1),
                      "project_bwd_adam_bytes": fused_bytes}})
        log(f"training step, Adam fused into the projection backward (captured): {ms_trf:.3f} ms/step; "
            f"fused kernel {ms_pba:.3f} ms against {ms_pb:.3f} + {ms_adam:.3f} ms unfused "
            f"({fused_bytes / (ms_pba * 1e-3) / 1e9:.0f} GB/s)")
        del gf, opt_f
        # the same fused training step with the 3D Gaussian Splatting training
        # loss, (1 - 0.2) L1 + 0.2 (1 - SSIM), in place of L2
        r_main.set_loss("ssim_l1", 0.2)
        opt_s = R.Adam(P_tr)
        gss = r_main.capture_train(P_tr, cams, tg, None, opt_s, warmup=1, fused=True)
        for _ in range(max(1, args.warmup)):
            gss.replay()
        ms_trs = timed(gss.replay, args.steps, torch)
        extra["train_step"]["fused_ssim_l1"] = {"ms_per_step": round(ms_trs, 4),
                                                "mp_per_s": round(pixels / ms_trs / 1e3, 3)}
        log(f"training step with the SSIM + L1 loss and Adam fused into the projection backward (captured): "
            f"{ms_trs:.3f} ms/step")
        del gss, opt_s, P_tr
        r_main.set_loss("l2")
        torch.cuda.empty_cache()

        # the other per-step calls of the training loop, alone: the fused SSIM
        # + L1 loss on the step's images (forward and image gradient), and the
        # 3-D Morton order of the means with the gather of all 59 parameter
        # planes (run at densification time, not every step)
        ws_s = torch.empty(B.ssim_workspace_size(scene.sizes), dtype=torch.uint8, device="cuda")
        loss_s = torch.empty(1, device="cuda")
        d_s = torch.empty_like(r_main.images)
        ms_ssim = timed(lambda: B.loss_ssim_l1(r_main.images, tg, scene.sizes, 0.2, loss_s, d_s, ws_s),
                        args.steps, torch)
        n = scene.n
        means = P["means"]
        ws_m = torch.empty(max(1, B.morton_workspace_size(n)), dtype=torch.uint8, device="cuda")
        order = torch.empty(n, dtype=torch.int32, device="cuda")
        lo = means.min(dim=1).values.cpu().numpy().astype(np.float32)
        hi = means.max(dim=1).values.cpu().numpy().astype(np.float32)
        inv = ((1 << 10) / np.maximum(hi.astype(np.float64) - lo, 1e-30)).astype(np.float32)
        ms_morton = timed(lambda: B.morton_order(means, lo, inv, ws_m, order), args.steps, torch)
        cols = {k: torch.empty_like(v) for k, v in P.items()}
        ms_gather = timed(lambda: [B.gather_columns(P[k], order, cols[k]) for k in P], args.steps, torch)
        n_el = sum(t.numel() for t in P.values())
        extra["ssim_l1"] = {"ms": round(ms_ssim, 4), "mp_per_s": round(pixels / ms_ssim / 1e3, 1)}
        extra["morton"] = {"order_ms": round(ms_morton, 4), "gather_ms": round(ms_gather, 4),
                           "gather_gb_s": round(n_el * 4 * 2 / (ms_gather * 1e-3) / 1e9, 1)}
        log(f"SSIM + L1 loss and image gradient: {ms_ssim:.3f} ms; Morton order {ms_morton:.3f} ms, "
            f"gather of the parameters {ms_gather:.3f} ms")
        del ws_s, loss_s, d_s, ws_m, order, cols
        torch.cuda.empty_cache()

    cpu = None
    cpu_small = None
    if not args.no_cpu_baseline and scene.n_views == 1:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(scene, args.tile)
        log(f"cpu baseline: {cpu['value']} MP/s on {cpu['cores']} threads ({cpu['seconds_measured']} s), "
            f"{cpu['one_core']['value']} MP/s on one; {cpu['cpu_model']}")
        if scene.name == "uhd":
            cpu_small = cpu_baseline_small_configs(args.tile)
            log(f"cpu baseline, small workloads: {cpu_small}")

    line = {
        "metric": "fwd+bwd megapixels/s at 4K, 5M Gaussians: batched vs plain path, 1 MI355X",
        "value": round(pixels / ms_main / 1e3, 3),
        "unit": "megapixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_main, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{scene.name}: {scene.n} Gaussians, SH degree {scene.sh_degree}, "
                               f"{scene.n_views} view(s) {'+'.join(f'{w}x{h}' for w, h in scene.sizes)}, "
                               f"FP32 forward + L2 loss + backward",
                   "tile": r_main.tile, "wave_block_fwd": list(r_main.block),
                   "wave_block_bwd": list(r_main.block_bwd), "tile_order_fwd": r_main.order,
                   "tile_order_bwd": r_main.order_bwd,
                   "path": "batched" if args.only != "plain" else "plain",
                   "gaussians": scene.n, "views": scene.n_views, "pixels": pixels,
                   "intersections": int(info[B.INFO_ISECT]), "visible": int(info[B.INFO_VISIBLE]),
                   "gaussian_order": "3-D Morton (applied once before timing)",
                   "parallelism": "1 GPU"},
        "gaussians_per_s": round(gauss / ms_main * 1e3, 1),
        "plain": {k: round(v, 4) for k, v in result.get("plain", {}).items()},
        "batched_same_tile": result.get("batched_same_tile"),
        "ms_per_step_spread": ({k: round(v, 4) for k, v in result["per_step"].items()}
                               if "per_step" in result else None),
        "batched_generator_order": ({k: round(v, 4) for k, v in result["batched_generator_order"].items()}
                                    if "batched_generator_order" in result else None),
        "batched_opacity_radius": ({k: round(v, 4) for k, v in result["batched_opacity_radius"].items()}
                                   if "batched_opacity_radius" in result else None),
        "autotuned": tuned,
        "stage_ms": {k: round(v, 4) for k, v in st.items()},
        "visits": {"forward": fwd_visits, "backward": bwd_visits},
        "roofline": roofline,
        "roofline_all": rooflines,
        **extra,
        "cpu_baseline": cpu,
        "cpu_baseline_small_workloads": cpu_small,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
