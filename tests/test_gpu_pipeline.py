"""GPU whole-path tests: end to end against the oracle, batched against plain
per-view launches, persistent against grid scheduling, HIP-graph replay
against eager execution, and the autograd wrapper against the fused step.

End to end, the GPU's own float32 projection feeds its binning and
compositing, so its image differs from the FP64 pipeline by the float32
rounding of the projected means and conics propagated through the falloff
(see the bound in ``_e2e_tol``), not by the 1e-5 of the stage-isolated tests.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2606_11390_amd import binding as B
from paper_2606_11390_amd import render as R
from paper_2606_11390_amd import scenes
from tests import gpu_util as G

pytestmark = pytest.mark.gpu



def _run_step(s, tile=16, persistent=False, capacity=1 << 16, order=None, order_bwd=None):
    r = R.Renderer(s.n, s.sh_degree, s.sizes, tile=tile, capacity=capacity, persistent=persistent, order=order,
                   order_bwd=order_bwd)
    P, cams = R.params_to_device(s)
    r.fit_capacity(P, cams)
    tg = R.packed_targets(s)
    grads = R.zeros_like_params(P)
    r.step(P, cams, tg, grads)
    torch.cuda.synchronize()
    return r, P, cams, tg, grads


@pytest.mark.parametrize("name", ["tiny", "ragged"])
def test_end_to_end_against_oracle(name):
    """The whole GPU step (projection feeding binning, compositing, loss and
    both backward passes) against the all-FP64 oracle at the target
    tolerances: images within 1e-5 (max |x - y| / max |y|) and every parameter
    gradient within 1e-4 (relative L2), outside the set where float32 may
    legitimately take another discrete decision.  That set comes from the
    oracle's own decision margins (``gpu_util.ambiguity``); its size is
    reported and bounded, and its pixels must still lie within one decision
    flip of the oracle."""
    s = scenes.tiny() if name == "tiny" else scenes.tiny(seed=21, n_gaussians=1500, width=100, height=75,
                                                         focal=90.0)
    G.say(f"[e2e] {name}")
    r, P, cams, tg, grads = _run_step(s)
    o = oracle.step(s)
    pmasks, gmask = G.ambiguity(s, o, 16)
    W, H = (int(x) for x in s.sizes[0])
    img = G.host(r.images).reshape(3, H, W)
    ref = o["imgs"][0]
    keep = ~pmasks[0]
    e_img = float(np.max(np.abs(img - ref)[:, keep]) / np.max(np.abs(ref)))
    e_all = float(np.max(np.abs(img - ref)) / np.max(np.abs(ref)))
    loss = float(G.host(r.loss)[0])
    gn = {k: G.host(v) for k, v in grads.items()}
    pairs = (("means", "means"), ("log_scales", "log_scales"), ("quats", "quats"), ("opac", "opacity_logits"),
             ("sh", "sh"))
    errs = {k: G.rel_l2(gn[k2][..., ~gmask], o["grads"][k][..., ~gmask]) for k, k2 in pairs}
    errs_all = {k: G.rel_l2(gn[k2], o["grads"][k]) for k, k2 in pairs}
    G.say(f"  ambiguous: {int(pmasks[0].sum())} of {W * H} pixels, {int(gmask.sum())} of {s.n} Gaussians")
    G.say(f"  image {e_img:.2e} outside them ({e_all:.2e} everywhere), loss {loss:.7f} vs {o['loss']:.7f}")
    G.say("  grads outside: " + " ".join(f"{k} {e:.1e}" for k, e in errs.items()) +
          "; everywhere: " + " ".join(f"{k} {e:.1e}" for k, e in errs_all.items()))
    assert pmasks[0].mean() <= 0.005
    assert gmask.mean() <= 0.2
    assert e_img <= 1e-5
    assert max(errs.values()) <= 1e-4
    # one decision flip changes a pixel by at most ~sigma alpha |dc|: < 2e-2
    assert e_all <= 2e-2
    assert loss == pytest.approx(o["loss"], rel=1e-5)


def _multi():
    return scenes.blobs(5, 30_000, 64, 20.0, [(320, 240, 250.0), (200, 150, 156.0), (128, 96, 100.0),
                                              (257, 131, 200.0)], name="multi")


def test_opacity_radius_changes_work_not_images():
    """The opacity-aware screen box renders the same images and transmittance
    as the 3-sigma box, bit for bit, from fewer intersections, and its
    gradients agree to float32 accumulation order."""
    s = scenes.tiny(seed=21, n_gaussians=1500, width=100, height=75, focal=90.0)
    # wide splats across the whole opacity range, so that many are clipped
    s.opacity_logits[:] = np.linspace(-5.5, 4.0, s.n).astype(np.float32)
    s.log_scales[:] += np.float32(1.0)
    out = []
    for mode in (0, 1):
        r = R.Renderer(s.n, s.sh_degree, s.sizes, tile=16, capacity=1 << 16, radius_mode=mode)
        P, cams = R.params_to_device(s)
        r.fit_capacity(P, cams)
        grads = R.zeros_like_params(P)
        r.step(P, cams, R.packed_targets(s), grads)
        torch.cuda.synchronize()
        out.append((G.host(r.images), G.host(r.T_final), int(G.host(r.info)[1]),
                    {k: G.host(v) for k, v in grads.items()}))
    G.say(f"[opacity radius] intersections {out[0][2]} -> {out[1][2]}")
    assert out[1][2] < out[0][2]
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])
    for k in out[0][3]:
        assert G.rel_l2(out[1][3][k], out[0][3][k]) <= 1e-5, k


def test_morton_permutation_preserves_step():
    """Reordering the Gaussians into Morton order changes no image bit (depths
    are distinct, so every pixel composites the same splats in the same order)
    and permutes the gradients with them."""
    s = _multi()
    r0, P, cams, tg, g0 = _run_step(s)
    img0 = G.host(r0.images)
    Pm, order = R.morton_permute(P)
    order = G.host(order).astype(np.int64)
    assert np.array_equal(np.sort(order), np.arange(s.n))
    np.testing.assert_array_equal(G.host(Pm["sh"]), G.host(P["sh"])[..., order])
    r1 = R.Renderer(s.n, s.sh_degree, s.sizes, tile=16, capacity=1 << 16)
    r1.fit_capacity(Pm, cams)
    g1 = R.zeros_like_params(Pm)
    r1.step(Pm, cams, tg, g1)
    torch.cuda.synchronize()
    # equal depths in one tile list would be ordered by the new indices
    M = int(G.host(r0.info)[1])
    tiles = G.host(r0.isect_tile)[:M]
    gids = G.host(r0.isect_gid)[:M].astype(np.int64)
    _, toff, _ = B.tile_grid(s.sizes, 16)
    view = np.searchsorted(np.asarray(toff), tiles, side="right") - 1
    z = G.host(r0.depths).reshape(s.n_views, s.n)[view, gids]
    ties = int(np.sum((tiles[1:] == tiles[:-1]) & (z[1:] == z[:-1])))
    G.say(f"[morton] M={M} equal-depth neighbours {ties}")
    if ties == 0:
        np.testing.assert_array_equal(G.host(r1.images), img0)
    else:
        assert G.rel_max(G.host(r1.images), img0) <= 1e-2
    for k in g0:
        e = G.rel_l2(G.host(g1[k]), G.host(g0[k])[..., order])
        G.say(f"  morton grad {k}: rel L2 {e:.1e}")
        assert e <= (1e-5 if ties == 0 else 1e-2), k


def test_batched_equals_plain_views():
    s = _multi()
    G.say("[batched == plain]")
    rb, P, cams, tg, gb = _run_step(s)
    imgs_b = G.unpack(G.host(rb.images), s.sizes, 3)
    gsum = {k: np.zeros_like(G.host(v)) for k, v in gb.items()}
    ranges_b = G.host(rb.ranges).reshape(-1, 2)
    gid_b = G.host(rb.isect_gid)
    _, toff, _ = B.tile_grid(s.sizes, 16)
    for v in range(s.n_views):
        sv = scenes.Scene(s.means, s.log_scales, s.quats, s.opacity_logits, s.sh, s.sh_degree,
                          s.viewmats[v:v + 1], s.intrinsics[v:v + 1], s.sizes[v:v + 1], [s.targets[v]])
        # the plain path's loss is a mean over its own view: rescale to the batch mean
        r1, P1, c1, t1, g1 = _run_step(sv)
        np.testing.assert_array_equal(G.host(r1.images).reshape(imgs_b[v].shape), imgs_b[v])
        r1r = G.host(r1.ranges).reshape(-1, 2)
        rbv = ranges_b[toff[v]:toff[v + 1]]
        gid1 = G.host(r1.isect_gid)
        for t in np.nonzero(r1r[:, 1] > r1r[:, 0])[0]:
            np.testing.assert_array_equal(gid1[r1r[t, 0]:r1r[t, 1]], gid_b[rbv[t, 0]:rbv[t, 1]])
        scale = (3 * int(s.sizes[v][0]) * int(s.sizes[v][1])) / (3 * s.pixels)
        for k in gsum:
            gsum[k] += G.host(g1[k]) * scale
    for k in gsum:
        e = G.rel_l2(G.host(gb[k]), gsum[k])
        G.say(f"  grad {k}: rel L2 {e:.1e}")
        assert e <= 1e-5


def _sixteen():
    """The 16-view workload's layout at reduced size: 16 view sizes drawn as
    for the 20M-Gaussian benchmark, each scaled by 1/8 per axis (80x60 ...
    480x270, fx = 0.78125 W), 60,000 Gaussians from 256 blobs in a 50 m cube."""
    rng = np.random.default_rng(4 + 1000)
    picks = rng.integers(0, len(scenes.VIEW_SIZES), size=16)
    views = [(scenes.VIEW_SIZES[i][0] // 8, scenes.VIEW_SIZES[i][1] // 8, 0.78125 * scenes.VIEW_SIZES[i][0] / 8)
             for i in picks]
    return scenes.blobs(4, 60_000, 256, 25.0, views, name="sixteen")


@pytest.mark.parametrize("tile", [8, 16])
def test_sixteen_views_batched_equals_plain_and_oracle(tile):
    """All 16 views in one launch per call against 16 one-view runs (images and
    every tile list bit-identical, summed gradients to float32 accumulation
    order) and against the FP64 oracle (images outside the ambiguity set within
    1e-5 plus the float32 rounding of the projected mean)."""
    s = _sixteen()
    G.say(f"[16 views, tile {tile}]")
    rb, P, cams, tg, gb = _run_step(s, tile=tile, capacity=1 << 18, order="heavy", order_bwd="heavy")
    assert int(G.host(rb.info)[2]) == 0
    imgs_b = G.unpack(G.host(rb.images), s.sizes, 3)
    ranges_b = G.host(rb.ranges).reshape(-1, 2)
    gid_b = G.host(rb.isect_gid)
    _, toff, _ = B.tile_grid(s.sizes, tile)
    gsum = {k: np.zeros_like(G.host(v)) for k, v in gb.items()}
    for v in range(s.n_views):
        sv = scenes.Scene(s.means, s.log_scales, s.quats, s.opacity_logits, s.sh, s.sh_degree,
                          s.viewmats[v:v + 1], s.intrinsics[v:v + 1], s.sizes[v:v + 1], [s.targets[v]])
        r1, _, _, _, g1 = _run_step(sv, tile=tile, capacity=1 << 16)
        np.testing.assert_array_equal(G.host(r1.images).reshape(imgs_b[v].shape), imgs_b[v])
        r1r = G.host(r1.ranges).reshape(-1, 2)
        rbv = ranges_b[toff[v]:toff[v + 1]]
        np.testing.assert_array_equal(r1r[:, 1] - r1r[:, 0], rbv[:, 1] - rbv[:, 0])
        gid1 = G.host(r1.isect_gid)
        for t in np.nonzero(r1r[:, 1] > r1r[:, 0])[0]:
            np.testing.assert_array_equal(gid1[r1r[t, 0]:r1r[t, 1]], gid_b[rbv[t, 0]:rbv[t, 1]])
        scale = (3 * int(s.sizes[v][0]) * int(s.sizes[v][1])) / (3 * s.pixels)
        for k in gsum:
            gsum[k] += G.host(g1[k]) * scale
    for k in gsum:
        e = G.rel_l2(G.host(gb[k]), gsum[k])
        G.say(f"  grad {k}: rel L2 {e:.1e}")
        assert e <= 1e-5
    # against the oracle: besides its discrete decisions, the image carries
    # the float32 rounding of the projected mean (the record's pixel
    # coordinates), which moves the falloff exponent of a compact splat by up
    # to ~2 |Q d| ulp(u) with |Q d| <= ~3.3 / px (the 0.3 px^2 dilation bounds
    # the conic's eigenvalues by 1 / 0.3): a few ulps of the view's largest
    # coordinate, relative
    o = oracle.step(s, tile=tile, backward=False)
    pm, _ = G.ambiguity(s, o, tile)
    errs = []
    for v in range(s.n_views):
        ref = o["imgs"][v]
        keep = ~pm[v]
        e = float(np.max(np.abs(imgs_b[v] - ref)[:, keep]) / np.max(np.abs(ref)))
        bound = 1e-5 + 4.0 * float(np.spacing(np.float32(max(s.sizes[v]))))
        errs.append((e, bound))
    G.say(f"  images vs oracle outside {sum(int(m.sum()) for m in pm)} ambiguous pixels: " +
          " ".join(f"{e:.1e}/{b:.1e}" for e, b in errs))
    assert sum(int(m.sum()) for m in pm) <= 0.005 * s.pixels
    assert all(e <= b for e, b in errs)


@pytest.mark.parametrize("order,order_bwd", [("queue", "queue"), ("xcd", "heavy"), ("heavy", "xcd")])
def test_tile_orders_equal_grid(order, order_bwd):
    s = _multi()
    G.say(f"[{order}/{order_bwd} == grid]")
    ra, *_, ga = _run_step(s, persistent=False)
    rp, *_, gp = _run_step(s, order=order, order_bwd=order_bwd)
    np.testing.assert_array_equal(G.host(ra.images), G.host(rp.images))
    np.testing.assert_array_equal(G.host(ra.n_contrib), G.host(rp.n_contrib))
    for k in ga:
        assert G.rel_l2(G.host(gp[k]), G.host(ga[k])) <= 1e-5


@pytest.mark.parametrize("order", ["tile", "heavy", "queue"])
def test_graph_replay_matches_eager(order):
    s = _multi()
    G.say(f"[graph replay] order={order}")
    r, P, cams, tg, grads = _run_step(s, order=order)
    eager = {k: G.host(v).copy() for k, v in grads.items()}
    eager_img = G.host(r.images).copy()
    eager_loss = float(G.host(r.loss)[0])
    r.capture(P, cams, tg, grads)
    for rep in range(3):
        for v in grads.values():
            v.fill_(float("nan"))
        r.images.fill_(float("nan"))
        # the projection zeroes the 2-D gradient records the step adds to
        r.grad2d.fill_(float("nan"))
        torch.cuda.synchronize()
        r.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(G.host(r.images), eager_img)
        assert float(G.host(r.loss)[0]) == pytest.approx(eager_loss, rel=1e-6)
        for k, v in grads.items():
            assert G.rel_l2(G.host(v), eager[k]) <= 1e-5, (rep, k)
        # unrelated eager work between replays
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()


def test_step_writes_unseen_zeros_in_raster_bwd():
    """The step with the unseen Gaussians' zero gradients written by the fused
    L2 compositing backward and the seen ones by the projection backward
    equals the step with one whole projection backward: no gradient left
    unwritten, exact zeros where no view sees the Gaussian, the rest equal up
    to the backward's atomic order."""
    s = _multi()
    G.say("[unseen zeros in the compositing backward]")
    out = []
    for split in (True, False):
        r = R.Renderer(s.n, s.sh_degree, s.sizes, tile=16, capacity=1 << 16, unseen_in_bwd=split)
        P, cams = R.params_to_device(s)
        # Morton order, so that whole groups of 64 Gaussians go unseen
        P, _ = R.morton_permute(P)
        r.fit_capacity(P, cams)
        tg = R.packed_targets(s)
        grads = {k: torch.full_like(v, float("nan")) for k, v in P.items()}
        r.step(P, cams, tg, grads)
        torch.cuda.synchronize()
        out.append(({k: G.host(v).copy() for k, v in grads.items()}, G.host(r.flags).copy()))
    (ga, fl), (gb, _) = out
    seen = np.any(fl.reshape(s.n_views, s.n) & 1, axis=0)
    grp = np.arange(s.n) // 64
    gseen = np.zeros(grp[-1] + 1, bool)
    np.logical_or.at(gseen, grp, seen)
    G.say(f"  groups of 64 that no view sees: {int((~gseen).sum())} of {gseen.size}")
    assert (~gseen).any() and gseen.any()
    for k in ga:
        assert not np.isnan(ga[k]).any(), k
        assert (ga[k].reshape(-1, s.n)[:, ~seen] == 0).all(), k
        assert G.rel_l2(ga[k], gb[k]) <= 1e-5, k


def test_ssim_l1_step_matches_separate_calls():
    """The step with the SSIM + L1 training loss equals the loss call and the
    backward run by hand (same images and loss bit for bit, gradients up to
    atomic order), and its loss is the oracle's SSIM + L1 of the rendered
    images; a captured training step with it replays."""
    s = scenes.tiny(seed=7, n_gaussians=1200, width=100, height=75, focal=90.0)
    W, H = (int(x) for x in s.sizes[0])
    P, cams = R.params_to_device(s)
    tg = R.packed_targets(s)
    r = R.Renderer(s.n, s.sh_degree, s.sizes, tile=16, capacity=1 << 16, loss="ssim_l1")
    r.fit_capacity(P, cams)
    grads = R.zeros_like_params(P)
    r.step(P, cams, tg, grads)
    torch.cuda.synchronize()
    loss = float(G.host(r.loss)[0])
    img = G.host(r.images).copy()
    r2 = R.Renderer(s.n, s.sh_degree, s.sizes, tile=16, capacity=1 << 16)
    r2.fit_capacity(P, cams)
    r2.forward(P, cams)
    ws = torch.empty(B.ssim_workspace_size(s.sizes), dtype=torch.uint8, device="cuda")
    l2 = torch.zeros(1, device="cuda")
    d = torch.empty_like(r2.images)
    B.loss_ssim_l1(r2.images, tg, s.sizes, 0.2, l2, d, ws)
    g2 = R.zeros_like_params(P)
    r2.backward(P, cams, d, g2)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(G.host(r2.images), img)
    assert float(G.host(l2)[0]) == loss
    for k in grads:
        assert G.rel_l2(G.host(grads[k]), G.host(g2[k])) <= 1e-5, k
    L, _ = oracle.ssim_l1_loss([img.reshape(3, H, W)], [G.host(tg).reshape(3, H, W)], lam=0.2)
    G.say(f"[ssim step] loss {loss:.8f} oracle {L:.8f}")
    assert loss == pytest.approx(L, rel=1e-5)
    opt = R.Adam({k: v.clone() for k, v in P.items()})
    g = r.capture_train(opt.P, cams, tg, None, opt, warmup=1, fused=True)
    g.replay()
    torch.cuda.synchronize()
    assert np.isfinite(G.host(r.loss)[0])


def test_captured_graph_keeps_its_tensors():
    """The captured step reads and writes the parameters, targets and gradient
    tensors it was captured with on every replay, and torch does not track
    tensors used by library launches: the graph object must keep them alive,
    so that a caller's temporary dicts are not freed and reused under it.
    Checked by weak references only (no replay touches released memory)."""
    import gc
    import weakref
    s = scenes.tiny(seed=5, n_gaussians=800, width=96, height=64, focal=80.0)
    r, P, cams, tg, _ = _run_step(s)
    grads = R.zeros_like_params(P)
    tg2 = tg.clone()
    refs = [weakref.ref(t) for t in list(grads.values()) + [tg2]]
    g = r.capture(P, cams, tg2, grads, warmup=1)
    del grads, tg2
    gc.collect()
    assert all(ref() is not None for ref in refs)
    g.replay()
    torch.cuda.synchronize()
    del g
    r.graph = None
    gc.collect()
    assert all(ref() is None for ref in refs)


def test_autograd_matches_fused_step():
    s = scenes.tiny(seed=9, n_gaussians=3000, width=160, height=96, focal=110.0)
    G.say("[autograd]")
    r, P, cams, tg, grads = _run_step(s)
    Pt = {k: v.clone().requires_grad_(True) for k, v in P.items()}
    img = R.render(r, Pt, cams)
    loss = ((img - tg) ** 2).mean()
    loss.backward()
    assert float(loss) == pytest.approx(float(G.host(r.loss)[0]), rel=1e-5)
    for k in grads:
        assert G.rel_l2(G.host(Pt[k].grad), G.host(grads[k])) <= 1e-5, k


def test_autograd_l2_matches_fused_step():
    """render -> l2_loss -> backward through the autograd functions (eager)
    against the fused step."""
    s = scenes.tiny(seed=10, n_gaussians=3000, width=160, height=96, focal=110.0)
    G.say("[autograd l2]")
    r, P, cams, tg, grads = _run_step(s)
    ref_loss = float(G.host(r.loss)[0])
    ref = {k: G.host(v).copy() for k, v in grads.items()}
    Pt = {k: v.clone().requires_grad_(True) for k, v in P.items()}
    loss = R.l2_loss(r, R.render(r, Pt, cams), tg)
    loss.backward()
    assert float(loss.detach()) == pytest.approx(ref_loss, rel=1e-6)
    for k in ref:
        assert G.rel_l2(G.host(Pt[k].grad), ref[k]) <= 1e-5, k


@pytest.mark.skip(reason="capturing loss.backward() through the autograd functions in a HIP graph ended in a "
                         "segmentation fault inside torch's capture_end on the GPU box; the cause is not shown, "
                         "so the captured form of the step stays Renderer.capture / capture_train")
def test_autograd_graph_capture():
    pass


def test_captured_train_step_matches_eager():
    """forward, loss, backward and the fused Adam update replayed from one
    graph (one warm-up step, then two replays) against three eager training
    steps from the same start: parameters and both Adam moments agree."""
    s = scenes.blobs(12, 20000, 32, 10.0, [(320, 180, 250.0)], name="hd_small")
    G.say("[train step graph]")
    P0, cams = R.params_to_device(s)
    tg = R.packed_targets(s)
    r = R.Renderer(s.n, s.sh_degree, s.sizes, tile=16, capacity=1 << 16, order="heavy")
    r.fit_capacity(P0, cams)
    PA = {k: v.clone() for k, v in P0.items()}
    PB = {k: v.clone() for k, v in P0.items()}
    oa, ob = R.Adam(PA), R.Adam(PB)
    ga, gb = R.zeros_like_params(PA), R.zeros_like_params(PB)
    for _ in range(3):
        r.train_step(PA, cams, tg, ga, oa)
    g = r.capture_train(PB, cams, tg, gb, ob, warmup=1)
    for _ in range(2):
        g.replay()
    torch.cuda.synchronize()
    assert int(G.host(oa.t)[0]) == 3 and int(G.host(ob.t)[0]) == 3
    for k in P0:
        p0 = G.host(P0[k]).astype(np.float64)
        da, db = G.host(PA[k]) - p0, G.host(PB[k]) - p0
        assert np.linalg.norm(da) > 0, k
        # the updates (not the parameters, which barely move) agree
        assert G.rel_l2(db, da) <= 1e-3, k
        assert G.rel_l2(G.host(ob.m[k]), G.host(oa.m[k])) <= 1e-4, k
        assert G.rel_l2(G.host(ob.v[k]), G.host(oa.v[k])) <= 1e-4, k


@pytest.mark.parametrize("which", ["one view", "four views"])
def test_fused_projection_backward_adam_equals_unfused(which):
    """gs_project_bwd_adam against gs_project_bwd followed by gs_adam on the
    same 2-D gradients, over three steps (the third replayed from a graph):
    parameters and both Adam moments agree element by element, including the
    Gaussians no view sees (zero gradient; their moments decay and their
    parameters keep moving)."""
    s = (scenes.blobs(13, 20000, 24, 10.0, [(320, 180, 250.0)], name="hd_small") if which == "one view"
         else _multi())
    G.say(f"[fused projection backward + Adam, {which}]")
    r, P, cams, tg, grads = _run_step(s)
    unseen = int(np.sum(~np.any(G.host(r.flags).reshape(len(s.sizes), s.n) & B.FLAG_VISIBLE, axis=0)))
    assert 0 < unseen < s.n, unseen
    PA = {k: v.clone() for k, v in P.items()}
    PB = {k: v.clone() for k, v in P.items()}
    oa, ob = R.Adam(PA), R.Adam(PB)
    ga = R.zeros_like_params(PA)
    graph = None
    for step in range(3):
        r.project_bwd(PA, cams, ga)
        oa.update(ga)
        if step < 2:
            ob.update_fused(r, PB, cams)
        else:
            graph = torch.cuda.CUDAGraph()
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.graph(graph, stream=side):
                ob.update_fused(r, PB, cams)
            graph.replay()
    torch.cuda.synchronize()
    assert int(G.host(oa.t)[0]) == 3 and int(G.host(ob.t)[0]) == 3
    # the two forms run the same float32 operations (explicit fmas, the same
    # gradient code), so every parameter and moment is the same bits
    for k in R.PARAM_KEYS:
        p0 = G.host(P[k])
        assert np.linalg.norm(G.host(PA[k]).astype(np.float64) - p0) > 0, k
        for name, a, b in (("p", PA[k], PB[k]), ("m", oa.m[k], ob.m[k]), ("v", oa.v[k], ob.v[k])):
            a, b = G.host(a), G.host(b)
            diff = int(np.sum(a != b))
            if diff:
                G.say(f"  {k}.{name}: {diff} of {a.size} differ, rel_max {G.rel_max(b, a):.2e}")
            np.testing.assert_array_equal(b, a, err_msg=f"{k}.{name}")
    G.say(f"  all parameters and moments bit-identical; {unseen} of {s.n} Gaussians unseen")


def test_renderer_reports_overflow():
    s = scenes.tiny()
    r = R.Renderer(s.n, s.sh_degree, s.sizes, capacity=100)
    P, cams = R.params_to_device(s)
    R.render(r, P, cams)
    with pytest.raises(B.GSError):
        r.check_overflow()
    m = r.fit_capacity(P, cams)
    assert r.capacity >= m
    R.render(r, P, cams)
    r.check_overflow()
