"""Gradient spot check of the 5,000,000-Gaussian 3840x2160 workload on the
FP64 oracle (CPU): for 1,000 seeded (Gaussian, parameter) samples, the
oracle's analytic gradient against a central finite difference (h = 1e-4) of
the L2 loss, each perturbed render re-running only the pixels of the tiles the
Gaussian touches (the loss is a sum over pixels; the others do not change).
Agreement is to 1e-4 relative, plus twice the difference's own truncation
error estimated from the same difference at 2h (where a gradient is a sum of
cancelling pixel terms, that error can exceed 1e-4 of the small total).
Samples whose discrete decisions change between the two perturbed renders
(projection: visibility, radii, tile rectangle, SH clamps, its place in each
depth-sorted tile list; compositing: the per-pixel signature of composited
Gaussians, 0.99 clamps and stop) are skipped and counted."""
import os

import numpy as np
import pytest

import oracle
from paper_2606_11390_amd import scenes

H_STEP = 1e-4
TILE = 16
GROUPS = (("means", 3), ("log_scales", 3), ("quats", 4), ("opac", 1), ("sh", 48))


def _param_array(P, group):
    return {"means": P.means, "log_scales": P.log_scales, "quats": P.quats, "opac": P.opac[None, :],
            "sh": P.sh.reshape(-1, P.n)}[group]


def _one(P, g):
    """The parameters of Gaussian g alone (copies)."""
    return oracle.Params(P.means[:, g:g + 1].copy(), P.log_scales[:, g:g + 1].copy(), P.quats[:, g:g + 1].copy(),
                         P.opac[g:g + 1].copy(), P.sh[..., g:g + 1].copy(), P.deg)


PROJ_KEYS = ("u", "v", "depth", "conic", "sigma", "rgb")


def _swap_in(pr, g, q):
    """Write Gaussian g's projected quantities from the one-Gaussian projection
    q into pr; returns the previous values."""
    old = {}
    for k in PROJ_KEYS:
        a = pr[k]
        if a.ndim == 1:
            old[k] = a[g].copy()
            a[g] = q[k][0]
        else:
            old[k] = a[:, g].copy()
            a[:, g] = q[k][:, 0]
    return old


def _restore(pr, g, old):
    for k, val in old.items():
        if pr[k].ndim == 1:
            pr[k][g] = val
        else:
            pr[k][:, g] = val


def _keys_in_order(z32, g, lists):
    """Does Gaussian g with float32 depth z32[g] keep its place (key = depth
    bits, ties by index) in every tile list that holds it?"""
    kg = (np.float32(z32[g]).view(np.uint32), g)
    for lst in lists:
        k = int(np.nonzero(lst == g)[0][0])
        if k > 0:
            a = lst[k - 1]
            if not (np.float32(z32[a]).view(np.uint32), a) < kg:
                return False
        if k + 1 < len(lst):
            b = lst[k + 1]
            if not kg < (np.float32(z32[b]).view(np.uint32), b):
                return False
    return True


@pytest.mark.slow
def test_uhd_gradient_spot_check_against_finite_differences():
    s = scenes.uhd()
    W, H = (int(x) for x in s.sizes[0])
    vm, it = s.viewmats[0], s.intrinsics[0]
    oracle.set_threads(os.cpu_count() or 1)
    try:
        o = oracle.step(s, tile=TILE)
    finally:
        oracle.set_threads(1)
    P = oracle.Params.of(s)
    pr = o["projs"][0]
    ranges, vals = o["ranges"], o["vals"]
    target = s.targets[0].astype(np.float64)
    n_el = 3 * W * H
    z32 = pr["depth"].astype(np.float32)
    TX = (W + TILE - 1) // TILE
    rng = np.random.default_rng(2024)
    # Gaussians the view sees whose tile rectangle spans at most 16 tiles
    cand = np.nonzero(pr["visible"].astype(bool) & (pr["tiles"] <= 16))[0]
    samples = rng.choice(cand, size=1000, replace=False)
    agree, plain, skipped, worst, bad = 0, 0, {"projection": 0, "order": 0, "compositing": 0}, 0.0, []
    for g in samples:
        gi = int(rng.integers(len(GROUPS)))
        group, width = GROUPS[gi]
        j = int(rng.integers(width))
        base_rect = oracle.tile_rect(np.float32(pr["u"][g]), np.float32(pr["v"][g]), int(pr["radii"][0][g]),
                                     int(pr["radii"][1][g]), TILE, W, H)
        x0, y0, x1, y1 = base_rect
        lists = [vals[ranges[ty * TX + tx][0]:ranges[ty * TX + tx][1]] for ty in range(y0, y1) for tx in range(x0, x1)]
        px = (x0 * TILE, y0 * TILE, min(W, x1 * TILE), min(H, y1 * TILE))
        _, sig0 = oracle.raster_fwd_rect(W, H, TILE, ranges, vals, pr, *px)
        losses, ok = [], "ok"
        for sgn in (1.0, -1.0, 2.0, -2.0):
            Pg = _one(P, g)
            _param_array(Pg, group)[j, 0] += sgn * H_STEP
            q = oracle.project(Pg, vm, it, W, H, tile=TILE)
            rect = oracle.tile_rect(np.float32(q["u"][0]), np.float32(q["v"][0]), int(q["radii"][0][0]),
                                    int(q["radii"][1][0]), TILE, W, H)
            if (not q["visible"][0] or rect != base_rect or q["clamp"][0] != pr["clamp"][g]
                    or q["radii"][0][0] != pr["radii"][0][g] or q["radii"][1][0] != pr["radii"][1][g]):
                ok = "projection"
                break
            # the Jacobian's clamp of x/z and y/z (|u - cx| > 0.65 W, |v - cy| > 0.65 H) is a kink
            if ((abs(q["u"][0] - it[2]) > 0.65 * W) != (abs(pr["u"][g] - it[2]) > 0.65 * W) or
                    (abs(q["v"][0] - it[3]) > 0.65 * H) != (abs(pr["v"][g] - it[3]) > 0.65 * H)):
                ok = "projection"
                break
            zg = z32[g]
            z32[g] = np.float32(q["depth"][0])
            in_order = _keys_in_order(z32, g, lists)
            z32[g] = zg
            if not in_order:
                ok = "order"
                break
            old = _swap_in(pr, g, q)
            try:
                img, sg = oracle.raster_fwd_rect(W, H, TILE, ranges, vals, pr, *px)
            finally:
                _restore(pr, g, old)
            if not np.array_equal(sg, sig0):
                ok = "compositing"
                break
            d = img - target[:, px[1]:px[3], px[0]:px[2]]
            losses.append(float(np.sum(d * d)) / n_el)
        if ok != "ok":
            skipped[ok] += 1
            continue
        fd = (losses[0] - losses[1]) / (2.0 * H_STEP)
        fd2 = (losses[2] - losses[3]) / (4.0 * H_STEP)
        # the central difference's own O(h^2) truncation error, estimated from
        # the same difference at 2h (error 4x larger): (fd2 - fd) / 3
        trunc = abs(fd2 - fd) / 3.0
        an = float(o["grads"][group].reshape(-1, s.n)[j, g])
        err = abs(fd - an)
        plain += err <= 1e-4 * abs(an)
        if err <= 1e-4 * abs(an) + 2.0 * trunc + 1e-16:
            agree += 1
        else:
            bad.append((int(g), group, j, an, fd, trunc))
        worst = max(worst, err / max(abs(an), 1e-30))
    n_skip = sum(skipped.values())
    print(f"uhd FD spot check: {agree} of {len(samples)} agree to 1e-4 (plus the difference's truncation "
          f"error), {plain} within 1e-4 outright; skipped {skipped}, disagree {len(bad)}, worst relative "
          f"{worst:.2e}; first disagreements {bad[:5]}", flush=True)
    assert agree >= 900
    assert not bad
    assert n_skip <= 100
