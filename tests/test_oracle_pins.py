"""Pins of the FP64 oracle against things other than itself.

Each test ties one part of the oracle to an independent fact: a library
routine (scipy's complex spherical harmonics and rotations, numpy's sort), a
closed form, a numerical Jacobian, a brute-force re-implementation in Python,
an invariant of front-to-back compositing, or central finite differences of
the oracle's own forward pass.  A dropped term, a wrong sign or index or a
transposed operand anywhere in the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy.special import sph_harm_y

import oracle
from tests import records as RC
from paper_2606_11390_amd import scenes

PI = math.pi
F32 = np.float32


def _params(means, log_scales, quats, opac, sh, deg):
    return oracle.Params(np.asarray(means, float).reshape(3, -1), np.asarray(log_scales, float).reshape(3, -1),
                         np.asarray(quats, float).reshape(4, -1), np.asarray(opac, float).reshape(-1),
                         np.asarray(sh, float).reshape((deg + 1) ** 2, 3, -1), deg)


IDENT = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1).reshape(12)


# --------------------------------------------------------------------------
# spherical harmonics
# --------------------------------------------------------------------------
def _real_sh_scipy(l, m, d):
    theta = math.acos(max(-1.0, min(1.0, d[2])))
    phi = math.atan2(d[1], d[0]) % (2 * PI)
    if m > 0:
        return math.sqrt(2) * sph_harm_y(l, m, theta, phi).real
    if m < 0:
        return math.sqrt(2) * sph_harm_y(l, -m, theta, phi).imag
    return sph_harm_y(l, 0, theta, phi).real


def test_sh_basis_matches_scipy_condon_shortley():
    rng = np.random.default_rng(0)
    for _ in range(40):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        y = oracle.sh_basis(d)
        for l in range(4):
            for m in range(-l, l + 1):
                assert y[l * l + l + m] == pytest.approx(_real_sh_scipy(l, m, d), abs=1e-12)
    # Condon-Shortley phase: Y_{1,1} along +x is negative
    assert oracle.sh_basis([1.0, 0.0, 0.0])[3] == pytest.approx(-math.sqrt(3 / (4 * PI)))


def test_sh_basis_orthonormal_by_exact_quadrature():
    # Gauss-Legendre in cos(theta) (8 nodes, exact to degree 15) times 16
    # uniform azimuths (exact for trigonometric degree < 16): exact for every
    # product of two degree-3 harmonics.
    xs, ws = np.polynomial.legendre.leggauss(8)
    phis = 2 * PI * np.arange(16) / 16
    gram = np.zeros((16, 16))
    for x, w in zip(xs, ws):
        s = math.sqrt(1 - x * x)
        for ph in phis:
            y = oracle.sh_basis([s * math.cos(ph), s * math.sin(ph), x])
            gram += w * (2 * PI / 16) * np.outer(y, y)
    np.testing.assert_allclose(gram, np.eye(16), atol=1e-12)


# --------------------------------------------------------------------------
# rotations
# --------------------------------------------------------------------------
def test_quaternion_rotation_matches_scipy():
    rng = np.random.default_rng(1)
    for _ in range(20):
        q = rng.standard_normal(4) * 3.0          # not unit: the oracle normalises
        r = oracle.quat_rot(q)
        ref = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()   # scipy is (x, y, z, w)
        np.testing.assert_allclose(r, ref, atol=1e-13)
    th = 0.7
    r = oracle.quat_rot([math.cos(th / 2), 0, 0, math.sin(th / 2)])
    np.testing.assert_allclose(r, [[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]],
                               atol=1e-15)


# --------------------------------------------------------------------------
# projection
# --------------------------------------------------------------------------
def _proj1(mu, ls, q, o=2.0, sh0=0.0, deg=0, W=64, H=64, f=50.0, vm=IDENT, tile=16, near=0.01, eps=0.3):
    K = (deg + 1) ** 2
    sh = np.zeros((K, 3, 1))
    sh[0, :, 0] = sh0
    P = _params(mu, ls, q, [o], sh, deg)
    return oracle.project(P, vm, [f, f, W / 2, H / 2], W, H, near=near, eps2d=eps, tile=tile)


def test_projection_isotropic_on_axis_closed_form():
    z0, s, f = 4.0, 0.05, 50.0
    pr = _proj1([0, 0, z0], [math.log(s)] * 3, [0.3, -0.2, 0.9, 0.1], f=f)
    var = (f * s / z0) ** 2 + 0.3
    assert pr["visible"][0] == 1
    assert pr["u"][0] == pytest.approx(32.0) and pr["v"][0] == pytest.approx(32.0)
    assert pr["depth"][0] == pytest.approx(z0)
    np.testing.assert_allclose(pr["cov"][:, 0], [var, 0.0, var], atol=1e-14)
    np.testing.assert_allclose(pr["conic"][:, 0], [1 / var, 0.0, 1 / var], rtol=1e-13, atol=1e-15)
    assert tuple(pr["radii"][:, 0]) == (math.ceil(3 * math.sqrt(var)),) * 2


def test_projection_rotated_anisotropic_on_axis_closed_form():
    z0, f, th = 3.0, 60.0, 0.4
    s1, s2, s3 = 0.08, 0.02, 0.5
    pr = _proj1([0, 0, z0], np.log([s1, s2, s3]), [math.cos(th / 2), 0, 0, math.sin(th / 2)], f=f)
    R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    S2 = (f / z0) ** 2 * R @ np.diag([s1 * s1, s2 * s2]) @ R.T + 0.3 * np.eye(2)
    np.testing.assert_allclose(pr["cov"][:, 0], [S2[0, 0], S2[0, 1], S2[1, 1]], rtol=1e-12)
    inv = np.linalg.inv(S2)
    np.testing.assert_allclose(pr["conic"][:, 0], [inv[0, 0], inv[0, 1], inv[1, 1]], rtol=1e-12)
    assert pr["radii"][0, 0] == math.ceil(3 * math.sqrt(S2[0, 0]))
    assert pr["radii"][1, 0] == math.ceil(3 * math.sqrt(S2[1, 1]))


def _num_jac(fun, p, h=1e-6):
    J = np.zeros((2, 3))
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        J[:, k] = (fun(p + e) - fun(p - e)) / (2 * h)
    return J


def test_projection_off_axis_matches_numerical_jacobian():
    rng = np.random.default_rng(2)
    W, H, fx, fy = 80, 60, 70.0, 55.0
    cx, cy = 41.0, 28.5
    for _ in range(10):
        mu = np.array([rng.uniform(-0.5, 0.5), rng.uniform(-0.4, 0.4), rng.uniform(1.5, 3.0)])
        ls = rng.normal(-2.5, 0.5, 3)
        q = rng.standard_normal(4)
        P = _params(mu, ls, q, [1.0], np.zeros((1, 3, 1)), 0)
        pr = oracle.project(P, IDENT, [fx, fy, cx, cy], W, H)
        pix = lambda p: np.array([fx * p[0] / p[2] + cx, fy * p[1] / p[2] + cy])
        J = _num_jac(pix, mu)
        Rm = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        Sig = Rm @ np.diag(np.exp(2 * ls)) @ Rm.T
        S2 = J @ Sig @ J.T + 0.3 * np.eye(2)
        np.testing.assert_allclose([pr["u"][0], pr["v"][0]], pix(mu), rtol=1e-13)
        np.testing.assert_allclose(pr["cov"][:, 0], [S2[0, 0], S2[0, 1], S2[1, 1]], rtol=1e-7, atol=1e-9)


def test_projection_clamps_jacobian_not_mean():
    W = H = 64
    f = 50.0
    lim = float(np.float32(1.3)) * 0.5 * W / f
    mu = np.array([2.0, 0.1, 1.0])               # x/z = 2 > lim
    ls = np.log([0.05, 0.07, 0.03])
    q = np.array([0.9, 0.1, -0.3, 0.2])
    P = _params(mu, ls, q, [1.0], np.zeros((1, 3, 1)), 0)
    pr = oracle.project(P, IDENT, [f, f, W / 2, H / 2], W, H)
    x, y, z = mu
    J = np.array([[f / z, 0, -f * lim / z], [0, f / z, -f * (y / z) / z]])
    Rm = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    S2 = J @ (Rm @ np.diag(np.exp(2 * ls)) @ Rm.T) @ J.T + 0.3 * np.eye(2)
    np.testing.assert_allclose(pr["cov"][:, 0], [S2[0, 0], S2[0, 1], S2[1, 1]], rtol=1e-12)
    assert pr["u"][0] == pytest.approx(f * x / z + W / 2)     # the mean is not clamped


def test_projection_invariant_under_rigid_motion():
    s = scenes.tiny(seed=7, n_gaussians=50, width=96, height=80, focal=70.0)
    P = oracle.Params.of(s)
    a = oracle.project(P, s.viewmats[0], s.intrinsics[0], 96, 80)
    rng = np.random.default_rng(3)
    RG = Rotation.random(random_state=4).as_matrix()
    tG = rng.standard_normal(3) * 5
    means2 = RG @ P.means + tG[:, None]
    qs = []
    for g in range(P.n):
        q = P.quats[:, g]
        Rq = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        x, y, z, w = Rotation.from_matrix(RG @ Rq).as_quat()
        qs.append([w, x, y, z])
    P2 = oracle.Params(means2, P.log_scales, np.array(qs).T, P.opac, P.sh, P.deg)
    vm = s.viewmats[0].astype(float).reshape(3, 4)
    Wn = vm[:, :3] @ RG.T
    tn = vm[:, 3] - Wn @ tG
    b = oracle.project(P2, np.concatenate([Wn, tn[:, None]], 1).reshape(12), s.intrinsics[0], 96, 80)
    for k in ("u", "v", "depth", "cov", "conic", "rgb"):
        np.testing.assert_allclose(b[k], a[k], rtol=1e-9, atol=1e-9)
    np.testing.assert_array_equal(b["radii"], a["radii"])


def test_projection_culling():
    W = H = 64
    mus = np.array([[0, 0, 0.005], [0, 0, 3.0], [0, 0, 3.0], [50, 0, 3.0], [0, 0, 3.0], [0, 0, -2.0]]).T
    ls = np.full((3, 6), math.log(0.05))
    q = np.tile([[1.0], [0], [0], [0]], (1, 6))
    o = np.array([2.0, -6.0, 2.0, 2.0, float("nan"), 2.0])     # sigmoid(-6) < 1/255
    P = _params(mus, ls, q, o, np.zeros((1, 3, 6)), 0)
    pr = oracle.project(P, IDENT, [50.0, 50.0, 32, 32], W, H)
    np.testing.assert_array_equal(pr["visible"], [0, 0, 1, 0, 0, 0])
    np.testing.assert_array_equal(pr["tiles"], [0, 0, 4, 0, 0, 0])
    np.testing.assert_array_equal(pr["radii"][:, [0, 1, 3, 4, 5]], 0)


def test_colour_degree0_closed_form_and_clamp():
    for k, want, clamped in ((0.4, 0.4 / (2 * math.sqrt(PI)) + 0.5, 0), (-3.0, 0.0, 1)):
        pr = _proj1([0.1, -0.2, 3.0], [-3.0] * 3, [1, 0, 0, 0], sh0=k)
        np.testing.assert_allclose(pr["rgb"][:, 0], [want] * 3, atol=1e-15)
        assert pr["clamp"][0] == (7 if clamped else 0)


def test_colour_uses_ray_from_camera_centre():
    # camera at c = (1, 2, -3) looking down +z (world == camera axes); only the
    # l=1, m=0 (z) coefficient is set, so rgb = c1 * d_z * k + 0.5
    c = np.array([1.0, 2.0, -3.0])
    vm = np.concatenate([np.eye(3), -c[:, None]], axis=1).reshape(12)
    mu = np.array([1.5, 1.0, 1.0])
    sh = np.zeros((4, 3, 1))
    sh[2, :, 0] = [0.3, -0.2, 0.1]
    P = _params(mu, [-3.0] * 3, [1, 0, 0, 0], [2.0], sh, 1)
    pr = oracle.project(P, vm, [50.0, 50.0, 32, 32], 64, 64)
    d = (mu - c) / np.linalg.norm(mu - c)
    np.testing.assert_allclose(pr["rgb"][:, 0], math.sqrt(3 / (4 * PI)) * d[2] * sh[2, :, 0] + 0.5, atol=1e-15)


# --------------------------------------------------------------------------
# compositing closed forms and invariants
# --------------------------------------------------------------------------
def _alpha(sig, conic, dx, dy):
    A, B, C = conic
    a = sig * math.exp(-0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy)
    a = min(a, oracle.ALPHA_MAX)
    return a if a >= oracle.ALPHA_MIN else 0.0


def _splats(u, v, conic, sig, rgb):
    return dict(u=np.array(u, float), v=np.array(v, float), conic=np.array(conic, float).reshape(3, -1),
                sigma=np.array(sig, float), rgb=np.array(rgb, float).reshape(3, -1))


def test_single_gaussian_composite_closed_form():
    W, H, tile = 32, 32, 16
    sp = _splats([13.3], [17.8], [[0.02], [0.005], [0.03]], [0.8], [[0.7], [0.2], [0.4]])
    ranges = np.array([[0, 1]] * 4, np.int32)
    vals = np.array([0], np.int32)
    f = oracle.raster_fwd(W, H, tile, ranges, vals, sp)
    for j in range(H):
        for i in range(W):
            a = _alpha(0.8, (0.02, 0.005, 0.03), 13.3 - (i + 0.5), 17.8 - (j + 0.5))
            np.testing.assert_allclose(f["img"][:, j, i], a * np.array([0.7, 0.2, 0.4]), rtol=1e-14, atol=1e-16)
            assert f["T"][j, i] == pytest.approx(1 - a, rel=1e-14)
            assert f["last"][j, i] == (1 if a > 0 else 0)


def test_two_gaussians_composite_closed_form_with_background():
    W, H, tile = 16, 16, 16
    sp = _splats([7.0, 9.5], [8.0, 6.5], [[0.05, 0.04], [0.01, -0.02], [0.06, 0.05]], [0.7, 0.9],
                 [[0.9, 0.1], [0.3, 0.8], [0.2, 0.5]])
    bg = np.array([0.25, 0.5, 0.75])
    f = oracle.raster_fwd(W, H, tile, np.array([[0, 2]], np.int32), np.array([0, 1], np.int32), sp, bg)
    c1, c2 = sp["rgb"][:, 0], sp["rgb"][:, 1]
    for j in range(H):
        for i in range(W):
            a1 = _alpha(0.7, sp["conic"][:, 0], 7.0 - i - 0.5, 8.0 - j - 0.5)
            a2 = _alpha(0.9, sp["conic"][:, 1], 9.5 - i - 0.5, 6.5 - j - 0.5)
            want = a1 * c1 + (1 - a1) * a2 * c2 + (1 - a1) * (1 - a2) * bg
            np.testing.assert_allclose(f["img"][:, j, i], want, rtol=1e-14, atol=1e-16)


def test_two_opaque_layers_stop_compositing():
    # alpha clamps at 0.99f; (1 - 0.99f)^2 < 1e-4f, so the second opaque layer
    # is not composited and at most 1 % of what lies behind the first shows.
    sp = _splats([8.5, 8.5, 8.5], [8.5, 8.5, 8.5], [[0.1] * 3, [0.0] * 3, [0.1] * 3], [1.0, 1.0, 1.0],
                 [[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    f = oracle.raster_fwd(16, 16, 16, np.array([[0, 3]], np.int32), np.array([0, 1, 2], np.int32), sp)
    assert f["last"][8, 8] == 1
    assert f["T"][8, 8] == pytest.approx(1 - oracle.ALPHA_MAX)
    assert f["img"][1, 8, 8] == 0.0 and f["img"][2, 8, 8] == 0.0
    assert f["img"][0, 8, 8] == pytest.approx(oracle.ALPHA_MAX)


def _tiny_setup(seed=11, n=300, W=48, H=40, f=45.0, tile=16, deg=0):
    s = scenes.tiny(seed=seed, n_gaussians=n, width=W, height=H, focal=f)
    P = oracle.Params.of(s)
    pr = oracle.project(P, s.viewmats[0], s.intrinsics[0], W, H, tile=tile)
    keys, vals, ranges, offs = oracle.bin_views(
        [(pr["u"].astype(F32), pr["v"].astype(F32), pr["depth"].astype(F32), pr["radii"])], s.sizes, tile)
    return s, P, pr, keys, vals, ranges


def test_composite_invariants():
    s, P, pr, keys, vals, ranges = _tiny_setup()
    W, H = 48, 40
    # weights sum with the final transmittance to one: rgb = 1, bg = 0
    ones = dict(pr, rgb=np.ones_like(pr["rgb"]))
    f1 = oracle.raster_fwd(W, H, 16, ranges, vals, ones)
    np.testing.assert_allclose(f1["img"][0], 1 - f1["T"], atol=1e-13)
    # final transmittance never below the stop threshold, alpha in [0, 1 - 1e-4f]
    assert f1["T"].min() >= oracle.T_MIN and f1["T"].max() <= 1.0
    # background enters linearly through the final transmittance
    bg = np.array([0.3, 0.6, 0.9])
    f0 = oracle.raster_fwd(W, H, 16, ranges, vals, pr)
    fb = oracle.raster_fwd(W, H, 16, ranges, vals, pr, bg)
    np.testing.assert_allclose(fb["img"] - f0["img"], f0["T"][None] * bg[:, None, None], atol=1e-13)
    # transmittance is non-increasing: truncating every list can only raise T
    half = ranges.copy()
    half[:, 1] = (ranges[:, 0] + ranges[:, 1]) // 2
    fh = oracle.raster_fwd(W, H, 16, half, vals, pr)
    assert np.all(fh["T"] >= f0["T"] - 1e-15)


def test_permuting_gaussians_leaves_image_unchanged():
    s, P, pr, keys, vals, ranges = _tiny_setup(seed=12)
    perm = np.random.default_rng(5).permutation(P.n)
    s2 = scenes.tiny(seed=12, n_gaussians=300, width=48, height=40, focal=45.0)
    P2 = oracle.Params(P.means[:, perm], P.log_scales[:, perm], P.quats[:, perm], P.opac[perm],
                       P.sh[:, :, perm], P.deg)
    pr2 = oracle.project(P2, s2.viewmats[0], s2.intrinsics[0], 48, 40)
    k2, v2, r2, _ = oracle.bin_views(
        [(pr2["u"].astype(F32), pr2["v"].astype(F32), pr2["depth"].astype(F32), pr2["radii"])], s2.sizes, 16)
    z = pr["depth"][pr["visible"] > 0].astype(F32)
    assert len(np.unique(z)) == len(z)            # distinct depths
    a = oracle.raster_fwd(48, 40, 16, ranges, vals, pr)
    b = oracle.raster_fwd(48, 40, 16, r2, v2, pr2)
    np.testing.assert_array_equal(a["img"], b["img"])
    np.testing.assert_array_equal(perm[v2], vals)


# --------------------------------------------------------------------------
# binning and sort: brute force
# --------------------------------------------------------------------------
def _rect_f32(u, v, rx, ry, tile, W, H):
    TX, TY = -(-W // tile), -(-H // tile)
    u, v, ts = F32(u), F32(v), F32(tile)
    x0 = np.floor((u - F32(rx)) / ts)
    x1 = np.floor((u + F32(rx)) / ts) + F32(1)
    y0 = np.floor((v - F32(ry)) / ts)
    y1 = np.floor((v + F32(ry)) / ts) + F32(1)
    c = lambda a, hi: int(min(max(float(a), 0.0), float(hi)))
    return c(x0, TX), c(y0, TY), c(x1, TX), c(y1, TY)


@pytest.mark.parametrize("tile", [8, 16])
def test_tiled_composite_equals_brute_force_per_pixel(tile):
    W, H = 40, 36
    s, P, pr, keys, vals, ranges = _tiny_setup(seed=13, n=150, W=W, H=H, f=40.0, tile=tile)
    f = oracle.raster_fwd(W, H, tile, ranges, vals, pr)
    zb = pr["depth"].astype(F32).view(np.uint32)
    vis = [g for g in range(P.n) if pr["visible"][g]]
    rects = {g: _rect_f32(pr["u"][g], pr["v"][g], pr["radii"][0, g], pr["radii"][1, g], tile, W, H) for g in vis}
    for j in range(H):
        for i in range(W):
            tx, ty = i // tile, j // tile
            cand = [g for g in vis if rects[g][0] <= tx < rects[g][2] and rects[g][1] <= ty < rects[g][3]]
            cand.sort(key=lambda g: (int(zb[g]), g))
            T, C, last = 1.0, np.zeros(3), 0
            for k, g in enumerate(cand):
                dx, dy = pr["u"][g] - (i + 0.5), pr["v"][g] - (j + 0.5)
                A, B, Cc = pr["conic"][:, g]
                power = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy
                if power > 0:
                    continue
                a = min(pr["sigma"][g] * math.exp(power), oracle.ALPHA_MAX)
                if a < oracle.ALPHA_MIN:
                    continue
                Tn = T * (1 - a)
                if Tn < oracle.T_MIN:
                    break
                C += a * T * pr["rgb"][:, g]
                T, last = Tn, k + 1
            np.testing.assert_allclose(f["img"][:, j, i], C, rtol=0, atol=1e-14)
            assert f["last"][j, i] == last


def test_sort_is_stable_and_matches_numpy_lexsort():
    rng = np.random.default_rng(6)
    keys = rng.integers(0, 40, 5000).astype(np.uint64) << np.uint64(32) | rng.integers(0, 20, 5000).astype(np.uint64)
    vals = np.arange(5000, dtype=np.int32)
    k, v = oracle.sort_pairs(keys, vals)
    order = np.argsort(keys, kind="stable")
    np.testing.assert_array_equal(k, keys[order])
    np.testing.assert_array_equal(v, vals[order])
    r = oracle.tile_ranges(k, 45)
    for t in range(45):
        idx = np.nonzero((k >> np.uint64(32)) == t)[0]
        want = (idx[0], idx[-1] + 1) if len(idx) else (0, 0)
        assert tuple(r[t]) == want


def test_bin_keys_and_emission_match_python():
    W, H, tile = 40, 36, 8
    s, P, pr, keys, vals, ranges = _tiny_setup(seed=14, n=120, W=W, H=H, f=40.0, tile=tile)
    TX = -(-W // tile)
    want = []
    z = pr["depth"].astype(F32).view(np.uint32)
    for g in range(P.n):
        if not pr["visible"][g]:
            continue
        x0, y0, x1, y1 = _rect_f32(pr["u"][g], pr["v"][g], pr["radii"][0, g], pr["radii"][1, g], tile, W, H)
        assert (x1 - x0) * (y1 - y0) == pr["tiles"][g]
        for ty in range(y0, y1):
            for tx in range(x0, x1):
                want.append(((ty * TX + tx) << 32 | int(z[g]), g))
    want.sort(key=lambda kv: kv[0])          # Python's sort is stable
    np.testing.assert_array_equal(keys, np.array([k for k, _ in want], np.uint64))
    np.testing.assert_array_equal(vals, np.array([g for _, g in want], np.int32))


# --------------------------------------------------------------------------
# backward: finite differences of the oracle's own forward, closed forms
# --------------------------------------------------------------------------
def test_raster_backward_matches_finite_differences():
    W, H, tile = 48, 40, 16
    s, P, pr, keys, vals, ranges = _tiny_setup(seed=15, W=W, H=H, tile=tile)
    rng = np.random.default_rng(7)
    bg = np.array([0.1, 0.2, 0.3])
    d_img = rng.standard_normal((3, H, W))
    d_alpha = rng.standard_normal((H, W))
    g = oracle.raster_bwd(W, H, tile, ranges, vals, pr, d_img, d_alpha, bg)
    base = oracle.raster_fwd(W, H, tile, ranges, vals, pr, bg)

    def objective(sp):
        f = oracle.raster_fwd(W, H, tile, ranges, vals, sp, bg)
        return float(np.sum(f["img"] * d_img) + np.sum((1 - f["T"]) * d_alpha)), f

    for key in ("u", "v", "conic", "sigma", "rgb"):
        delta = rng.standard_normal(pr[key].shape) * (pr["visible"] > 0)
        h = 1e-6
        sp_p = dict(pr)
        sp_p[key] = pr[key] + h * delta
        sp_m = dict(pr)
        sp_m[key] = pr[key] - h * delta
        fp, a = objective(sp_p)
        fm, b = objective(sp_m)
        assert np.array_equal(a["last"], base["last"]) and np.array_equal(b["last"], base["last"])
        fd = (fp - fm) / (2 * h)
        an = float(np.sum(g[key] * delta))
        assert an == pytest.approx(fd, rel=2e-6, abs=1e-9), key


def test_projection_backward_matches_finite_differences():
    s = scenes.hd(seed=8, n_gaussians=400)
    # bring the blob scene into a small view so that many Gaussians are visible
    P = oracle.Params.of(s)
    W, H = 64, 48
    intr = np.array([60.0, 60.0, 32.0, 24.0])
    vm = s.viewmats[0]
    pr = oracle.project(P, vm, intr, W, H)
    vis = pr["visible"] > 0
    assert vis.sum() > 20
    rng = np.random.default_rng(9)
    g = dict(u=rng.standard_normal(P.n), v=rng.standard_normal(P.n), conic=rng.standard_normal((3, P.n)),
             sigma=rng.standard_normal(P.n), rgb=rng.standard_normal((3, P.n)))
    acc = oracle.project_bwd(P, vm, intr, W, H, g)

    def objective(Pp):
        o = oracle.project(Pp, vm, intr, W, H)
        assert np.array_equal(o["visible"], pr["visible"]) and np.array_equal(o["clamp"], pr["clamp"])
        return sum(float(np.sum(g[k] * o[k] * vis)) for k in ("u", "v", "conic", "sigma", "rgb"))

    for name, attr in (("means", "means"), ("log_scales", "log_scales"), ("quats", "quats"),
                       ("opac", "opac"), ("sh", "sh")):
        delta = rng.standard_normal(getattr(P, attr).shape)
        h = 1e-7
        Pp, Pm = P.copy(), P.copy()
        setattr(Pp, attr, getattr(P, attr) + h * delta)
        setattr(Pm, attr, getattr(P, attr) - h * delta)
        fd = (objective(Pp) - objective(Pm)) / (2 * h)
        an = float(np.sum(acc[name] * delta))
        assert an == pytest.approx(fd, rel=1e-5), name


def _decisions(o):
    return (o["keys"].tobytes(), o["vals"].tobytes(), *[f["last"].tobytes() for f in o["fwds"]],
            *[p["clamp"].tobytes() for p in o["projs"]])


def test_whole_step_gradient_matches_finite_differences():
    s = scenes.tiny(seed=16, n_gaussians=400, width=64, height=48, focal=60.0)
    P = oracle.Params.of(s)
    base = oracle.step(s, P)
    sig = _decisions(base)
    rng = np.random.default_rng(10)
    checked = 0
    for attr, gname in (("means", "means"), ("log_scales", "log_scales"), ("quats", "quats"),
                        ("opac", "opac"), ("sh", "sh")):
        arr = getattr(P, attr)
        for _ in range(6):
            idx = tuple(int(rng.integers(0, n)) for n in arr.shape)
            an = base["grads"][gname][idx]
            h = 1e-6
            Pp, Pm = P.copy(), P.copy()
            getattr(Pp, attr)[idx] += h
            getattr(Pm, attr)[idx] -= h
            op, om = oracle.step(s, Pp, backward=False), oracle.step(s, Pm, backward=False)
            if _decisions(op) != sig or _decisions(om) != sig:
                continue
            fd = (op["loss"] - om["loss"]) / (2 * h)
            assert an == pytest.approx(fd, rel=1e-4, abs=1e-10), (attr, idx)
            checked += 1
    assert checked >= 20


def test_single_gaussian_gradient_closed_form():
    # one Gaussian in front of the camera, degree 0: d img_c / d k00_c = alpha / (2 sqrt(pi))
    # and d img_c / d sigma = G rgb_c while alpha is not clamped
    W = H = 32
    mu, ls = [0.05, -0.03, 3.0], np.log([0.04, 0.03, 0.05])
    P = _params(mu, ls, [0.9, 0.2, 0.1, -0.3], [0.2], np.full((1, 3, 1), 0.3), 0)
    intr = [30.0, 30.0, 16.0, 16.0]
    pr = oracle.project(P, IDENT, intr, W, H)
    ranges = np.array([[0, 1]] * 4, np.int32)
    vals = np.array([0], np.int32)
    f = oracle.raster_fwd(W, H, 16, ranges, vals, pr)
    j, i = 17, 15
    d_img = np.zeros((3, H, W))
    d_img[1, j, i] = 1.0
    g2 = oracle.raster_bwd(W, H, 16, ranges, vals, pr, d_img)
    acc = oracle.project_bwd(P, IDENT, intr, W, H, g2)
    alpha = 1 - f["T"][j, i]
    assert 0 < alpha < oracle.ALPHA_MAX
    assert acc["sh"][0, 1, 0] == pytest.approx(alpha / (2 * math.sqrt(PI)), rel=1e-12)
    assert acc["sh"][0, 0, 0] == 0.0
    G = alpha / pr["sigma"][0]
    assert g2["sigma"][0] == pytest.approx(G * pr["rgb"][1, 0], rel=1e-12)


def test_record_round_trip_and_factor_definition():
    s, P, pr, keys, vals, ranges = _tiny_setup(seed=17)
    rec = RC.to_record(pr)
    back = RC.from_record(rec)
    vis = pr["visible"] > 0
    m = RC.factor(pr["conic"])[:, vis]
    A, B, C = pr["conic"][:, vis]
    np.testing.assert_allclose(m[0] ** 2, RC.C0 * A, rtol=1e-13)
    np.testing.assert_allclose(m[0] * m[1], RC.C0 * B, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(m[1] ** 2 + m[2] ** 2, RC.C0 * C, rtol=1e-13)
    assert np.all(m[0] > 0) and np.all(m[2] > 0)
    np.testing.assert_allclose(back["conic"][:, vis], pr["conic"][:, vis], rtol=2e-6, atol=1e-9)
    np.testing.assert_allclose(back["u"][vis], pr["u"][vis], rtol=1e-7)


def test_alpha_box_contains_every_pixel_with_alpha_above_threshold():
    # brute force over a pixel window around each splat: every pixel whose
    # FP64 alpha reaches 1/255 lies inside the record's packed box
    s, P, pr, keys, vals, ranges = _tiny_setup(seed=18, n=200, W=64, H=48, f=50.0)
    rec = RC.to_record(pr)
    x_lo, x_hi = RC.unpack_box(rec[:, 10])
    y_lo, y_hi = RC.unpack_box(rec[:, 11])
    inside = 0
    for g in np.nonzero(pr["visible"])[0]:
        A, B, C = pr["conic"][:, g]
        u, v = pr["u"][g], pr["v"][g]
        ii, jj = np.meshgrid(np.arange(int(u) - 40, int(u) + 41), np.arange(int(v) - 40, int(v) + 41))
        dx, dy = u - (ii + 0.5), v - (jj + 0.5)
        a = pr["sigma"][g] * np.exp(-0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy)
        hit = a >= oracle.ALPHA_MIN
        assert np.all(ii[hit] >= x_lo[g]) and np.all(ii[hit] <= x_hi[g])
        assert np.all(jj[hit] >= y_lo[g]) and np.all(jj[hit] <= y_hi[g])
        inside += hit.sum()
        # and the box is tight to within the padding
        if hit.any():
            assert x_hi[g] - ii[hit].max() <= 3 and ii[hit].min() - x_lo[g] <= 3
    assert inside > 0


def test_eigen_square_radius_matches_largest_eigenvalue():
    # the 3D Gaussian Splatting square: 3 sqrt(lambda_max) on both axes, the
    # eigenvalue cross-checked with numpy's symmetric eigensolver
    z0, f, th = 3.0, 60.0, 0.4
    s1, s2 = 0.08, 0.02
    q = [math.cos(th / 2), 0, 0, math.sin(th / 2)]
    P = _params([0, 0, z0], np.log([s1, s2, 0.5]), q, [2.0], np.zeros((1, 3, 1)), 0)
    pr = oracle.project(P, IDENT, [f, f, 32, 32], 64, 64, radius_mode=oracle.RADIUS_EIGEN)
    a, b, c = pr["cov"][:, 0]
    lam = np.linalg.eigvalsh(np.array([[a, b], [b, c]])).max()
    assert tuple(pr["radii"][:, 0]) == (math.ceil(3 * math.sqrt(lam)),) * 2
    # never smaller than the per-axis 3-sigma box
    p0 = oracle.project(P, IDENT, [f, f, 32, 32], 64, 64)
    assert np.all(pr["radii"] >= p0["radii"])


def test_opacity_aware_radius_changes_work_not_images():
    # the opacity-aware box drops only tiles where every pixel has
    # alpha < 1/255: images and gradients are identical to the 3-sigma box,
    # with fewer intersections; opaque splats (tau >= 9) keep the 3-sigma box
    s = scenes.tiny(seed=31, n_gaussians=400, width=64, height=48, focal=50.0)
    s.opacity_logits[:] = np.linspace(-5.5, 4.0, 400).astype(np.float32)
    s.log_scales[:] += np.float32(1.0)
    o0 = oracle.step(s, tile=8)
    o1 = oracle.step(s, tile=8, radius_mode=oracle.RADIUS_OPACITY)
    r0, r1 = o0["projs"][0]["radii"], o1["projs"][0]["radii"]
    assert np.all(r1 <= r0)
    assert len(o1["vals"]) < 0.9 * len(o0["vals"])
    assert np.array_equal(o0["imgs"][0], o1["imgs"][0])
    for k in o0["grads"]:
        assert np.array_equal(o0["grads"][k], o1["grads"][k]), k
    pr = o1["projs"][0]
    tau = 2 * np.log(255 * pr["sigma"]) * 1.001 + 0.01
    opaque = pr["visible"].astype(bool) & (tau >= 9.0)
    assert opaque.any() and np.array_equal(r1[:, opaque], r0[:, opaque])
    # brute force: an axis the opacity rule clipped still holds every pixel
    # centre whose alpha reaches 1/255, and is within three pixels of the
    # tightest such half-width
    clipped = 0
    for g in np.nonzero(pr["visible"])[0]:
        A, B, C = pr["conic"][:, g]
        u, v = pr["u"][g], pr["v"][g]
        ii, jj = np.meshgrid(np.arange(int(u) - 60, int(u) + 61), np.arange(int(v) - 60, int(v) + 61))
        dx, dy = ii + 0.5 - u, jj + 0.5 - v
        hit = pr["sigma"][g] * np.exp(-0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy) >= oracle.ALPHA_MIN
        for ax, d in ((0, dx), (1, dy)):
            if r1[ax, g] < r0[ax, g]:
                clipped += 1
                ext = np.abs(d[hit]).max() if hit.any() else 0.0
                assert ext <= r1[ax, g] <= ext + 3
    assert clipped > 100


def test_densify_stats_hand_example():
    # two views (4 x 6 and 2 x 2 pixels, so d/dx_ndc = (2, 3) and (1, 1) times
    # d/du, d/dv), three Gaussians; the third is never visible
    g_uv = [np.array([[1.5, 0.0, 9.0], [1.0, 2.0, 9.0]]), np.array([[3.0, 0.5, 9.0], [4.0, 0.0, 9.0]])]
    visible = [np.array([1, 1, 0]), np.array([1, 0, 0])]
    radii = [np.array([[3, 7, 50], [5, 2, 50]]), np.array([[9, 1, 50], [4, 1, 50]])]
    acc = oracle.densify_stats(g_uv, visible, radii, [(4, 6), (2, 2)])
    # G0: |(3, 3)| + |(3, 4)| = 3 sqrt 2 + 5; G1: |(0, 6)| = 6
    np.testing.assert_allclose(acc["grad"], [3 * math.sqrt(2) + 5, 6.0, 0.0], rtol=1e-15)
    np.testing.assert_array_equal(acc["count"], [2, 1, 0])
    np.testing.assert_array_equal(acc["max_radius"], [9, 7, 0])
    # accumulation continues from a previous call
    acc = oracle.densify_stats(g_uv[:1], visible[:1], radii[:1], [(4, 6)], acc)
    np.testing.assert_array_equal(acc["count"], [3, 2, 0])


def test_adam_matches_torch_optim_adam():
    # library pin: torch.optim.Adam (CPU, float64) over several steps
    import torch
    rng = np.random.default_rng(19)
    p0 = rng.standard_normal(257)
    grads = [rng.standard_normal(257) for _ in range(5)]
    t = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([t], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(257), np.zeros(257)
    for k, g in enumerate(grads, start=1):
        t.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        p, m, v = oracle.adam(p, g, m, v, k, 3e-3, 0.9, 0.999, 1e-8)
        np.testing.assert_allclose(p, t.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_morton_codes_interleave_and_visit_octants_contiguously():
    # decoding the interleaved bits gives back the cells
    rng = np.random.default_rng(21)
    means = rng.uniform(-5, 5, (3, 500)).astype(np.float32)
    org, inv = np.array([-5, -5, -5], np.float32), np.array([102.4, 102.4, 102.4], np.float32)
    cells = oracle.morton_cells(means, org, inv)
    codes = oracle.morton_codes(means, org, inv)
    for k in range(3):
        dec = np.zeros_like(codes)
        for b in range(10):
            dec |= ((codes >> (3 * b + k)) & 1) << b
        np.testing.assert_array_equal(dec, cells[k])
    # a 4x4x4 lattice: Morton order visits each 2x2x2 octant in one run of 8,
    # and the x coordinate varies fastest
    g = np.stack(np.meshgrid(np.arange(4), np.arange(4), np.arange(4), indexing="ij")).reshape(3, -1)
    lat = (g.astype(np.float32) + 0.5) * 256
    order = oracle.morton_order(lat, np.zeros(3, np.float32), np.ones(3, np.float32))
    pts = g[:, order]
    octant = (pts[0] // 2) + 2 * (pts[1] // 2) + 4 * (pts[2] // 2)
    np.testing.assert_array_equal(octant, np.repeat(np.arange(8), 8))
    np.testing.assert_array_equal(pts[:, 1], [1, 0, 0])
    # non-finite and out-of-box coordinates clamp into the grid
    bad = np.array([[np.nan, -1e9, 1e9], [0, 0, 0], [0, 0, 0]], np.float32)
    np.testing.assert_array_equal(oracle.morton_cells(bad, org, inv)[0], [0, 0, 1023])


def test_ssim_window_blur_and_closed_forms():
    import scipy.ndimage as ndi
    w = oracle.ssim_window()
    assert w.sum() == pytest.approx(1.0) and np.allclose(w, w[::-1])
    np.testing.assert_allclose(w / w[5], np.exp(-(np.arange(11) - 5) ** 2 / 4.5), rtol=1e-14)
    # separable zero-padded blur == 2-D correlation with the outer-product window
    img = np.random.default_rng(22).uniform(0, 1, (3, 23, 31))
    ref = np.stack([ndi.correlate(c, np.outer(w, w), mode="constant") for c in img])
    np.testing.assert_allclose(oracle._blur(img, w), ref, atol=1e-14)
    # axes shorter than the window (down to 1 x 1) keep their length
    for shp in [(1, 1, 1), (2, 4, 3), (1, 7, 12)]:
        small = np.random.default_rng(24).uniform(0, 1, shp)
        ref = np.stack([ndi.correlate(c, np.outer(w, w), mode="constant") for c in small])
        np.testing.assert_allclose(oracle._blur(small, w), ref, atol=1e-14)
    # constant images: interior SSIM = (2ab + C1) / (a^2 + b^2 + C1)
    a, b = 0.3, 0.7
    S, _ = oracle.ssim_map(np.full((1, 30, 30), a), np.full((1, 30, 30), b))
    want = (2 * a * b + oracle.SSIM_C1) / (a * a + b * b + oracle.SSIM_C1)
    np.testing.assert_allclose(S[0, 5:-5, 5:-5], want, rtol=1e-12)
    # identical images: SSIM = 1, loss = 0
    S, _ = oracle.ssim_map(img, img)
    np.testing.assert_allclose(S, 1.0, rtol=1e-12)


def test_ssim_l1_gradient_matches_finite_differences():
    rng = np.random.default_rng(23)
    x = rng.uniform(0, 1, (3, 17, 21))
    y = rng.uniform(0, 1, (3, 17, 21))
    L, (g,) = oracle.ssim_l1_loss([x], [y])
    for _ in range(25):
        idx = tuple(int(rng.integers(0, n)) for n in x.shape)
        h = 1e-6
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (oracle.ssim_l1_loss([xp], [y])[0] - oracle.ssim_l1_loss([xm], [y])[0]) / (2 * h)
        assert g[idx] == pytest.approx(fd, rel=1e-5, abs=1e-12)


def test_rectangle_render_matches_full_render_and_signatures_track_decisions():
    """The local re-render the finite-difference spot check uses: any pixel
    rectangle renders bit-identically to the same pixels of the whole-view
    render, and its per-pixel decision signature changes when (and only when)
    a pixel's composited set changes."""
    s = scenes.tiny(seed=21, n_gaussians=1500, width=100, height=75, focal=90.0)
    o = oracle.step(s, backward=False)
    pr = o["projs"][0]
    W, H = 100, 75
    full = o["imgs"][0]
    for x0, y0, x1, y1 in ((0, 0, 100, 75), (13, 7, 61, 40), (96, 64, 100, 75), (16, 16, 32, 32)):
        img, sg = oracle.raster_fwd_rect(W, H, 16, o["ranges"], o["vals"], pr, x0, y0, x1, y1)
        np.testing.assert_array_equal(img, full[:, y0:y1, x0:x1])
        assert sg.shape == (y1 - y0, x1 - x0)
    img0, sg0 = oracle.raster_fwd_rect(W, H, 16, o["ranges"], o["vals"], pr, 0, 0, W, H)
    # a tiny colour change keeps every decision; making one Gaussian fully
    # transparent removes it from every pixel that composited it
    vis = np.nonzero(pr["visible"])[0]
    g = int(vis[np.argmax(pr["sigma"][vis])])
    rgb = pr["rgb"][:, g].copy()
    pr["rgb"][:, g] += 1e-3
    _, sg1 = oracle.raster_fwd_rect(W, H, 16, o["ranges"], o["vals"], pr, 0, 0, W, H)
    pr["rgb"][:, g] = rgb
    np.testing.assert_array_equal(sg1, sg0)
    sig = pr["sigma"][g]
    pr["sigma"][g] = 0.0
    img2, sg2 = oracle.raster_fwd_rect(W, H, 16, o["ranges"], o["vals"], pr, 0, 0, W, H)
    pr["sigma"][g] = sig
    changed = sg2 != sg0
    assert changed.any()
    np.testing.assert_array_equal(img2[:, ~changed], img0[:, ~changed])
