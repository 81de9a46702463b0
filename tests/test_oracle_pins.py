"""Pins of the FP64 oracle against what the mathematics fixes (CPU only).

Each test names the part of the method it pins (paper Sec. 2.3: projection,
per-tile depth sort, front-to-back blend; Sec. 3.5: reuse across layers;
Sec. 2.2: foveal layers) and the independent source of truth it uses.
"""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation
from scipy.special import sph_harm_y

import oracle
import synth
from synth import Scene

F32 = np.float32


def tiny_scene(means, scales, quats, opac, sh0, deg_rest=None):
    n = len(means)
    sh = np.zeros((16, 3, n), F32)
    sh[0] = np.asarray(sh0, F32).T
    if deg_rest is not None:
        sh[1:] = deg_rest
    sc = np.asarray(scales, F32).T.copy()
    return Scene(n=n, mean=np.asarray(means, F32).T.copy(), log_scale=np.log(sc).astype(F32), scale=sc,
                 quat=np.asarray(quats, F32).T.copy(), logit=np.zeros(n, F32), opacity=np.asarray(opac, F32),
                 sh=sh)


def origin_cam(w=64, h=64, fov=60.0, bg=(0.0, 0.0, 0.0)):
    return synth.make_camera(w, h, fov, (0.0, 0.0, 0.0), bg=bg)


Y00 = 0.5 / math.sqrt(math.pi)


def dc_colour(f0):
    return np.maximum(0.0, 0.5 + Y00 * np.asarray(f0, np.float64).astype(F32).astype(np.float64))


# --------------------------------------------------------------------------
# projection
# --------------------------------------------------------------------------
def test_single_isotropic_gaussian_closed_form():
    """On-axis isotropic Gaussian (sigma) at depth z: Sigma2D = ((f sigma/z)^2 + 0.3) I,
    centre = principal point; pixel = c min(0.99, o exp(-r^2 / (2 s2))), T = 1 - alpha."""
    sigma, z, o, f0 = 0.0625, 2.0, 0.75, (1.0, -0.5, -3.0)
    sc = tiny_scene([(0, 0, z)], [(sigma,) * 3], [(1, 0, 0, 0)], [o], [f0])
    cam = origin_cam()
    r = oracle.render(sc, [oracle.full_view(cam)])
    s2 = (cam.fx * sigma / z) ** 2 + 0.3
    np.testing.assert_allclose(r["cov"][0, 0], [s2, 0.0, s2], rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(r["mu"][0, 0], [cam.cx, cam.cy], rtol=0, atol=1e-12)
    ys, xs = np.mgrid[0:64, 0:64]
    r2 = (xs + 0.5 - cam.cx) ** 2 + (ys + 0.5 - cam.cy) ** 2
    alpha = np.minimum(0.99, float(F32(o)) * np.exp(-0.5 * r2 / s2))
    alpha = np.where(alpha < 1 / 255, 0.0, alpha)
    c = dc_colour(f0)
    img = r["images"][0]
    for ch in range(3):
        np.testing.assert_allclose(img["rgb"][ch], c[ch] * alpha, rtol=0, atol=1e-12)
    np.testing.assert_allclose(img["T"], 1.0 - alpha, rtol=0, atol=1e-12)
    assert c[2] == 0.0  # the negative channel is clamped at zero


def test_two_gaussians_front_to_back():
    """Two on-axis Gaussians: pixel = c1 a1 + c2 a2 (1 - a1), the nearer first,
    whatever their index order."""
    z = (3.0, 2.0)  # index 0 is the far one
    sig = (float(F32(0.09)), float(F32(0.05)))
    o = (0.6, 0.8)
    f0 = [(1.2, 0.1, 0.4), (-0.3, 0.9, 0.2)]
    sc = tiny_scene([(0, 0, z[0]), (0, 0, z[1])], [(s,) * 3 for s in sig], [(1, 0, 0, 0)] * 2, o, f0)
    cam = origin_cam()
    r = oracle.render(sc, [oracle.full_view(cam)])
    ys, xs = np.mgrid[0:64, 0:64]
    r2 = (xs + 0.5 - cam.cx) ** 2 + (ys + 0.5 - cam.cy) ** 2

    def alpha(k):
        s2 = (cam.fx * sig[k] / z[k]) ** 2 + 0.3
        a = np.minimum(0.99, float(F32(o[k])) * np.exp(-0.5 * r2 / s2))
        return np.where(a < 1 / 255, 0.0, a)

    a_near, a_far = alpha(1), alpha(0)
    c_near, c_far = dc_colour(f0[1]), dc_colour(f0[0])
    for ch in range(3):
        want = c_near[ch] * a_near + c_far[ch] * a_far * (1 - a_near)
        np.testing.assert_allclose(r["images"][0]["rgb"][ch], want, rtol=0, atol=1e-12)
    np.testing.assert_allclose(r["images"][0]["T"], (1 - a_near) * (1 - a_far), rtol=0, atol=1e-12)


def _random_gauss(rng, n, spread=0.6, z0=2.5):
    means = np.stack([rng.uniform(-spread, spread, n), rng.uniform(-spread, spread, n), rng.uniform(z0 - 0.5, z0 + 0.5, n)], 1)
    scales = np.exp(rng.normal(-2.5, 0.6, (n, 3)))
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return means, scales, q


def test_rotation_and_covariance_vs_scipy():
    """Sigma3D = R(q) diag(s^2) R(q)^T with R from scipy's Rotation (quaternion
    order (w,x,y,z) here, (x,y,z,w) in scipy); q and -q give the same matrix;
    Sigma_view = R_w Sigma3D R_w^T for a rotated camera."""
    rng = np.random.default_rng(3)
    means, scales, q = _random_gauss(rng, 40)
    sc = tiny_scene(means, scales, q, [0.5] * 40, [(0, 0, 0)] * 40)
    scn = tiny_scene(means, scales, -q, [0.5] * 40, [(0, 0, 0)] * 40)
    ident = oracle.full_view(origin_cam())
    c2w = synth.rot_yaw_pitch(17.0, -9.0)
    rot = oracle.full_view(synth.make_camera(64, 64, 60, (0.1, -0.2, -0.5), c2w))
    for i in range(40):
        qq = sc.quat[:, i].astype(np.float64)
        Rs = Rotation.from_quat([qq[1], qq[2], qq[3], qq[0]]).as_matrix()
        S3 = Rs @ np.diag(sc.scale[:, i].astype(np.float64) ** 2) @ Rs.T
        ok, p, Sv = oracle.view_cov(sc, ident, i)
        assert ok
        np.testing.assert_allclose(Sv, S3, rtol=1e-11, atol=1e-15)
        ok2, _, Svn = oracle.view_cov(scn, ident, i)
        np.testing.assert_allclose(Svn, Sv, rtol=1e-13, atol=1e-17)
        okr, pr, Svr = oracle.view_cov(sc, rot, i)
        if okr:
            np.testing.assert_allclose(Svr, rot.R @ S3 @ rot.R.T, rtol=1e-10, atol=1e-15)
            np.testing.assert_allclose(pr, rot.R @ sc.mean[:, i].astype(np.float64) + rot.t, rtol=1e-13, atol=1e-13)


def _pinhole(v, p):
    return np.array([v.fx * p[0] / p[2] + v.cx, v.fy * p[1] / p[2] + v.cy])


def _fd_jacobian(v, p, h=1e-6):
    J = np.zeros((2, 3))
    for k in range(3):
        e = np.zeros(3)
        e[k] = h * max(1.0, abs(p[k]))
        J[:, k] = (_pinhole(v, p + e) - _pinhole(v, p - e)) / (2 * e[k])
    return J


def test_projection_matches_numerical_jacobian():
    """Sigma2D - 0.3 I = J Sigma_view J^T with J the finite-difference Jacobian of
    the pinhole map at the view-space mean (clamped to the guard band); the
    centre is the pinhole image of the mean; a layer at 1/s resolution has
    (Sigma2D - 0.3)/s^2."""
    rng = np.random.default_rng(5)
    n = 60
    means, scales, q = _random_gauss(rng, n, spread=2.5)  # some beyond the guard band
    sc = tiny_scene(means, scales, q, [0.5] * n, [(0, 0, 0)] * n)
    cam = synth.make_camera(96, 64, 60, (0.05, 0.02, -0.3), synth.rot_yaw_pitch(5.0, 3.0))
    views = [oracle.full_view(cam)]
    half = oracle.foveated_views([cam], [(48.0, 32.0)], (10.0, 20.0))[1]
    r = oracle.render(sc, views, blend=False)
    rh = oracle.render(sc, [half], blend=False)
    v = views[0]
    limx = 1.3 * 0.5 * v.width / v.fx
    limy = 1.3 * 0.5 * v.height / v.fy
    clamped = 0
    for i in range(n):
        ok, p, Sv = oracle.view_cov(sc, v, i)
        if not ok or not r["proj"][0, i]:
            continue
        pc = p.copy()
        tx, ty = p[0] / p[2], p[1] / p[2]
        if abs(tx) > limx or abs(ty) > limy:
            clamped += 1
            pc[0] = np.clip(tx, -limx, limx) * p[2]
            pc[1] = np.clip(ty, -limy, limy) * p[2]
        J = _fd_jacobian(v, pc)
        want = J @ Sv @ J.T
        a, b, c = r["cov"][0, i]
        got = np.array([[a - 0.3, b], [b, c - 0.3]])
        np.testing.assert_allclose(got, want, rtol=2e-7, atol=1e-9 * np.abs(want).max())
        np.testing.assert_allclose(r["mu"][0, i], _pinhole(v, p), rtol=1e-13)
        ah, bh, ch = rh["cov"][0, i]
        np.testing.assert_allclose([ah - 0.3, bh, ch - 0.3], [(a - 0.3) / 4, b / 4, (c - 0.3) / 4], rtol=1e-12,
                                   atol=1e-14)
        assert r["depth_bits"][0, i] == np.float32(p[2]).view(np.uint32)
    assert clamped > 0


# --------------------------------------------------------------------------
# colour
# --------------------------------------------------------------------------
def _real_sh_scipy(l, m, theta, phi):
    if m == 0:
        return sph_harm_y(l, 0, theta, phi).real
    y = sph_harm_y(l, abs(m), theta, phi)
    return math.sqrt(2.0) * (y.imag if m < 0 else y.real)


def test_sh_basis_vs_scipy_legendre():
    """Real SH of degree <= 3 (Condon-Shortley phase, m = -l..l) against scipy's
    complex spherical harmonics built from associated Legendre functions."""
    rng = np.random.default_rng(7)
    d = rng.normal(size=(2000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    for x, y, z in d[:400]:
        theta = math.acos(max(-1.0, min(1.0, z)))
        phi = math.atan2(y, x)
        want = [_real_sh_scipy(l, m, theta, phi) for l in range(4) for m in range(-l, l + 1)]
        np.testing.assert_allclose(oracle.sh_basis((x, y, z)), want, rtol=1e-12, atol=1e-14)


def test_colour_view_dependence_and_clamp():
    """colour = max(0, 0.5 + sum_k Y_k(d) f_k) with d from the eye centre to the mean."""
    rng = np.random.default_rng(9)
    sc = synth.make_scene(50, 1.0, 11)
    eye = np.array([0.3, -0.1, -3.0])
    col = oracle.colour(sc, [eye])[0]
    for i in range(50):
        d = sc.mean[:, i].astype(np.float64) - eye
        d /= np.linalg.norm(d)
        theta, phi = math.acos(d[2]), math.atan2(d[1], d[0])
        Y = np.array([_real_sh_scipy(l, m, theta, phi) for l in range(4) for m in range(-l, l + 1)])
        want = np.maximum(0.0, 0.5 + Y @ sc.sh[:, :, i].astype(np.float64))
        np.testing.assert_allclose(col[i], want, rtol=1e-12, atol=1e-13)
    assert (col == 0).any() or (col > 0).all()


# --------------------------------------------------------------------------
# blend invariants
# --------------------------------------------------------------------------
def test_zero_opacity_gives_background():
    sc = synth.make_scene(300, 1.0, 13)
    sc.opacity[:] = 0.0
    cam = synth.make_camera(48, 40, 60, (0, 0, -3), bg=(0.2, 0.4, 0.6))
    r = oracle.render(sc, [oracle.full_view(cam)])
    img = r["images"][0]
    for ch, b in enumerate((0.2, 0.4, 0.6)):
        assert np.all(img["rgb"][ch] == b)
    assert np.all(img["T"] == 1.0) and np.all(img["last"] == 0)


def test_partition_of_unity():
    """All colours 1 and background 1: every pixel is exactly sum(a T) + T = 1."""
    sc = synth.make_scene(400, 1.0, 17, log_scale_mean=-2.5)
    cam = synth.make_camera(64, 48, 60, (0, 0, -3), bg=(1.0, 1.0, 1.0))
    ones = np.ones((1, sc.n, 3))
    r = oracle.render(sc, [oracle.full_view(cam)], colours=ones)
    np.testing.assert_allclose(r["images"][0]["rgb"], 1.0, rtol=0, atol=1e-12)
    assert (r["images"][0]["T"] < 0.5).mean() > 0.3  # the scene does cover the image


def test_transmittance_monotone_and_bounded():
    sc = synth.make_scene(2000, 1.0, 19)
    cam = synth.make_camera(64, 64, 60, (0, 0, -3))
    views = [oracle.full_view(cam)]
    r = oracle.render(sc, views)
    rng = np.random.default_rng(0)
    for _ in range(40):
        x, y = rng.integers(0, 64, 2)
        tr = oracle.pixel_trace(r, 0, x, y, views=views)
        assert np.all(np.diff(tr) <= 0) and np.all(tr >= 1e-4) and np.all(tr <= 1.0)
        assert tr.size == 0 or tr[-1] == r["images"][0]["T"][y, x]
    assert np.all(r["T"] >= 1e-4) and np.all(r["T"] <= 1.0)


@pytest.mark.parametrize("tw,th", [(16, 16), (32, 8), (8, 32), (32, 32), (16, 8)])
def test_tiled_equals_brute_force(tw, th):
    """The tiled pipeline (rectangles, keys, stable sort, ranges) reproduces the
    plain per-pixel definition exactly, for any tile shape, on a ragged image."""
    sc = synth.make_scene(180, 1.0, 23, log_scale_mean=-2.3)
    cam = synth.make_camera(72, 40, 60, (0, 0, -3), bg=(0.1, 0.2, 0.3))
    views = [oracle.full_view(cam)]
    r = oracle.render(sc, views, tw=tw, th=th)
    b = oracle.render_brute(sc, views, tw=tw, th=th)
    np.testing.assert_array_equal(r["images"][0]["rgb"], b[0]["rgb"])
    np.testing.assert_array_equal(r["images"][0]["T"], b[0]["T"])


def test_foveated_layers_equal_brute_force_on_active_tiles():
    """Masked and subset layers: every active tile equals the brute force of that
    layer's camera (with the kept subset for the periphery)."""
    sc = synth.make_scene(200, 1.0, 29, log_scale_mean=-2.3)
    cams = synth.stereo_cameras((0, 0, -3), 96, 64, 60)
    gz = [(40.0, 30.0), (50.0, 28.0)]
    views = oracle.foveated_views(cams, gz, (0.15 * 96, 0.35 * 96))
    r = oracle.render(sc, views)
    b = oracle.render_brute(sc, views, keep=r["keep"])
    for v, vw in enumerate(views):
        TX = (vw.width + 15) // 16
        act = r["active"][r["aoff"][v]: r["aoff"][v + 1]].reshape(-1, TX)
        pm = np.kron(act, np.ones((16, 16), np.uint8))[: vw.height, : vw.width].astype(bool)
        assert pm.any()
        for ch in range(3):
            np.testing.assert_array_equal(r["images"][v]["rgb"][ch][pm], b[v]["rgb"][ch][pm])


# --------------------------------------------------------------------------
# keys
# --------------------------------------------------------------------------
def test_footprint_bound_brackets_the_alpha_threshold():
    """Q(o) is a step of 1/8 above 2 ln(1.001 x 255 o) -- every q with
    o exp(-q/2) >= 1/255 (with the margin) is inside -- and at most 11.1,
    the bound for opacity 1 (2 ln 255 < 11.1)."""
    rng = np.random.default_rng(5)
    for o in np.concatenate([rng.uniform(0.0, 1.0, 2000), [1e-6, 1.0 / 255.0, 0.5, 0.97, 0.99, 1.0]]):
        q = oracle.footprint_q(o)
        lo = 2.0 * math.log(max(1.001 * 255.0 * o, 1e-300))
        assert q <= 11.1 and q >= lo - 1e-12
        assert q == 11.1 or (q * 8.0 == round(q * 8.0) and (q - 0.125 < lo or q == 0.125))
    assert oracle.footprint_q(1.0) == 11.1 and oracle.footprint_q(0.0) == 0.125


def test_tile_rectangles_equal_brute_force_overlap():
    """Tile range of each Gaussian = the tiles holding a pixel centre inside the
    box [u - e_x, u + e_x] x [v - e_y, v + e_y], e = sqrt(Q(o) diag(Sigma2D));
    every pixel centre outside the box has alpha < 1/255."""
    sc = synth.make_scene(400, 1.0, 31, log_scale_mean=-2.6)
    cam = synth.make_camera(88, 56, 60, (0, 0, -3))
    for tw, th in [(16, 16), (8, 32)]:
        v = oracle.full_view(cam)
        r = oracle.render(sc, [v], tw=tw, th=th, blend=False)
        TX, TY = (88 + tw - 1) // tw, (56 + th - 1) // th
        xs, ys = np.arange(88) + 0.5, np.arange(56) + 0.5
        for i in range(sc.n):
            if not r["proj"][0, i]:
                assert not r["vis"][0, i]
                continue
            u, vv = r["mu"][0, i]
            a, b, c = r["cov"][0, i]
            q_o = oracle.footprint_q(float(sc.opacity[i]))
            ex, ey = math.sqrt(q_o * a), math.sqrt(q_o * c)
            inx = (xs >= u - ex) & (xs <= u + ex)
            iny = (ys >= vv - ey) & (ys <= vv + ey)
            want = set()
            for tx in range(TX):
                for ty in range(TY):
                    if inx[tx * tw:(tx + 1) * tw].any() and iny[ty * th:(ty + 1) * th].any():
                        want.add((tx, ty))
            x0, x1, y0, y1 = r["rect"][0, i]
            got = {(tx, ty) for tx in range(x0, x1 + 1) for ty in range(y0, y1 + 1)} if r["vis"][0, i] else set()
            assert got == want, i
            # footprint guarantee
            X, Y = np.meshgrid(xs, ys)
            det = a * c - b * b
            q = (c * (X - u) ** 2 - 2 * b * (X - u) * (Y - vv) + a * (Y - vv) ** 2) / det
            alpha = float(sc.opacity[i]) * np.exp(-0.5 * q)
            outside = ~(np.abs(X - u) <= ex) | ~(np.abs(Y - vv) <= ey)
            assert np.all(alpha[outside] < 1 / 255)


def test_emission_order_sort_and_ranges():
    """Keys are emitted (view, index, row, column); the sorted order equals a
    lexicographic sort on (tile, depth bits, index); ranges delimit the runs."""
    sc = synth.make_scene(3000, 1.0, 37)
    cams = synth.stereo_cameras((0, 0, -3), 128, 96, 60)
    views = oracle.foveated_views(cams, [(60.0, 50.0), (70.0, 40.0)], (0.15 * 128, 0.35 * 128))
    r = oracle.render(sc, views, blend=False)
    keys, vals = r["keys"], r["vals"]
    # emission order
    tile = (keys >> np.uint64(32)).astype(np.int64)
    view = np.searchsorted(r["tile_off"], tile, side="right") - 1
    order = np.lexsort((tile, vals.astype(np.int64), view))
    np.testing.assert_array_equal(order, np.arange(keys.size))
    cnt = (r["count"] * np.where([[vw.select] for vw in views], r["keep"], 1)).sum()
    assert cnt == keys.size
    # sort
    o = np.lexsort((vals, keys & np.uint64(0xFFFFFFFF), keys >> np.uint64(32)))
    np.testing.assert_array_equal(r["sorted_keys"], keys[o])
    np.testing.assert_array_equal(r["sorted_vals"], vals[o])
    # ranges
    st = (r["sorted_keys"] >> np.uint64(32)).astype(np.int64)
    for t in np.unique(st):
        s, e = r["ranges"][t]
        assert np.all(st[s:e] == t) and (s == 0 or st[s - 1] != t) and (e == st.size or st[e] != t)
    empty = np.setdiff1d(np.arange(r["ranges"].shape[0]), st)
    assert np.all(r["ranges"][empty] == 0)


def test_select_equals_argsort():
    """Periphery subset: the top ceil(3/10 N_vis) by (score desc, index asc)."""
    rng = np.random.default_rng(41)
    n = 5000
    vis = (rng.uniform(size=n) < 0.7).astype(np.uint8)
    score = np.round(rng.exponential(size=n), 2)  # many ties
    keep, k = oracle.select(vis, score)
    nv = int(vis.sum())
    assert k == -(-3 * nv // 10)
    idx = np.nonzero(vis)[0]
    o = idx[np.lexsort((idx, -score[idx]))][:k]
    want = np.zeros(n, np.uint8)
    want[o] = 1
    np.testing.assert_array_equal(keep, want)


# --------------------------------------------------------------------------
# foveation: masks, composite, PSNR
# --------------------------------------------------------------------------
def _layer_active_pixels(r, v, vw):
    TX = (vw.width + 15) // 16
    act = r["active"][r["aoff"][v]: r["aoff"][v + 1]].reshape(-1, TX)
    return np.kron(act, np.ones((16, 16), np.uint8))[: vw.height, : vw.width].astype(bool)


@pytest.mark.parametrize("gaze", [(100.0, 60.0), (3.0, 120.0), (180.0, 5.0)])
def test_masks_cover_what_the_composite_reads(gaze):
    W, H = 192, 128
    cam = synth.make_camera(W, H, 60, (0, 0, -3))
    rf, rm = 0.15 * W, 0.35 * W
    views = oracle.foveated_views([cam], [gaze], (rf, rm))
    sc = synth.make_scene(10, 1.0, 1)
    r = oracle.render(sc, views, blend=False)
    fov, mid = _layer_active_pixels(r, 0, views[0]), _layer_active_pixels(r, 1, views[1])
    assert not mid.all() and not fov.all()
    ys, xs = np.mgrid[0:H, 0:W]
    rho2 = (xs + 0.5 - gaze[0]) ** 2 + (ys + 0.5 - gaze[1]) ** 2
    assert fov[rho2 <= rf * rf].all()
    # mid: bilinear taps of every pixel in r_f < rho <= r_m
    sel = (rho2 > rf * rf) & (rho2 <= rm * rm)
    Wm, Hm = W // 2, H // 2
    sx = np.clip((xs[sel] + 0.5) / 2 - 0.5, 0, Wm - 1)
    sy = np.clip((ys[sel] + 0.5) / 2 - 0.5, 0, Hm - 1)
    x0, y0 = np.floor(sx).astype(int), np.floor(sy).astype(int)
    x1, y1 = np.minimum(x0 + 1, Wm - 1), np.minimum(y0 + 1, Hm - 1)
    for yy in (y0, y1):
        for xx in (x0, x1):
            assert mid[yy, xx].all()
    # and through the composite itself: inactive pixels hold NaN, output has none
    f = np.full((3, H, W), np.nan)
    f[:, fov] = 0.25
    m = np.full((3, Hm, Wm), np.nan)
    m[:, mid] = 0.5
    p = np.full((3, H // 4, W // 4), 0.75)
    out = oracle.composite(W, H, gaze, (rf, rm), f, m, p)
    assert not np.isnan(out).any()


def test_bilinear_matches_torch_interpolate():
    rng = np.random.default_rng(43)
    W, H = 64, 48
    mid = rng.uniform(size=(3, H // 2, W // 2))
    per = rng.uniform(size=(3, H // 4, W // 4))
    fov = np.zeros((3, H, W))
    far = (-1e9, -1e9)
    out_mid = oracle.composite(W, H, far, (0.0, 1e12), fov, mid, per)
    want = torch.nn.functional.interpolate(torch.from_numpy(mid)[None], scale_factor=2, mode="bilinear",
                                           align_corners=False)[0].numpy()
    np.testing.assert_allclose(out_mid, want, rtol=0, atol=1e-13)
    out_per = oracle.composite(W, H, far, (0.0, 0.0), fov, mid, per)
    want = torch.nn.functional.interpolate(torch.from_numpy(per)[None], scale_factor=4, mode="bilinear",
                                           align_corners=False)[0].numpy()
    np.testing.assert_allclose(out_per, want, rtol=0, atol=1e-13)
    # inside r_f the fovea is taken verbatim
    out_f = oracle.composite(W, H, (32.0, 24.0), (1e9, 1e9), rng.uniform(size=(3, H, W)), mid, per)
    assert out_f.shape == (3, H, W)


def test_psnr_closed_forms():
    W, H = 40, 32
    rng = np.random.default_rng(47)
    a = rng.uniform(0.2, 0.8, size=(3, H, W))
    p, po = oracle.periphery_psnr(W, H, (20.0, 16.0), (5.0, 10.0), a, a)
    assert p == math.inf and po == math.inf
    b = a + 0.01
    p, po = oracle.periphery_psnr(W, H, (20.0, 16.0), (5.0, 10.0), a, b)
    assert abs(p - 40.0) < 1e-9 and abs(po - 40.0) < 1e-9
    # values are clamped to [0,1] before the error
    c = np.full((3, H, W), 1.5)
    d = np.ones((3, H, W))
    assert oracle.periphery_psnr(W, H, (20.0, 16.0), (5.0, 10.0), c, d)[0] == math.inf


# --------------------------------------------------------------------------
# tolerance of ambiguous pixels: the colour change of the reversed decision
# --------------------------------------------------------------------------
def test_ambiguity_tolerance_of_a_skip_decision():
    """A near Gaussian whose alpha at one pixel centre is 1/255 up to float32
    rounding of its opacity: the pixel is ambiguous, and its tolerance is the
    closed-form difference between blending that Gaussian and skipping it,
    max over channels of |a1 (c1 - c2 a2)| (two on-axis Gaussians, bg 0)."""
    z, sig = (3.0, 2.0), (float(F32(0.09)), float(F32(0.05)))
    f0 = [(1.2, 0.1, 0.4), (-0.3, 0.9, 0.2)]
    cam = origin_cam()
    px, py = 34, 33
    r2p = (px + 0.5 - cam.cx) ** 2 + (py + 0.5 - cam.cy) ** 2
    s2n = (cam.fx * sig[1] / z[1]) ** 2 + 0.3
    o_near = float(F32((1.0 / 255.0) / math.exp(-0.5 * r2p / s2n)))
    assert o_near < 0.99
    sc = tiny_scene([(0, 0, z[0]), (0, 0, z[1])], [(s,) * 3 for s in sig], [(1, 0, 0, 0)] * 2, (0.6, o_near), f0)
    r = oracle.render(sc, [oracle.full_view(cam)])
    img = r["images"][0]
    s2f = (cam.fx * sig[0] / z[0]) ** 2 + 0.3
    a1 = o_near * math.exp(-0.5 * r2p / s2n)
    a2 = min(0.99, float(F32(0.6)) * math.exp(-0.5 * r2p / s2f))
    c1, c2 = dc_colour(f0[1]), dc_colour(f0[0])
    assert abs(a1 - 1 / 255) <= oracle.EPS_ALPHA / 255
    assert img["amb"][py, px] == 1
    want = np.max(np.abs(a1 * (c1 - c2 * a2)))
    np.testing.assert_allclose(img["amb_tol"][py, px], want, rtol=1e-12)
    # pixels with no near-threshold decision carry no tolerance
    assert np.all(img["amb_tol"][img["amb"] == 0] == 0.0)


def test_ambiguity_tolerance_of_a_stop_decision():
    """Two opaque on-axis Gaussians (alpha clamped at 0.99): after both,
    T = (1 - 0.99)^2, which is 1e-4 up to rounding, so the stop decision at
    the second is ambiguous.  Blending it or stopping before it differ by
    0.99 (1 - 0.99) c2 + ((1 - 0.99)^2 - (1 - 0.99)) bg, the tolerance."""
    bg = (0.25, 0.5, 0.75)
    f0 = [(1.2, 0.1, 0.4), (-0.3, 0.9, 0.2)]
    sc = tiny_scene([(0, 0, 3.0), (0, 0, 2.0)], [(0.3,) * 3, (0.3,) * 3], [(1, 0, 0, 0)] * 2, (0.999, 0.999), f0)
    cam = origin_cam(bg=bg)
    r = oracle.render(sc, [oracle.full_view(cam)])
    img = r["images"][0]
    py, px = 31, 31  # pixel centre 0.5 px from the principal point: both alphas clamp
    c2 = dc_colour(f0[0])
    t1 = 1.0 - 0.99
    want = np.max(np.abs(0.99 * t1 * c2 + (t1 * t1 - t1) * np.asarray(bg)))
    assert img["amb"][py, px] == 1 and img["last"][py, px] == 2
    np.testing.assert_allclose(img["amb_tol"][py, px], want, rtol=1e-12)
    assert want > 5e-3  # a stop decision can move a colour far more than 1e-4
