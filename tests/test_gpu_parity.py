"""GPU parity of the HIP path against the FP64 oracle (MI355X only).

Bar: integer outputs (per-(view, Gaussian) counts, depth keys, tile
rectangles, offsets, keys in emission order, sorted keys and values, tile
ranges, active tiles, periphery subset, last-contributor index) bit-exact;
float32 colours within 1e-4 absolute of the FP64 oracle, except on pixels the
oracle flags as ambiguous (a skip/stop decision inside the float32 error bound
of its threshold), which are counted and checked at 2e-2.
"""
import math

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

COLOUR_TOL = 1e-4
AMB_TOL = 2e-2


@pytest.fixture(scope="module")
def pkg():
    import paper_2507_04147_amd as p
    p.lib()
    assert torch.cuda.is_available()
    return p


@pytest.fixture(scope="module")
def ctx(pkg):
    c = pkg.Context()
    yield c
    c.close()


def _u(t, dt):
    return t.cpu().numpy().view(dt)


def gpu_render(pkg, ctx, scene, views, keep=(3, 10), debug=True):
    ds = pkg.DeviceScene.from_host(scene)
    ctx.set_debug(debug)
    ctx.preprocess(ds, views, keep)
    K = ctx.bin_sort()
    npx = sum(v.width * v.height for v in views)
    rgb = torch.full((3 * npx,), float("nan"), device="cuda")
    T = torch.full((npx,), float("nan"), device="cuda")
    last = torch.zeros(npx, dtype=torch.int32, device="cuda")
    ctx.blend(rgb, T, last)
    ctx.sync()
    return ds, K, rgb, T, last


def compare_stage_outputs(ctx, ref, views, n):
    nv = len(views)
    counts = _u(ctx.inspect("counts", torch.int32), np.uint32).reshape(nv, n)
    vis = ref["vis"].astype(bool)
    np.testing.assert_array_equal(counts, ref["count"].astype(np.uint32) * vis)
    depth = _u(ctx.inspect("depth", torch.int32), np.uint32).reshape(nv, n)
    np.testing.assert_array_equal(depth[vis], ref["depth_bits"][vis])
    rect = _u(ctx.inspect("rect", torch.int64), np.uint64).reshape(nv, n)
    r = ref["rect"].astype(np.uint64)
    want = r[..., 0] | (r[..., 1] << np.uint64(16)) | (r[..., 2] << np.uint64(32)) | (r[..., 3] << np.uint64(48))
    np.testing.assert_array_equal(rect[vis], want[vis])
    act = ctx.inspect("active", torch.uint8).cpu().numpy()
    np.testing.assert_array_equal(act, ref["active"])
    if any(v.select for v in views):
        keep = ctx.inspect("keep", torch.uint8).cpu().numpy().reshape(nv, n)
        for v, vw in enumerate(views):
            if vw.select:
                np.testing.assert_array_equal(keep[v], ref["keep"][v])
    keys = _u(ctx.inspect("keys", torch.int64), np.uint64)
    vals = _u(ctx.inspect("vals", torch.int32), np.uint32)
    np.testing.assert_array_equal(keys, ref["keys"])
    np.testing.assert_array_equal(vals, ref["vals"])
    sk = _u(ctx.inspect("sorted_keys", torch.int64), np.uint64)
    sv = _u(ctx.inspect("sorted_vals", torch.int32), np.uint32)
    np.testing.assert_array_equal(sk, ref["sorted_keys"])
    np.testing.assert_array_equal(sv, ref["sorted_vals"])
    rg = _u(ctx.inspect("ranges", torch.int32), np.uint32).reshape(-1, 2)
    np.testing.assert_array_equal(rg.astype(np.int64), ref["ranges"])


def compare_images(views, ref, rgb, T, last, active):
    rgb, T, last = rgb.cpu().numpy(), T.cpu().numpy(), last.cpu().numpy()
    n_amb = 0
    for v, vw in enumerate(views):
        a, b = int(ref["img_off"][v]), int(ref["img_off"][v + 1])
        H, W = vw.height, vw.width
        TX = (W + 15) // 16
        act = active[ref["aoff"][v]: ref["aoff"][v + 1]].reshape(-1, TX)
        pm = np.kron(act, np.ones((16, 16), np.uint8))[:H, :W].astype(bool)
        amb = ref["amb"][a:b].reshape(H, W).astype(bool) & pm
        ok = pm & ~amb
        g = rgb[3 * a: 3 * b].reshape(3, H, W)
        o = ref["rgb"][3 * a: 3 * b].reshape(3, H, W)
        err = np.abs(g - o)
        assert np.isfinite(g[:, pm]).all()
        assert err[:, ok].max(initial=0.0) <= COLOUR_TOL, (v, err[:, ok].max())
        assert err[:, amb].max(initial=0.0) <= AMB_TOL, (v, err[:, amb].max())
        gT = T[a:b].reshape(H, W)
        oT = ref["T"][a:b].reshape(H, W)
        assert np.abs(gT - oT)[ok].max(initial=0.0) <= COLOUR_TOL
        gl = last[a:b].reshape(H, W)
        ol = ref["last"][a:b].reshape(H, W)
        np.testing.assert_array_equal(gl[ok], ol[ok])
        n_amb += int(amb.sum())
    return n_amb


# ---------------------------------------------------------------------------
def test_fp64_sqrt_and_division_are_correctly_rounded(pkg, ctx):
    """The key path needs IEEE float64 sqrt and division on the device."""
    rng = np.random.default_rng(0)
    n = 1 << 22
    x = np.exp(rng.uniform(-60, 60, n)) * rng.uniform(0.5, 2.0, n)
    y = np.exp(rng.uniform(-30, 30, n)) * np.where(rng.uniform(size=n) < 0.5, -1.0, 1.0)
    x[:4] = [0.0, 1.0, 2.0, 4.0]
    sq, dv = ctx.fp64_probe(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
    ctx.sync()
    np.testing.assert_array_equal(sq.cpu().numpy().view(np.uint64), np.sqrt(x).view(np.uint64))
    np.testing.assert_array_equal(dv.cpu().numpy().view(np.uint64), (x / y).view(np.uint64))


def test_single_view_parity(pkg, ctx):
    """Single view, no foveation: 10,000 Gaussians in [-1,1]^3, 256 x 256."""
    scene, cam = synth.single_view()
    views = [oracle.full_view(cam)]
    ref = oracle.render(scene, views)
    _, K, rgb, T, last = gpu_render(pkg, ctx, scene, views)
    assert K == ref["keys"].size
    compare_stage_outputs(ctx, ref, views, scene.n)
    n_amb = compare_images(views, ref, rgb, T, last, ref["active"])
    assert n_amb < 0.002 * 256 * 256


@pytest.mark.parametrize("size,gaze,n", [((232, 240), "centre", 60_000), ((200, 136), (3.0, 120.0), 40_000),
                                         ((232, 240), (220.0, 10.0), 60_000)])
def test_foveated_stereo_layers_parity(pkg, ctx, size, gaze, n):
    """Foveated stereo (fovea disc, mid annulus at 1/2, periphery subset at 1/4)
    on a ragged tile grid: every stage and every active tile."""
    W, H = size
    scene, cams = synth.foveated_stereo(n=n, width=W, height=H, seed=2)
    gz = [(c.cx, c.cy) for c in cams] if gaze == "centre" else [gaze, (gaze[0] - 6.0, gaze[1] + 2.0)]
    rad = (0.15 * W, 0.35 * W)
    views = oracle.foveated_views(cams, gz, rad)
    ref = oracle.render(scene, views)
    _, K, rgb, T, last = gpu_render(pkg, ctx, scene, views)
    assert K == ref["keys"].size
    compare_stage_outputs(ctx, ref, views, scene.n)
    compare_images(views, ref, rgb, T, last, ref["active"])


def test_full_render_and_composite_parity(pkg, ctx):
    """render_full (FRR) and render_foveated (layers + composite) against the
    oracle's, on the same small stereo scene."""
    W, H = 232, 240
    scene, cams = synth.foveated_stereo(n=50_000, width=W, height=H, seed=5)
    gz = [(100.5, 130.25), (110.0, 128.0)]
    rad = (0.15 * W, 0.35 * W)
    ds = pkg.DeviceScene.from_host(scene)
    out = torch.zeros((2, 3, H, W), device="cuda")
    ctx.set_debug(False)
    ctx.render_full(ds, cams, out)
    ctx.sync()
    fr = oracle.render_full(scene, cams)
    for e in range(2):
        amb = fr["images"][e]["amb"].astype(bool)
        err = np.abs(out[e].cpu().numpy() - fr["out"][e])
        assert err[:, ~amb].max() <= COLOUR_TOL
        assert err[:, amb].max(initial=0.0) <= AMB_TOL
    fv = oracle.render_foveated(scene, cams, gz, rad)
    outf = torch.zeros((2, 3, H, W), device="cuda")
    ctx.render_foveated(ds, cams, gz, pkg.fovea_struct(*rad), outf)
    ctx.sync()
    for e in range(2):
        amb = composite_ambiguity(W, H, gz[e], rad, fv["images"][3 * e: 3 * e + 3])
        err = np.abs(outf[e].cpu().numpy() - fv["out"][e])
        assert err[:, ~amb].max() <= COLOUR_TOL
        assert err[:, amb].max(initial=0.0) <= AMB_TOL
    # the quality judge on the GPU equals the oracle's region sums
    sse, cnt = ctx.region_sse(W, H, gz[0], rad[0], rad[1], outf[0], out[0])
    osse, ocnt = oracle.region_sse(W, H, gz[0], rad, outf[0].cpu().numpy().astype(np.float64),
                                   out[0].cpu().numpy().astype(np.float64))
    np.testing.assert_array_equal(cnt, ocnt)
    np.testing.assert_allclose(sse, osse, rtol=1e-9, atol=1e-12)


def composite_ambiguity(W, H, gaze, rad, layers):
    """Full-resolution pixels whose composite reads an ambiguous layer pixel."""
    ys, xs = np.mgrid[0:H, 0:W]
    px, py = xs + 0.5, ys + 0.5
    r2 = (px - gaze[0]) ** 2 + (py - gaze[1]) ** 2
    out = np.zeros((H, W), bool)
    f = r2 <= rad[0] ** 2
    out[f] = layers[0]["amb"][f].astype(bool)
    for reg, s, L in ((1, 2, layers[1]), (2, 4, layers[2])):
        sel = (~f & (r2 <= rad[1] ** 2)) if reg == 1 else (r2 > rad[1] ** 2)
        Hl, Wl = H // s, W // s
        sx = np.clip(px[sel] / s - 0.5, 0, Wl - 1)
        sy = np.clip(py[sel] / s - 0.5, 0, Hl - 1)
        x0, y0 = np.floor(sx).astype(int), np.floor(sy).astype(int)
        x1, y1 = np.minimum(x0 + 1, Wl - 1), np.minimum(y0 + 1, Hl - 1)
        a = L["amb"].astype(bool)
        out[sel] = a[y0, x0] | a[y0, x1] | a[y1, x0] | a[y1, x1]
    return out


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------
def test_empty_scene_and_all_culled(pkg, ctx):
    cam = synth.make_camera(40, 24, 60, (0, 0, -3), bg=(0.25, 0.5, 0.75))
    for n, behind in ((0, False), (500, True)):
        scene = synth.make_scene(max(n, 1), 1.0, 3)
        if n == 0:
            scene = scene.subset(np.arange(0))
        if behind:
            scene.mean[2] = -10.0  # every point behind the camera
        _, K, rgb, T, last = gpu_render(pkg, ctx, scene, [oracle.full_view(cam)])
        assert K == 0
        img = rgb.cpu().numpy().reshape(3, 24, 40)
        for ch, b in enumerate((0.25, 0.5, 0.75)):
            assert np.all(img[ch] == np.float32(b))
        assert np.all(T.cpu().numpy() == 1.0) and np.all(last.cpu().numpy() == 0)


@pytest.mark.parametrize("keep", [(0, 10), (10, 10), (1, 1000)])
def test_periphery_keep_extremes(pkg, ctx, keep):
    W, H = 96, 64
    scene, cams = synth.foveated_stereo(n=8000, width=W, height=H, seed=7)
    views = oracle.foveated_views(cams, [(40.0, 30.0), (44.0, 30.0)], (0.15 * W, 0.35 * W))
    ref = oracle.render(scene, views, keep_frac=keep)
    _, K, rgb, T, last = gpu_render(pkg, ctx, scene, views, keep=keep)
    assert K == ref["keys"].size
    compare_stage_outputs(ctx, ref, views, scene.n)
    compare_images(views, ref, rgb, T, last, ref["active"])


def test_gaze_outside_image_and_zero_fovea(pkg, ctx):
    W, H = 128, 96
    scene, cams = synth.foveated_stereo(n=10000, width=W, height=H, seed=9)
    views = oracle.foveated_views(cams, [(-500.0, 40.0), (60.0, 1e4)], (0.0, 0.35 * W))
    ref = oracle.render(scene, views)
    _, K, rgb, T, last = gpu_render(pkg, ctx, scene, views)
    compare_stage_outputs(ctx, ref, views, scene.n)
    compare_images(views, ref, rgb, T, last, ref["active"])


def test_deterministic_across_runs(pkg, ctx):
    scene, cam = synth.single_view(n=20000)
    views = [oracle.full_view(cam)]
    _, _, rgb1, T1, l1 = gpu_render(pkg, ctx, scene, views, debug=False)
    _, _, rgb2, T2, l2 = gpu_render(pkg, ctx, scene, views, debug=False)
    assert torch.equal(rgb1, rgb2) and torch.equal(T1, T2) and torch.equal(l1, l2)


def test_invalid_arguments_enqueue_nothing(pkg, ctx):
    scene, cam = synth.single_view(n=100)
    ds = pkg.DeviceScene.from_host(scene)
    v = oracle.full_view(cam)
    v.width = 0
    with pytest.raises(pkg.A3FRError) as e:
        ctx.preprocess(ds, [v])
    assert e.value.status == pkg.A3FR_EINVAL
    v = oracle.full_view(cam)
    v.mask = 7
    with pytest.raises(pkg.A3FRError):
        ctx.preprocess(ds, [v])
