"""GPU parity of the AMR levels (MI355X only).

Rendered positions are the plain full-resolution render's pixels and the
other positions copies (inheritance) or float32 means (interpolation) of
them, so the AMR image must equal the GPU's own full-resolution render
gathered by the oracle's level and fill rule bit for bit, and the oracle's AMR
image within the colour tolerances (ambiguous pixels of the plain render,
gathered the same way, within 1e-4 plus the tolerance the oracle derives for
each; an interpolated pixel's bound is the mean of its samples' bounds plus
the float32 rounding of the mean).  The tile levels of the count modes must
equal the oracle's ranking of the oracle's own per-tile key counts."""
import numpy as np
import pytest

import oracle.amr as oa
import synth
from test_gpu_parity import COLOUR_TOL, assert_amb_within

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    import paper_2507_04147_amd as p
    p.lib()
    assert torch.cuda.is_available()
    return p


def _gpu(pkg, scene, cams, gz, radii, mode=0, fill=0, fracs=(0.25, 0.5, 0.75), want_ranges=False):
    ds = pkg.DeviceScene.from_host(scene)
    ctx = pkg.Context()
    H, W = cams[0].height, cams[0].width
    out = torch.full((len(cams), 3, H, W), float("nan"), device="cuda")
    ctx.render_amr(ds, cams, gz, pkg.amr_struct(*radii, mode=mode, fill=fill, fracs=fracs), out)
    lv = ctx.inspect("amr_levels", torch.uint8).cpu().numpy().astype(np.int32)
    rg = ctx.inspect("ranges", torch.int32).cpu().numpy().view(np.uint32).reshape(-1, 2) if want_ranges else None
    full = torch.empty_like(out)
    ctx.render_full(ds, cams, full)
    ctx.sync()
    ctx.close()
    if want_ranges:
        return out.cpu().numpy(), full.cpu().numpy(), lv, rg
    return out.cpu().numpy(), full.cpu().numpy()


def _split(a, cams):
    T = [((c.height + 15) // 16) * ((c.width + 15) // 16) for c in cams]
    return np.split(a, np.cumsum(T)[:-1])


@pytest.mark.parametrize("radii", [(60.0, 110.0, 170.0), (0.0, 0.0, 0.0), (1e9, 1e9, 1e9)])
def test_amr_small_vs_full_render_and_oracle(pkg, radii):
    W, H = 236, 244
    scene, cams = synth.foveated_stereo(n=60_000, width=W, height=H, seed=9)
    gz = [(0.4 * W, 0.55 * H), (0.4 * W + 3.0, 0.55 * H)]
    amr, full = _gpu(pkg, scene, cams, gz, radii)
    for e in range(2):
        lv = oa.tile_levels(cams[e], gz[e], radii)
        assert np.array_equal(amr[e], oa.amr_image(full[e], lv, W, H))
    ref = oa.render_amr(scene, cams, gz, radii)
    for e in range(2):
        lv = oa.tile_levels(cams[e], gz[e], radii)
        amb = oa.amr_image(ref["images"][e]["amb"][None].astype(np.float64), lv, W, H)[0] != 0
        tol = oa.amr_image(ref["images"][e]["amb_tol"][None], lv, W, H)[0]
        err = np.abs(amr[e] - ref["amr"][e])
        assert err.max(axis=0)[~amb].max() <= COLOUR_TOL
        assert_amb_within(err, amb, tol)


FILL = {0: "inherit", 1: "interpolate"}


@pytest.mark.parametrize("mode,fill,fracs", [(1, 0, (0.25, 0.5, 0.75)), (1, 1, (0.1, 0.3, 0.6)),
                                             (2, 1, (0.25, 0.5, 0.75)), (2, 0, (0.3, 0.3, 0.9)),
                                             (0, 1, (0.0, 0.0, 0.0)), (1, 1, (0.0, 0.0, 0.0)),
                                             (1, 0, (1.0, 1.0, 1.0))])
def test_amr_count_modes_and_interpolation(pkg, mode, fill, fracs):
    """Odd 235 x 243 eyes (ragged tiles and a half block at the edges): tile
    levels by eccentricity, Gaussian count (rank of the tile's key count, ties
    to the lower index) and their minimum; inherited or interpolated fill.
    Levels bit-exact against the oracle's, the image bit-exact against the GPU's
    full render gathered by the oracle's rule, and within tolerance of the
    oracle's AMR image."""
    W, H = 235, 243
    radii = (50.0, 90.0, 140.0)
    scene, cams = synth.foveated_stereo(n=60_000, width=W, height=H, seed=11)
    gz = [(0.45 * W, 0.5 * H), (0.45 * W + 3.0, 0.5 * H)]
    amr, full, lv, rg = _gpu(pkg, scene, cams, gz, radii, mode, fill, fracs, want_ranges=True)
    ref = oa.render_amr(scene, cams, gz, radii, mode=mode, fracs=fracs, fill=FILL[fill])
    np.testing.assert_array_equal(rg, ref["ranges"])
    for e, lv_e in enumerate(_split(lv, cams)):
        np.testing.assert_array_equal(lv_e, ref["levels"][e])
        if mode == 1 and fracs == (1.0, 1.0, 1.0):
            assert (lv_e == 4).all()
        if mode == 1 and fracs == (0.0, 0.0, 0.0):
            assert (lv_e == 1).all()
        assert np.array_equal(amr[e], oa.amr_image(full[e], lv_e, W, H, FILL[fill]))
        amb = oa.amr_image(ref["images"][e]["amb"][None].astype(np.float64), lv_e, W, H, FILL[fill])[0] != 0
        tol = oa.amr_image(ref["images"][e]["amb_tol"][None], lv_e, W, H, FILL[fill])[0]
        err = np.abs(amr[e] - ref["amr"][e])
        slack = 1e-6 if fill else 0.0  # float32 rounding of an interpolated mean
        assert err.max(axis=0)[~amb].max() <= COLOUR_TOL + slack
        assert_amb_within(np.maximum(err - slack, 0.0), amb, tol)


@pytest.mark.parametrize("mode,fill", [(1, 1), (2, 0)])
def test_amr_count_levels_full_size(pkg, mode, fill):
    """1M Gaussians, 2 x 1832 x 1920 (13 800 tiles a view): count levels
    against the oracle's ranking of the GPU's own per-tile counts (the tile
    ranges are bit-exact against the oracle in the parity tests), the image
    against the GPU's full render gathered by that rule."""
    scene, cams = synth.foveated_stereo()
    W, H = cams[0].width, cams[0].height
    gz = [(c.cx + 200.0, c.cy - 150.0) for c in cams]
    radii = (0.15 * W, 0.25 * W, 0.35 * W)
    fracs = (0.2, 0.45, 0.7)
    amr, full, lv, rg = _gpu(pkg, scene, cams, gz, radii, mode, fill, fracs, want_ranges=True)
    rgs = _split(rg, cams)
    for e, lv_e in enumerate(_split(lv, cams)):
        cnt = oa.count_levels(rgs[e][:, 1].astype(np.int64) - rgs[e][:, 0], fracs)
        want = oa.combine_levels(oa.tile_levels(cams[e], gz[e], radii), cnt, mode)
        np.testing.assert_array_equal(lv_e, want)
        assert np.array_equal(amr[e], oa.amr_image(full[e], lv_e, W, H, FILL[fill]))


def test_amr_full_size(pkg):
    """1M Gaussians, 2 x 1832 x 1920, levels at the fovea, between, mid and beyond."""
    scene, cams = synth.foveated_stereo()
    W, H = cams[0].width, cams[0].height
    gz = [(c.cx, c.cy) for c in cams]
    radii = (0.15 * W, 0.25 * W, 0.35 * W)
    amr, full = _gpu(pkg, scene, cams, gz, radii)
    for e in range(2):
        assert np.array_equal(amr[e], oa.amr_image(full[e], oa.tile_levels(cams[e], gz[e], radii), W, H))


def test_amr_arguments(pkg):
    scene, cams = synth.foveated_stereo(n=1000, width=64, height=64, seed=9)
    ds = pkg.DeviceScene.from_host(scene)
    ctx = pkg.Context()
    out = torch.empty((2, 3, 64, 64), device="cuda")
    gz = [(32.0, 32.0)] * 2
    for bad in ((10.0, 5.0, 20.0), (-1.0, 5.0, 20.0), (1.0, 2.0, float("inf"))):
        with pytest.raises(pkg.A3FRError) as e:
            ctx.render_amr(ds, cams, gz, pkg.amr_struct(*bad), out)
        assert e.value.status == pkg.A3FR_EINVAL
    for kw in (dict(mode=3), dict(mode=-1), dict(fill=2), dict(mode=1, fracs=(0.5, 0.2, 0.9)),
               dict(mode=2, fracs=(0.1, 0.2, 1.5)), dict(mode=1, fracs=(-0.1, 0.2, 0.5)),
               dict(mode=1, fracs=(0.1, 0.2, float("nan")))):
        with pytest.raises(pkg.A3FRError) as e:
            ctx.render_amr(ds, cams, gz, pkg.amr_struct(1.0, 2.0, 3.0, **kw), out)
        assert e.value.status == pkg.A3FR_EINVAL
    # the count mode ignores the radii
    ctx.render_amr(ds, cams, gz, pkg.amr_struct(10.0, 5.0, 1.0, mode=1), out)
    ctx.sync()
    with pytest.raises(pkg.A3FRError) as e:  # levels exist only after an AMR frame
        ctx.render_full(ds, cams, out)
        ctx.inspect("amr_levels", torch.uint8)
    assert e.value.status == pkg.A3FR_ENOTREADY
    ctx.close()
