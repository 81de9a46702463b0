"""Pins of the oracle's periphery error estimate and full-resolution fallback
(CPU only): mass conservation of the dropped-opacity map, the threshold
extremes of the flags, and the fallback layer against the plain
full-resolution render."""
import numpy as np

import oracle
import synth


def _frame(n=20_000, W=232, H=240, seed=5):
    scene, cams = synth.foveated_stereo(n=n, width=W, height=H, seed=seed)
    gz = [(100.5, 130.25), (110.0, 128.0)]
    rad = (0.15 * W, 0.35 * W)
    return scene, cams, gz, rad, oracle.foveated_views(cams, gz, rad)


def test_tile_mass_conserves_mass_and_estimate_vanishes_when_all_kept():
    scene, cams, gz, rad, views = _frame()
    ref = oracle.render(scene, views, blend=False)
    for e in range(2):
        pv = 3 * e + 2
        D, K = oracle.tile_mass(ref, views, pv)
        vis = ref["count"][pv] > 0
        drop = vis & (ref["keep"][pv] == 0)
        assert drop.sum() > 0
        np.testing.assert_allclose(D.sum() * 256.0, 2.0 * ref["score"][pv][drop].sum(), rtol=1e-12)
        np.testing.assert_allclose(K.sum() * 256.0, 2.0 * ref["score"][pv][vis & ~drop].sum(), rtol=1e-12)
    ref_all = oracle.render(scene, views, keep_frac=(1, 1), blend=False)
    D, K = oracle.tile_mass(ref_all, views, 2)
    assert not D.any() and not oracle.fallback_estimate(D, K, 1.0, 1.0).any()
    # the transmittance rise is 1 - exp(-D) on an empty tile and vanishes under saturation
    est = oracle.fallback_estimate(np.array([1.0, 1.0]), np.array([0.0, 50.0]), 1.0, 1.0)
    assert abs(est[0] - (1 - np.exp(-1.0)) ** 2) < 1e-15 and est[1] < 1e-40


def test_flags_threshold_extremes_and_monotone():
    scene, cams, gz, rad, views = _frame()
    ref = oracle.render(scene, views, blend=False)
    D, K = oracle.tile_mass(ref, views, 2)
    E = oracle.fallback_estimate(D, K, 1.0, 1.0)
    vp, vf = views[2], views[0]
    f0, x0 = oracle.fallback_flags(D, K, vp, vf, rad[1], 0.0, 1.0, 1.0)
    finf, xinf = oracle.fallback_flags(D, K, vp, vf, rad[1], np.inf, 1.0, 1.0)
    assert not finf.any() and not xinf.any()
    # threshold 0: exactly the periphery tiles that reach outside r_mid
    assert f0.any() and not f0.all()
    prev = f0
    for thr in np.quantile(E[E > 0], [0.2, 0.5, 0.8]):
        f, _ = oracle.fallback_flags(D, K, vp, vf, rad[1], thr, 1.0, 1.0)
        assert not (f & ~prev).any()
        prev = f
    # each flagged periphery tile covers 4 x 4 full-resolution tiles
    assert x0.sum() <= 16 * f0.sum() and x0.sum() > 0


def test_fallback_everywhere_equals_full_resolution_render():
    """Threshold 0: the full-resolution layer's flagged tiles are rendered with
    every Gaussian, so outside r_mid the composite equals the plain
    full-resolution render exactly."""
    scene, cams, gz, rad, views = _frame(n=8000, W=160, H=128)
    ref0 = oracle.render(scene, views, blend=False)
    extra = {}
    flags = []
    for e in range(2):
        D, K = oracle.tile_mass(ref0, views, 3 * e + 2)
        f, x = oracle.fallback_flags(D, K, views[3 * e + 2], views[3 * e], rad[1], 0.0, 1.0, 1.0)
        extra[3 * e] = x
        flags.append(f)
    ref = oracle.render(scene, views, extra_active=extra)
    frr = oracle.render_full(scene, cams)
    W, H = cams[0].width, cams[0].height
    for e in range(2):
        L = ref["images"][3 * e: 3 * e + 3]
        out = oracle.composite(W, H, gz[e], rad, L[0]["rgb"], L[1]["rgb"], L[2]["rgb"])
        out = oracle.composite_fallback(out, L[0]["rgb"], flags[e], W, H, gz[e], rad[1], 64)
        ys, xs = np.mgrid[0:H, 0:W]
        outer = (xs + 0.5 - gz[e][0]) ** 2 + (ys + 0.5 - gz[e][1]) ** 2 > rad[1] ** 2
        np.testing.assert_array_equal(out[:, outer], frr["out"][e][:, outer])
