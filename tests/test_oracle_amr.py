"""Pins of the AMR oracle (CPU only): the inheritance table, nested levels,
level 4 everywhere = the plain render, level 1 = constant 2 x 2 blocks, and
the rendered positions equal the plain render's pixels."""
import numpy as np

import oracle.amr as oa
import oracle.core as oc
import synth


def test_source_table():
    want = {1: [0, 0, 0, 0], 2: [0, 1, 0, 1], 3: [0, 1, 2, 1], 4: [0, 1, 2, 3]}
    for L, row in want.items():
        assert [oa.source_position(k, L) for k in range(4)] == row


def test_levels_nested_and_monotone():
    cam = synth.foveated_stereo(n=10)[1][0]
    lv = oa.tile_levels(cam, (700.0, 900.0), (200.0, 400.0, 650.0))
    assert lv.min() >= 1 and lv.max() <= 4
    tx = (cam.width + 15) // 16
    # a tile's level never increases away from the gaze along a row
    row = lv.reshape(-1, tx)[900 // 16]
    left = row[: 700 // 16 + 1][::-1]
    assert np.all(np.diff(left) <= 0)


def _small():
    sc = synth.make_scene(3000, 1.0, seed=21)
    cams = [synth.make_camera(70, 54, 60.0, (0.0, 0.0, -3.0))]
    return sc, cams


def test_level4_is_full_render_and_level1_blocks_constant():
    sc, cams = _small()
    r = oa.render_amr(sc, cams, [(35.0, 27.0)], (1e9, 1e9, 1e9))
    np.testing.assert_array_equal(r["amr"][0], r["out"][0])
    r1 = oa.render_amr(sc, cams, [(35.0, 27.0)], (-1.0, -1.0, -1.0))
    img = r1["amr"][0]
    H, W = img.shape[1:]
    for y in range(0, H, 2):
        for x in range(0, W, 2):
            blk = img[:, y:y + 2, x:x + 2].reshape(3, -1)
            assert np.all(blk == blk[:, :1])
            assert np.all(blk[:, 0] == r1["out"][0][:, y, x])


def test_rendered_positions_are_full_render():
    sc, cams = _small()
    r = oa.render_amr(sc, cams, [(10.0, 40.0)], (12.0, 25.0, 40.0))
    lv = oa.tile_levels(cams[0], (10.0, 40.0), (12.0, 25.0, 40.0))
    full, amr = r["out"][0], r["amr"][0]
    H, W = amr.shape[1:]
    tx = (W + 15) // 16
    for y in range(H):
        for x in range(W):
            k = (x & 1) + 2 * (y & 1)
            if k < lv[(y // 16) * tx + x // 16]:
                assert np.array_equal(amr[:, y, x], full[:, y, x])


def test_count_levels_rank_tiles_by_their_gaussians():
    """Count levels: the top ceil(f T) tiles by (count desc, index asc) reach
    each level; ties go to the lower tile index; levels are monotone in the
    count; fractions 0 and 1 give all level 1 and all level 4."""
    rng = np.random.default_rng(5)
    c = rng.integers(0, 40, 101)
    lv = oa.count_levels(c, (0.1, 0.3, 0.6))
    for f, L in ((0.1, 4), (0.3, 3), (0.6, 2)):
        assert int((lv >= L).sum()) == int(np.ceil(f * c.size))
    # a tile with more Gaussians never has a lower level
    for i in range(c.size):
        for j in range(c.size):
            if c[i] > c[j]:
                assert lv[i] >= lv[j]
    # ties: equal counts, the lower index first
    eq = oa.count_levels(np.full(8, 3), (0.25, 0.5, 0.75))
    assert list(eq) == [4, 4, 3, 3, 2, 2, 1, 1]
    assert np.all(oa.count_levels(c, (0.0, 0.0, 0.0)) == 1) and np.all(oa.count_levels(c, (1.0, 1.0, 1.0)) == 4)
    assert np.all(oa.combine_levels(np.full(4, 2), np.array([1, 2, 3, 4]), 2) == [1, 2, 2, 2])


def test_interpolation_reproduces_a_linear_image():
    """Bilinear interpolation of the top-left samples is exact for an image
    linear in x and y (away from the last row and column, where it clamps);
    rendered positions keep the full render's pixels; level 4 interpolates nothing."""
    H, W = 36, 42
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    full = np.stack([0.01 * xs + 0.02 * ys, 0.5 - 0.003 * xs, 0.001 * ys + 0.2])
    tx = (W + 15) // 16
    lv = np.array([1, 2, 3, 4, 1, 2, 3, 4, 1][: tx * ((H + 15) // 16)], np.int32)
    img = oa.amr_image(full, lv, W, H, fill="interpolate")
    np.testing.assert_allclose(img[:, : H - 1, : W - 1], full[:, : H - 1, : W - 1], rtol=0, atol=1e-14)
    np.testing.assert_array_equal(oa.amr_image(full, np.full_like(lv, 4), W, H, fill="interpolate"), full)
    # a level-1 tile of a constant image stays constant
    const = np.full((3, H, W), 0.25)
    np.testing.assert_array_equal(oa.amr_image(const, np.ones_like(lv), W, H, fill="interpolate"), const)


def test_interpolated_positions_are_means_of_top_left_samples():
    sc, cams = _small()
    r = oa.render_amr(sc, cams, [(35.0, 27.0)], (-1.0, -1.0, -1.0), fill="interpolate")
    full, img = r["out"][0], r["amr"][0]
    H, W = img.shape[1:]
    x, y = 21, 13  # odd, odd: four samples
    np.testing.assert_allclose(img[:, y, x], 0.25 * (full[:, 12, 20] + full[:, 12, 22] + full[:, 14, 20] +
                                                     full[:, 14, 22]), rtol=0, atol=1e-15)
    np.testing.assert_array_equal(img[:, 12, 20], full[:, 12, 20])
    # the last (odd, odd) pixel of the even-sized image clamps to its own block's sample
    assert H % 2 == 0 and W % 2 == 0
    np.testing.assert_array_equal(img[:, H - 1, W - 1], full[:, H - 2, W - 2])
