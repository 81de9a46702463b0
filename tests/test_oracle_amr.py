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
