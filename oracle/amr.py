"""Oracle of the AMR levels (TEST INFRASTRUCTURE ONLY: used by tests/ and the
benchmark's checks, never by the library).

Sec. 3.4: pixels are grouped in 2 x 2 blocks; nearer the gaze more positions
of each block are rendered (Fig. 8: top-left first), the others inherit or
interpolate from the rendered ones; Sec. 3.5 labels each tile with a level
1..4 by eccentricity.  Reading used here: positions in the order top-left,
top-right, bottom-left, bottom-right; a tile of level L renders the first L;
an unrendered position takes the rendered pixel above it, else the top-left
one; the level is 4, 3, 2 within r4 <= r3 <= r2 of the gaze (distance to the
tile's pixel-centre rectangle, the disc-mask test) and 1 beyond.  Rendered
positions are the plain full-resolution render's pixels.
"""
from __future__ import annotations

import numpy as np

from . import core


def tile_levels(cam, gaze, radii):
    """Level per tile [tiles_y * tiles_x]: 1 + membership in the nested discs."""
    lv = np.ones(((cam.height + core.TILE - 1) // core.TILE) * ((cam.width + core.TILE - 1) // core.TILE), np.int32)
    for r in radii:
        v = core.full_view(cam)
        v.mask, v.gx, v.gy, v.r_out = 1, float(gaze[0]), float(gaze[1]), float(r)
        act, _ = core.tile_masks([v])
        lv += act.astype(np.int32)
    return lv


def source_position(k, level):
    """Block position (0 top-left, 1 top-right, 2 bottom-left, 3 bottom-right)
    whose rendered pixel position k shows at this level."""
    if k < level:
        return k
    if 0 <= k - 2 < level:
        return k - 2
    return 0


def amr_image(full_rgb, levels, W, H):
    """The AMR image from the full-resolution render [3][H][W] and the tile levels."""
    ys, xs = np.mgrid[0:H, 0:W]
    tiles_x = (W + core.TILE - 1) // core.TILE
    lv = levels[(ys // core.TILE) * tiles_x + xs // core.TILE]
    k = (xs & 1) + 2 * (ys & 1)
    table = np.array([[source_position(kk, L) for kk in range(4)] for L in range(5)])
    src = table[lv, k]
    sx = (xs & ~1) + (src & 1)
    sy = (ys & ~1) + (src >> 1)
    return full_rgb[:, sy, sx]


def render_amr(scene, cams, gazes, radii, nthreads=None):
    full = core.render_full(scene, cams, nthreads=nthreads)
    outs = []
    for e, cam in enumerate(cams):
        outs.append(amr_image(full["out"][e], tile_levels(cam, gazes[e], radii), cam.width, cam.height))
    full["amr"] = np.stack(outs)
    return full
