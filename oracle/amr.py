"""Oracle of the AMR levels (TEST INFRASTRUCTURE ONLY: used by tests/ and the
benchmark's checks, never by the library).

Sec. 3.4: pixels are grouped in 2 x 2 blocks; nearer the gaze more positions
of each block are rendered (Fig. 8: top-left first), the others inherit or
interpolate from the rendered ones; Sec. 3.5 labels each tile with a level
1..4 by eccentricity, and the framework (Sec. 3.6, Sec. 4.6) also sets a
tile's resolution by the number of Gaussians intersecting it, tiles sorted by
that number.  Readings used here:
  * positions in the order top-left, top-right, bottom-left, bottom-right; a
    tile of level L renders the first L;
  * eccentricity levels: 4, 3, 2 within r4 <= r3 <= r2 of the gaze (distance
    to the tile's pixel-centre rectangle, the disc-mask test), 1 beyond;
  * count levels: the view's tiles sorted by their number of Gaussians (key
    count of the tile, ties to the lower tile index first); the first
    ceil(f4 T) of the T tiles level 4, the first ceil(f3 T) at least 3, the
    first ceil(f2 T) at least 2, the rest 1 (f4 <= f3 <= f2): few Gaussians, a
    smooth tile, fewer samples;
  * combined: the smaller of the two levels;
  * inheritance: an unrendered position takes the rendered pixel above it,
    else the top-left one;
  * interpolation: an unrendered position takes the bilinear interpolation of
    the blocks' top-left samples (rendered at every level) at its own position
    on that half-resolution grid, clamped at the last block: the mean of two
    (odd x or odd y) or four (both) top-left samples, in float32 as
    0.5 (a + b) and 0.25 ((a + b) + (c + d));
  * rendered positions are the plain full-resolution render's pixels.
"""
from __future__ import annotations

import math

import numpy as np

from . import core


def tile_levels(cam, gaze, radii):
    """Eccentricity level per tile [tiles_y * tiles_x]: 1 + membership in the nested discs."""
    lv = np.ones(((cam.height + core.TILE - 1) // core.TILE) * ((cam.width + core.TILE - 1) // core.TILE), np.int32)
    for r in radii:
        v = core.full_view(cam)
        v.mask, v.gx, v.gy, v.r_out = 1, float(gaze[0]), float(gaze[1]), float(r)
        act, _ = core.tile_masks([v])
        lv += act.astype(np.int32)
    return lv


def count_levels(tile_counts, fracs):
    """Count level per tile from its number of Gaussians (tile_counts, one view):
    rank the tiles by (count descending, tile index ascending); the first
    ceil(f T) of them reach the level of fraction f, fracs = (f4, f3, f2)."""
    c = np.asarray(tile_counts, np.int64)
    T = c.size
    order = np.lexsort((np.arange(T), -c))  # count descending, then index ascending
    rank = np.empty(T, np.int64)
    rank[order] = np.arange(T)
    lv = np.ones(T, np.int32)
    for f in fracs:
        lv += (rank < math.ceil(f * T)).astype(np.int32)
    return lv


def combine_levels(ecc, cnt, mode):
    """mode 0: eccentricity, 1: count, 2: the smaller of the two."""
    return {0: ecc, 1: cnt, 2: np.minimum(ecc, cnt)}[mode].astype(np.int32)


def source_position(k, level):
    """Block position (0 top-left, 1 top-right, 2 bottom-left, 3 bottom-right)
    whose rendered pixel position k shows at this level."""
    if k < level:
        return k
    if 0 <= k - 2 < level:
        return k - 2
    return 0


def amr_image(full_rgb, levels, W, H, fill="inherit"):
    """The AMR image from the full-resolution render [C][H][W] (C = 3, or one
    plane such as a mask) and the tile levels."""
    ys, xs = np.mgrid[0:H, 0:W]
    tiles_x = (W + core.TILE - 1) // core.TILE
    lv = levels[(ys // core.TILE) * tiles_x + xs // core.TILE]
    k = (xs & 1) + 2 * (ys & 1)
    if fill == "inherit":
        table = np.array([[source_position(kk, L) for kk in range(4)] for L in range(5)])
        src = table[lv, k]
        sx = (xs & ~1) + (src & 1)
        sy = (ys & ~1) + (src >> 1)
        return full_rgb[:, sy, sx]
    # interpolation of the top-left samples (even pixels), in the image's dtype
    out = full_rgb.copy()
    miss = k >= lv
    bx, by = xs >> 1, ys >> 1
    BX, BY = (W + 1) // 2, (H + 1) // 2
    x0, y0 = 2 * bx, 2 * by
    x1, y1 = 2 * np.minimum(bx + 1, BX - 1), 2 * np.minimum(by + 1, BY - 1)
    f = full_rgb
    dt = f.dtype.type
    half, quarter = dt(0.5), dt(0.25)
    for ch in range(f.shape[0]):
        a, b = f[ch, y0, x0], f[ch, y0, x1]
        c, d = f[ch, y1, x0], f[ch, y1, x1]
        v = np.where((xs & 1) & (ys & 1), quarter * ((a + b) + (c + d)),
                     np.where(xs & 1, half * (a + b), np.where(ys & 1, half * (a + c), a)))
        out[ch][miss] = v[miss]
    return out


def render_amr(scene, cams, gazes, radii, nthreads=None, mode=0, fracs=(0.25, 0.5, 0.75), fill="inherit"):
    full = core.render_full(scene, cams, nthreads=nthreads)
    outs, levels = [], []
    for e, cam in enumerate(cams):
        ecc = tile_levels(cam, gazes[e], radii)
        T = ecc.size
        rg = full["ranges"][int(full["tile_off"][e]): int(full["tile_off"][e]) + T]
        cnt = count_levels(rg[:, 1] - rg[:, 0], fracs)
        lv = combine_levels(ecc, cnt, mode)
        levels.append(lv)
        outs.append(amr_image(full["out"][e], lv, cam.width, cam.height, fill))
    full["amr"] = np.stack(outs)
    full["levels"] = levels
    return full
