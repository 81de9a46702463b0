"""Oracle of the incremental foveal rendering (TEST INFRASTRUCTURE ONLY: used by
tests/ and the benchmark's checks, never by the library).

Sec. 3.3: prediction u_i of gaze-network exit i starts rendering before the
final prediction u_N.  Round i renders the fovea region C_i of radius

    r_i = max(0, r_f - E[dist(u_i, u_N)])     (Eq. 4; Eq. 3 with the distance known)

around u_i, only where earlier rounds did not render; with no newer
prediction, rendering continues around u_j up to r_f + E[dist(u_j, u_N)]
(Eq. 5).  The final round renders what C_N (radius r_f around u_N) still
lacks, and the frame is composited around u_N -- so the result is the plain
foveated frame for gaze u_N, which `oracle.render_foveated` defines.

Here: the expected distance for independent normal offsets (through the
complete elliptic integral of the second kind), the radii of Eq. 4 and 5, the
tile sets of each round (the same tile test as the fovea layer's disc mask),
and the key count a round's tiles receive from the projected rectangles.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import ellipe

from . import core


def expected_distance(sx, sy):
    """E[sqrt(X^2 + Y^2)], X ~ N(0, sx^2), Y ~ N(0, sy^2) independent: with
    a = max(sx, sy), b = min, the polar form gives sqrt(pi/2) times the mean
    radius of the ellipse with semi-axes (a, b), i.e. sqrt(2/pi) a E(1 - b^2/a^2)
    with E the complete elliptic integral of the second kind (parameter m)."""
    a, b = max(abs(sx), abs(sy)), min(abs(sx), abs(sy))
    if a == 0.0:
        return 0.0
    return math.sqrt(2.0 / math.pi) * a * float(ellipe(1.0 - (b / a) ** 2))


def round_radius(r_f, e):
    """Eq. 4."""
    return max(0.0, r_f - e)


def speculative_radius(r_f, e):
    """Eq. 5."""
    return r_f + e


def _empty(v):
    tx, ty = (v.width + core.TILE - 1) // core.TILE, (v.height + core.TILE - 1) // core.TILE
    return np.zeros(tx * ty, np.uint8)


def disc_tiles(cam, gaze, radius, scale=1):
    """Active flags [tiles_y * tiles_x] of the disc mask of the given radius
    (in this layer's pixels) around gaze (full-resolution pixels) on the layer
    of the given scale; radius <= 0: none."""
    v = core.foveated_views([cam], [gaze], (1.0, 2.0), scales=(scale, scale, scale))[0]
    if radius <= 0.0:
        return _empty(v)
    v.mask, v.r_in, v.r_out = 1, 0.0, float(radius)
    act, _ = core.tile_masks([v])
    return act


def layer_rounds(masks):
    """New tiles of each round of one layer, given each round's tile mask (the
    last one the final round's): a tile is new where its round's mask has it
    and no earlier round rendered it.  Returns the list and the union."""
    done = np.zeros_like(masks[0])
    out = []
    for a in masks:
        new = ((a != 0) & (done == 0)).astype(np.uint8)
        done = done | new
        out.append(new)
    return out, done


def round_tiles(cam, rounds, final_gaze, r_f):
    """Fovea layer: rounds = [(gaze, radius)] then (final_gaze, r_f)."""
    return layer_rounds([disc_tiles(cam, g, r) for g, r in rounds] + [disc_tiles(cam, final_gaze, r_f)])


def mid_round_tiles(cam, rounds, final_gaze, radius_px, scale=2, margin=core.MID_MARGIN):
    """Mid layer: a round with fovea radius r renders the disc of radius
    r + (r_m - r_f) (full-resolution pixels; Eq. 4 and 5 offset the mid
    layer's outer radius by the same expected distance) plus the bilinear
    margin, in its own pixels; the final round its annulus around the final gaze."""
    rf, rm = radius_px
    masks = []
    for g, r in rounds:
        rr = r + (rm - rf)
        masks.append(disc_tiles(cam, g, rr / scale + margin, scale) if rr > 0.0 else
                     disc_tiles(cam, g, -1.0, scale))
    fin = core.foveated_views([cam], [final_gaze], radius_px)[1]
    act, _ = core.tile_masks([fin])
    masks.append(act)
    return layer_rounds(masks)


def keys_for_tiles(rect, vis, tiles, tiles_x, tiles_y):
    """Keys the visible Gaussians emit into the flagged tiles: for each, the
    flagged tiles inside its rectangle (x0, x1, y0, y1), summed (2D prefix)."""
    m = tiles.reshape(tiles_y, tiles_x).astype(np.int64)
    P = np.zeros((tiles_y + 1, tiles_x + 1), np.int64)
    P[1:, 1:] = m.cumsum(0).cumsum(1)
    r = rect[vis.astype(bool)].astype(np.int64)
    x0, x1, y0, y1 = r[:, 0], r[:, 1], r[:, 2], r[:, 3]
    return int((P[y1 + 1, x1 + 1] - P[y0, x1 + 1] - P[y1 + 1, x0] + P[y0, x0]).sum())
