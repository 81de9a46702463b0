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


def disc_tiles(cam, gaze, radius, tw=core.TILE, th=core.TILE):
    """Active flags [tiles_y * tiles_x] of a full-resolution disc mask of the
    given radius around gaze (the fovea layer's tile test); radius <= 0: none."""
    if radius <= 0.0:
        tx, ty = (cam.width + tw - 1) // tw, (cam.height + th - 1) // th
        return np.zeros(tx * ty, np.uint8)
    v = core.full_view(cam)
    v.mask, v.gx, v.gy, v.r_out = 1, float(gaze[0]), float(gaze[1]), float(radius)
    act, _ = core.tile_masks([v], tw, th)
    return act


def round_tiles(cam, rounds, final_gaze, r_f):
    """New fovea tiles of each round for one eye: rounds = [(gaze, radius)];
    the final round is (final_gaze, r_f).  Returns the list of new-tile flag
    arrays (rounds then final) and the union."""
    done = None
    out = []
    for g, r in list(rounds) + [(final_gaze, r_f)]:
        a = disc_tiles(cam, g, r)
        if done is None:
            done = np.zeros_like(a)
        new = (a != 0) & (done == 0)
        done = done | new
        out.append(new.astype(np.uint8))
    return out, done


def keys_for_tiles(rect, vis, tiles, tiles_x, tiles_y):
    """Keys the visible Gaussians emit into the flagged tiles: for each, the
    flagged tiles inside its rectangle (x0, x1, y0, y1), summed (2D prefix)."""
    m = tiles.reshape(tiles_y, tiles_x).astype(np.int64)
    P = np.zeros((tiles_y + 1, tiles_x + 1), np.int64)
    P[1:, 1:] = m.cumsum(0).cumsum(1)
    r = rect[vis.astype(bool)].astype(np.int64)
    x0, x1, y0, y1 = r[:, 0], r[:, 1], r[:, 2], r[:, 3]
    return int((P[y1 + 1, x1 + 1] - P[y0, x1 + 1] - P[y1 + 1, x0] + P[y0, x0]).sum())
