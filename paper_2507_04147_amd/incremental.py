"""Round schedule of the incremental foveal rendering (Sec. 3.3).

The gaze network yields predictions u_1 .. u_N of increasing accuracy; the
renderer starts on the fovea before u_N is known.  With E_i the expected
distance between u_i and the final prediction u_N (profiled offline,
Sec. 3.3.2), round i renders the fovea tiles within

    r_i = max(0, r_f - E_i)                                   (Eq. 4)

of u_i that earlier rounds did not render; a disc of that radius lies inside
the final fovea whenever the prediction is no farther from u_N than expected
(the containment of Eq. 3).  When the renderer is done before the next
prediction arrives it keeps growing the region around the same prediction, up
to (speculative incremental rendering)

    r_max_j = r_f + E_j                                        (Eq. 5)

which covers the final fovea under the same condition.  The last round uses
u_N and r_f, and the frame is composited around u_N
(`Context.incremental_finish`).

Prediction errors are taken as independent normal offsets of u_i from u_N
per axis, with standard deviations (s_x, s_y) in pixels; E_i is then the mean
length of such an offset.  This module is host logic only: the rendering is
the library's.
"""
from __future__ import annotations

import math

import numpy as np


def degrees_to_pixels(deg, focal_px):
    """An angular error at the image centre in pixels: f tan(theta) (Eq. 1 with
    the gaze in front, rho d = the focal length in pixels)."""
    return focal_px * math.tan(math.radians(deg))


def expected_distance(sx, sy, samples=8192):
    """E[sqrt(X^2 + Y^2)] for independent X ~ N(0, sx^2), Y ~ N(0, sy^2).

    In polar form (X, Y) = R (sx cos t, sy sin t) with R the radius of a
    standard 2D normal (mean sqrt(pi/2)) and t uniform and independent, so
    E = sqrt(pi/2) * mean over t of sqrt(sx^2 cos^2 t + sy^2 sin^2 t); the
    mean of this smooth periodic function is taken with the trapezoid rule on
    `samples` equally spaced angles (exact to rounding up to axis ratios of
    about 50)."""
    sx, sy = abs(float(sx)), abs(float(sy))
    t = (np.arange(samples) + 0.5) * (2.0 * math.pi / samples)
    ring = np.sqrt((sx * np.cos(t)) ** 2 + (sy * np.sin(t)) ** 2)
    return math.sqrt(math.pi / 2.0) * float(ring.mean())


def round_radius(r_f, e_dist):
    """Eq. 4: the largest fovea radius around u_i that stays inside the final
    fovea when u_i lies at the expected distance from u_N."""
    return max(0.0, r_f - e_dist)


def speculative_radius(r_f, e_dist):
    """Eq. 5: the radius up to which rendering continues around u_j when no
    newer prediction has arrived."""
    return r_f + e_dist


def schedule(exits, sigmas_px, r_f, speculative=True):
    """Rounds for one frame.

    exits: per exit i = 1..N-1 the predicted gazes (one (x, y) per eye);
    sigmas_px: per exit the (s_x, s_y) spread around the final prediction.
    Returns [(gazes, radius, kind)] with kind "exit" (Eq. 4) or "speculative"
    (Eq. 5), in order; the final round (u_N, r_f) is the caller's
    `incremental_finish`.  With speculative rendering every exit round is
    followed by its growth to r_max (the renderer finishes a round long
    before the next prediction: a few tens of microseconds against
    milliseconds per network layer)."""
    out = []
    for gz, (sx, sy) in zip(exits, sigmas_px):
        e = expected_distance(sx, sy)
        out.append((gz, round_radius(r_f, e), "exit"))
        if speculative:
            out.append((gz, speculative_radius(r_f, e), "speculative"))
    return out


def run_frame(ctx, scene, cams, fovea, rounds, final_gazes, out, timed=None):
    """Begin, the scheduled rounds, finish.  Returns per-step dicts with the
    tiles and keys of each step (and milliseconds when `timed(fn)` is given,
    a function that runs fn and returns its duration)."""
    steps = []

    def go(name, fn, radius=None):
        ms = timed(fn) if timed else (fn() or None)
        cnt = ctx.get_counts()
        steps.append(dict(step=name, radius=radius, tiles=cnt["n_active_tiles"], keys=cnt["n_keys"], ms=ms))

    go("begin", lambda: ctx.incremental_begin(scene, cams, fovea))
    for gz, r, kind in rounds:
        go(kind, (lambda g=gz, rr=r: ctx.incremental_round(g, rr)), r)
    go("finish", lambda: ctx.incremental_finish(final_gazes, out), fovea.r_fovea)
    return steps
