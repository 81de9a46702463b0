"""Concurrent gaze tracking and incremental rendering (Algorithm 1).

Two activities share one variable S = (exit index, gaze): the gaze tracker
runs its network layer by layer on the CPU and publishes each exit's
prediction; the renderer, on the GPU, renders round 0 (projection and
periphery) at once, then whenever it is free takes the newest prediction in S
and renders the next round of the foveal region (Eq. 4), continuing around the
same prediction up to r_f + E (Eq. 5) when nothing newer has arrived, and
finishes the frame when the last exit's prediction is there.  Total latency
T_s + T_c + max(T_d, T_r) against T_s + T_c + T_d + T_r for the sequential
pipeline (Sec. 3.1).

The tracker is a stand-in: it publishes the predictions of a synthetic
early-exit stream at given times (the per-exit CPU latencies of the network,
scaled by a load factor), so the rendering side -- the part on this GPU -- is
what is measured.  Host threads; the library calls release the interpreter
lock while they run.
"""
from __future__ import annotations

import sys
import threading
import time

from . import incremental as inc


class Shared:
    """S of Algorithm 1: the newest (exit index, gazes), with a condition to wait on."""

    def __init__(self):
        self.cv = threading.Condition()
        self.layer = 0
        self.gaze = None
        self.stamp = {}

    def publish(self, layer, gaze, t):
        with self.cv:
            self.layer, self.gaze = layer, gaze
            self.stamp[layer] = t
            self.cv.notify_all()

    def newest(self):
        with self.cv:
            return self.layer, self.gaze

    def wait_newer(self, layer):
        with self.cv:
            while self.layer <= layer:
                self.cv.wait()
            return self.layer, self.gaze


def run(ctx, scene, cams, fovea, exits, final, sigmas_px, exit_times_ms, sync, load=1.0, out=None,
        speculative=True, network=None, eye_image=None):
    """One frame of Algorithm 1.

    exits: predictions of exits 1..N-1 (gazes per eye); final: exit N's;
    exit_times_ms: cumulative tracker latency of exits 1..N (ms); load scales
    them (a busier CPU); sync(): waits for the GPU.  With network (an
    early-exit model with exits_iter, see gaze_vit) and eye_image, the tracker
    runs that network on the CPU instead and publishes exit l's prediction of
    the synthetic stream when its layer l is done (the timing is the
    network's, the gazes the stream's).  Returns the timeline (ms from the
    start) and the rendering-complete time."""
    n = len(exit_times_ms)
    assert len(exits) == n - 1 and len(sigmas_px) == n - 1
    S = Shared()
    t0 = time.perf_counter()
    now = lambda: (time.perf_counter() - t0) * 1000.0

    errors = []

    def tracker():
        try:
            if network is not None:
                for l, _ in network.exits_iter(eye_image):
                    S.publish(l, exits[l - 1] if l < n else final, now())
                return
            for l in range(1, n + 1):
                target = exit_times_ms[l - 1] * load
                while True:
                    left = target - now()
                    if left <= 0.0:
                        break
                    time.sleep(min(left, 0.5) / 1000.0)
                S.publish(l, exits[l - 1] if l < n else final, now())
        except BaseException as e:  # the renderer must not wait for an exit that never comes
            errors.append(e)
        finally:
            if S.newest()[0] < n:
                S.publish(n, final, now())

    events = []
    old = sys.getswitchinterval()
    sys.setswitchinterval(1e-5)
    th = threading.Thread(target=tracker, daemon=True)
    th.start()
    try:
        t = now()
        ctx.incremental_begin(scene, cams, fovea)
        sync()
        events.append(("round 0", 0, t, now()))
        layer = 0
        while True:
            l, g = S.newest()
            if l == layer:
                l, g = S.wait_newer(layer)
            layer = l
            if l == n:
                t = now()
                ctx.incremental_finish(g, out)
                sync()
                events.append(("finish", l, t, now()))
                break
            e = inc.expected_distance(*sigmas_px[l - 1])
            t = now()
            ctx.incremental_round(g, inc.round_radius(fovea.r_fovea, e))
            sync()
            events.append(("exit", l, t, now()))
            if speculative and S.newest()[0] == layer:
                t = now()
                ctx.incremental_round(g, inc.speculative_radius(fovea.r_fovea, e))
                sync()
                events.append(("speculative", l, t, now()))
    finally:
        th.join()
        sys.setswitchinterval(old)
    if errors:
        raise errors[0]
    return dict(events=events, exit_ms=[S.stamp[l] for l in range(1, n + 1)], render_done_ms=events[-1][3])
