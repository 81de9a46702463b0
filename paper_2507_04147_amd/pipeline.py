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

The tracker either runs the early-exit network on the CPU (gaze_vit; the
predictions published are those of a synthetic early-exit stream, the timing
is the network's) or is a stand-in that publishes the stream at given times.
Host threads; the library calls release the interpreter lock while they run,
and the renderer's waits sleep (a3fr_set_host_wait) so that the tracker keeps
the CPU.  CpuLoad reproduces the paper's load experiment (Sec. 4.5): other
processes take the CPU, their utilisation alternating between 50% and 100%
every 0.1 s.
"""
from __future__ import annotations

import os
import subprocess
import sys
import threading
import time

from . import incremental as inc

# One load process: alternates its duty between 100% and 50% every period
# seconds, in slices of 2 ms (busy for duty x slice, then asleep); it exits when
# its parent is gone or after max_s seconds.
_LOAD_CODE = r"""
import os, sys, time
ppid, period, max_s = int(sys.argv[1]), float(sys.argv[2]), float(sys.argv[3])
sl = 0.002
t0 = time.perf_counter()
while True:
    now = time.perf_counter() - t0
    if now > max_s or os.getppid() != ppid:
        break
    duty = 1.0 if int(now / period) % 2 == 0 else 0.5
    end = time.perf_counter() + duty * sl
    while time.perf_counter() < end:
        pass
    if duty < 1.0:
        time.sleep((1.0 - duty) * sl)
"""


class CpuLoad:
    """Context manager: n_procs child processes loading the host CPU, each
    alternating 100% and 50% utilisation every period seconds."""

    def __init__(self, n_procs, period_s=0.1, max_s=600.0):
        self.n, self.period, self.max_s = int(n_procs), float(period_s), float(max_s)
        self.procs = []

    def __enter__(self):
        for _ in range(self.n):
            self.procs.append(subprocess.Popen([sys.executable, "-c", _LOAD_CODE, str(os.getpid()), str(self.period),
                                                str(self.max_s)]))
        time.sleep(0.05)
        return self

    def __exit__(self, *exc):
        for p in self.procs:
            p.terminate()
        for p in self.procs:
            try:
                p.wait(timeout=5)
            except subprocess.TimeoutExpired:
                p.kill()
                p.wait()
        self.procs = []
        return False


def tracker_main(argv=None):
    """Body of the tracker process (python -m paper_2507_04147_amd.pipeline
    PRUNE SEED THREADS IMAGE_SEED): the early-exit ViT on THREADS CPU threads.
    It prints "ready THREADS", then on each "go" line runs the network on the
    eye image and prints "EXIT TIME" (time.perf_counter()) as each block
    finishes; "stop" or the end of its input ends it."""
    import torch

    from . import gaze_vit as gv
    prune, seed, threads, image_seed = argv if argv is not None else sys.argv[1:5]
    torch.set_num_threads(int(threads))
    net = gv.EarlyExitViT(prune=float(prune), seed=int(seed))
    img = torch.rand(1, 1, 400, 640, generator=torch.Generator().manual_seed(int(image_seed)))
    for _ in net.exits_iter(img):  # warm-up
        pass
    out = sys.stdout
    out.write(f"ready {torch.get_num_threads()}\n")
    out.flush()
    for line in sys.stdin:
        if line.strip() != "go":
            break
        for l, _ in net.exits_iter(img):
            out.write(f"{l} {time.perf_counter()!r}\n")
            out.flush()


class TrackerProcess:
    """Algorithm 1's first process: the gaze tracker (the early-exit ViT) in a
    process of its own on the CPU, so that it shares neither the interpreter
    nor its lock with the renderer.  start() sets it going on one eye image;
    the renderer takes its exits through newest() / wait_newer(), which read the
    child's pipe (wait_newer sleeps in poll() until a line comes).  Times are
    time.perf_counter() (CLOCK_MONOTONIC, shared by the two processes)."""

    def __init__(self, prune=0.0, seed=5, threads=8, image_seed=5):
        import select
        self.proc = subprocess.Popen([sys.executable, "-m", "paper_2507_04147_amd.pipeline", str(float(prune)),
                                      str(int(seed)), str(int(threads)), str(int(image_seed))],
                                     stdin=subprocess.PIPE, stdout=subprocess.PIPE, bufsize=0,
                                     cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
        self.fd = self.proc.stdout.fileno()
        self.poller = select.poll()
        self.poller.register(self.fd, select.POLLIN)
        self.buf = b""
        tag, th = self._line(block=True).split()
        assert tag == "ready"
        self.threads = int(th)
        self.n, self.latest, self.stamp = 0, 0, {}

    def _line(self, block):
        while b"\n" not in self.buf:
            if not self.poller.poll(None if block else 0):
                return None
            chunk = os.read(self.fd, 4096)
            if not chunk:
                raise RuntimeError("the tracker process ended")
            self.buf += chunk
        line, self.buf = self.buf.split(b"\n", 1)
        return line.decode()

    def start(self, n_exits):
        self.n, self.latest, self.stamp = n_exits, 0, {}
        self.proc.stdin.write(b"go\n")
        self.proc.stdin.flush()

    def _take(self, line):
        l, t = line.split()
        self.latest = max(self.latest, int(l))
        self.stamp[int(l)] = float(t)

    def newest(self):
        while True:
            line = self._line(block=False)
            if line is None:
                return self.latest
            self._take(line)

    def wait_newer(self, layer):
        while self.newest() <= layer:
            self._take(self._line(block=True))
        return self.latest

    def run_alone(self, n_exits):
        """Exit times (perf_counter) of one run with the renderer idle."""
        self.start(n_exits)
        self.wait_newer(n_exits - 1)
        return [self.stamp[l] for l in range(1, n_exits + 1)]

    def close(self):
        if self.proc.poll() is None:
            try:
                self.proc.stdin.write(b"stop\n")
                self.proc.stdin.close()
            except OSError:
                pass
            try:
                self.proc.wait(timeout=10)
            except subprocess.TimeoutExpired:
                self.proc.terminate()
                self.proc.wait()


def run_process(ctx, scene, cams, fovea, exits, final, sigmas_px, tracker: TrackerProcess, sync=None, out=None,
                speculative=True):
    """One frame of Algorithm 1 with the tracker in its own process: it is set
    going, round 0 is rendered at once, then each round takes the newest exit
    (its prediction from the synthetic stream: exits[l - 1], final for the
    last), with speculative growth to r_f + E when nothing newer has come
    (speculative=False: wait for it), and the finish on the last exit.
    Returns the timeline (ms from the start) like run()."""
    if sync is None:
        sync = ctx.sync
    n = len(exits) + 1
    assert len(sigmas_px) == n - 1
    t0 = time.perf_counter()
    now = lambda: (time.perf_counter() - t0) * 1000.0
    tracker.start(n)
    events = []
    t = now()
    ctx.incremental_begin(scene, cams, fovea)
    sync()
    events.append(("round 0", 0, t, now()))
    layer = 0
    while True:
        l = tracker.newest()
        if l == layer:
            l = tracker.wait_newer(layer)
        layer = l
        g = exits[l - 1] if l < n else final
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
        if speculative and tracker.newest() == layer:
            t = now()
            ctx.incremental_round(g, inc.speculative_radius(fovea.r_fovea, e))
            sync()
            events.append(("speculative", l, t, now()))
    exit_ms = [(tracker.stamp[l] - t0) * 1000.0 for l in range(1, n + 1)]
    return dict(events=events, exit_ms=exit_ms, render_done_ms=events[-1][3])


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


def run(ctx, scene, cams, fovea, exits, final, sigmas_px, exit_times_ms, sync=None, load=1.0, out=None,
        speculative=True, network=None, eye_image=None):
    """One frame of Algorithm 1.

    exits: predictions of exits 1..N-1 (gazes per eye); final: exit N's;
    exit_times_ms: cumulative latency of exits 1..N (ms) of the stand-in
    tracker, scaled by load (the tests use it to vary which rounds run);
    sync(): waits for the GPU (default: the context's own wait, which sleeps
    after ctx.set_host_wait(True)).  With network (an early-exit model with
    exits_iter, see gaze_vit) and eye_image, the tracker runs that network on
    the CPU instead and publishes exit l's prediction of the synthetic stream
    when its layer l is done (the timing is the network's, the gazes the
    stream's).  speculative=False is the paper's baseline without speculative
    rounds: after a round the renderer waits for the next prediction.  Returns
    the timeline (ms from the start) and the rendering-complete time."""
    if sync is None:
        sync = ctx.sync
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
    if errors:
        raise errors[0]
    return dict(events=events, exit_ms=[S.stamp[l] for l in range(1, n + 1)], render_done_ms=events[-1][3])


if __name__ == "__main__":
    tracker_main()
