"""Host logic of Algorithm 1 (CPU only): the render loop's control flow with a
recording stand-in for the library context, and the CPU load generator."""
import time

import pytest

from paper_2507_04147_amd import pipeline


class FakeCtx:
    """Records the library calls of the render loop; each call takes ms_per_call."""

    def __init__(self, ms_per_call=0.2):
        self.calls, self.ms = [], ms_per_call

    def _t(self):
        time.sleep(self.ms / 1000.0)

    def incremental_begin(self, scene, cams, fovea):
        self.calls.append(("begin",))
        self._t()

    def incremental_round(self, gaze, radius):
        self.calls.append(("round", gaze, radius))
        self._t()

    def incremental_finish(self, gaze, out):
        self.calls.append(("finish", gaze))
        self._t()

    def sync(self):
        pass


class Fovea:
    r_fovea = 100.0


def _stream(n=6):
    exits = [[(float(l), 0.0)] for l in range(1, n)]
    return exits, [(10.0 / l, 10.0 / l) for l in range(1, n)], [(99.0, 0.0)]


@pytest.mark.parametrize("speculative", [True, False])
def test_render_loop_follows_the_exits(speculative):
    exits, sig, final = _stream()
    # exits 30 ms apart: far slower than a call, and than a scheduling hiccup of the test process
    times = [30.0, 60.0, 90.0, 120.0, 150.0, 180.0]
    ctx = FakeCtx()
    r = pipeline.run(ctx, None, None, Fovea(), exits, final, sig, times, speculative=speculative)
    kinds = [e[0] for e in r["events"]]
    assert kinds[0] == "round 0" and kinds[-1] == "finish"
    assert ctx.calls[0] == ("begin",) and ctx.calls[-1] == ("finish", final)
    layers = [e[1] for e in r["events"][1:]]
    assert layers == sorted(layers)
    # every exit's prediction is rendered (the stand-in publishes far slower than a call)
    assert [e[1] for e in r["events"] if e[0] == "exit"] == [1, 2, 3, 4, 5]
    # speculative rounds grow around the same prediction (Eq. 5 radius >= Eq. 4 radius)
    spec = [e for e in r["events"] if e[0] == "speculative"]
    assert bool(spec) == speculative
    rounds = [c for c in ctx.calls if c[0] == "round"]
    for a, b in zip(rounds, rounds[1:]):
        if a[1] == b[1]:
            assert b[2] >= a[2]
    assert r["events"][-1][2] >= r["exit_ms"][-1] - 1e-6


def test_cpu_load_processes_start_and_stop():
    with pipeline.CpuLoad(2, period_s=0.05, max_s=30.0) as load:
        assert len(load.procs) == 2 and all(p.poll() is None for p in load.procs)
        procs = list(load.procs)
    assert all(p.poll() is not None for p in procs)


@pytest.mark.parametrize("speculative", [True, False])
def test_render_loop_with_the_tracker_in_its_own_process(speculative):
    """Algorithm 1's two processes: the early-exit ViT in a child process sends
    its six exits in order; the render loop (recording stand-in context) takes
    them from the pipe, renders a round per exit it sees and finishes on the
    last, after it is out."""
    exits, sig, final = _stream()
    tr = pipeline.TrackerProcess(prune=0.0, seed=5, threads=2)
    try:
        t = time.perf_counter()
        alone = tr.run_alone(6)
        assert alone == sorted(alone) and alone[0] > t
        ctx = FakeCtx(ms_per_call=0.1)
        r = pipeline.run_process(ctx, None, None, Fovea(), exits, final, sig, tr, speculative=speculative)
    finally:
        tr.close()
    assert tr.proc.returncode == 0
    kinds = [e[0] for e in r["events"]]
    assert kinds[0] == "round 0" and kinds[-1] == "finish"
    assert ctx.calls[-1] == ("finish", final)
    layers = [e[1] for e in r["events"][1:]]
    assert layers == sorted(layers) and layers[-1] == 6
    assert r["exit_ms"] == sorted(r["exit_ms"]) and r["events"][-1][2] >= r["exit_ms"][-1] - 1e-6
    assert bool([e for e in r["events"] if e[0] == "speculative"]) <= speculative
