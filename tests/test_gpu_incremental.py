"""GPU parity of the incremental foveal rounds (MI355X only).

The frame built by a3fr_incremental_begin / _round / _finish must equal the
one-shot a3fr_render_foveated with the final gaze bit for bit (every tile is
blended from the same list whichever round renders it), and the oracle's
foveated frame within the composite tolerances.  Each round's rendered tiles
and emitted keys must equal the oracle's: the round's new tiles (Eq. 4 / Eq. 5
discs minus earlier rounds, same tile test as the fovea disc mask) and the
keys the projected rectangles give them.
"""
import numpy as np
import pytest

import oracle
import oracle.incremental as oi
import synth
from test_gpu_parity import COLOUR_TOL, assert_amb_within, composite_ambiguity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    import paper_2507_04147_amd as p
    p.lib()
    assert torch.cuda.is_available()
    return p


def _setup(n, W, H, seed, n_trials):
    scene, cams = synth.foveated_stereo(n=n, width=W, height=H, seed=seed)
    trials, sig = synth.gaze_exits(seed=seed + 60, n_trials=n_trials, width=W, height=H)
    rad = (0.15 * W, 0.35 * W)
    return scene, cams, trials, sig, rad


def _oracle_rounds(scene, cams, final, rounds, rad):
    """Per round (then the finish): new fovea and mid tiles and their keys over
    both eyes."""
    views = oracle.foveated_views(cams, final, rad)
    pr = oracle.project(scene, views)
    out = [[0, 0] for _ in range(len(rounds) + 1)]
    for e, cam in enumerate(cams):
        per_eye = [(g[e], r) for g, r, _ in rounds]
        for lvl, (news, _) in enumerate((oi.round_tiles(cam, per_eye, final[e], rad[0]),
                                         oi.mid_round_tiles(cam, per_eye, final[e], rad))):
            v = views[3 * e + lvl]
            tx, ty = (v.width + 15) // 16, (v.height + 15) // 16
            for k, nw in enumerate(news):
                out[k][0] += int(nw.sum())
                out[k][1] += oi.keys_for_tiles(pr["rect"][3 * e + lvl], pr["vis"][3 * e + lvl], nw, tx, ty)
    return out


def _run(pkg, ctx, ds, cams, fov, rounds, final, out):
    from paper_2507_04147_amd import incremental as inc
    steps = inc.run_frame(ctx, ds, cams, fov, rounds, final, out)
    ctx.sync()
    return steps


@pytest.mark.parametrize("speculative", [True, False])
def test_incremental_equals_one_shot_and_oracle(pkg, speculative):
    from paper_2507_04147_amd import incremental as inc
    W, H = 464, 480
    scene, cams, trials, sig, rad = _setup(100_000, W, H, 3, 2)
    ds = pkg.DeviceScene.from_host(scene)
    fov = pkg.fovea_struct(*rad)
    ctx = pkg.Context()
    for final, exits in trials:
        rounds = inc.schedule(exits, sig, rad[0], speculative=speculative)
        out = torch.full((2, 3, H, W), float("nan"), device="cuda")
        steps = _run(pkg, ctx, ds, cams, fov, rounds, final, out)
        ref = torch.zeros_like(out)
        ctx.render_foveated(ds, cams, final, fov, ref)
        ctx.sync()
        assert torch.equal(out, ref)
        want = _oracle_rounds(scene, cams, final, rounds, rad)
        got = [[s["tiles"], s["keys"]] for s in steps[1:]]
        print("rounds (tiles, keys):", got, flush=True)
        assert got == want
    # the last frame against the oracle's foveated frame
    o = oracle.render_foveated(scene, cams, final, rad)
    img = out.cpu().numpy()
    for e in range(2):
        err = np.abs(img[e] - o["out"][e])
        amb, tol = composite_ambiguity(W, H, final[e], rad, o["images"][3 * e: 3 * e + 3])
        assert err.max(axis=0)[~amb].max() <= COLOUR_TOL
        assert_amb_within(err, amb, tol)
    ctx.close()


def test_incremental_full_size(pkg):
    """The 1M-Gaussian stereo frame at 2 x 1832 x 1920 (the benchmark's
    launches): one trial of the early-exit stream with speculative rounds."""
    from paper_2507_04147_amd import incremental as inc
    scene, cams, trials, sig, rad = _setup(1_000_000, 1832, 1920, 2, 1)
    ds = pkg.DeviceScene.from_host(scene)
    fov = pkg.fovea_struct(*rad)
    ctx = pkg.Context()
    final, exits = trials[0]
    rounds = inc.schedule(exits, sig, rad[0])
    out = torch.empty((2, 3, 1920, 1832), device="cuda")
    steps = _run(pkg, ctx, ds, cams, fov, rounds, final, out)
    ref = torch.empty_like(out)
    ctx.render_foveated(ds, cams, final, fov, ref)
    ctx.sync()
    assert torch.equal(out, ref)
    got = [[s["tiles"], s["keys"]] for s in steps[1:]]
    assert got == _oracle_rounds(scene, cams, final, rounds, rad)
    ctx.close()


def test_incremental_call_order_and_args(pkg):
    W, H = 128, 96
    scene, cams, trials, sig, rad = _setup(2_000, W, H, 4, 1)
    ds = pkg.DeviceScene.from_host(scene)
    fov = pkg.fovea_struct(*rad)
    ctx = pkg.Context()
    final, exits = trials[0]
    out = torch.zeros((2, 3, H, W), device="cuda")
    ctx._inc_eyes = 2
    with pytest.raises(pkg.A3FRError) as e:
        ctx.incremental_round(final, 10.0)
    assert e.value.status == pkg.A3FR_ENOTREADY
    ctx.incremental_begin(ds, cams, fov)
    with pytest.raises(pkg.A3FRError) as e:
        ctx.incremental_round(final, -1.0)
    assert e.value.status == pkg.A3FR_EINVAL
    ctx.incremental_round(final, 0.0)  # radius 0: no fovea tile; the mid disc of radius r_m - r_f
    cnt = ctx.get_counts()
    assert [cnt["n_active_tiles"], cnt["n_keys"]] == _oracle_rounds(scene, cams, final, [(final, 0.0, "exit")],
                                                                     rad)[0]
    with pytest.raises(ValueError):
        ctx.incremental_round(final[:1], 5.0)
    # another frame on the context ends the incremental one
    ctx.render_foveated(ds, cams, final, fov, out)
    with pytest.raises(pkg.A3FRError) as e:
        ctx.incremental_finish(final, out)
    assert e.value.status == pkg.A3FR_ENOTREADY
    # a finished frame takes no further round
    ctx.incremental_begin(ds, cams, fov)
    ctx.incremental_finish(final, out)
    with pytest.raises(pkg.A3FRError) as e:
        ctx.incremental_round(final, 5.0)
    assert e.value.status == pkg.A3FR_ENOTREADY
    ctx.sync()
    ctx.close()


@pytest.mark.parametrize("load,speculative", [(0.05, True), (0.5, True), (0.5, False)])
def test_concurrent_pipeline_frame_is_exact(pkg, load, speculative):
    """Algorithm 1 with a stand-in tracker publishing exits at the network's
    latencies (scaled by load, so which rounds run depends on timing): the frame
    is the one-shot frame of the last prediction whatever the rounds were, the
    rounds follow the exits in order and the finish comes after the last exit;
    the frame also equals the FP64 oracle's frame of the last prediction
    (colours within 1e-4, ambiguous pixels within their derived tolerance)."""
    from paper_2507_04147_amd import pipeline
    W, H = 464, 480
    scene, cams, trials, sig, rad = _setup(100_000, W, H, 7, 2)
    ds = pkg.DeviceScene.from_host(scene)
    fov = pkg.fovea_struct(*rad)
    ctx = pkg.Context()
    ctx.set_host_wait(True)  # the renderer's waits sleep, as beside a CPU tracker
    for final, exits in trials:
        out = torch.full((2, 3, H, W), float("nan"), device="cuda")
        res = pipeline.run(ctx, ds, cams, fov, exits, final, sig, list(synth.EXIT_LATENCY_MS), load=load, out=out,
                           speculative=speculative)
        ref = torch.zeros_like(out)
        ctx.render_foveated(ds, cams, final, fov, ref)
        ctx.sync()
        assert torch.equal(out, ref)
        # and the frame against the FP64 oracle's foveated frame of the final gaze
        o = oracle.render_foveated(scene, cams, final, rad)
        img = out.cpu().numpy()
        for e in range(2):
            err = np.abs(img[e] - o["out"][e])
            amb, tol = composite_ambiguity(W, H, final[e], rad, o["images"][3 * e: 3 * e + 3])
            assert err.max(axis=0)[~amb].max() <= COLOUR_TOL
            assert_amb_within(err, amb, tol)
        ev = res["events"]
        assert ev[0][0] == "round 0" and ev[-1][0] == "finish"
        layers = [e[1] for e in ev[1:]]
        assert layers == sorted(layers) and layers[-1] == len(synth.EXIT_LATENCY_MS)
        assert ev[-1][2] >= res["exit_ms"][-1] - 1e-6  # the finish starts once the last exit is published
        for a, b in zip(ev, ev[1:]):
            assert b[2] >= a[3] - 1e-6  # one round at a time
        if not speculative:
            assert all(e[0] != "speculative" for e in ev)
    ctx.close()
