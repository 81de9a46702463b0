"""HIP-graph replay of the foveated frame and batched frames (MI355X only).

Bars: every replay of the captured frame, with new poses and gazes, equals the
eager render of the same frame bit for bit (replays interleaved with eager
work); a frame over the key capacity is reported as A3FR_ECAPACITY without
touching memory beyond the buffers, and later frames work again; several
frames rendered in one batch equal the frames rendered one at a time.
"""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    import paper_2507_04147_amd as p
    p.lib()
    assert torch.cuda.is_available()
    return p


def _eager(pkg, ctx, ds, cams, gz, fov, W, H):
    out = torch.zeros((len(cams), 3, H, W), device="cuda")
    ctx.render_foveated(ds, cams, gz, fov, out)
    ctx.sync()
    return out, ctx.get_counts()["n_keys"]


def _setup(pkg, n, W, H, n_frames, seed):
    scene, _ = synth.foveated_stereo(n=n, width=W, height=H, seed=seed)
    trace = synth.gaze_trace(seed=31, n_frames=n_frames, width=W, height=H)
    return scene, pkg.DeviceScene.from_host(scene), trace, pkg.fovea_struct(0.15 * W, 0.35 * W)


@pytest.mark.parametrize("options", ["plain", "fallback+net+queue", "fallback+net"])
def test_graph_replays_match_eager(pkg, options):
    """Graph replays equal eager frames bit for bit.  With the network and a
    grid blend variant ("fallback+net") the frame blends the fovea and mid
    layers on a second stream beside the periphery's blend and the network,
    in the eager frames and in the captured graph (fork and join recorded)."""
    W, H = 232, 240
    scene, ds, trace, fov = _setup(pkg, 60_000, W, H, 6, 11)
    ce, cg = pkg.Context(), pkg.Context()
    if options != "plain":
        theta = torch.from_numpy(synth.net_init(47, last_scale=1.0)).cuda()
        for c in (ce, cg):
            c.set_fallback(1e-3, 20.0, 1.0)
            c.set_upsampler(theta)
            if "queue" in options:
                c.set_blend_variant(7)  # 64-record batches, 4 x 1 pixels, longest-first queue
    refs, keys = [], []
    for cams, gz in trace:
        o, k = _eager(pkg, ce, ds, cams, gz, fov, W, H)
        refs.append(o.cpu())
        keys.append(k)
    cap = int(max(keys) * 1.25) + 64
    out = torch.zeros((2, 3, H, W), device="cuda")
    cg.graph_capture(ds, trace[0][0], trace[0][1], fov, out, cap)
    cg.sync()
    assert torch.equal(out.cpu(), refs[0])
    for rep in range(2):
        for k, (cams, gz) in enumerate(trace):
            out.fill_(float("nan"))
            torch.cuda.synchronize()
            cg.graph_launch(cams, gz)
            cg.sync()
            assert torch.equal(out.cpu(), refs[k]), (rep, k)
            assert cg.get_counts()["n_keys"] == keys[k]
            # eager work between replays
            _eager(pkg, ce, ds, cams, gz, fov, W, H)
    cg.graph_destroy()
    o, _ = _eager(pkg, cg, ds, trace[2][0], trace[2][1], fov, W, H)
    assert torch.equal(o.cpu(), refs[2])
    ce.close()
    cg.close()


def test_graph_capacity_overflow_is_reported(pkg):
    W, H = 232, 240
    scene, ds, trace, fov = _setup(pkg, 60_000, W, H, 12, 12)
    ce, cg = pkg.Context(), pkg.Context()
    keys = [_eager(pkg, ce, ds, c, g, fov, W, H)[1] for c, g in trace]
    order = np.argsort(keys)
    small, big = int(order[0]), int(order[-1])
    assert keys[big] > keys[small]
    out = torch.zeros((2, 3, H, W), device="cuda")
    # too small for the warm-up frame itself
    with pytest.raises(pkg.A3FRError) as e:
        cg.graph_capture(ds, trace[big][0], trace[big][1], fov, out, keys[big] - 1)
    assert e.value.status == pkg.A3FR_ECAPACITY
    cg.graph_capture(ds, trace[small][0], trace[small][1], fov, out, keys[small])
    cg.sync()
    cg.graph_launch(trace[big][0], trace[big][1])
    with pytest.raises(pkg.A3FRError) as e:
        cg.sync()
    assert e.value.status == pkg.A3FR_ECAPACITY
    cg.graph_launch(trace[small][0], trace[small][1])
    cg.sync()
    ref, _ = _eager(pkg, ce, ds, trace[small][0], trace[small][1], fov, W, H)
    assert torch.equal(out, ref)
    cg.graph_destroy()
    ce.close()
    cg.close()


def test_batched_frames_equal_single_frames(pkg):
    """Four stereo frames (8 eyes, 24 layer views with uneven tile counts) in
    one preprocess / sort / persistent blend equal the frames one by one."""
    W, H = 232, 240
    scene, ds, trace, fov = _setup(pkg, 60_000, W, H, 4, 13)
    ctx = pkg.Context()
    ctx.set_blend_variant(7)
    cams = [c for f in trace for c in f[0]]
    gz = [g for f in trace for g in f[1]]
    out = torch.zeros((8, 3, H, W), device="cuda")
    ctx.render_foveated(ds, cams, gz, fov, out)
    ctx.sync()
    for k, (c, g) in enumerate(trace):
        o, _ = _eager(pkg, ctx, ds, c, g, fov, W, H)
        assert torch.equal(out[2 * k: 2 * k + 2], o), k
    ctx.close()


def test_graph_batched_full_size(pkg):
    """Eight stereo frames of the 1M-Gaussian scene at 1832 x 1920 (16 eyes,
    48 layer views) captured once and replayed for another window of the
    gaze trace; each replay equals the eager batch."""
    W, H = 1832, 1920
    scene, ds, trace, fov = _setup(pkg, 1_000_000, W, H, 16, 2)
    ce, cg = pkg.Context(), pkg.Context()
    cg.set_blend_variant(7)
    ce.set_blend_variant(7)
    wins = [trace[:8], trace[8:]]
    flat = [([c for f in w for c in f[0]], [g for f in w for g in f[1]]) for w in wins]
    refs, keys = [], []
    for cams, gz in flat:
        o, k = _eager(pkg, ce, ds, cams, gz, fov, W, H)
        refs.append(o)
        keys.append(k)
    out = torch.zeros((16, 3, H, W), device="cuda")
    cg.graph_capture(ds, flat[0][0], flat[0][1], fov, out, int(max(keys) * 1.2))
    for rep in range(2):
        for k, (cams, gz) in enumerate(flat):
            cg.graph_launch(cams, gz)
            cg.sync()
            assert torch.equal(out, refs[k]), (rep, k)
    cg.graph_destroy()
    ce.close()
    cg.close()


@pytest.mark.parametrize("variant", [1, 7])
def test_batched_frames_vs_oracle(pkg, variant):
    """Row 12 against the FP64 oracle: four stereo frames of a drifting gaze
    trace (head turning 1 deg/frame, saccades and jitter) in ONE a3fr_render_batch
    (8 eyes, 24 layer views with uneven tile counts, ragged 232 x 240 grids).
    Bit-exact against oracle.render on the same concatenated views: per-entry
    counts, depths and rectangles, the kept sets, the depth order, key offsets,
    keys in emission order, sorted keys and values, tile ranges; layer colours
    within 1e-4 (ambiguous pixels within their derived tolerance), T, last
    index; and the composite of every eye against the oracle's composite."""
    import oracle
    from test_gpu_parity import compare_images, compare_stage_outputs, composite_ambiguity, assert_amb_within, \
        COLOUR_TOL
    W, H = 232, 240
    scene, ds, trace, fov = _setup(pkg, 40_000, W, H, 4, 17)
    rad = (0.15 * W, 0.35 * W)
    cams = [c for f in trace for c in f[0]]
    gz = [g for f in trace for g in f[1]]
    views = oracle.foveated_views(cams, gz, rad)
    ref = oracle.render(scene, views)
    ctx = pkg.Context()
    ctx.set_blend_variant(variant)
    ctx.set_debug(True)
    out = torch.full((4, 2, 3, H, W), float("nan"), device="cuda")
    ctx.render_batch(ds, trace, fov, out)
    ctx.sync()
    assert ctx.get_counts()["n_keys"] == ref["keys"].size
    compare_stage_outputs(ctx, ref, views, scene.n)
    o = out.cpu().numpy().reshape(8, 3, H, W)
    for e in range(8):
        L = ref["images"][3 * e: 3 * e + 3]
        want = oracle.composite(W, H, gz[e], rad, L[0]["rgb"], L[1]["rgb"], L[2]["rgb"])
        amb, tol = composite_ambiguity(W, H, gz[e], rad, L)
        err = np.abs(o[e] - want)
        assert err[:, ~amb].max() <= COLOUR_TOL, e
        assert_amb_within(err, amb, tol, e)
    # the layer images of the same batch (stage calls on the same views)
    ctx.preprocess(ds, views)
    assert ctx.bin_sort() == ref["keys"].size
    npx = sum(v.width * v.height for v in views)
    rgb = torch.full((3 * npx,), float("nan"), device="cuda")
    T = torch.full((npx,), float("nan"), device="cuda")
    last = torch.zeros(npx, dtype=torch.int32, device="cuda")
    ctx.blend(rgb, T, last)
    ctx.sync()
    compare_images(views, ref, rgb, T, last, ref["active"])
    ctx.close()


def test_gaze_trace_64_frames_one_launch(pkg):
    """The batched gaze trace as one launch: 64 stereo frames of the 3M-Gaussian
    scene at 1832 x 1920 (128 eyes, 384 layer views: more than 2^30 (view,
    Gaussian) slots and more than 2^30 keys, addressed by 32-bit positions up
    to 2^32 - 1) in one a3fr_render_batch and in one captured graph.  Every
    frame equals the frame rendered alone (the path the single-frame parity
    tests check against the oracle), and the batch's keys are the sum of the
    frames' keys."""
    W, H = 1832, 1920
    scene, _ = synth.foveated_stereo(n=3_000_000, seed=3)
    ds = pkg.DeviceScene.from_host(scene)
    n = scene.n
    del scene
    trace = synth.gaze_trace(seed=31, n_frames=64, width=W, height=H)
    fov = pkg.fovea_struct(0.15 * W, 0.35 * W)
    cb = pkg.Context()
    out = torch.empty((64, 2, 3, H, W), device="cuda")
    cb.render_batch(ds, trace, fov, out)
    cb.sync()
    K = cb.get_counts()["n_keys"]
    print(f"64 frames: {384 * n} slots, {K} keys", flush=True)
    assert 384 * n > (1 << 30) and K > (1 << 30)
    cs = pkg.Context()
    one = torch.empty((2, 3, H, W), device="cuda")
    k_sum = 0
    for f, (cams, gz) in enumerate(trace):
        cs.render_foveated(ds, cams, gz, fov, one)
        cs.sync()
        k_sum += cs.get_counts()["n_keys"]
        assert torch.equal(out[f], one), f
    assert k_sum == K
    cs.close()
    # the same window from a captured graph (no host read-back), replayed twice
    ref = out.clone()
    cams = [c for fr in trace for c in fr[0]]
    gzs = [g for fr in trace for g in fr[1]]
    cb.graph_capture(ds, cams, gzs, fov, out.view(128, 3, H, W), int(K * 1.05))
    for _ in range(2):
        out.fill_(float("nan"))
        cb.graph_launch(cams, gzs)
        cb.sync()
        assert torch.equal(out, ref)
    cb.graph_destroy()
    cb.close()
