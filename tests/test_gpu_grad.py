"""GPU parity of the differentiable render against the FP64 oracle (MI355X only).

The HIP path is a3fr_activate -> a3fr_preprocess -> a3fr_bin_sort -> a3fr_blend
forward and a3fr_blend_backward -> a3fr_preprocess_backward backward, called
through the torch.autograd.Function of paper_2507_04147_amd.train.  The oracle
is the plain-definition render of the raw parameters with its analytic FP64
backward (oracle/a3fr_oracle_grad.c, pinned by finite differences on the CPU).

dL/dI is N(0,1) noise, set to zero on the pixels where the oracle flags a
skip or stop decision as lying within the float32 error bound of its
threshold (there the two sides may take different branches).

Bars: image within 1e-4 absolute; each gradient entry within
GRAD_RTOL x |oracle| + GRAD_ATOL x max |oracle| of its parameter group.  The
float32 path carries relative errors of a few 1e-6 per (pixel, Gaussian) term
(record rounding, exp2, the division that recovers T, which the 1/(1-alpha)
factor can amplify up to 100x near alpha = 0.99), and a Gaussian's gradient is
a sum of up to thousands of such terms with cancellation, so the bound is
relative to the group's scale rather than to each (possibly cancelled) entry.
"""
import numpy as np
import pytest

import oracle.core as oc
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

IMG_TOL = 1e-4
GRAD_RTOL = 1e-4
GRAD_ATOL = 2e-5
GROUPS = ("mean", "log_scale", "quat", "logit", "sh")


@pytest.fixture(scope="module")
def pkg():
    import paper_2507_04147_amd as p
    p.lib()
    assert torch.cuda.is_available()
    return p


def gpu_grads(pkg, sc, cam, wgt, sh_degree=3):
    from paper_2507_04147_amd import train
    a3 = pkg.Context()
    P = pkg.DeviceParams.from_host(sc, sh_degree=sh_degree)
    ts = [t.clone().requires_grad_(True) for t in P.tensors()]
    rgb = train.render(a3, train.view_from_camera(cam), *ts, sh_degree=sh_degree)
    rgb.backward(torch.from_numpy(np.ascontiguousarray(wgt, dtype=np.float32)).cuda())
    torch.cuda.synchronize()
    a3.sync()
    g = [t.grad.cpu().numpy().astype(np.float64) for t in ts]
    a3.close()
    return rgb.detach().cpu().numpy(), dict(mean=g[0], log_scale=g[1], quat=g[2], logit=g[3],
                                            sh=np.transpose(g[4], (1, 2, 0)))


def oracle_run(sc, cam, wgt, deg=3, window=None):
    return oc.render_grad(sc.mean, sc.log_scale, sc.quat, sc.logit, sc.sh, oc.full_view(cam), wgt, smooth=False,
                          deg=deg, window=window)


def masked_weights(sc, cam, seed, deg=3, windows=None):
    """N(0,1) dL/dI, zero on ambiguous pixels (and outside the windows, if given)."""
    rng = np.random.default_rng(seed)
    w = rng.normal(size=(3, cam.height, cam.width))
    if windows is None:
        amb = oracle_run(sc, cam, w, deg)["amb"]
    else:
        keep = np.zeros((cam.height, cam.width), bool)
        amb = np.zeros((cam.height, cam.width), np.uint8)
        for win in windows:
            x0, y0, ww, wh = win
            keep[y0:y0 + wh, x0:x0 + ww] = True
            r = oracle_run(sc, cam, np.zeros_like(w), deg, window=win)
            amb[y0:y0 + wh, x0:x0 + ww] = r["amb"][y0:y0 + wh, x0:x0 + ww]
        w[:, ~keep] = 0.0
    w[:, amb != 0] = 0.0
    return w, amb


def compare_grads(gpu, orc, label=""):
    report = {}
    for k in GROUPS:
        a, b = gpu[k], orc[k]
        assert a.shape == b.shape, (k, a.shape, b.shape)
        scale = float(np.abs(b).max())
        err = np.abs(a - b)
        bound = GRAD_RTOL * np.abs(b) + GRAD_ATOL * scale
        worst = float((err / np.maximum(bound, 1e-300)).max()) if scale > 0 else float(err.max())
        report[k] = (scale, float(err.max()), worst)
        print(f"{label} {k}: max|oracle|={scale:.3e} max err={err.max():.3e} worst err/bound={worst:.3f}",
              flush=True)
        if scale == 0.0:
            assert err.max() == 0.0, k
        else:
            bad = np.argwhere(err > bound)
            assert bad.size == 0, (k, bad[:5], a[tuple(bad[0])], b[tuple(bad[0])])
    return report


def _check(pkg, sc, cam, seed, deg=3):
    w, amb = masked_weights(sc, cam, seed, deg)
    orc = oracle_run(sc, cam, w, deg)
    img, g = gpu_grads(pkg, sc, cam, w, deg)
    ok = amb == 0
    d = np.abs(img - orc["image"]).max(axis=0)
    assert d[ok].max() <= IMG_TOL, d[ok].max()
    compare_grads(g, orc["grads"] if deg == 3 else {**orc["grads"]}, f"n={sc.n} {cam.width}x{cam.height}")
    return g, orc


def test_grad_small_ragged(pkg):
    """3,000 Gaussians, 100 x 70 (ragged tiles), coloured background."""
    sc = synth.make_scene(3000, 1.0, seed=31)
    cam = synth.make_camera(100, 70, 60.0, (0.0, 0.0, -3.0), bg=(0.1, 0.2, 0.3))
    _check(pkg, sc, cam, 1)


def test_grad_large_splats(pkg):
    """Fewer, larger splats (log-scale mean -2): long per-tile lists."""
    sc = synth.make_scene(800, 1.0, seed=32, log_scale_mean=-2.0)
    cam = synth.make_camera(96, 80, 60.0, (0.0, 0.0, -3.0))
    _check(pkg, sc, cam, 2)


def test_grad_opaque_clamp_and_stop(pkg):
    """Opaque Gaussians: alpha clamped at 0.99 and early stops."""
    sc = synth.make_scene(600, 1.0, seed=33, log_scale_mean=-2.2)
    sc.logit[:] = np.float32(5.0)
    sc.opacity[:] = np.float32(1.0 / (1.0 + np.exp(-5.0)))
    cam = synth.make_camera(64, 64, 60.0, (0.0, 0.0, -3.0))
    _check(pkg, sc, cam, 3)


def test_grad_sh_degree1(pkg):
    sc = synth.make_scene(1500, 1.0, seed=34)
    cam = synth.make_camera(80, 64, 60.0, (0.0, 0.0, -3.0))
    _check(pkg, sc, cam, 4, deg=1)


def test_grad_fd_subset(pkg):
    """The finite-difference subset of the differentiable-render workload: its
    first 1,000 Gaussians at 64 x 64 (the oracle's gradient there is the one
    pinned by central differences on the CPU)."""
    sc, _ = synth.differentiable()
    sub = sc.subset(np.arange(1000))
    cam = synth.make_camera(64, 64, 60.0, (0.0, 0.0, -3.0))
    _check(pkg, sub, cam, 5)


def test_grad_full_size_windows(pkg):
    """500,000 Gaussians at 1024 x 1024 (the launch configuration of the
    training step): dL/dI is nonzero only in three 32 x 32 windows (centre,
    corner, right edge), which the oracle differentiates pixel by pixel; every
    Gaussian's gradient is compared (the others must be exactly zero)."""
    sc, cam = synth.differentiable()
    wins = [(496, 496, 32, 32), (0, 0, 32, 32), (992, 300, 32, 32)]
    w, amb = masked_weights(sc, cam, 6, windows=wins)
    img, g = gpu_grads(pkg, sc, cam, w)
    tot = None
    for win in wins:
        x0, y0, ww, wh = win
        wi = np.zeros_like(w)
        wi[:, y0:y0 + wh, x0:x0 + ww] = w[:, y0:y0 + wh, x0:x0 + ww]
        r = oracle_run(sc, cam, wi, window=win)
        ok = amb[y0:y0 + wh, x0:x0 + ww] == 0
        d = np.abs(img[:, y0:y0 + wh, x0:x0 + ww] - r["image"][:, y0:y0 + wh, x0:x0 + ww]).max(axis=0)
        assert d[ok].max() <= IMG_TOL, (win, d[ok].max())
        tot = r["grads"] if tot is None else {k: tot[k] + r["grads"][k] for k in GROUPS}
    compare_grads(g, tot, "full size windows")


def test_zero_upstream_gives_zero_grads(pkg):
    sc = synth.make_scene(500, 1.0, seed=35)
    cam = synth.make_camera(48, 48, 60.0, (0.0, 0.0, -3.0))
    _, g = gpu_grads(pkg, sc, cam, np.zeros((3, 48, 48)))
    for k in GROUPS:
        assert not np.any(g[k]), k


def test_stale_context_raises(pkg):
    from paper_2507_04147_amd import train
    sc = synth.make_scene(200, 1.0, seed=36)
    cam = synth.make_camera(32, 32, 60.0, (0.0, 0.0, -3.0))
    a3 = pkg.Context()
    P = pkg.DeviceParams.from_host(sc)
    ts = [t.clone().requires_grad_(True) for t in P.tensors()]
    v = train.view_from_camera(cam)
    rgb1 = train.render(a3, v, *ts)
    train.render(a3, v, *ts)  # a second frame on the same context
    with pytest.raises(RuntimeError, match="another frame"):
        rgb1.sum().backward()
    a3.close()


def test_backward_call_order_and_args(pkg):
    sc = synth.make_scene(100, 1.0, seed=37)
    a3 = pkg.Context()
    P = pkg.DeviceParams.from_host(sc)
    g = [torch.empty_like(t) for t in P.tensors()]
    with pytest.raises(pkg.A3FRError) as e:
        a3.preprocess_backward(P.struct(), *g)
    assert e.value.status == pkg.A3FR_ENOTREADY
    with pytest.raises(pkg.A3FRError) as e:
        a3.blend_backward(g[0], g[0], g[0])
    assert e.value.status == pkg.A3FR_ENOTREADY
    a3.close()


def test_training_step_reduces_l1(pkg):
    """Differentiable-render workload: 500,000 Gaussians at 1024 x 1024, L1 loss
    against the render of the scene with perturbed means and logits; a few
    Adam steps on the means and logits from the unperturbed start lower it."""
    from paper_2507_04147_amd import train
    sc, cam = synth.differentiable()
    tgt = synth.perturbed(sc)
    a3 = pkg.Context()
    v = train.view_from_camera(cam)
    T = pkg.DeviceParams.from_host(tgt)
    with torch.no_grad():
        target = train.render(a3, v, *T.tensors())
    P = pkg.DeviceParams.from_host(sc)
    ts = [t.clone().requires_grad_(True) for t in P.tensors()]
    opt = torch.optim.Adam([ts[0], ts[3]], lr=2e-3)
    losses = []
    for it in range(12):
        opt.zero_grad()
        rgb = train.render(a3, v, *ts)
        loss = (rgb - target).abs().mean()
        loss.backward()
        opt.step()
        losses.append(float(loss.detach()))
        assert np.isfinite(losses[-1])
    print("L1:", ["%.5f" % x for x in losses], flush=True)
    assert losses[-1] < 0.8 * losses[0]
    a3.close()
