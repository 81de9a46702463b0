"""Pins of the oracle's differentiable render (CPU only).

The backward is the analytic chain rule of the forward (Sec. 2.3: projection,
depth order, front-to-back blend, evaluated from the raw parameters); it is
pinned here by central finite differences of the forward, by its forward
against the tiled/brute-force oracle render, and by linearity in dL/dI.
"""
import numpy as np
import pytest

import oracle.core as oc
import synth


def _setup(n=300, seed=5, w=48, h=40, half=1.0, log_scale_mean=-2.0, bg=(0.0, 0.0, 0.0)):
    sc = synth.make_scene(n, half, seed=seed, log_scale_mean=log_scale_mean)
    cam = synth.make_camera(w, h, 60.0, (0.0, 0.0, -3.0), bg=bg)
    v = oc.full_view(cam)
    wgt = np.random.default_rng(seed + 100).normal(size=(3, h, w))
    P = dict(mean=sc.mean.astype(np.float64), log_scale=sc.log_scale.astype(np.float64),
             quat=sc.quat.astype(np.float64), logit=sc.logit.astype(np.float64), sh=sc.sh.astype(np.float64))
    return sc, cam, v, wgt, P


def _run(P, v, wgt, smooth, deg=3):
    return oc.render_grad(P["mean"], P["log_scale"], P["quat"], P["logit"], P["sh"], v, wgt, smooth=smooth, deg=deg)


def _loss(P, v, wgt, smooth, deg=3):
    return float((wgt * _run(P, v, wgt, smooth, deg)["image"]).sum())


def _depth_order(P, v):
    R = np.asarray(v.R).reshape(3, 3)
    z = (R[2] @ P["mean"].astype(np.float32).astype(np.float64)) + float(v.t[2])
    return np.lexsort((np.arange(z.size), z.astype(np.float32)))


def _fd_check(P, v, wgt, smooth, name, idxs, rel_h, tol, floor_frac=1e-4, deg=3):
    ref = _run(P, v, wgt, smooth, deg)
    an_all = ref["grads"][name]
    floor = floor_frac * float(np.abs(an_all).max())
    arr = P[name]
    worst = 0.0
    checked = 0
    for idx in idxs:
        x0 = float(arr[idx])
        h = rel_h * max(1.0, abs(x0))
        xp, xm = float(np.float32(x0 + h)), float(np.float32(x0 - h))
        arr[idx] = xp
        order_p = _depth_order(P, v) if name == "mean" else None
        Lp = _loss(P, v, wgt, smooth, deg)
        arr[idx] = xm
        order_m = _depth_order(P, v) if name == "mean" else None
        Lm = _loss(P, v, wgt, smooth, deg)
        arr[idx] = x0
        if name == "mean" and not np.array_equal(order_p, order_m):
            continue  # the step crossed a depth-order swap: the render is not differentiable there
        fd = (Lp - Lm) / (xp - xm)
        an = float(an_all[idx])
        err = abs(fd - an) / max(abs(fd), abs(an), floor)
        worst = max(worst, err)
        checked += 1
        assert err <= tol, (name, idx, fd, an, err)
    assert checked >= len(idxs) // 2
    return worst


_SEEDS = dict(mean=1, log_scale=2, quat=3, logit=4, sh=5)


def _sample(shape, k, seed):
    rng = np.random.default_rng(seed)
    return [tuple(int(rng.integers(0, s)) for s in shape) for _ in range(k)]


@pytest.mark.parametrize("name", ["mean", "log_scale", "quat", "logit", "sh"])
def test_grad_fd_smooth(name):
    """Smooth mode (no skip, stop or clamps): the analytic gradient of every
    parameter group equals the central difference of the loss."""
    sc, cam, v, wgt, P = _setup()
    idxs = _sample(P[name].shape, 10, _SEEDS[name])
    _fd_check(P, v, wgt, True, name, idxs, rel_h=1e-4, tol=2e-4)


@pytest.mark.parametrize("name", ["mean", "log_scale", "quat", "logit", "sh"])
def test_grad_fd_thresholded(name):
    """The render as shipped (1/255 skip, 0.99 clamp, early stop, colour clamp at
    zero): away from the thresholds the gradient is still the central difference."""
    sc, cam, v, wgt, P = _setup(seed=7, log_scale_mean=-1.8)
    idxs = _sample(P[name].shape, 10, 17 + _SEEDS[name])
    _fd_check(P, v, wgt, False, name, idxs, rel_h=1e-6, tol=2e-3)


def test_grad_fd_clamped_projection():
    """A Gaussian whose centre lies outside the 1.3x guard band (the Jacobian is
    evaluated at the clamped direction) but whose footprint reaches the image."""
    sc, cam, v, wgt, P = _setup(n=3, seed=9, w=32, h=32)
    P["mean"][:, 0] = [1.9, 0.1, -1.0]   # x/z = 0.95 > 1.3 * tan(30 deg) = 0.75
    P["log_scale"][:, 0] = [-0.7, -0.9, -1.1]
    P["logit"][0] = 2.0
    P["mean"][:, 1] = [-0.1, 1.7, -1.2]  # y/z clamped
    P["log_scale"][:, 1] = [-0.8, -0.6, -1.0]
    P["mean"][:, 2] = [0.0, 0.0, 0.5]
    ref = _run(P, v, wgt, True)
    assert ref["n_proj"] == 3
    for name in ("mean", "log_scale", "quat"):
        idxs = [(c, g) for c in range(P[name].shape[0]) for g in (0, 1)]
        _fd_check(P, v, wgt, True, name, idxs, rel_h=1e-5, tol=1e-4)


def test_grad_forward_matches_oracle_render():
    """The thresholded forward equals the tiled and brute-force renders of the
    pinned oracle (same scene, activated in FP64) away from ambiguous pixels."""
    sc, cam, v, wgt, P = _setup(n=400, seed=11, w=64, h=48, bg=(0.2, 0.1, 0.4))
    r = _run(P, v, wgt, False)
    brute = oc.render_brute(sc, [v])[0]["rgb"]
    tiled = oc.render(sc, [v])["images"][0]["rgb"]
    ok = r["amb"] == 0
    assert ok.mean() > 0.95
    for ref in (brute, tiled):
        d = np.abs(r["image"] - ref).max(axis=0)
        assert d[ok].max() < 2e-5, d[ok].max()


def test_grad_linear_in_weights():
    """dL/dtheta is linear in dL/dI."""
    sc, cam, v, wgt, P = _setup(n=120, seed=13)
    w2 = np.random.default_rng(3).normal(size=wgt.shape)
    g1 = _run(P, v, wgt, False)["grads"]
    g2 = _run(P, v, w2, False)["grads"]
    g3 = _run(P, v, wgt + 2.0 * w2, False)["grads"]
    for k in g1:
        np.testing.assert_allclose(g3[k], g1[k] + 2.0 * g2[k], rtol=1e-9, atol=1e-12)


def test_grad_degree0_colour_is_view_independent():
    """With degree 0 the colour does not depend on the viewing direction, so
    colour gradients send nothing to the mean through the direction; the DC
    gradient is Y_0 times the colour gradient."""
    sc, cam, v, wgt, P = _setup(n=80, seed=15)
    r0 = _run(P, v, wgt, True, deg=0)
    assert r0["grads"]["sh"].shape == (1, 3, 80)
    # moving a mean along the camera ray through it keeps (u, v) and only changes
    # depth-dependent terms; an SH-only perturbation of degree > 0 coefficients
    # must not change the degree-0 render
    P2 = {k: a.copy() for k, a in P.items()}
    P2["sh"][1:] += 0.5
    np.testing.assert_array_equal(_run(P2, v, wgt, True, deg=0)["image"], r0["image"])
    idxs = _sample((1, 3, 80), 6, 5)
    _fd_check(P, v, wgt, True, "sh", idxs, rel_h=1e-4, tol=2e-4, deg=0)


@pytest.mark.parametrize("name", ["mean", "log_scale", "logit"])
def test_grad_fd_alpha_clamp_and_stop(name):
    """Opaque Gaussians: alpha is clamped at 0.99 near their centres (no
    gradient through alpha there) and pixels stop early once T drops below
    1e-4; the gradient is still the central difference away from the thresholds."""
    sc, cam, v, wgt, P = _setup(n=150, seed=19, log_scale_mean=-1.6)
    P["logit"][:] = 6.0 + 0.1 * np.arange(150) / 150.0   # opacity ~0.9975
    idxs = _sample(P[name].shape, 10, 40 + _SEEDS[name])
    _fd_check(P, v, wgt, False, name, idxs, rel_h=1e-6, tol=2e-3)


def test_grad_window_equals_restricted_full_render():
    """Rendering and differentiating a pixel window (with the exact footprint
    cull of the thresholded mode) equals the whole-view run with dL/dI zero
    outside the window."""
    sc, cam, v, wgt, P = _setup(n=300, seed=21, w=64, h=48)
    win = (16, 8, 24, 20)
    wz = np.zeros_like(wgt)
    wz[:, 8:28, 16:40] = wgt[:, 8:28, 16:40]
    full = _run(P, v, wz, False)
    part = oc.render_grad(P["mean"], P["log_scale"], P["quat"], P["logit"], P["sh"], v, wgt, window=win)
    np.testing.assert_allclose(part["image"][:, 8:28, 16:40], full["image"][:, 8:28, 16:40], rtol=0, atol=1e-15)
    assert not part["image"][:, :8].any() and not part["image"][:, :, :16].any()
    assert part["n_proj"] < full["n_proj"]
    for k in full["grads"]:
        np.testing.assert_allclose(part["grads"][k], full["grads"][k], rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("name", ["mean", "log_scale", "quat", "logit", "sh"])
def test_grad_fd_differentiable_workload_subset(name):
    """The finite-difference subset of the differentiable-render workload (its
    first 1,000 Gaussians at 64 x 64, 60 degree FOV, f = 55.4 px), smooth mode."""
    sc, _ = synth.differentiable()
    sub = sc.subset(np.arange(1000))
    cam = synth.make_camera(64, 64, 60.0, (0.0, 0.0, -3.0))
    assert abs(cam.fx - 55.4256) < 1e-3
    v = oc.full_view(cam)
    wgt = np.random.default_rng(77).normal(size=(3, 64, 64))
    P = dict(mean=sub.mean.astype(np.float64), log_scale=sub.log_scale.astype(np.float64),
             quat=sub.quat.astype(np.float64), logit=sub.logit.astype(np.float64), sh=sub.sh.astype(np.float64))
    idxs = _sample(P[name].shape, 6, 60 + _SEEDS[name])
    _fd_check(P, v, wgt, True, name, idxs, rel_h=1e-4, tol=2e-4)
