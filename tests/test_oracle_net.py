"""Pins of the upsampler oracle (CPU only).

Each piece is checked against an independent implementation (torch's float64
CPU conv2d, pixel_shuffle, bilinear interpolate, bfloat16 cast and Adam), the
unquantised backward against central differences and against torch autograd,
and the quantised forward/backward for the properties its rounding points fix.
"""
import numpy as np
import pytest

import oracle.upsampler as up

torch = pytest.importorskip("torch")
F = torch.nn.functional


def _theta(seed, scale3=1.0):
    rng = np.random.default_rng(seed)
    layers = []
    for k, (ci, co) in enumerate(up.LAYERS):
        bound = 1.0 / np.sqrt(ci * 9)
        s = scale3 if k == 2 else 1.0
        layers.append((rng.uniform(-bound, bound, (co, ci, 3, 3)) * s, rng.uniform(-bound, bound, co) * s))
    return up.pack(layers)


def test_param_count_and_flops():
    assert up.N_PARAMS == 24016
    macs = sum(ci * co * 9 for ci, co in up.LAYERS)
    assert 2 * macs == 47808


def test_conv_matches_torch():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 5, 7, 6))
    W = rng.normal(size=(4, 5, 3, 3))
    b = rng.normal(size=4)
    ref = F.conv2d(torch.from_numpy(x), torch.from_numpy(W), torch.from_numpy(b), padding=1).numpy()
    np.testing.assert_allclose(up.conv3x3(x, W, b), ref, rtol=1e-12, atol=1e-12)


def test_conv_grads_match_torch():
    rng = np.random.default_rng(2)
    x = torch.from_numpy(rng.normal(size=(2, 5, 7, 6))).requires_grad_(True)
    W = torch.from_numpy(rng.normal(size=(4, 5, 3, 3))).requires_grad_(True)
    b = torch.from_numpy(rng.normal(size=4)).requires_grad_(True)
    g = rng.normal(size=(2, 4, 7, 6))
    F.conv2d(x, W, b, padding=1).backward(torch.from_numpy(g))
    np.testing.assert_allclose(up.conv3x3_input_grad(g, W.detach().numpy(), 7, 6), x.grad.numpy(), rtol=1e-12,
                               atol=1e-12)
    dW, db = up.conv3x3_weight_grad(g, x.detach().numpy())
    np.testing.assert_allclose(dW, W.grad.numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(db, b.grad.numpy(), rtol=1e-12, atol=1e-12)


def test_pixel_shuffle_and_bilinear_match_torch():
    rng = np.random.default_rng(3)
    y = rng.normal(size=(2, 48, 5, 7))
    np.testing.assert_array_equal(up.pixel_shuffle(y), F.pixel_shuffle(torch.from_numpy(y), 4).numpy())
    g = rng.normal(size=(2, 3, 20, 28))
    np.testing.assert_array_equal(up.pixel_unshuffle(g), F.pixel_unshuffle(torch.from_numpy(g), 4).numpy())
    x = rng.normal(size=(2, 3, 5, 7))
    ref = F.interpolate(torch.from_numpy(x), scale_factor=4, mode="bilinear", align_corners=False).numpy()
    np.testing.assert_allclose(up.bilinear_up(x), ref, rtol=1e-12, atol=1e-12)


def test_bf16_rounding_matches_torch_cast():
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.normal(size=20000).astype(np.float32),
                        (rng.normal(size=2000) * 1e-30).astype(np.float32),
                        (rng.normal(size=2000) * 1e30).astype(np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(up.bf16(x.astype(np.float64)), ref)


def test_bf16_ties_to_even():
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: ties go to the even mantissa (1)
    assert up.bf16(1.0 + 2.0 ** -8) == 1.0
    # 1 + 3 * 2^-8 lies halfway between 1 + 2^-7 and 1 + 2^-6: goes to 1 + 2^-6
    assert up.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert up.bf16(-(1.0 + 2.0 ** -8)) == -1.0
    assert up.bf16(255.5) == 256.0 and up.bf16(0.0) == 0.0


def _loss_fd(theta, x, t, idx, h):
    tp, tm = theta.copy(), theta.copy()
    tp[idx] += h
    tm[idx] -= h
    Lp = up.mse(up.forward(tp, x, quantize=False)["out"], t)
    Lm = up.mse(up.forward(tm, x, quantize=False)["out"], t)
    return (Lp - Lm) / (2 * h)


def test_backward_fd_unquantised():
    rng = np.random.default_rng(5)
    theta = _theta(6)
    x = rng.uniform(0, 1, (2, 3, 5, 6))
    t = rng.uniform(0, 1, (2, 3, 20, 24))
    loss, g, _ = up.backward(theta, x, t, quantize=False)
    # sample entries of every block: W1, b1, W2, b2, W3, b3
    offs = np.cumsum([0] + [n for ci, co in up.LAYERS for n in (co * ci * 9, co)])
    for blk in range(6):
        for idx in rng.integers(offs[blk], offs[blk + 1], 4):
            fd = _loss_fd(theta, x, t, idx, 1e-6)
            assert abs(fd - g[idx]) <= 1e-6 * max(1e-3, abs(fd)), (blk, idx, fd, g[idx])


def test_backward_matches_torch_autograd_unquantised():
    rng = np.random.default_rng(7)
    theta = _theta(8)
    x = rng.uniform(0, 1, (2, 3, 6, 5))
    t = rng.uniform(0, 1, (2, 3, 24, 20))
    loss, g, _ = up.backward(theta, x, t, quantize=False)
    th = torch.from_numpy(theta.copy()).requires_grad_(True)
    o, ps = 0, []
    for ci, co in up.LAYERS:
        ps.append((th[o:o + co * ci * 9].view(co, ci, 3, 3), th[o + co * ci * 9:o + co * ci * 9 + co]))
        o += co * ci * 9 + co
    xt = torch.from_numpy(x)
    a = F.relu(F.conv2d(xt, *ps[0], padding=1))
    a = F.relu(F.conv2d(a, *ps[1], padding=1))
    out = F.pixel_shuffle(F.conv2d(a, *ps[2], padding=1), 4) + F.interpolate(xt, scale_factor=4, mode="bilinear",
                                                                               align_corners=False)
    lt = ((out - torch.from_numpy(t)) ** 2).mean()
    lt.backward()
    assert abs(float(lt.detach()) - loss) < 1e-12
    np.testing.assert_allclose(g, th.grad.numpy(), rtol=1e-9, atol=1e-14)


def test_quantised_rounding_points():
    """Rounded quantities are bfloat16 values; the quantised forward equals the
    unquantised one on bfloat16 weights and inputs up to the activation
    rounding; the quantised backward differs from the unquantised one only
    through the rounded gradients and activations."""
    rng = np.random.default_rng(9)
    theta = _theta(10)
    x = rng.uniform(0, 1, (1, 3, 6, 6))
    fw = up.forward(theta, x)
    for k in ("x0", "a1", "a2"):
        np.testing.assert_array_equal(up.bf16(fw[k]), fw[k])
    # weights already bfloat16 and input already bfloat16: z1 is the same either way
    layers = [(up.bf16(W), b) for W, b in up.unpack(theta)]
    tq = up.pack(layers)
    xq = up.bf16(x)
    np.testing.assert_allclose(up.forward(tq, xq)["z1"], up.forward(tq, xq, quantize=False)["z1"], rtol=0, atol=0)
    t = rng.uniform(0, 1, (1, 3, 24, 24))
    _, _, gs = up.backward(theta, x, t, fw)
    for k in ("g3", "g2", "g1"):
        np.testing.assert_array_equal(up.bf16(gs[k]), gs[k])
    # the unrounded and rounded gradients are close (relative 2^-8 per rounding)
    l0, g0, _ = up.backward(theta, x, t, quantize=False)
    l1, g1, _ = up.backward(theta, x, t)
    assert np.abs(g1 - g0).max() < 0.05 * np.abs(g0).max()


def test_adam_matches_torch():
    rng = np.random.default_rng(11)
    theta = rng.normal(size=50)
    m, v = np.zeros(50), np.zeros(50)
    tt = torch.from_numpy(theta.copy()).requires_grad_(True)
    opt = torch.optim.Adam([tt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 6):
        g = rng.normal(size=50)
        theta, m, v = up.adam(theta, g, m, v, step, lr=1e-2)
        tt.grad = torch.from_numpy(g)
        opt.step()
    np.testing.assert_allclose(theta, tt.detach().numpy(), rtol=1e-12, atol=1e-14)
