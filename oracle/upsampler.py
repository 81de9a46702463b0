"""FP64 oracle of the learned peripheral upsampler (TEST INFRASTRUCTURE ONLY:
used by tests/, the smoke check and the benchmark's CPU baseline, never by the
library).

The paper's periphery is rendered at reduced resolution and brought back to
full resolution (Sec. 2.2: progressively lower detail away from the fovea;
Sec. 3.5: coarser regions are interpolated from the rendered samples).  The
learned part replaces the bilinear x4 of the periphery by

    out = pixel_shuffle_x4(conv3(relu(conv2(relu(conv1(x)))))) + bilinear_x4(x)

with 3x3 convolutions (stride 1, zero padding 1, bias) of 3->32, 32->32 and
32->48 channels; channel c*16 + 4i + j of the last layer becomes output pixel
(c, 4y+i, 4x+j).  Loss: mean squared error against the full-resolution render.

Precision model (the one the GPU path computes): the convolution input, the
weights and the post-ReLU activations are rounded to bfloat16 (round to
nearest, ties to even); products are accumulated exactly here (float64) and in
float32 on the GPU; the last layer, the shuffle and the bilinear residual (of
the unrounded input) are float32 / float64.  In the backward pass the
gradient entering each convolution's weight and input gradients (dL/dy3 and
dL/dz2, dL/dz1 after the ReLU masks) is rounded to bfloat16 at the same points
as on the GPU; the rounding itself is passed straight through.  With
quantize=False every rounding is skipped and the backward is the exact
gradient of the float64 network.

Parameters are one flat float vector of 24,016 values:
  W1 [32][3][3][3], b1 [32], W2 [32][32][3][3], b2 [32], W3 [48][32][3][3], b3 [48]
(weights [out][in][ky][kx]).
"""
from __future__ import annotations

import numpy as np

LAYERS = ((3, 32), (32, 32), (32, 48))
N_PARAMS = sum(co * ci * 9 + co for ci, co in LAYERS)  # 24,016
SCALE = 4


def unpack(theta):
    """Flat parameter vector -> [(W [co][ci][3][3], b [co]), ...] (views)."""
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (N_PARAMS,)
    out, o = [], 0
    for ci, co in LAYERS:
        W = theta[o:o + co * ci * 9].reshape(co, ci, 3, 3)
        o += co * ci * 9
        b = theta[o:o + co]
        o += co
        out.append((W, b))
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.reshape(-1), b.reshape(-1)]) for W, b in layers])


def bf16(x):
    """Round float64 values to the nearest bfloat16 (8 significant bits), ties
    to even, returned as float64.  Written from the format's definition:
    x = m 2^e with m in [0.5, 1); keep round_half_even(m 2^8) 2^(e-8).
    Values below the smallest normal bfloat16 are rounded on that grid."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)
    e = np.maximum(e, -125)  # subnormal range: fixed spacing 2^-133
    m = x / np.ldexp(1.0, e)
    return np.ldexp(np.rint(m * 256.0), e - 8)


def conv3x3(x, W, b):
    """out[n, co, y, x] = b[co] + sum_{ci, ky, kx} W[co, ci, ky, kx] xpad[n, ci, y+ky, x+kx]
    with xpad the input zero-padded by one pixel (the taps are summed one by
    one; the sum over input channels is a matrix product)."""
    n, ci, h, w = x.shape
    co = W.shape[0]
    xp = np.zeros((n, ci, h + 2, w + 2))
    xp[:, :, 1:h + 1, 1:w + 1] = x
    out = np.broadcast_to(b.reshape(1, co, 1, 1), (n, co, h, w)).copy()
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, :, ky:ky + h, kx:kx + w]                 # [n][ci][h][w]
            out += np.einsum("oc,nchw->nohw", W[:, :, ky, kx], patch)
    return out


def conv3x3_input_grad(g, W, h, w):
    """dL/dx of conv3x3 for dL/dout = g: dx[n, ci, y, x] = sum over taps and
    co of W[co, ci, ky, kx] g[n, co, y-ky+1, x-kx+1] (zero outside)."""
    n, co = g.shape[:2]
    ci = W.shape[1]
    dxp = np.zeros((n, ci, h + 2, w + 2))
    for ky in range(3):
        for kx in range(3):
            dxp[:, :, ky:ky + h, kx:kx + w] += np.einsum("oc,nohw->nchw", W[:, :, ky, kx], g)
    return dxp[:, :, 1:h + 1, 1:w + 1]


def conv3x3_weight_grad(g, x):
    """dL/dW[co, ci, ky, kx] = sum_{n, y, x} g[n, co, y, x] xpad[n, ci, y+ky, x+kx];
    dL/db[co] = sum g[n, co, :, :]."""
    n, ci, h, w = x.shape
    xp = np.zeros((n, ci, h + 2, w + 2))
    xp[:, :, 1:h + 1, 1:w + 1] = x
    dW = np.zeros((g.shape[1], ci, 3, 3))
    for ky in range(3):
        for kx in range(3):
            dW[:, :, ky, kx] = np.einsum("nohw,nchw->oc", g, xp[:, :, ky:ky + h, kx:kx + w])
    return dW, g.sum(axis=(0, 2, 3))


def pixel_shuffle(y, r=SCALE):
    """[n][c r^2][h][w] -> [n][c][r h][r w]: channel c r^2 + r i + j goes to (c, r y + i, r x + j)."""
    n, C, h, w = y.shape
    c = C // (r * r)
    out = np.zeros((n, c, r * h, r * w))
    for i in range(r):
        for j in range(r):
            out[:, :, i::r, j::r] = y[:, [cc * r * r + r * i + j for cc in range(c)]]
    return out


def pixel_unshuffle(g, r=SCALE):
    """Adjoint of pixel_shuffle."""
    n, c, H, W = g.shape
    out = np.zeros((n, c * r * r, H // r, W // r))
    for i in range(r):
        for j in range(r):
            for cc in range(c):
                out[:, cc * r * r + r * i + j] = g[:, cc, i::r, j::r]
    return out


def bilinear_up(x, r=SCALE):
    """Bilinear x r with align_corners = false and clamp to edge: output pixel
    X samples source coordinate (X + 0.5)/r - 0.5, clamped to [0, w-1]."""
    n, c, h, w = x.shape

    def axis(L):
        s = (np.arange(L * r) + 0.5) / r - 0.5
        s = np.clip(s, 0.0, L - 1)
        i0 = np.floor(s).astype(int)
        i1 = np.minimum(i0 + 1, L - 1)
        return i0, i1, s - i0

    y0, y1, fy = axis(h)
    x0, x1, fx = axis(w)
    top = x[:, :, y0][:, :, :, x0] * (1 - fx) + x[:, :, y0][:, :, :, x1] * fx
    bot = x[:, :, y1][:, :, :, x0] * (1 - fx) + x[:, :, y1][:, :, :, x1] * fx
    return top * (1 - fy)[:, None] + bot * fy[:, None]


def forward(theta, x, quantize=True):
    """x: [n][3][h][w] (float32 values).  Returns the intermediates and out."""
    q = bf16 if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    (W1, b1), (W2, b2), (W3, b3) = unpack(theta)
    x = np.asarray(x, dtype=np.float64)
    x0 = q(x)
    z1 = conv3x3(x0, q(W1), b1)
    a1 = q(np.maximum(z1, 0.0))
    z2 = conv3x3(a1, q(W2), b2)
    a2 = q(np.maximum(z2, 0.0))
    y3 = conv3x3(a2, q(W3), b3)
    out = pixel_shuffle(y3) + bilinear_up(x)
    return dict(x0=x0, z1=z1, a1=a1, z2=z2, a2=a2, y3=y3, out=out)


def mse(out, target):
    return float(np.mean((np.asarray(out, np.float64) - np.asarray(target, np.float64)) ** 2))


def backward(theta, x, target, fw=None, quantize=True):
    """Loss (mean squared error) and its gradient w.r.t. theta.  Also returns
    the bfloat16-rounded gradients entering each convolution (g3, g2, g1)."""
    q = bf16 if quantize else (lambda a: a)
    if fw is None:
        fw = forward(theta, x, quantize)
    (W1, b1), (W2, b2), (W3, b3) = unpack(theta)
    qW2, qW3 = (bf16(W2), bf16(W3)) if quantize else (W2, W3)
    out = fw["out"]
    t = np.asarray(target, np.float64)
    loss = mse(out, t)
    h, w = fw["x0"].shape[2:]
    g3 = q(pixel_unshuffle(2.0 * (out - t) / out.size))
    dW3, db3 = conv3x3_weight_grad(g3, fw["a2"])
    g2 = q(conv3x3_input_grad(g3, qW3, h, w) * (fw["a2"] > 0))
    dW2, db2 = conv3x3_weight_grad(g2, fw["a1"])
    g1 = q(conv3x3_input_grad(g2, qW2, h, w) * (fw["a1"] > 0))
    dW1, db1 = conv3x3_weight_grad(g1, fw["x0"])
    grad = pack([(dW1, db1), (dW2, db2), (dW3, db3)])
    return loss, grad, dict(g3=g3, g2=g2, g1=g1)


def adam(theta, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (bias-corrected first and second moments); returns new
    (theta, m, v).  step counts from 1."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
