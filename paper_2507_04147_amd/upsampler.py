"""Learned peripheral upsampler: training pairs from the renderer, training
and inference, all on the library's kernels (a3fr_preprocess / a3fr_bin_sort /
a3fr_blend for the pairs; a3fr_net_forward / a3fr_net_backward / a3fr_net_adam
for the network).

A training pair is a crop of an eye frame: the target is the full-resolution
render of a crop x crop window with every Gaussian, the input the periphery
recipe over the same window -- 1/scale resolution per axis, drawing only the
ceil(keep_num/keep_den x N_vis) visible Gaussians of largest opacity x area.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import MASK_ALL, NET_PARAMS, Context, DeviceScene, View_

MAX_EYES = 16


def _crop_view(cam, x0, y0, crop, scale, eye, select):
    v = View_()
    v.R[:] = [float(a) for a in np.asarray(cam.R, np.float64).reshape(9)]
    v.t[:] = [float(a) for a in np.asarray(cam.t, np.float64).reshape(3)]
    v.campos[:] = [float(a) for a in np.asarray(cam.campos, np.float64).reshape(3)]
    v.fx, v.fy = cam.fx / scale, cam.fy / scale
    v.cx, v.cy = (cam.cx - x0) / scale, (cam.cy - y0) / scale
    v.width = v.height = crop // scale
    v.eye, v.mask, v.select = eye, MASK_ALL, select
    v.bg[:] = [float(a) for a in cam.bg]
    return v


def make_pairs(ctx: Context, scene: DeviceScene, poses, crop=256, scale=4, keep=(3, 10)):
    """(inputs [n][3][crop/scale][crop/scale], targets [n][3][crop][crop]) on the
    device for poses = [(camera, x0, y0), ...]; 16 poses per render call."""
    n = len(poses)
    lo = crop // scale
    xs = torch.empty((n, 3, lo, lo), device="cuda")
    ts = torch.empty((n, 3, crop, crop), device="cuda")
    per = 3 * (crop * crop + lo * lo)
    buf = torch.empty(MAX_EYES * per, device="cuda")
    for s in range(0, n, MAX_EYES):
        grp = poses[s:s + MAX_EYES]
        views = []
        for e, (cam, x0, y0) in enumerate(grp):
            views.append(_crop_view(cam, x0, y0, crop, 1, e, 0))
            views.append(_crop_view(cam, x0, y0, crop, scale, e, 1))
        ctx.preprocess(scene, views, keep)
        ctx.bin_sort()
        ctx.blend(buf)
        o = 0
        for e in range(len(grp)):
            ts[s + e] = buf[o:o + 3 * crop * crop].view(3, crop, crop)
            o += 3 * crop * crop
            xs[s + e] = buf[o:o + 3 * lo * lo].view(3, lo, lo)
            o += 3 * lo * lo
    return xs, ts


class Upsampler:
    """Parameters, Adam state and the training / inference calls."""

    def __init__(self, ctx: Context, theta0):
        self.ctx = ctx
        self.theta = torch.as_tensor(np.asarray(theta0, np.float32)).to("cuda").contiguous()
        assert self.theta.numel() == NET_PARAMS
        self.grad = torch.zeros_like(self.theta)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.loss = torch.zeros(1, device="cuda")
        self.step = 0

    def forward(self, x, out=None, for_training=False):
        B, _, h, w = x.shape
        if out is None:
            out = torch.empty((B, 3, 4 * h, 4 * w), device="cuda")
        self.ctx.net_forward(self.theta, x, out, for_training)
        return out

    def train_step(self, x, target, lr=1e-3):
        out = self.forward(x, for_training=True)
        self.ctx.net_backward(self.theta, out, target, self.grad, self.loss)
        self.step += 1
        self.ctx.net_adam(self.theta, self.grad, self.m, self.v, self.step, lr)
        return self.loss

    def fit(self, xs, ts, epochs=20, batch=32, lr=1e-3, seed=0):
        """Adam on mini-batches of a seeded permutation each epoch; lr is one
        rate or one per epoch (a step schedule).  Returns the mean training
        loss of each epoch."""
        n = xs.shape[0]
        rng = np.random.default_rng(seed)
        rates = list(lr) if isinstance(lr, (list, tuple)) else [lr] * epochs
        if len(rates) != epochs:
            raise ValueError("one learning rate per epoch")
        hist = []
        for ep in range(epochs):
            lr = rates[ep]
            perm = torch.as_tensor(rng.permutation(n), device="cuda")
            tot, cnt = torch.zeros(1, device="cuda"), 0
            for s in range(0, n - batch + 1, batch):
                idx = perm[s:s + batch]
                tot += self.train_step(xs[idx].contiguous(), ts[idx].contiguous(), lr)
                cnt += 1
            hist.append(float(tot) / max(1, cnt))
        return hist


def psnr(a, b):
    """PSNR of two images (clamped to [0,1]) over all pixels and channels."""
    mse = float(((a.clamp(0, 1) - b.clamp(0, 1)) ** 2).mean())
    return math.inf if mse == 0 else 10.0 * math.log10(1.0 / mse)
