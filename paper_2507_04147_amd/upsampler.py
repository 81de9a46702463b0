"""Learned peripheral upsampler: training pairs from the renderer, training
and inference, all on the library's kernels (a3fr_preprocess / a3fr_bin_sort /
a3fr_blend for the pairs; a3fr_net_forward / a3fr_net_backward / a3fr_net_adam
for the network).

A training pair is a crop of an eye frame, rendered the way the foveated
frame renders it: the target is the full-resolution render of a crop x crop
window with every Gaussian; the input is the same window of the frame's
periphery layer -- the whole eye frame at 1/scale resolution per axis,
drawing only the ceil(keep_num/keep_den x N_vis) Gaussians of largest
opacity x area among those visible in the frame (the subset the frame's
periphery draws, not one chosen within the crop).
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


def _periphery_view(cam, scale, eye):
    """The frame's periphery layer of an eye camera: 1/scale per axis, every
    tile, drawing the kept subset (a3fr_make_foveated_views' third layer)."""
    v = _crop_view(cam, 0, 0, 0, scale, eye, 1)
    v.width, v.height = cam.width // scale, cam.height // scale
    return v


def make_pairs(ctx: Context, scene: DeviceScene, poses, crop=256, scale=4, keep=(3, 10)):
    """(inputs [n][3][crop/scale][crop/scale], targets [n][3][crop][crop]) on the
    device for poses = [(camera, x0, y0), ...] (x0, y0 multiples of scale); 16
    poses per render call, each rendering its full-resolution crop and its
    whole periphery layer."""
    n = len(poses)
    lo = crop // scale
    xs = torch.empty((n, 3, lo, lo), device="cuda")
    ts = torch.empty((n, 3, crop, crop), device="cuda")
    for cam, x0, y0 in poses:
        if x0 % scale or y0 % scale or x0 + crop > cam.width or y0 + crop > cam.height:
            raise ValueError("crop origin must be a multiple of the scale, the crop inside the frame")
    buf = None
    for s in range(0, n, MAX_EYES):
        grp = poses[s:s + MAX_EYES]
        views = []
        for e, (cam, x0, y0) in enumerate(grp):
            views.append(_crop_view(cam, x0, y0, crop, 1, e, 0))
            views.append(_periphery_view(cam, scale, e))
        tot = 3 * sum(v.width * v.height for v in views)
        if buf is None or buf.numel() < tot:
            buf = torch.empty(tot, device="cuda")
        ctx.preprocess(scene, views, keep)
        ctx.bin_sort()
        ctx.blend(buf)
        o = 0
        for e, (cam, x0, y0) in enumerate(grp):
            ts[s + e] = buf[o:o + 3 * crop * crop].view(3, crop, crop)
            o += 3 * crop * crop
            pw, ph = views[2 * e + 1].width, views[2 * e + 1].height
            per = buf[o:o + 3 * pw * ph].view(3, ph, pw)
            xs[s + e] = per[:, y0 // scale: y0 // scale + lo, x0 // scale: x0 // scale + lo]
            o += 3 * pw * ph
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


# ---------------------------------------------------------------------------
# saved weights: raw little-endian float32 plus a JSON header
# ---------------------------------------------------------------------------
WEIGHTS_LAYOUT = "W1 [32][3][3][3], b1 [32], W2 [32][32][3][3], b2 [32], W3 [48][32][3][3], b3 [48]"


def save_weights(path, theta, meta):
    """Writes path + '.bin' (NET_PARAMS float32, little-endian) and path + '.json'
    (meta plus the format fields and the sha256 of the .bin)."""
    import hashlib
    import json
    raw = np.ascontiguousarray(np.asarray(theta, dtype="<f4")).tobytes()
    if len(raw) != 4 * NET_PARAMS:
        raise ValueError("theta must hold NET_PARAMS values")
    with open(path + ".bin", "wb") as fh:
        fh.write(raw)
    head = dict(format="a3fr upsampler weights", dtype="float32", byteorder="little", params=NET_PARAMS,
                layout=WEIGHTS_LAYOUT, sha256=hashlib.sha256(raw).hexdigest())
    head.update(meta)
    with open(path + ".json", "w") as fh:
        json.dump(head, fh, indent=1)
        fh.write("\n")


def load_weights(path):
    """(theta float32 [NET_PARAMS], header dict) from save_weights' files; raises
    if the size, byte order or checksum does not match the header."""
    import hashlib
    import json
    with open(path + ".json") as fh:
        head = json.load(fh)
    with open(path + ".bin", "rb") as fh:
        raw = fh.read()
    if head.get("params") != NET_PARAMS or len(raw) != 4 * NET_PARAMS or head.get("byteorder") != "little":
        raise ValueError(f"{path}: not a {NET_PARAMS}-parameter little-endian weight file")
    if hashlib.sha256(raw).hexdigest() != head.get("sha256"):
        raise ValueError(f"{path}.bin does not match the checksum in its header")
    return np.frombuffer(raw, dtype="<f4").astype(np.float32), head
