"""Differentiable render of one view behind torch.autograd.Function.

Forward: a3fr_activate (exp of the log-scales, sigmoid of the logits) ->
a3fr_preprocess -> a3fr_bin_sort -> a3fr_blend, with the final transmittance
and last-blended index kept.  Backward: a3fr_blend_backward (reverse walk of
each tile's list, transmittance recovered by division) -> a3fr_preprocess_backward
(float64 chain rule to the raw parameters).  Every step runs in the library's
HIP kernels; this module only allocates the tensors and orders the calls.

The points' parameters are the trainable quantities of Sec. 2.3 (position,
scale, rotation, opacity, SH colour).
"""
from __future__ import annotations

import torch

from . import MASK_ALL, Context, DeviceScene, View_, params_struct


def view_from_camera(cam, eye: int = 0) -> View_:
    """A full-resolution view of every tile from a camera-like object (R, t,
    campos, fx, fy, cx, cy, width, height, bg)."""
    import numpy as np
    v = View_()
    v.R[:] = [float(x) for x in np.asarray(cam.R, np.float64).reshape(9)]
    v.t[:] = [float(x) for x in np.asarray(cam.t, np.float64).reshape(3)]
    v.campos[:] = [float(x) for x in np.asarray(cam.campos, np.float64).reshape(3)]
    v.fx, v.fy, v.cx, v.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    v.width, v.height, v.eye, v.mask, v.select = int(cam.width), int(cam.height), int(eye), MASK_ALL, 0
    v.bg[:] = [float(x) for x in cam.bg]
    return v


class RenderView(torch.autograd.Function):
    """rgb [3][H][W] = render(mean [3][n], log_scale [3][n], quat [4][n], logit [n],
    sh [n][(deg+1)^2][3]) for one view; gradients w.r.t. all five."""

    @staticmethod
    def forward(fctx, mean, log_scale, quat, logit, sh, a3: Context, view: View_, sh_degree: int):
        n = int(logit.shape[0])
        p = params_struct(n, sh_degree, mean, log_scale, quat, logit, sh)
        scale = torch.empty_like(log_scale)
        opacity = torch.empty_like(logit)
        a3.activate(p, scale, opacity)
        scene = DeviceScene(mean, scale, quat, opacity, sh, sh_degree)
        a3.preprocess(scene, [view])
        a3.bin_sort()
        H, W = int(view.height), int(view.width)
        rgb = torch.empty((3, H, W), device=mean.device, dtype=torch.float32)
        T = torch.empty((H, W), device=mean.device, dtype=torch.float32)
        last = torch.empty((H, W), device=mean.device, dtype=torch.int32)
        a3.blend(rgb, T, last)
        fctx.save_for_backward(mean, log_scale, quat, logit, sh, T, last)
        fctx.a3, fctx.gen, fctx.sh_degree = a3, a3.generation, sh_degree
        fctx.hold = (scale, opacity)  # the scene the context's buffers were built from
        return rgb

    @staticmethod
    def backward(fctx, grad_rgb):
        a3 = fctx.a3
        if a3.generation != fctx.gen:
            raise RuntimeError("the context has rendered another frame since this forward; run backward first "
                               "or give each differentiable render its own Context")
        mean, log_scale, quat, logit, sh, T, last = fctx.saved_tensors
        n = int(logit.shape[0])
        p = params_struct(n, fctx.sh_degree, mean, log_scale, quat, logit, sh)
        if grad_rgb is None:
            grad_rgb = torch.zeros((3,) + tuple(T.shape), device=T.device, dtype=torch.float32)
        grad_rgb = grad_rgb.to(torch.float32).contiguous()
        a3.blend_backward(grad_rgb, T, last)
        g = [torch.empty_like(t) for t in (mean, log_scale, quat, logit, sh)]
        a3.preprocess_backward(p, *g)
        return (*g, None, None, None)


def render(a3: Context, view: View_, mean, log_scale, quat, logit, sh, sh_degree: int = 3):
    """Differentiable render of one view (see RenderView)."""
    return RenderView.apply(mean, log_scale, quat, logit, sh, a3, view, sh_degree)
