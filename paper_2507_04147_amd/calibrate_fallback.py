"""Calibrate the periphery error estimate coef x (dT^2)^power of the
full-resolution fallback (a3fr_set_fallback).

For frames rendered at the upsampler's training poses (one eye, gaze at the
image centre), every periphery tile that reaches outside r_mid gets its
transmittance rise dT = exp(-K) - exp(-(K + D)) (D, K: the library's own
dropped and kept opacity mass per pixel, computed with an unreachable
threshold so nothing falls back) and its measured squared error against the
plain full-resolution render over its pixels outside r_mid (images clamped
to [0,1]).  With power 1, coef is set so that the estimate reaches the
threshold (1e-3, the squared error of 30 dB) at the given quantile of dT^2:
the fallback then takes that fraction of tiles, highest dT^2 first.  The
script prints what share of the measured squared error, and of the tiles
above the threshold, each flagged fraction captures.

    python -m paper_2507_04147_amd.calibrate_fallback [--poses 64] [--flag-fraction 0.10]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

import numpy as np


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--poses", type=int, default=64)
    ap.add_argument("--seed", type=int, default=41)
    ap.add_argument("--threshold", type=float, default=1e-3)
    ap.add_argument("--flag-fraction", type=float, default=0.10)
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch

    import paper_2507_04147_amd as pkg
    import synth

    scene, cams0 = synth.foveated_stereo()
    W, H = cams0[0].width, cams0[0].height
    rad = (0.15 * W, 0.35 * W)
    fov = pkg.fovea_struct(*rad)
    ds = pkg.DeviceScene.from_host(scene)
    ctx = pkg.Context()
    ctx.set_fallback(1e300, 1.0, 1.0)
    span = 64
    TX, TY = (W // 4 + 15) // 16, (H // 4 + 15) // 16
    ys, xs = torch.meshgrid(torch.arange(H, device="cuda"), torch.arange(W, device="cuda"), indexing="ij")
    outer = ((xs + 0.5 - W / 2) ** 2 + (ys + 0.5 - H / 2) ** 2) > rad[1] ** 2
    tid = (ys // span) * TX + (xs // span)
    Fs, Ms = [], []
    out = torch.empty((1, 3, H, W), device="cuda")
    ref = torch.empty_like(out)
    for cam, _, _ in synth.crop_poses(args.seed, args.poses):
        ctx.render_foveated(ds, [cam], [(cam.cx, cam.cy)], fov, out)
        en = ctx.inspect("fb_energy", torch.float32).double()
        nt = en.numel() // 2
        D, K = en[nt - TX * TY:nt], en[2 * nt - TX * TY:]  # the periphery view's tiles come last
        dT2 = (torch.exp(-K) - torch.exp(-(K + D))) ** 2
        ctx.render_full(ds, [cam], ref)
        d2 = ((out[0].clamp(0, 1) - ref[0].clamp(0, 1)) ** 2).sum(0)
        sse = torch.zeros(TX * TY, device="cuda", dtype=torch.float64).index_add_(
            0, tid[outer], d2[outer].double())
        cnt = torch.zeros(TX * TY, device="cuda", dtype=torch.float64).index_add_(
            0, tid[outer], torch.ones_like(d2[outer], dtype=torch.float64))
        ok = cnt >= 64
        Fs.append(dT2[ok].cpu().numpy())
        Ms.append((sse[ok] / (3.0 * cnt[ok])).cpu().numpy())
    F, M = np.concatenate(Fs), np.concatenate(Ms)
    order = np.argsort(-F)
    bad = M > args.threshold
    table = []
    for frac in (0.01, 0.02, 0.05, 0.1, 0.2):
        k = max(1, int(frac * F.size))
        table.append(dict(flagged=frac, mse_share=float(M[order[:k]].sum() / M.sum()),
                          tiles_above_threshold_caught=float(np.isin(np.nonzero(bad)[0], order[:k]).mean())
                          if bad.any() else None))
    q = float(np.quantile(F, 1.0 - args.flag_fraction))
    coef = args.threshold / q if q > 0 else 0.0
    res = dict(tiles=int(F.size), tiles_above_threshold=int(bad.sum()),
               above_threshold_mse_share=float(M[bad].sum() / M.sum()), dT2_quantile=q, coef=coef, table=table)
    print(json.dumps(res))
    print(f"FALLBACK_DEFAULT = ({args.threshold!r}, {coef:.6g}, 1.0)")


if __name__ == "__main__":
    main()
