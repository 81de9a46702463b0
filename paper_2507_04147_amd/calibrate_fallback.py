"""Calibrate the periphery error estimate coef x (dT^2)^power of the
full-resolution fallback (a3fr_set_fallback).

Frames are rendered at the upsampler's training poses of a workload (one eye;
the first gaze at the image centre, the others seeded within 20 degrees of
it; the periphery through the given network or bilinear).  Every periphery tile that reaches outside r_mid gets its
transmittance rise dT = exp(-K) - exp(-(K + D)) (D, K: the library's own
dropped and kept opacity mass per pixel, computed with an unreachable
threshold so that nothing falls back) and its measured squared error against
the plain full-resolution render over its pixels outside r_mid (images
clamped to [0,1]); the mid annulus's error is measured too.  A fallen-back
tile equals the full-resolution render outside r_mid, so with the tiles of
dT^2 >= q flagged, a frame's periphery PSNR (every pixel outside r_fovea)
follows from the measured errors of the tiles left.  With power 1, coef =
threshold / q for the largest q at which every calibration frame keeps its
periphery PSNR at or above target + margin dB: the fewest tiles, taken in
order of dT^2, that bring each frame to the target.

    python -m paper_2507_04147_amd.calibrate_fallback --workload outside \
        [--weights paper_2507_04147_amd/weights/upsampler_outside] [--poses 64]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

import numpy as np


def measure(pkg, synth, torch, workload, weights, n_poses, seed, keep=(3, 10)):
    """Per frame: dT^2 and squared-error sum of each periphery tile reaching
    outside r_mid, and the mid annulus's error sum and pixel counts."""
    scene, cams0 = synth.foveated_stereo()
    W, H = cams0[0].width, cams0[0].height
    rad = (0.15 * W, 0.35 * W)
    fov = pkg.fovea_struct(*rad, keep=keep)
    ds = pkg.DeviceScene.from_host(scene)
    ctx = pkg.Context()
    theta = None
    if weights:
        from . import upsampler as U
        theta = torch.from_numpy(U.load_weights(weights)[0]).cuda()
        ctx.set_upsampler(theta)
    ctx.set_fallback(1e300, 1.0, 1.0)
    span = 64
    TX, TY = (W // 4 + 15) // 16, (H // 4 + 15) // 16
    ys, xs = torch.meshgrid(torch.arange(H, device="cuda"), torch.arange(W, device="cuda"), indexing="ij")
    tid = (ys // span) * TX + (xs // span)
    frames = []
    out = torch.empty((1, 3, H, W), device="cuda")
    ref = torch.empty_like(out)
    poses = synth.crop_poses(seed, n_poses) if workload == "inside" else synth.crop_poses_outside(seed, n_poses)
    gazes = synth.gaze_points(seed + 1000, n_poses, cams0[0])
    for (cam, _, _), g in zip(poses, gazes):
        r2 = (xs + 0.5 - g[0]) ** 2 + (ys + 0.5 - g[1]) ** 2
        outer = r2 > rad[1] ** 2
        mid = (r2 > rad[0] ** 2) & ~outer
        ctx.render_foveated(ds, [cam], [g], fov, out)
        en = ctx.inspect("fb_energy", torch.float32).double()
        nt = en.numel() // 2
        D, K = en[nt - TX * TY:nt], en[2 * nt - TX * TY:]  # the periphery view's tiles come last
        dT2 = (torch.exp(-K) - torch.exp(-(K + D))) ** 2
        ctx.render_full(ds, [cam], ref)
        d2 = ((out[0].clamp(0, 1) - ref[0].clamp(0, 1)) ** 2).sum(0).double()
        sse = torch.zeros(TX * TY, device="cuda", dtype=torch.float64).index_add_(0, tid[outer], d2[outer])
        cnt = torch.zeros(TX * TY, device="cuda", dtype=torch.float64).index_add_(
            0, tid[outer], torch.ones_like(d2[outer]))
        ok = cnt > 0
        frames.append(dict(dT2=dT2[ok].cpu().numpy(), sse=sse[ok].cpu().numpy(), cnt=cnt[ok].cpu().numpy(),
                           mid_sse=float(d2[mid].sum()), mid_cnt=int(mid.sum())))
    ctx.close()
    return frames


def frame_psnr(f, q):
    """Periphery PSNR of frame f when the tiles with dT^2 >= q fall back."""
    left = f["dT2"] < q
    sse = f["mid_sse"] + float(f["sse"][left].sum())
    n = 3.0 * (f["mid_cnt"] + float(f["cnt"].sum()))
    return math.inf if sse == 0 else 10.0 * math.log10(n / sse)


def calibrate(frames, threshold=1e-3, target_db=30.0, margin_db=1.0):
    F = np.concatenate([f["dT2"] for f in frames])
    cand = np.unique(F)[::-1]  # descending: the first q flags the fewest tiles
    need = target_db + margin_db
    q_best = None
    if all(frame_psnr(f, math.inf) >= need for f in frames):
        q_best = math.inf  # no tile needs the fallback
    else:
        # the worst frame's PSNR only rises as q falls: bisect over the candidates
        lo, hi = 0, cand.size - 1
        if min(frame_psnr(f, cand[hi]) for f in frames) >= need:
            while lo < hi:
                m = (lo + hi) // 2
                if min(frame_psnr(f, cand[m]) for f in frames) >= need:
                    hi = m
                else:
                    lo = m + 1
            q_best = float(cand[lo])
    coef = 0.0 if q_best is None else (0.0 if q_best == math.inf else threshold / q_best)
    flagged = 0.0 if q_best in (None, math.inf) else float((F >= q_best).mean())
    before = [frame_psnr(f, math.inf) for f in frames]
    after = [frame_psnr(f, q_best if q_best is not None else 0.0) for f in frames]
    order = np.argsort(-F)
    M = np.concatenate([f["sse"] / (3.0 * f["cnt"]) for f in frames])
    table = [dict(flagged=fr, mse_share=float(M[order[:max(1, int(fr * F.size))]].sum() / max(M.sum(), 1e-300)))
             for fr in (0.01, 0.05, 0.1, 0.2, 0.4)]
    return dict(tiles=int(F.size), tiles_above_threshold=int((M > threshold).sum()), dT2_threshold=q_best,
                coef=coef, flagged_fraction=flagged, psnr_before_db=dict(min=min(before), median=float(np.median(before))),
                psnr_after_db=dict(min=min(after), median=float(np.median(after))), target_db=target_db,
                margin_db=margin_db, table=table)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=("inside", "outside"), default="outside")
    ap.add_argument("--weights", default=None, help="upsampler weights (path without extension); default bilinear")
    ap.add_argument("--poses", type=int, default=64)
    ap.add_argument("--seed", type=int, default=41)
    ap.add_argument("--threshold", type=float, default=1e-3)
    ap.add_argument("--target-db", type=float, default=30.0)
    ap.add_argument("--margin-db", type=float, default=1.0)
    ap.add_argument("--keep", type=int, nargs=2, default=(3, 10), metavar=("NUM", "DEN"))
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch

    import paper_2507_04147_amd as pkg
    import synth
    frames = measure(pkg, synth, torch, args.workload, args.weights, args.poses, args.seed, tuple(args.keep))
    res = calibrate(frames, args.threshold, args.target_db, args.margin_db)
    res.update(workload=args.workload, weights=args.weights, poses=args.poses, seed=args.seed, keep=list(args.keep))
    print(json.dumps(res))
    print(f"({args.threshold!r}, {res['coef']:.6g}, 1.0)")


if __name__ == "__main__":
    main()
