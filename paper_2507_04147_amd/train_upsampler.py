"""Train the peripheral upsampler at the size of its configuration and save it.

10,000 (quarter-resolution, full-resolution) 256 x 256 crop pairs rendered by
the library from the 1M-Gaussian scene at the workload's random poses (9,000
to train, 1,000 held out), 20 epochs of Adam (batch 32, lr 1e-3) from the
seeded initial weights, all on the library's kernels.  Writes the weights
(raw little-endian float32 + JSON header with the held-out PSNR of the
network and of bilinear x4, the method without the network).

    python -m paper_2507_04147_amd.train_upsampler --workload outside \
        --out paper_2507_04147_amd/weights/upsampler_outside
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

WORKLOADS = ("inside", "outside")


def poses_for(synth, workload, seed, n):
    return synth.crop_poses(seed, n) if workload == "inside" else synth.crop_poses_outside(seed, n)


def held_out_psnr(U, pkg, ctx, theta, xs, ts):
    """Held-out PSNR of the network theta and of bilinear x4 (theta = 0)."""
    net = U.Upsampler(ctx, theta)
    bil = U.Upsampler(ctx, np.zeros(pkg.NET_PARAMS, np.float32))
    return U.psnr(net.forward(xs), ts), U.psnr(bil.forward(xs), ts)


def train(workload="outside", pairs=10_000, held=1_000, epochs=20, batch=32, lr=1e-3, seed_poses=41, seed_init=42):
    import torch  # noqa: F401  (device memory)

    import paper_2507_04147_amd as pkg
    import synth
    from . import upsampler as U
    scene, _ = synth.foveated_stereo()
    ds = pkg.DeviceScene.from_host(scene)
    ctx = pkg.Context()
    t0 = time.perf_counter()
    xs, ts = U.make_pairs(ctx, ds, poses_for(synth, workload, seed_poses, pairs))
    ntr = pairs - held
    net = U.Upsampler(ctx, synth.net_init(seed_init))
    hist = net.fit(xs[:ntr], ts[:ntr], epochs=epochs, batch=batch, lr=lr)
    theta = net.theta.cpu().numpy()
    p_net, p_bil = held_out_psnr(U, pkg, ctx, theta, xs[ntr:].contiguous(), ts[ntr:].contiguous())
    ctx.close()
    meta = dict(workload=workload, scene="1M-Gaussian uniform cloud over [-5,5]^3 (seed 2)", pairs=pairs,
                train_pairs=ntr, held_out_pairs=held, epochs=epochs, batch=batch, lr=lr, seed_poses=seed_poses,
                seed_init=seed_init, train_loss_first_epoch=hist[0], train_loss_last_epoch=hist[-1],
                held_out_psnr_db=dict(network=p_net, bilinear=p_bil), seconds=time.perf_counter() - t0)
    return theta, meta


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=WORKLOADS, default="outside")
    ap.add_argument("--out", required=True, help="path without extension (.bin and .json are written)")
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from . import upsampler as U
    theta, meta = train(args.workload)
    d = os.path.dirname(args.out)
    if d:
        os.makedirs(d, exist_ok=True)
    U.save_weights(args.out, theta, meta)
    print(f"{args.workload}: held-out PSNR network {meta['held_out_psnr_db']['network']:.4f} dB, "
          f"bilinear {meta['held_out_psnr_db']['bilinear']:.4f} dB -> {args.out}.bin", flush=True)


if __name__ == "__main__":
    main()
