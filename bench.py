#!/usr/bin/env python
"""Stereo frames/s of the gaze-tracked foveated 3DGS renderer on one MI355X.

Workload: the foveated stereo frame -- 1,000,000 Gaussians drawn uniformly over
[-5,5]^3 (log-scales N(-3,0.5), random unit quaternions, opacity sigmoid(N(0,1)),
degree-3 SH coefficients N(0,0.3)), head at (0,0,-3) looking +z, two eyes 64 mm
apart, 1832 x 1920 per eye, 60 degree horizontal FOV; foveal layer at full
resolution within 0.15 W of the gaze (image centre), mid layer at 1/2 resolution
to 0.35 W, periphery at 1/4 resolution over the whole frame drawing the top 30%
of visible Gaussians by opacity x projected area; composited to full resolution.
One step = one whole stereo frame through the C ABI (preprocess, periphery
select, scan, key emission, radix sort, ranges, blend, composite), scene
resident in HBM, output [2][3][1920][1832] float32 in HBM.

The plain full-resolution render (FRR) of the same frame is timed in the same
process, and the periphery PSNR of the foveated frame against it is reported.
A second timed pass with per-stage HIP events gives the roofline of the
dominant kernel; the FP64 CPU oracle is timed on the host as the CPU baseline.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "stereo frames/s @1M Gaussians, foveated vs full-res on GPU, periphery PSNR≥30dB"
HBM_PEAK_GBS = 8000.0         # MI355X HBM3E
FP32_VECTOR_PEAK_TF = 157.3   # MI355X FP32 vector (packed) peak
SORT_BYTES_PER_KEY_PASS = 16  # tile-id sort scatter: read key (4) + value (4), write key (4) + value (4)
BLEND_FLOPS_PER_PAIR = 18
# HBM traffic per dispatch from the hardware counters: rocprofv3 --pmc
# FETCH_SIZE, then WRITE_SIZE (KiB per dispatch) of the profiled benchmark
# command, each scaled by the factor that maps what the same counter reads for
# a device-to-device copy of known size to that size.  A table entry is used
# only while the kernel source it was measured on is unchanged (sha256), else
# traffic is null.  Keys: the blend variant "batch,block,schedule", else the
# kernel name.
# Calibration (bench.py --calibrate-copy 512): a 512 MiB device copy reads
# FETCH_SIZE = 262,166.6 KiB (its reads are 128-byte requests, which that
# counter's expression weighs as 64 bytes) and writes WRITE_SIZE = 524,288 KiB.
PMC_FETCH_FACTOR = 524288.0 / 262166.6
PMC_WRITE_FACTOR = 1.0
PMC_TRAFFIC = {  # stage -> source under the package, its sha256, {key: (FETCH KiB, WRITE KiB) per dispatch}
    "blend": dict(source="csrc/blend.hip",
                  sha256="56f821fff9a95f00860d8993a5417dd80d0363ec35df19f2aad1ddd6a39f7747",
                  kib={"32,4x1,grid": (7391.3, 21750.0),
                       "32,4x1,queue": (6907.5, 23917.3),
                       "32,2x2,grid": (7394.2, 21750.0),
                       "32,2x2,queue": (6863.3, 21967.7),
                       "64,4x1,grid": (10525.8, 21750.0),
                       "64,4x1,queue": (9891.7, 24541.2),
                       "64,2x2,grid": (10541.1, 21750.0),
                       "64,2x2,queue": (9785.6, 22118.5),
                       "128,4x1,grid": (18967.4, 21750.0),
                       "128,4x1,queue": (18750.9, 25320.5),
                       "128,2x2,grid": (18933.1, 21750.0),
                       "128,2x2,queue": (18566.8, 22442.3),
                       "64,8x8q,grid": (10183.4, 21750.0),
                       "128,8x8q,grid": (18054.5, 21750.0),
                       "256,8x8q,grid": (32726.9, 21750.0)}),
    "preprocess": dict(source="csrc/preprocess.hip",
                       sha256="044dc8100cd9684f7154eb5e94863f28896b7b63b5a8875195212cefd947bc8a",
                       kib={"k_preprocess": (21722.5, 100987.8)}),
    "colour": dict(source="csrc/preprocess.hip",
                   sha256="044dc8100cd9684f7154eb5e94863f28896b7b63b5a8875195212cefd947bc8a",
                   kib={"k_entry_record": (85767.5, 33774.9)}),
    "sort_pass": dict(source="csrc/sort.hip",  # the scatter of each tile-id pass
                      sha256="166153c8db95ae1265c358d997265e86b9ad0b13047e449c838020c17afb1a0a",
                      kib={"k_sort_scatter": (40104.4, 81888.8)}),
}
# projection, one launch for both eyes (each with its fovea, mid and periphery
# views): the float32 mean, scale, quaternion and opacity of every Gaussian
# (44 B) once per frame; a 4-byte key count per (view, Gaussian) slot; the
# 4-byte depth key of every slot that emits keys, an 8-byte score in the
# periphery (selecting) views, and an 8-byte rectangle for every slot of the
# views that keep them (with the fallback: each eye's fovea, recounted, and
# periphery, whose mass map reads them).
PREPROCESS_READ_PER_GAUSSIAN = 44
PREPROCESS_WRITE_PER_SLOT = 4
PREPROCESS_WRITE_PER_EMITTING = 4
PREPROCESS_WRITE_PER_SCORE = 8
PREPROCESS_WRITE_PER_RECT_SLOT = 8
# record pass, per entry (a kept slot that emits keys): its slot index (4), the
# Gaussian's geometry (44) and SH coefficients (4 x 3 x 16 at degree 3) read;
# its 48-byte blend record, 8-byte rectangle and 4-byte slot-to-entry map written
RECORD_BYTES_PER_ENTRY = 4 + 44 + 48 + 8 + 4
# key emission (chunk starts + emission): per entry its key offset (4), index
# (4) and rectangle (8) read; per key its tile id and Gaussian index written
EMIT_BYTES_PER_ENTRY = 4 + 4 + 8
EMIT_BYTES_PER_KEY = 8
# reverse blend: floating-point operations per revisited (pixel, Gaussian) pair
# (alpha recomputed: 8; transmittance recovery, colour and alpha gradients: 14;
# the nine per-Gaussian sums: 21)
BLEND_BWD_FLOPS_PER_PAIR = 43
# reverse projection: per Gaussian, parameters read once (mean 12, log-scale 12,
# quaternion 16, logit 4), the 48-byte accumulator read, gradients written once
# (236 B at SH degree 3); per drawn Gaussian also its 48-byte record and 192 B
# of SH coefficients
PREPROCESS_BWD_BYTES_PER_GAUSSIAN = 44 + 48 + 236
PREPROCESS_BWD_BYTES_PER_DRAWN = 48 + 192


def pmc_traffic(stage, key):
    """HBM bytes per dispatch of a stage's kernel from the counter table, or
    None when there is none or its source has changed since."""
    t = PMC_TRAFFIC.get(stage)
    if t is None or key is None or key not in t["kib"] or PMC_FETCH_FACTOR is None or PMC_WRITE_FACTOR is None:
        return None
    import hashlib
    with open(os.path.join(ROOT, "paper_2507_04147_amd", t["source"]), "rb") as fh:
        if hashlib.sha256(fh.read()).hexdigest() != t["sha256"]:
            return None
    fetch, write = t["kib"][key]
    return 1024.0 * (fetch * PMC_FETCH_FACTOR + write * PMC_WRITE_FACTOR)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--gaussians", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-frames", type=int, default=2, help="oracle frames timed for the CPU baseline")
    ap.add_argument("--only", choices=["both", "foveated", "full"], default="both",
                    help="restrict the timed loops (for profiling runs)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the graph, upsampler, fallback and gaze-trace legs")
    ap.add_argument("--trace-window", type=int, default=64, help="frames per graph launch in the gaze-trace leg")
    ap.add_argument("--train-steps", type=int, default=10,
                    help="timed steps of the differentiable-render training loop (0: skip)")
    ap.add_argument("--gazes", type=int, default=16, help="seeded gazes per workload in the workloads leg")
    ap.add_argument("--legs", default="all",
                    help="comma-separated extra legs to run (parts, workloads, incremental, amr, pipeline, "
                         "upsampler, net_training, trace, training) or 'all'")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device (reference dispatch for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the renderer has no multi-GPU path; "
              "see DESIGN.md for how it would shard.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2507_04147_amd as pkg
    import synth

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calibrate_copy} MiB read + {args.calibrate_copy} MiB written")
        del src, dst
    t0 = time.time()
    scene, cams = synth.foveated_stereo(n=args.gaussians)
    W, H = cams[0].width, cams[0].height
    gaze = [(c.cx, c.cy) for c in cams]
    rad = (synth.FOVEA_FRACTIONS[0] * W, synth.FOVEA_FRACTIONS[1] * W)
    ds = pkg.DeviceScene.from_host(scene)
    fov = pkg.fovea_struct(*rad, keep=synth.PERIPH_KEEP)
    ctx = pkg.Context()
    # the method's frame: the periphery through the upsampler trained for this
    # workload when that network beats bilinear on its held-out pairs (the
    # weights' header), else bilinear x4; and the per-tile error estimate with
    # full-resolution fallback, calibrated for that periphery
    nets = {w: load_net(pkg, torch, w) for w in ("inside", "outside")}
    theta, use_net = nets["inside"]["theta"], nets["inside"]["use"]

    fallback = pkg.FALLBACK_NET if use_net else pkg.FALLBACK_BILINEAR
    fallback_on = math.isfinite(fallback[0])

    def method_options(c):
        c.set_upsampler(theta if use_net else None)
        c.set_fallback(*fallback)

    method_options(ctx)
    out_f = torch.empty((2, 3, H, W), device="cuda")
    out_r = torch.empty((2, 3, H, W), device="cuda")
    log(f"scene ready in {time.time() - t0:.1f}s: {scene.n} Gaussians, {W}x{H} per eye")

    def step_fov():
        ctx.render_foveated(ds, cams, gaze, fov, out_f)

    def step_frr():
        ctx.render_full(ds, cams, out_r)

    def timed(fn, steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1000.0 / steps

    do_fov = args.only in ("both", "foveated")
    do_frr = args.only in ("both", "full")
    for _ in range(args.warmup):
        if do_fov:
            step_fov()
        if do_frr:
            step_frr()
    torch.cuda.synchronize()
    tuned = None
    if do_fov:
        # the blend autotuner (all variants give identical images) on this frame
        step_fov()
        ms_var, best = ctx.autotune_blend(reps=3)
        tuned = dict(variant=best, desc=list(pkg.blend_variant_desc(best)),
                     ms=[round(m, 4) for m in ms_var])
        log(f"blend autotuner: variant {best} {pkg.blend_variant_desc(best)}")
    log("warmup done")
    ms_f = timed(step_fov, args.steps) if do_fov else float("nan")
    ms_r = timed(step_frr, args.steps) if do_frr else float("nan")
    log(f"foveated {ms_f:.3f} ms/frame, full-res {ms_r:.3f} ms/frame")

    # the same frame replayed from a HIP graph (no host read-back inside the frame)
    ms_g = float("nan")
    if do_fov and not args.no_extra:
        ctx.render_foveated(ds, cams, gaze, fov, out_f)
        keys = ctx.get_counts()["n_keys"]
        ctxg = pkg.Context()
        method_options(ctxg)
        out_g = torch.empty_like(out_f)
        ctxg.graph_capture(ds, cams, gaze, fov, out_g, int(keys * 1.25) + 1024)
        for _ in range(args.warmup):
            ctxg.graph_launch(cams, gaze)
        ms_g = timed(lambda: ctxg.graph_launch(cams, gaze), args.steps)
        ctxg.sync()
        if not torch.equal(out_g, out_f):
            raise RuntimeError("graph replay differs from the eager frame")
        ctxg.graph_destroy()
        ctxg.close()
        log(f"foveated from a HIP graph {ms_g:.3f} ms/frame")

    # quality of the foveated frame against the full-resolution render
    psnr = []
    psnr_outer = []
    if do_fov and do_frr:
        step_fov()
        step_frr()
        for e in range(2):
            sse, cnt = ctx.region_sse(W, H, gaze[e], rad[0], rad[1], out_f[e], out_r[e])
            n_out = cnt[1] + cnt[2]
            mse = (sse[1] + sse[2]) / (3.0 * n_out)
            psnr.append(math.inf if mse == 0 else 10 * math.log10(1.0 / mse))
            mo = sse[2] / (3.0 * cnt[2])
            psnr_outer.append(math.inf if mo == 0 else 10 * math.log10(1.0 / mo))

    # per-stage event timing over a second timed pass (roofline)
    stages = {}
    roofline = None
    counts = {}
    if do_fov:
        # evaluated (pixel, Gaussian) pairs of one frame (counting variant of the blend)
        ctx.set_profiling(True, count_pairs=True)
        step_fov()
        pairs = ctx.get_profile()["blend_pairs"]
        # stage times with the blend variant used for rendering
        ctx.set_profiling(True, count_pairs=False)
        ms_f_prof = timed(step_fov, args.steps)
        prof = ctx.get_profile()
        ctx.set_profiling(False)
        counts = ctx.get_counts()
        K = prof["sort_keys"] / max(1, args.steps)
        st = prof["stages"]
        for name, v in st.items():
            if v["launches"]:
                stages[name] = dict(ms_per_frame=v["ms"] / args.steps, launches_per_frame=v["launches"] / args.steps,
                                    ms_per_launch=v["ms"] / v["launches"])
        # sort pass: bytes per launch = SORT_BYTES_PER_KEY_PASS x keys
        sp = st["sort_pass"]
        if sp["launches"]:
            per_launch_s = sp["ms"] / sp["launches"] / 1000.0
            gbs = SORT_BYTES_PER_KEY_PASS * K / per_launch_s / 1e9
            stages["sort_pass"].update(bound="hbm", achieved_GBs=gbs, frac=gbs / HBM_PEAK_GBS,
                                       bytes_per_launch=SORT_BYTES_PER_KEY_PASS * K)
        bl = st["blend"]
        if bl["launches"]:
            per_launch_s = bl["ms"] / bl["launches"] / 1000.0
            tf = BLEND_FLOPS_PER_PAIR * pairs / per_launch_s / 1e12
            stages["blend"].update(bound="alu", achieved_TFLOPs=tf, frac=tf / FP32_VECTOR_PEAK_TF,
                                   pairs_per_launch=pairs)
        # views of the frame: per eye fovea, mid, periphery (selecting, every tile active)
        cnt = ctx.inspect("counts", torch.int32).view(-1, scene.n)
        nz = (cnt != 0).sum(dim=1).tolist()
        n_periph = sum(nz[2::3])
        n_ent = int(ctx.inspect("offsets", torch.int32).numel()) - 1  # entries that emit keys (kept)

        def hbm_stage(name, bytes_per_frame):
            v = st[name]
            if not v["launches"]:
                return
            gbs = bytes_per_frame / (v["ms"] / args.steps / 1000.0) / 1e9
            stages[name].update(bound="hbm", achieved_GBs=gbs, frac=gbs / HBM_PEAK_GBS,
                                bytes_per_launch=bytes_per_frame * args.steps / v["launches"])

        rect_views = 2 * len(cams) if fallback_on else 0  # each eye's fovea and periphery views
        hbm_stage("preprocess", PREPROCESS_READ_PER_GAUSSIAN * scene.n + PREPROCESS_WRITE_PER_SLOT * cnt.numel() +
                  PREPROCESS_WRITE_PER_EMITTING * sum(nz) + PREPROCESS_WRITE_PER_SCORE * n_periph +
                  PREPROCESS_WRITE_PER_RECT_SLOT * rect_views * scene.n)
        sh_bytes = 4 * int(np.prod(scene.sh.shape[:-1]))  # [coef][channel][n]
        hbm_stage("colour", n_ent * (RECORD_BYTES_PER_ENTRY + sh_bytes))
        hbm_stage("emit", EMIT_BYTES_PER_ENTRY * n_ent + EMIT_BYTES_PER_KEY * K)
        if st["net"]["launches"]:
            flop = net_frame_flop(np, W, H, gaze, rad[1])
            tf = flop / (st["net"]["ms"] / args.steps / 1000.0) / 1e12
            stages["net"].update(bound="mfma", achieved_TFLOPs=tf, frac=tf / BF16_MFMA_PEAK_TF, flop_per_frame=flop)
        # dominant kernel: the single-kernel stage with the most time per frame
        cand = [s_ for s_ in ("sort_pass", "blend", "preprocess", "colour") if "bound" in stages.get(s_, {})]
        dom = max(cand, key=lambda s_: stages[s_]["ms_per_frame"])
        d = stages[dom]
        variant = tuned["variant"] if tuned else 1  # the library's default variant when not tuned
        key = {"blend": ",".join(str(x) for x in pkg.blend_variant_desc(variant)),
               "preprocess": "k_preprocess", "colour": "k_entry_record", "sort_pass": "k_sort_scatter"}[dom]
        traffic = pmc_traffic(dom, key)
        if d["bound"] == "hbm":
            roofline = dict(kernel=dom, bound="hbm", achieved=d["achieved_GBs"], peak=HBM_PEAK_GBS, unit="GB/s",
                            frac=d["frac"], traffic=traffic, ms_per_launch=d["ms_per_launch"],
                            algorithmic_bytes=d["bytes_per_launch"])
        else:
            roofline = dict(kernel=dom, bound="alu", achieved=d["achieved_TFLOPs"], peak=FP32_VECTOR_PEAK_TF,
                            unit="TFLOP/s", frac=d["frac"], traffic=traffic, ms_per_launch=d["ms_per_launch"])
        log(f"profiled pass {ms_f_prof:.3f} ms/frame; stages: " +
            ", ".join(f"{k}={v['ms_per_frame']:.3f}ms" for k, v in stages.items()))

    legs = set(args.legs.split(",")) if args.legs != "all" else {"parts", "workloads", "incremental", "amr", "pipeline",
                                                                "upsampler", "net_training", "trace", "training"}
    training = train_leg(pkg, synth, torch, np, args.train_steps) if args.train_steps > 0 and "training" in legs \
        else None
    extra = {}
    if do_fov and do_frr and not args.no_extra:
        if "parts" in legs:
            extra["frame_parts"] = parts_leg(pkg, torch, ctx, ds, cams, gaze, rad, fov, out_r, args, timed, theta)
            method_options(ctx)
        if "workloads" in legs:
            extra["workloads"] = workloads_leg(pkg, synth, torch, ds, rad, fov, args, timed, nets)
        if "incremental" in legs:
            extra["incremental"] = incremental_leg(pkg, synth, torch, ds, cams, fov, rad, method_options)
        if "amr" in legs:
            extra["amr"] = amr_leg(pkg, torch, ctx, ds, cams, gaze, rad, out_r, args, timed,
                                   layered=dict(ms_per_frame=ms_f, periphery_psnr_db=min(psnr) if psnr else None))
        if "pipeline" in legs:
            extra["concurrent_pipeline"] = pipeline_leg(pkg, synth, torch, ds, cams, fov, method_options)
        if "upsampler" in legs:
            extra["upsampler_inference"] = upsampler_leg(pkg, synth, torch, np, ds, rad, fov, args, nets)
        if "net_training" in legs:
            extra["upsampler_training"] = net_train_leg(pkg, synth, torch, np, ctx, ds)
        if "trace" in legs:
            extra["gaze_trace"] = trace_leg(pkg, synth, torch, args)

    cpu = None
    if not args.no_cpu_baseline and do_fov:
        import oracle
        times = []
        for _ in range(max(1, args.cpu_frames)):
            t = time.perf_counter()
            oracle.render_foveated(scene, cams, gaze, rad)
            times.append(time.perf_counter() - t)
        med = statistics.median(times)
        cpu = dict(value=1.0 / med, unit="stereo frames/s", cores=oracle.default_threads(), kind="oracle",
                   sample=f"{len(times)} whole foveated stereo frames of the same workload (FP64 oracle, "
                          f"median {med:.2f} s/frame, {oracle.default_threads()} threads)")
        log(f"cpu oracle {med:.2f} s/frame")

    # the frame as served: the faster of the eager call and the graph replay (identical output)
    best_ms = ms_f if not (ms_g == ms_g) else min(ms_f, ms_g)
    res = {
        "metric": METRIC,
        "value": 1000.0 / best_ms if do_fov else None,
        "unit": "stereo frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": best_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "foveated stereo frame: 1M-Gaussian uniform cloud over [-5,5]^3, head at (0,0,-3), "
                        "2 eyes x 1832x1920, fovea r=0.15W full res, mid r=0.35W at 1/2, periphery at 1/4 with "
                        "top-30% subset, " + ("periphery through the learned x4 upsampler" if use_net else
                                              "periphery through bilinear x4 (the upsampler trained for this "
                                              "workload gains nothing on its held-out pairs)") +
                        ", per-tile error estimate with full-resolution fallback",
            "gaussians": scene.n, "width": W, "height": H, "eyes": 2, "gaze": "image centre",
            "key_path": "f64", "blend": "f32",
            "upsampler": dict(used=use_net, weights="paper_2507_04147_amd/weights/upsampler_inside",
                              held_out_psnr_db=nets["inside"]["held_out_psnr_db"]),
            "fallback": list(pkg.FALLBACK_NET if use_net else pkg.FALLBACK_BILINEAR),
        },
        "full_res_fps": 1000.0 / ms_r if do_frr else None,
        "full_res_ms": ms_r,
        "speedup_vs_full_res": (ms_r / best_ms) if (do_fov and do_frr) else None,
        "periphery_psnr_db": min(psnr) if psnr else None,
        "periphery_psnr_db_per_eye": psnr,
        "outer_psnr_db_per_eye": psnr_outer,
        "keys_foveated": counts.get("n_keys"),
        "fallback_tiles": counts.get("n_fallback_tiles"),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "stages": stages,
        "blend_autotune": tuned,
        "eager_ms_per_step": ms_f,
        "graph_ms_per_step": ms_g,
        "training": training,
        **extra,
    }
    print(json.dumps(res), flush=True)


NET_FLOP_PER_INPUT_PIXEL = 47808    # 2 x (3x32 + 32x32 + 32x48) x 9 multiply-adds
BF16_MFMA_PEAK_TF = 2500.0          # MI355X dense bf16


def _psnr_outside_fovea(ctx, W, H, gaze, rad, out, ref):
    vals = []
    for e in range(len(gaze)):
        sse, cnt = ctx.region_sse(W, H, gaze[e], rad[0], rad[1], out[e], ref[e])
        mse = (sse[1] + sse[2]) / (3.0 * (cnt[1] + cnt[2]))
        vals.append(math.inf if mse == 0 else 10 * math.log10(1.0 / mse))
    return vals


def net_frame_flop(np, W, H, gaze, r_mid):
    """Multiply-add FLOPs the upsampler must spend on one stereo frame: layer 3
    on every quarter-resolution pixel whose x4 block has a pixel centre outside
    r_mid (the composite's periphery), layers 2 and 1 on those pixels widened by
    one and two pixels (their receptive field)."""
    h, w = H // 4, W // 4
    total = 0
    for gx, gy in gaze:
        # farthest full-resolution pixel centre of each x4 block from the gaze
        fx = np.maximum(np.abs(4.0 * np.arange(w) + 0.5 - gx), np.abs(4.0 * np.arange(w) + 3.5 - gx))
        fy = np.maximum(np.abs(4.0 * np.arange(h) + 0.5 - gy), np.abs(4.0 * np.arange(h) + 3.5 - gy))
        need = (fy[:, None] ** 2 + fx[None, :] ** 2) > r_mid * r_mid
        n3 = int(need.sum())
        grown = need.copy()
        counts = []
        for _ in range(2):
            g = grown.copy()
            g[1:, :] |= grown[:-1, :]; g[:-1, :] |= grown[1:, :]
            g2 = g.copy()
            g2[:, 1:] |= g[:, :-1]; g2[:, :-1] |= g[:, 1:]
            grown = g2
            counts.append(int(grown.sum()))
        n2, n1 = counts
        total += 2 * 9 * (3 * 32 * n1 + 32 * 32 * n2 + 32 * 48 * n3)
    return total


def load_net(pkg, torch, workload):
    """The committed upsampler weights of a workload and whether the frame uses
    them: only when the network beats bilinear on its held-out pairs."""
    from paper_2507_04147_amd import upsampler as U
    theta, head = U.load_weights(os.path.join(ROOT, "paper_2507_04147_amd", "weights", f"upsampler_{workload}"))
    p = head["held_out_psnr_db"]
    return dict(theta=torch.from_numpy(theta).cuda(), use=p["network"] > p["bilinear"] + 0.1, held_out_psnr_db=p,
                pairs=head["pairs"], epochs=head["epochs"])


FRAME_OPTIONS = (("bilinear", False, None), ("bilinear+fallback", False, "bilinear"), ("network", True, None),
                 ("network+fallback", True, "net"))


def set_frame_options(pkg, c, theta, net, fb):
    c.set_upsampler(theta if net else None)
    if fb is None:
        c.set_fallback(float("inf"), 1.0, 1.0)
    else:
        c.set_fallback(*(pkg.FALLBACK_NET if fb == "net" else pkg.FALLBACK_BILINEAR))


def parts_leg(pkg, torch, ctx, ds, cams, gaze, rad, fov, out_r, args, timed, theta):
    """The foveated frame with and without each of the method's additions:
    bilinear periphery, with the error estimate, the network trained for this
    workload, both (ms per frame, periphery PSNR, fallback tiles)."""
    W, H = cams[0].width, cams[0].height
    out = torch.empty((2, 3, H, W), device="cuda")
    res = {}
    for name, net, fb in FRAME_OPTIONS:
        set_frame_options(pkg, ctx, theta, net, fb)
        step = lambda: ctx.render_foveated(ds, cams, gaze, fov, out)
        for _ in range(args.warmup):
            step()
        ms = timed(step, args.steps)
        res[name] = dict(ms_per_frame=ms, periphery_psnr_db=min(_psnr_outside_fovea(ctx, W, H, gaze, rad, out, out_r)),
                         fallback_tiles=ctx.get_counts()["n_fallback_tiles"])
        log(f"frame {name}: {ms:.3f} ms")
    return res


def workloads_leg(pkg, synth, torch, ds, rad, fov, args, timed, nets):
    """Both workloads -- the head inside the cloud (0,0,-3) and the camera
    outside it (0,0,-15) -- at args.gazes seeded gazes within 20 degrees (the
    first at the image centre): for each periphery option (bilinear, with the
    error estimate, the workload's network, both) the frame time, the periphery
    PSNR against the full-resolution render (minimum over the eyes) and the
    fallback tiles; the full-resolution frame time of the pose."""
    import statistics as stats
    res = {}
    for w, head in (("inside", synth.HEAD_INSIDE), ("outside", synth.HEAD_OUTSIDE)):
        _, cams = synth.foveated_stereo(n=1, head=head)
        W, H = cams[0].width, cams[0].height
        gazes = synth.gaze_points(21, args.gazes, cams[0])
        c = pkg.Context()
        out = torch.empty((2, 3, H, W), device="cuda")
        ref = torch.empty_like(out)
        step_r = lambda: c.render_full(ds, cams, ref)
        for _ in range(2):
            step_r()
        ms_frr = timed(step_r, max(3, args.steps // 4))
        rows = {name: [] for name, _, _ in FRAME_OPTIONS}
        for g in gazes:
            gz = [g, g]
            for name, net, fb in FRAME_OPTIONS:
                set_frame_options(pkg, c, nets[w]["theta"], net, fb)
                step = lambda: c.render_foveated(ds, cams, gz, fov, out)
                for _ in range(2):
                    step()
                ms = timed(step, max(3, args.steps // 4))
                rows[name].append((ms, min(_psnr_outside_fovea(c, W, H, gz, rad, out, ref)),
                                   c.get_counts()["n_fallback_tiles"]))
        c.close()
        ntiles = 2 * ((W // 4 + 15) // 16) * ((H // 4 + 15) // 16)
        summ = {}
        for name, r in rows.items():
            summ[name] = dict(ms_median=stats.median(x[0] for x in r), psnr_min_db=min(x[1] for x in r),
                              psnr_median_db=stats.median(x[1] for x in r),
                              fallback_tile_fraction_mean=stats.mean(x[2] for x in r) / ntiles,
                              centre_gaze=dict(ms=r[0][0], psnr_db=r[0][1], fallback_tiles=r[0][2]))
        best = max((n_ for n_ in summ if summ[n_]["psnr_min_db"] >= 30.0),
                   key=lambda n_: 1.0 / summ[n_]["ms_median"], default=None)
        res[w] = dict(head=list(head), gazes=len(gazes), full_res_ms=ms_frr, options=summ,
                      network=dict(used_by_method=nets[w]["use"], held_out_psnr_db=nets[w]["held_out_psnr_db"],
                                   pairs=nets[w]["pairs"], epochs=nets[w]["epochs"]),
                      fastest_option_at_30db=best,
                      speedup_vs_full_res=(ms_frr / summ[best]["ms_median"]) if best else None)
        log(f"workload {w}: FRR {ms_frr:.3f} ms; " + "; ".join(
            f"{n_} {v['ms_median']:.3f} ms, PSNR min {v['psnr_min_db']:.2f} dB, fallback "
            f"{v['fallback_tile_fraction_mean']:.3f}" for n_, v in summ.items()))
    return res


def upsampler_leg(pkg, synth, torch, np, ds, rad, fov, args, nets):
    """The upsampler's inference forward (one fused launch): on the stereo
    periphery layer as a whole (a3fr_net_forward, 2 x 3 x H/4 x W/4 -> 4x) and
    as the foveated frame runs it (the camera-outside workload, whose network
    the method uses, centre gaze: tiles and units within r_mid skipped, only the
    periphery written), timed alone: the frame's network stage from a profiled
    frame (one stream).  FLOPs count the multiply-adds the method must spend
    (every pixel, resp. net_frame_flop)."""
    _, cams = synth.foveated_stereo(n=1, head=synth.HEAD_OUTSIDE)
    W, H = cams[0].width, cams[0].height
    theta = nets["outside"]["theta"]
    c = pkg.Context()
    x = torch.rand((2, 3, H // 4, W // 4), device="cuda", generator=torch.Generator(device="cuda").manual_seed(5))
    y = torch.empty((2, 3, H, W), device="cuda")
    n = max(5, args.steps)
    for _ in range(3):
        c.net_forward(theta, x, y, False)
    c.sync()
    t = time.perf_counter()
    for _ in range(n):
        c.net_forward(theta, x, y, False)
    c.sync()
    ms_whole = (time.perf_counter() - t) * 1000.0 / n
    flop_whole = NET_FLOP_PER_INPUT_PIXEL * 2 * (H // 4) * (W // 4)
    gz = [(cams[0].cx, cams[0].cy)] * 2
    out = torch.empty((2, 3, H, W), device="cuda")
    set_frame_options(pkg, c, theta, True, None)
    c.render_foveated(ds, cams, gz, fov, out)
    c.set_profiling(True, count_pairs=False)
    for _ in range(n):
        c.render_foveated(ds, cams, gz, fov, out)
    c.sync()
    st = c.get_profile()["stages"]["net"]
    c.set_profiling(False)
    c.close()
    ms_frame = st["ms"] / n
    flop_frame = net_frame_flop(np, W, H, gz, rad[1])

    def rate(flop, ms):
        tf = flop / (ms / 1000.0) / 1e12
        return dict(bound="mfma", achieved_TFLOPs=tf, peak_TFLOPs=BF16_MFMA_PEAK_TF, frac=tf / BF16_MFMA_PEAK_TF)

    res = dict(kernel="k_net_fused",
               whole_layer=dict(us_per_forward=ms_whole * 1000.0, flop=flop_whole, **rate(flop_whole, ms_whole)),
               frame_stage=dict(us_per_frame=ms_frame * 1000.0, launches_per_frame=st["launches"] / n,
                                flop=flop_frame, **rate(flop_frame, ms_frame)))
    log(f"upsampler: whole layer {ms_whole * 1000:.1f} us ({res['whole_layer']['achieved_TFLOPs']:.0f} TFLOP/s); "
        f"frame stage {ms_frame * 1000:.1f} us ({res['frame_stage']['achieved_TFLOPs']:.0f} TFLOP/s)")
    return res


def pipeline_leg(pkg, synth, torch, ds, cams, fov, method_options, n_trials=6, tracker_threads=8):
    """Algorithm 1 with the early-exit ViT (random weights, 640 x 400 eye
    image) running on this host's CPU beside the renderer, which renders round
    0 at once and then incremental rounds on the newest prediction; the
    renderer's waits sleep (a3fr_set_host_wait) so that the tracker keeps the
    CPU.  Latency with sensing and transfer T_s = T_c = 1 ms (Sec. 3.1):
    T_s + T_c + max(T_d, T_r) against the sequential T_s + T_c + T_d + T_r,
    with T_d the tracker alone and T_r the foveated frame rendered after the
    last prediction (medians over trials).
      * per pruning ratio 0 / 10% / 20% of tokens per block;
      * the paper's load experiment (Sec. 4.5): processes taking the CPU with
        utilisation alternating between 50% and 100% every 0.1 s, A3FR with
        and without speculative rounds (without: after a round the renderer
        waits for the next prediction);
      * a stand-in tracker publishing at the paper's per-exit latencies
        (Table 2, Orin CPU).
    The tracker is a process of its own (Algorithm 1's two processes: it shares
    no interpreter lock with the renderer) on tracker_threads CPU threads in
    both pipelines, leaving the renderer's host thread a core."""
    import statistics as stats
    from paper_2507_04147_amd import pipeline
    W, H = cams[0].width, cams[0].height
    trials, sig = synth.gaze_exits(seed=71, n_trials=n_trials, width=W, height=H)
    c = pkg.Context()
    method_options(c)
    c.set_fallback(float("inf"), 1.0, 1.0)
    c.set_host_wait(True)
    out = torch.empty((2, 3, H, W), device="cuda")
    t_sc = 2.0

    def frame_ms(final):
        t = time.perf_counter()
        c.render_foveated(ds, cams, final, fov, out)
        c.sync()
        return (time.perf_counter() - t) * 1000.0

    def measure(tracker, speculative=True, exit_ms=None):
        """Medians over the trials; tracker: a TrackerProcess (the ViT in its own
        process) or None (the stand-in publishing at exit_ms)."""
        rows = []
        for final, exits in trials:
            if tracker is not None:
                t = time.perf_counter()
                t_d = (tracker.run_alone(len(exits) + 1)[-1] - t) * 1000.0
            else:
                t_d = exit_ms[-1]
            sfr = frame_ms(final)
            if tracker is not None:
                r = pipeline.run_process(c, ds, cams, fov, exits, final, sig, tracker, out=out,
                                         speculative=speculative)
            else:
                r = pipeline.run(c, ds, cams, fov, exits, final, sig, exit_ms, out=out, speculative=speculative)
            rows.append(dict(t_d=t_d, beside=r["exit_ms"][-1], done=r["render_done_ms"], sfr=sfr,
                             rounds=len(r["events"]) - 2))
        med = lambda k: stats.median(x[k] for x in rows)
        a3fr, seq = t_sc + med("done"), t_sc + med("t_d") + med("sfr")
        return dict(tracker_alone_ms=med("t_d"), tracker_beside_renderer_ms=med("beside"),
                    render_after_last_prediction_ms=med("done") - med("beside"), sequential_render_ms=med("sfr"),
                    total_latency_ms=a3fr, sequential_total_latency_ms=seq, speedup=seq / a3fr,
                    incremental_rounds=med("rounds"))

    for _ in range(2):  # warm-up of the frame and the network
        frame_ms(trials[0][0])
    threads = min(tracker_threads, torch.get_num_threads())
    res = dict(tracker_threads=threads, host_threads=torch.get_num_threads())
    vit = {}
    for prune in (0.0, 0.1, 0.2):
        tr = pipeline.TrackerProcess(prune=prune, seed=5, threads=threads)
        try:
            tr.run_alone(6)
            vit[f"prune_{prune:g}"] = m = measure(tr)
        finally:
            tr.close()
        log(f"Algorithm 1, ViT on the CPU (prune {prune:g}): total {m['total_latency_ms']:.2f} ms vs sequential "
            f"{m['sequential_total_latency_ms']:.2f} ms (tracker {m['tracker_alone_ms']:.2f} ms alone, "
            f"{m['tracker_beside_renderer_ms']:.2f} ms beside the renderer)")
    res["cpu_tracker"] = vit
    tr = pipeline.TrackerProcess(prune=0.0, seed=5, threads=threads)
    try:
        tr.run_alone(6)
        with pipeline.CpuLoad(torch.get_num_threads()):
            spec = measure(tr, speculative=True)
            nospec = measure(tr, speculative=False)
    finally:
        tr.close()
    res["cpu_load_50_100"] = dict(load_processes=torch.get_num_threads(), period_s=0.1, speculative=spec,
                                  without_speculative=nospec)
    log(f"Algorithm 1 under CPU load (50%/100% every 0.1 s): total {spec['total_latency_ms']:.2f} ms with "
        f"speculative rounds, {nospec['total_latency_ms']:.2f} ms without; sequential "
        f"{spec['sequential_total_latency_ms']:.2f} ms")
    res["stand_in_table2"] = m = measure(None, exit_ms=list(synth.EXIT_LATENCY_MS))
    log(f"Algorithm 1, stand-in tracker at the paper's exit latencies: total {m['total_latency_ms']:.2f} ms vs "
        f"sequential {m['sequential_total_latency_ms']:.2f} ms")
    c.close()
    return res


def amr_leg(pkg, torch, ctx, ds, cams, gaze, rad, out_r, args, timed, layered=None):
    """AMR levels (Sec. 3.4) as the alternative foveation mode: one
    full-resolution view per eye, 2 x 2 blocks rendered at 4..1 positions by
    eccentricity (within r_f, (r_f + r_m)/2, r_m and beyond), by the tile's
    Gaussian count (the densest quarter, half, three quarters of a view's tiles
    at levels 4, 3, 2) or the smaller of the two; unrendered positions
    inherited or interpolated.  Frame time and periphery PSNR against the
    full-resolution render, beside the layered frame's (layered: its ms and
    PSNR) for the equal-quality comparison."""
    W, H = cams[0].width, cams[0].height
    radii = (rad[0], 0.5 * (rad[0] + rad[1]), rad[1])
    out = torch.empty((2, 3, H, W), device="cuda")
    configs = [("eccentricity/inherit", 0, 0), ("eccentricity/interpolate", 0, 1), ("count/interpolate", 1, 1),
               ("min/interpolate", 2, 1)]
    res = dict(radii=list(radii), count_fractions=[0.25, 0.5, 0.75], layered=layered, modes={})
    for name, mode, fill in configs:
        amr = pkg.amr_struct(*radii, mode=mode, fill=fill)
        step = lambda: ctx.render_amr(ds, cams, gaze, amr, out)
        for _ in range(args.warmup):
            step()
        ms = timed(step, args.steps)
        psnr = min(_psnr_outside_fovea(ctx, W, H, gaze, rad, out, out_r))
        res["modes"][name] = dict(ms_per_frame=ms, periphery_psnr_db=psnr)
        log(f"AMR {name}: frame {ms:.3f} ms, periphery PSNR {psnr:.2f} dB")
    # the first configuration keeps the flat fields of the leg
    res.update(ms_per_frame=res["modes"]["eccentricity/inherit"]["ms_per_frame"],
               periphery_psnr_db=res["modes"]["eccentricity/inherit"]["periphery_psnr_db"])
    return res


def incremental_leg(pkg, synth, torch, ds, cams, fov, rad, method_options, n_trials=8):
    """Incremental foveal rounds (Sec. 3.3) on the benchmark frame, driven by a
    seeded early-exit gaze stream (Table 2 spreads): round 0 (projection and
    periphery) before any gaze, per exit a round at r_f - E (Eq. 4) and its
    speculative growth to r_f + E (Eq. 5), the final round and composite at
    the last prediction.  Compared with the sequential frame (the whole
    foveated frame rendered after the last prediction, same options: the
    upsampler, no fallback): the time left after the last prediction."""
    import statistics as stats
    from paper_2507_04147_amd import incremental as inc
    W, H = cams[0].width, cams[0].height
    trials, sig = synth.gaze_exits(seed=61, n_trials=n_trials, width=W, height=H)
    c = pkg.Context()
    method_options(c)
    c.set_fallback(float("inf"), 1.0, 1.0)
    out = torch.empty((2, 3, H, W), device="cuda")

    def gpu_ms(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1000.0

    for _ in range(2):  # warm-up
        inc.run_frame(c, ds, cams, fov, inc.schedule(trials[0][1], sig, rad[0]), trials[0][0], out)
        c.render_foveated(ds, cams, trials[0][0], fov, out)
    rows = []
    for final, exits in trials:
        steps = inc.run_frame(c, ds, cams, fov, inc.schedule(exits, sig, rad[0]), final, out, timed=gpu_ms)
        sfr = gpu_ms(lambda: c.render_foveated(ds, cams, final, fov, out))
        one = c.get_counts()
        rows.append(dict(begin=steps[0]["ms"], rounds=sum(s["ms"] for s in steps[1:-1]), finish=steps[-1]["ms"],
                         sfr=sfr, tiles=sum(s["tiles"] for s in steps), tiles_one_shot=one["n_active_tiles"],
                         finish_tiles=steps[-1]["tiles"], steps=[(s["step"], round(s["radius"] or 0.0, 1),
                                                                 s["tiles"], s["keys"]) for s in steps]))
    c.close()
    med = lambda k: stats.median(r[k] for r in rows)
    res = dict(trials=n_trials, exits=len(sig), exit_latency_ms=list(synth.EXIT_LATENCY_MS),
               begin_ms=med("begin"), rounds_ms=med("rounds"), finish_ms=med("finish"), sequential_frame_ms=med("sfr"),
               latency_ratio_after_last_gaze=med("sfr") / med("finish"),
               extra_fovea_tiles=stats.median(r["tiles"] - r["tiles_one_shot"] for r in rows),
               finish_tiles=med("finish_tiles"), example_steps=rows[0]["steps"])
    log(f"incremental rounds: begin {res['begin_ms']:.3f} ms, rounds {res['rounds_ms']:.3f} ms, finish "
        f"{res['finish_ms']:.3f} ms after the last prediction vs {res['sequential_frame_ms']:.3f} ms sequential")
    return res


def net_train_leg(pkg, synth, torch, np, ctx, ds, n_pairs=2048, epochs=2, batch=32):
    """Training throughput of the upsampler: pairs rendered by the library at
    the camera-outside training poses (each a 256x256 full-resolution crop and
    its frame's whole periphery layer, cut to 64x64), Adam steps of batch 32."""
    from paper_2507_04147_amd import upsampler as U
    torch.cuda.synchronize()
    t = time.perf_counter()
    xs, ts = U.make_pairs(ctx, ds, synth.crop_poses_outside(41, n_pairs))
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t
    net = U.Upsampler(ctx, synth.net_init(42))
    net.fit(xs[:256], ts[:256], epochs=1, batch=batch)  # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    net.fit(xs, ts, epochs=epochs, batch=batch)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t
    steps = epochs * (n_pairs // batch)
    flop = 3 * 64 * 64 * NET_FLOP_PER_INPUT_PIXEL * batch * steps  # forward + input and weight gradients
    tf = flop / train_s / 1e12
    log(f"upsampler training: {n_pairs} pairs rendered in {gen_s:.2f} s; {steps} steps in {train_s:.2f} s "
        f"({tf:.1f} TFLOP/s)")
    return dict(pairs=n_pairs, pair_render_s=gen_s, pairs_per_s=n_pairs / gen_s, steps=steps, batch=batch,
                step_ms=1000.0 * train_s / steps, achieved_TFLOPs=tf, frac=tf / BF16_MFMA_PEAK_TF)


def trace_leg(pkg, synth, torch, args, n=3_000_000, n_frames=64):
    """Batched gaze trace: a 3M-Gaussian cloud over [-5,5]^3, 64 frames of a
    seeded gaze walk with head drift, rendered as windows of stereo frames
    (2 eyes x 3 layers per frame, uneven tile counts) in one preprocess / sort /
    blend each, every window replayed from one captured HIP graph."""
    win = max(1, min(args.trace_window, 64))
    scene, _ = synth.foveated_stereo(n=n, seed=3)
    ds = pkg.DeviceScene.from_host(scene)
    del scene
    trace = synth.gaze_trace(seed=31, n_frames=n_frames)
    W, H = trace[0][0][0].width, trace[0][0][0].height
    fov = pkg.fovea_struct(synth.FOVEA_FRACTIONS[0] * W, synth.FOVEA_FRACTIONS[1] * W, keep=synth.PERIPH_KEEP)
    wins = [trace[k:k + win] for k in range(0, n_frames, win)]
    flat = [([c for f in w for c in f[0]], [g for f in w for g in f[1]]) for w in wins]
    ctx = pkg.Context()
    out = torch.empty((2 * win, 3, H, W), device="cuda")
    keys = 0
    for cams, gz in flat:
        ctx.render_foveated(ds, cams, gz, fov, out[:len(cams)])
        keys = max(keys, ctx.get_counts()["n_keys"])
    ctx.graph_capture(ds, flat[0][0], flat[0][1], fov, out, min(int(keys * 1.2) + 4096, (1 << 32) - 1))
    for cams, gz in flat:
        ctx.graph_launch(cams, gz)
    ctx.sync()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for cams, gz in flat:
        ctx.graph_launch(cams, gz)
    ctx.sync()
    torch.cuda.synchronize()
    s = time.perf_counter() - t
    ctx.graph_destroy()
    ctx.close()
    log(f"gaze trace: {n_frames} stereo frames of {n} Gaussians in windows of {win}: {s * 1000:.1f} ms "
        f"({n_frames / s:.1f} frames/s), max {keys} keys per window")
    return dict(gaussians=n, frames=n_frames, window=win, views_per_launch=6 * win, max_keys_per_window=keys,
                ms_total=s * 1000.0, stereo_frames_per_s=n_frames / s)


def train_leg(pkg, synth, torch, np, steps):
    """Differentiable-render training step: 500,000 Gaussians at 1024 x 1024,
    L1 loss against the render of the scene with perturbed means and logits,
    Adam on all five parameter groups.  One step = activation, preprocess, key
    sort, blend, loss, reverse blend, reverse projection, Adam update."""
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
    opt = torch.optim.Adam(ts, lr=1e-3)
    losses = []

    def step():
        opt.zero_grad(set_to_none=False)
        rgb = train.render(a3, v, *ts)
        loss = (rgb - target).abs().mean()
        loss.backward()
        opt.step()
        return loss

    for _ in range(3):
        losses.append(float(step().detach()))
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        loss = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1000.0 / steps
    losses.append(float(loss.detach()))
    log(f"training step {ms:.3f} ms (L1 {losses[0]:.5f} -> {losses[-1]:.5f})")

    # one profiled step through the C entry points, keeping T and last
    H, W = cam.height, cam.width
    n = sc.n
    with torch.no_grad():
        pr = pkg.params_struct(n, 3, *[x.detach() for x in ts])
        scale, opac = torch.empty_like(ts[1]), torch.empty_like(ts[3])
        rgb = torch.empty((3, H, W), device="cuda")
        Tt = torch.empty((H, W), device="cuda")
        last = torch.empty((H, W), dtype=torch.int32, device="cuda")
        g = [torch.empty_like(x) for x in ts]
        a3.set_profiling(True, count_pairs=False)
        for _ in range(steps):
            a3.activate(pr, scale, opac)
            a3.preprocess(pkg.DeviceScene(ts[0].detach(), scale, ts[2].detach(), opac, ts[4].detach()), [v])
            a3.bin_sort()
            a3.blend(rgb, Tt, last)
            dl = torch.sign(rgb - target) / rgb.numel()
            a3.blend_backward(dl, Tt, last)
            a3.preprocess_backward(pr, *g)
        prof = a3.get_profile()
        a3.set_profiling(False)
        pairs_bwd = int(last.to(torch.int64).sum().item())
        drawn = int((a3.inspect("counts", torch.int32) != 0).sum().item())
    st = {}
    for name, rec in prof["stages"].items():
        if rec["launches"]:
            st[name] = dict(ms_per_step=rec["ms"] / steps, ms_per_launch=rec["ms"] / rec["launches"])
    bb = st.get("blend_bwd")
    if bb:
        tf = BLEND_BWD_FLOPS_PER_PAIR * pairs_bwd / (bb["ms_per_launch"] / 1000.0) / 1e12
        bb.update(bound="alu", pairs_per_launch=pairs_bwd, achieved_TFLOPs=tf, frac=tf / FP32_VECTOR_PEAK_TF)
    pb = st.get("preprocess_bwd")
    if pb:
        byts = PREPROCESS_BWD_BYTES_PER_GAUSSIAN * n + PREPROCESS_BWD_BYTES_PER_DRAWN * drawn
        gbs = byts / (pb["ms_per_launch"] / 1000.0) / 1e9
        pb.update(bound="hbm", bytes_per_launch=byts, achieved_GBs=gbs, frac=gbs / HBM_PEAK_GBS)
    a3.close()
    return dict(workload="differentiable render: 500k-Gaussian uniform cloud over [-1,1]^3, 1024x1024, L1 vs "
                         "perturbed target, Adam", ms_per_step=ms, steps_per_s=1000.0 / ms,
                l1_first=losses[0], l1_last=losses[-1], stages=st)


if __name__ == "__main__":
    main()
