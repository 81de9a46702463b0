"""Host logic of the fallback calibration (CPU only): the coefficient it picks
flags the fewest tiles, in order of dT^2, that keep every calibration frame's
periphery PSNR at or above the target plus the margin."""
import math

import numpy as np

from paper_2507_04147_amd.calibrate_fallback import calibrate, frame_psnr


def _frames(seed, n=6, tiles=200):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        dT2 = rng.uniform(0.0, 1.0, tiles)
        cnt = np.full(tiles, 4096.0)
        mse = 1.5e-3 * dT2 + rng.uniform(0.0, 4e-4, tiles)  # error grows with dT^2, with noise
        out.append(dict(dT2=dT2, sse=mse * 3.0 * cnt, cnt=cnt, mid_sse=3.0 * 20000 * 1e-5, mid_cnt=20000))
    return out


def test_frame_psnr_counts_only_the_tiles_left():
    f = dict(dT2=np.array([0.1, 0.9]), sse=np.array([3.0, 30.0]), cnt=np.array([100.0, 100.0]), mid_sse=0.0,
             mid_cnt=100)
    assert math.isclose(frame_psnr(f, math.inf), 10 * math.log10(900.0 / 33.0))
    assert math.isclose(frame_psnr(f, 0.5), 10 * math.log10(900.0 / 3.0))   # the 0.9 tile falls back
    assert frame_psnr(f, 0.0) == math.inf                                     # every tile falls back


def test_calibration_is_the_smallest_sufficient_set():
    frames = _frames(3)
    res = calibrate(frames, 1e-3, 30.0, 1.0)
    q = res["dT2_threshold"]
    assert 0.0 < q < 1.0 and math.isclose(res["coef"], 1e-3 / q)
    assert min(frame_psnr(f, q) for f in frames) >= 31.0
    # the next larger dT^2 value (one tile fewer flagged) misses the target
    F = np.unique(np.concatenate([f["dT2"] for f in frames]))
    nxt = F[F > q].min()
    assert min(frame_psnr(f, nxt) for f in frames) < 31.0
    assert res["psnr_before_db"]["min"] < 31.0 <= res["psnr_after_db"]["min"]


def test_calibration_flags_nothing_when_every_frame_passes():
    frames = _frames(4)
    for f in frames:
        f["sse"] *= 1e-3
    res = calibrate(frames, 1e-3, 30.0, 1.0)
    assert res["coef"] == 0.0 and res["flagged_fraction"] == 0.0
