"""Seeded synthetic inputs shared by the HIP path's tests/bench and the CPU oracle.

This module only draws inputs: Gaussian clouds, pinhole cameras and gaze points.
It holds none of the renderer's arithmetic (no projection, no colour, no blending),
so that the oracle and the GPU path can both take their inputs from it without
sharing any of the method.

The paper renders trained 3DGS scenes (Tanks & Temples, Deep Blending; Sec. 4.1).
Those are not available, so seeded uniform Gaussian clouds of the same parameter
layout stand in (Sec. 2.3 describes the representation: position, anisotropic
scale, rotation, opacity and spherical-harmonic colour per point).

Layout (structure of arrays, float32, as the GPU loads it):
  mean[3][N], scale[3][N] (already exp(log_scale)), quat[4][N] as (w, x, y, z),
  opacity[N] (already sigmoid(logit)), sh[16][3][N] (coefficient, channel, point).
The raw draws (log_scale, logit) are kept too, for the differentiable render.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SH_COEFFS = 16  # degree 3


@dataclass
class Scene:
    n: int
    mean: np.ndarray       # f32 [3][N]
    log_scale: np.ndarray  # f32 [3][N]
    scale: np.ndarray      # f32 [3][N]
    quat: np.ndarray       # f32 [4][N] (w, x, y, z), unit norm up to f32 rounding
    logit: np.ndarray      # f32 [N]
    opacity: np.ndarray    # f32 [N]
    sh: np.ndarray         # f32 [16][3][N]

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(
            n=int(idx.size),
            mean=np.ascontiguousarray(self.mean[:, idx]),
            log_scale=np.ascontiguousarray(self.log_scale[:, idx]),
            scale=np.ascontiguousarray(self.scale[:, idx]),
            quat=np.ascontiguousarray(self.quat[:, idx]),
            logit=np.ascontiguousarray(self.logit[idx]),
            opacity=np.ascontiguousarray(self.opacity[idx]),
            sh=np.ascontiguousarray(self.sh[:, :, idx]),
        )


def make_scene(n: int, half_extent: float, seed: int,
               log_scale_mean: float = -3.0, log_scale_std: float = 0.5,
               sh_std: float = 0.3) -> Scene:
    """Uniform cloud: mean ~ U[-h,h]^3, log-scale ~ N(-3,0.5) per axis, quaternion
    uniform on S^3 (normal draw then normalised), logit ~ N(0,1), 48 SH
    coefficients ~ N(0,0.3). Draw order: means, log-scales, quaternions, logits, SH.
    Values are drawn in float64 and rounded once to float32; the activated
    scale/opacity are the float64 exp/sigmoid of the drawn values, rounded once."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mean = rng.uniform(-half_extent, half_extent, size=(3, n))
    log_s = rng.normal(log_scale_mean, log_scale_std, size=(3, n))
    q = rng.normal(0.0, 1.0, size=(4, n))
    q = q / np.sqrt((q * q).sum(axis=0, keepdims=True))
    logit = rng.normal(0.0, 1.0, size=n)
    sh = rng.normal(0.0, sh_std, size=(SH_COEFFS, 3, n))
    log_s32 = log_s.astype(np.float32)
    logit32 = logit.astype(np.float32)
    return Scene(
        n=n,
        mean=mean.astype(np.float32),
        log_scale=log_s32,
        scale=np.exp(log_s32.astype(np.float64)).astype(np.float32),
        quat=q.astype(np.float32),
        logit=logit32,
        opacity=(1.0 / (1.0 + np.exp(-logit32.astype(np.float64)))).astype(np.float32),
        sh=sh.astype(np.float32),
    )


@dataclass
class Camera:
    """Pinhole camera, OpenCV axes (x right, y down, z forward).
    World->camera: p = R @ x + t. Pixel (i, j) is sampled at (i + 0.5, j + 0.5)."""
    R: np.ndarray          # f64 [3][3]
    t: np.ndarray          # f64 [3]
    campos: np.ndarray     # f64 [3], camera centre in world space
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    bg: tuple = (0.0, 0.0, 0.0)


def rot_yaw_pitch(yaw_deg: float, pitch_deg: float) -> np.ndarray:
    """Camera-to-world rotation for a head turned by yaw (about +y) then pitch
    (about +x): R_c2w = R_y(yaw) @ R_x(pitch)."""
    a, b = math.radians(yaw_deg), math.radians(pitch_deg)
    ry = np.array([[math.cos(a), 0.0, math.sin(a)], [0.0, 1.0, 0.0], [-math.sin(a), 0.0, math.cos(a)]])
    rx = np.array([[1.0, 0.0, 0.0], [0.0, math.cos(b), -math.sin(b)], [0.0, math.sin(b), math.cos(b)]])
    return ry @ rx


def make_camera(width: int, height: int, fov_x_deg: float, position, c2w=None,
                bg=(0.0, 0.0, 0.0)) -> Camera:
    """Square-pixel pinhole camera with the horizontal field of view on the width;
    principal point at the image centre."""
    c2w = np.eye(3) if c2w is None else np.asarray(c2w, dtype=np.float64)
    pos = np.asarray(position, dtype=np.float64)
    R = c2w.T.copy()
    t = -(R @ pos)
    f = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    return Camera(R=R, t=t, campos=pos.copy(), fx=f, fy=f, cx=width / 2.0, cy=height / 2.0,
                  width=width, height=height, bg=tuple(float(x) for x in bg))


def stereo_cameras(head, width, height, fov_x_deg, c2w=None, ipd=0.064):
    """Two parallel-axis eye cameras at head -/+ ipd/2 along the camera's right axis."""
    c2w = np.eye(3) if c2w is None else np.asarray(c2w, dtype=np.float64)
    right = c2w[:, 0]
    head = np.asarray(head, dtype=np.float64)
    return [make_camera(width, height, fov_x_deg, head + s * 0.5 * ipd * right, c2w) for s in (-1.0, 1.0)]


def gaze_points(seed: int, n: int, cam: Camera, ecc_max_deg: float = 20.0):
    """n seeded gaze points (pixel coordinates) uniform in eccentricity disc of
    ecc_max_deg around the optical axis; the first is the image centre."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = [(cam.cx, cam.cy)]
    while len(pts) < n:
        ecc = math.radians(ecc_max_deg) * math.sqrt(rng.uniform())
        ang = rng.uniform(0.0, 2.0 * math.pi)
        tx, ty = math.tan(ecc) * math.cos(ang), math.tan(ecc) * math.sin(ang)
        pts.append((cam.cx + cam.fx * tx, cam.cy + cam.fy * ty))
    return pts


# ---------------------------------------------------------------------------
# The workloads, with the sizes of the rendering configurations.
# ---------------------------------------------------------------------------

def single_view(n=10_000, size=256, seed=1):
    """Single view, no foveation: n Gaussians in [-1,1]^3, camera at z=-3 looking
    +z, 60 degree horizontal FOV, size x size, black background."""
    scene = make_scene(n, 1.0, seed)
    cam = make_camera(size, size, 60.0, (0.0, 0.0, -3.0))
    return scene, cam


HEAD_INSIDE = (0.0, 0.0, -3.0)    # the VR reading: the head inside the [-5,5]^3 cloud
HEAD_OUTSIDE = (0.0, 0.0, -15.0)  # the secondary row: the whole cloud in front of the eyes


def foveated_stereo(n=1_000_000, width=1832, height=1920, seed=2, half_extent=5.0, head=HEAD_INSIDE):
    """Foveated stereo frame: n Gaussians over [-h,h]^3, head at `head` (by
    default (0,0,-3), inside the cloud) looking +z, eyes 64 mm apart, width x
    height per eye. Returns scene and two cameras."""
    scene = make_scene(n, half_extent, seed)
    cams = stereo_cameras(head, width, height, 60.0)
    return scene, cams


FOVEA_FRACTIONS = (0.15, 0.35)   # fovea and mid radii as fractions of the image width
PERIPH_KEEP = (3, 10)            # periphery keeps ceil(3/10 of the visible points)


def differentiable(n=500_000, size=1024, seed=5):
    """Differentiable render: n Gaussians in [-1,1]^3 (the single-view recipe),
    camera at z=-3 looking +z, 60 degree horizontal FOV, size x size."""
    scene = make_scene(n, 1.0, seed)
    cam = make_camera(size, size, 60.0, (0.0, 0.0, -3.0))
    return scene, cam


def perturbed(scene: Scene, seed=51, mean_std=0.01, logit_std=0.1) -> Scene:
    """The optimisation target: a copy of the scene with means + N(0, mean_std)
    and opacity logits + N(0, logit_std) (drawn in that order, float64, added to
    the float32 values and rounded once); the opacity is re-activated like
    make_scene does."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dm = rng.normal(0.0, mean_std, size=scene.mean.shape)
    dl = rng.normal(0.0, logit_std, size=scene.logit.shape)
    logit = (scene.logit.astype(np.float64) + dl).astype(np.float32)
    return Scene(
        n=scene.n,
        mean=(scene.mean.astype(np.float64) + dm).astype(np.float32),
        log_scale=scene.log_scale.copy(),
        scale=scene.scale.copy(),
        quat=scene.quat.copy(),
        logit=logit,
        opacity=(1.0 / (1.0 + np.exp(-logit.astype(np.float64)))).astype(np.float32),
        sh=scene.sh.copy(),
    )


NET_LAYERS = ((3, 32), (32, 32), (32, 48))  # upsampler convolutions (in, out channels)


def net_init(seed=42, last_scale=0.01) -> np.ndarray:
    """Initial upsampler parameters, flat float32 [24016] in the order
    W1 [32][3][3][3], b1, W2 [32][32][3][3], b2, W3 [48][32][3][3], b3:
    each weight and bias ~ U(-1/sqrt(9 in), 1/sqrt(9 in)), the last layer's
    scaled by last_scale so that the network starts close to its bilinear
    residual."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for k, (ci, co) in enumerate(NET_LAYERS):
        bound = 1.0 / math.sqrt(ci * 9)
        s = last_scale if k == len(NET_LAYERS) - 1 else 1.0
        parts.append(rng.uniform(-bound, bound, co * ci * 9) * s)
        parts.append(rng.uniform(-bound, bound, co) * s)
    return np.concatenate(parts).astype(np.float32)


def crop_poses(seed=41, n=10_000, width=1832, height=1920, crop=256, fov_x_deg=60.0, scale=4,
               centre=HEAD_INSIDE, yaw_deg=180.0, pitch_deg=30.0):
    """Camera poses and crop offsets of the upsampler's training pairs: camera
    at centre + U(-1,1)^3 (centre (0,0,-3) by default), yaw U(-yaw_deg,
    yaw_deg), pitch U(-pitch_deg, pitch_deg), an eye camera of width x height;
    crop origin uniform over the frame, a multiple of `scale` so that the
    reduced-resolution crop is pixel-aligned.  Returns a list of (Camera, x0, y0).
    The camera-outside workload takes centre (0,0,-15) and 10 degrees of yaw
    and pitch (crop_poses_outside)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n):
        pos = np.asarray(centre, dtype=np.float64) + rng.uniform(-1.0, 1.0, 3)
        yaw, pitch = rng.uniform(-yaw_deg, yaw_deg), rng.uniform(-pitch_deg, pitch_deg)
        x0 = scale * int(rng.integers(0, (width - crop) // scale + 1))
        y0 = scale * int(rng.integers(0, (height - crop) // scale + 1))
        out.append((make_camera(width, height, fov_x_deg, pos, rot_yaw_pitch(yaw, pitch)), x0, y0))
    return out


def crop_poses_outside(seed=41, n=10_000, **kw):
    """Training poses of the camera-outside workload: the head within U(-1,1)^3
    of (0,0,-15), yaw and pitch U(-10,10) degrees, so that the cloud fills the
    central part of the frame as in its foveated frame."""
    return crop_poses(seed, n, centre=HEAD_OUTSIDE, yaw_deg=10.0, pitch_deg=10.0, **kw)


def gaze_trace(seed=31, n_frames=64, width=1832, height=1920, fov_x_deg=60.0, hz=90.0, head=(0.0, 0.0, -3.0),
               drift_deg=1.0, saccade_deg=(5.0, 20.0), interval_s=(0.2, 0.4), jitter_deg=0.3, max_ecc_deg=25.0):
    """Frames of a seeded gaze walk: fixations with Gaussian jitter (jitter_deg
    per axis), saccades of saccade_deg amplitude in a uniform direction every
    interval_s seconds (frames at hz), the gaze kept within max_ecc_deg of the
    optical axis; the head turns by drift_deg of yaw and of pitch per frame.
    Returns [(stereo cameras, [gaze left, gaze right] in pixels)] per frame."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gx = gy = 0.0
    t_next = rng.uniform(*interval_s)
    frames = []
    for k in range(n_frames):
        t = k / hz
        if t >= t_next:
            amp, ang = rng.uniform(*saccade_deg), rng.uniform(0.0, 2.0 * math.pi)
            gx = float(np.clip(gx + amp * math.cos(ang), -max_ecc_deg, max_ecc_deg))
            gy = float(np.clip(gy + amp * math.sin(ang), -max_ecc_deg, max_ecc_deg))
            t_next += rng.uniform(*interval_s)
        jx, jy = rng.normal(0.0, jitter_deg, 2)
        cams = stereo_cameras(head, width, height, fov_x_deg, c2w=rot_yaw_pitch(drift_deg * k, drift_deg * k))
        c = cams[0]
        px = c.cx + c.fx * math.tan(math.radians(gx + jx))
        py = c.cy + c.fy * math.tan(math.radians(gy + jy))
        frames.append((cams, [(px, py), (px, py)]))
    return frames


# Early-exit gaze predictions (Table 2, A3FR-ViT without pruning): per exit
# 1..6 the error spread (sigma_x, sigma_y) in degrees and the cumulative CPU
# latency in milliseconds at which the prediction is available.
EXIT_SIGMA_DEG = ((8.40, 9.33), (6.08, 7.05), (4.50, 4.46), (3.58, 3.38), (2.97, 2.85), (2.05, 2.16))
EXIT_LATENCY_MS = (5.11, 9.45, 13.91, 18.31, 22.21, 26.28)


def gaze_exits(seed=61, n_trials=16, width=1832, height=1920, fov_x_deg=60.0, max_ecc_deg=15.0, n_eyes=2):
    """Synthetic early-exit gaze streams for the incremental rounds: per trial a
    final gaze u_N (uniform direction, eccentricity uniform in [0, max_ecc_deg],
    the same pixel for every eye) and the predictions of exits 1..N-1, each
    u_N plus independent normal offsets with the exit's spread (Table 2,
    degrees at the image centre turned into pixels with f tan(theta)).
    Returns (trials, sigmas_px): trials = [(final [(x, y)] * n_eyes,
    [[(x, y)] * n_eyes for each exit 1..N-1])], sigmas_px = [(sx, sy)] for
    exits 1..N-1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = stereo_cameras((0.0, 0.0, -3.0), width, height, fov_x_deg)[0]
    sig = [(c.fx * math.tan(math.radians(sx)), c.fy * math.tan(math.radians(sy))) for sx, sy in EXIT_SIGMA_DEG[:-1]]
    trials = []
    for _ in range(n_trials):
        ecc, ang = rng.uniform(0.0, max_ecc_deg), rng.uniform(0.0, 2.0 * math.pi)
        ux = c.cx + c.fx * math.tan(math.radians(ecc * math.cos(ang)))
        uy = c.cy + c.fy * math.tan(math.radians(ecc * math.sin(ang)))
        exits = []
        for sx, sy in sig:
            ox, oy = rng.normal(0.0, 1.0, 2)
            exits.append([(float(ux + sx * ox), float(uy + sy * oy))] * n_eyes)
        trials.append(([(float(ux), float(uy))] * n_eyes, exits))
    return trials, sig
