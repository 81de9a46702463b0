"""ctypes front-end of the FP64 oracle (TEST INFRASTRUCTURE).

Each wrapper cites the part of the paper the computation follows:
  * projection, per-tile depth sort and front-to-back blend: Sec. 2.3 (the three
    stages of 3D Gaussian Splatting, and the 3DGS-process figure);
  * reuse of the projected data by several layers: Sec. 3.5;
  * foveal / coarser surrounding regions: Sec. 2.2, Eq. 1 (the foveal radius);
  * the periphery subset, layer radii and image sizes come from the rendering
    configuration (fovea radius 0.15 W, mid 0.35 W at 1/2 resolution, periphery
    at 1/4 resolution keeping the top 30% of points by opacity x projected area).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "a3fr_oracle.c")
_SRC_GRAD = os.path.join(_HERE, "a3fr_oracle_grad.c")
_LIB_PATH = os.path.join(_HERE, "liba3fr_oracle.so")
_lib = None

TILE = 16


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: FP64, no contraction, no fast-math."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-pthread",
               "-ffp-contract=off", "-fno-fast-math", "-fno-finite-math-only",
               _SRC, _SRC_GRAD, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class ORView(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("t", C.c_double * 3), ("campos", C.c_double * 3),
                ("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("width", C.c_int32), ("height", C.c_int32), ("eye", C.c_int32), ("mask", C.c_int32),
                ("select", C.c_int32), ("pad_", C.c_int32),
                ("gx", C.c_double), ("gy", C.c_double), ("r_in", C.c_double), ("r_out", C.c_double),
                ("bg", C.c_double * 3)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        I64, I32, D = C.c_int64, C.c_int32, C.c_double
        L.or_tile_masks.argtypes = [I32, P, I32, I32, P, P]
        L.or_project.argtypes = [I64, P, P, P, P, I32, P, I32, I32, P, P, P, P, P, P, P, P, P, P, P, C.c_int]
        L.or_sh_basis.argtypes = [D, D, D, P]
        L.or_view_cov.argtypes = [P, P, P, I64, I64, P, P, P]
        L.or_view_cov.restype = C.c_int
        L.or_footprint_q.argtypes = [D]
        L.or_footprint_q.restype = D
        L.or_colour.argtypes = [I64, P, P, I32, I32, P, P]
        L.or_select.argtypes = [I64, P, P, I32, I32, P]
        L.or_select.restype = I64
        L.or_emit.argtypes = [I64, I32, P, I32, I32, P, P, P, P, P, P, P, P, P, I64]
        L.or_emit.restype = I64
        L.or_sort.argtypes = [I64, P, P]
        L.or_ranges.argtypes = [I64, P, I64, P]
        L.or_blend.argtypes = [I32, P, I32, I32, P, P, P, P, P, P, I64, P, P, P, P, P, D, D,
                               P, P, P, P, P, P, C.c_int]
        L.or_blend_brute.argtypes = [I64, I32, P, P, P, P, P, P, P, P, P, P, P, P]
        L.or_blend_pixels.argtypes = [I64, I32, P, P, P, P, P, P, P, P, P, D, D, I64, P, P, P, P, P, P, C.c_int]
        L.or_pixel_trace.argtypes = [I32, D, D, P, I64, I64, P, P, P, P, P]
        L.or_pixel_trace.restype = I64
        L.or_composite.argtypes = [I32, I32, D, D, D, D, P, P, I32, P, I32, P, P]
        L.or_region_sse.argtypes = [I32, I32, D, D, D, D, P, P, P, P]
        L.or_render_grad.argtypes = [I64, P, P, P, P, P, I32, P, I32, P, D, D, I64, I64, I64, I64,
                                     P, P, P, P, P, P, P, C.c_int]
        L.or_render_grad.restype = I64
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def footprint_q(opacity):
    """Q(o) of the footprint box {d' Sigma2D^-1 d <= Q(o)} (Sec. 2.3): the
    smallest k/8 (k = 1..88) with exp(k/16) >= 1.001 x 255 o, else 11.1."""
    return float(lib().or_footprint_q(float(opacity)))


def default_threads() -> int:
    return max(1, os.cpu_count() or 1)


# ---------------------------------------------------------------------------
# views
# ---------------------------------------------------------------------------
@dataclass
class View:
    """One rendered layer of one eye (camera at this layer's resolution)."""
    R: np.ndarray
    t: np.ndarray
    campos: np.ndarray
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    eye: int = 0
    mask: int = 0        # 0 every tile, 1 disc, 2 annulus
    select: int = 0      # 1: periphery subset only
    gx: float = 0.0
    gy: float = 0.0
    r_in: float = 0.0
    r_out: float = 0.0
    bg: tuple = (0.0, 0.0, 0.0)

    def to_c(self) -> ORView:
        v = ORView()
        v.R[:] = [float(x) for x in np.asarray(self.R, dtype=np.float64).reshape(9)]
        v.t[:] = [float(x) for x in np.asarray(self.t, dtype=np.float64).reshape(3)]
        v.campos[:] = [float(x) for x in np.asarray(self.campos, dtype=np.float64).reshape(3)]
        v.fx, v.fy, v.cx, v.cy = self.fx, self.fy, self.cx, self.cy
        v.width, v.height, v.eye, v.mask, v.select = self.width, self.height, self.eye, self.mask, self.select
        v.gx, v.gy, v.r_in, v.r_out = self.gx, self.gy, self.r_in, self.r_out
        v.bg[:] = [float(x) for x in self.bg]
        return v


def full_view(cam, eye: int = 0) -> View:
    """A full-resolution layer with every tile active (the plain render)."""
    return View(R=cam.R, t=cam.t, campos=cam.campos, fx=cam.fx, fy=cam.fy, cx=cam.cx, cy=cam.cy,
                width=cam.width, height=cam.height, eye=eye, bg=tuple(cam.bg))


MID_MARGIN = 2.0  # layer pixels of bilinear support around the mid layer's disc edges


def foveated_views(cams, gazes, radius_px, scales=(1, 2, 4)):
    """The three layers of each eye (views ordered eye-major, layer-minor):
    fovea at full resolution over the tiles within r_f of the gaze (a disc);
    mid at 1/scales[1] over the annulus between r_f and r_m, with MID_MARGIN
    layer pixels of bilinear support on both edges; periphery at 1/scales[2] over
    every tile, drawing only the kept subset.  Each layer is the eye camera with
    focal lengths, principal point and size divided by its scale."""
    rf, rm = radius_px
    out = []
    for e, (cam, g) in enumerate(zip(cams, gazes)):
        for li, s in enumerate(scales):
            v = View(R=cam.R, t=cam.t, campos=cam.campos, fx=cam.fx / s, fy=cam.fy / s,
                     cx=cam.cx / s, cy=cam.cy / s, width=cam.width // s, height=cam.height // s,
                     eye=e, gx=g[0] / s, gy=g[1] / s, bg=tuple(cam.bg))
            if li == 0:
                v.mask, v.r_out = 1, rf / s
            elif li == 1:
                v.mask, v.r_in, v.r_out = 2, rf / s - MID_MARGIN, rm / s + MID_MARGIN
            else:
                v.select = 1
            out.append(v)
    return out


def _views_c(views):
    arr = (ORView * len(views))()
    for k, v in enumerate(views):
        arr[k] = v.to_c()
    return arr


def tile_grid(views, tw=TILE, th=TILE):
    tx = np.array([(v.width + tw - 1) // tw for v in views], dtype=np.int64)
    ty = np.array([(v.height + th - 1) // th for v in views], dtype=np.int64)
    off = np.zeros(len(views) + 1, dtype=np.int64)
    off[1:] = np.cumsum(tx * ty)
    return tx, ty, off


def image_offsets(views):
    off = np.zeros(len(views) + 1, dtype=np.int64)
    off[1:] = np.cumsum([v.width * v.height for v in views])
    return off


# ---------------------------------------------------------------------------
# stages
# ---------------------------------------------------------------------------
def tile_masks(views, tw=TILE, th=TILE):
    """uint8 active flag per (view, tile), concatenated in view order."""
    _, _, off = tile_grid(views, tw, th)
    act = np.zeros(int(off[-1]), dtype=np.uint8)
    vc = _views_c(views)
    lib().or_tile_masks(len(views), vc, tw, th, _p(off), _p(act))
    return act, off


def project(scene, views, tw=TILE, th=TILE, active=None, aoff=None, nthreads=None):
    n, nv = scene.n, len(views)
    out = dict(proj=np.zeros((nv, n), np.uint8), vis=np.zeros((nv, n), np.uint8),
               depth_bits=np.zeros((nv, n), np.uint32), rect=np.zeros((nv, n, 4), np.int32),
               count=np.zeros((nv, n), np.int32), mu=np.zeros((nv, n, 2)), cov=np.zeros((nv, n, 3)),
               det=np.zeros((nv, n)), score=np.zeros((nv, n)))
    vc = _views_c(views)
    m = [np.ascontiguousarray(a, dtype=np.float32) for a in (scene.mean, scene.scale, scene.quat, scene.opacity)]
    lib().or_project(n, *[_p(a) for a in m], nv, vc, tw, th, _p(active), _p(aoff),
                     _p(out["proj"]), _p(out["vis"]), _p(out["depth_bits"]), _p(out["rect"]),
                     _p(out["count"]), _p(out["mu"]), _p(out["cov"]), _p(out["det"]), _p(out["score"]),
                     nthreads or default_threads())
    return out


def view_cov(scene, view, i):
    """(ok, p_view[3], Sigma_view 3x3) of Gaussian i in the view's camera."""
    p, sv = np.zeros(3), np.zeros(6)
    m = [np.ascontiguousarray(a, dtype=np.float32) for a in (scene.mean, scene.scale, scene.quat)]
    vc = view.to_c()
    ok = lib().or_view_cov(*[_p(a) for a in m], scene.n, i, C.byref(vc), _p(p), _p(sv))
    S = np.array([[sv[0], sv[1], sv[2]], [sv[1], sv[3], sv[4]], [sv[2], sv[4], sv[5]]])
    return bool(ok), p, S


def sh_basis(d):
    """Real SH basis (16 values) at unit direction d."""
    Y = np.zeros(16)
    lib().or_sh_basis(float(d[0]), float(d[1]), float(d[2]), _p(Y))
    return Y


def colour(scene, campos_list, deg=3):
    """[n_eyes][n][3] float64 colours seen from each eye centre."""
    ne = len(campos_list)
    cp = np.ascontiguousarray(np.asarray(campos_list, dtype=np.float64).reshape(ne, 3))
    out = np.zeros((ne, scene.n, 3))
    lib().or_colour(scene.n, _p(np.ascontiguousarray(scene.mean, np.float32)),
                    _p(np.ascontiguousarray(scene.sh, np.float32)), deg, ne, _p(cp), _p(out))
    return out


def select(vis_row, score_row, num=3, den=10):
    keep = np.zeros(vis_row.shape[0], np.uint8)
    k = lib().or_select(vis_row.shape[0], _p(np.ascontiguousarray(vis_row)),
                        _p(np.ascontiguousarray(score_row)), num, den, _p(keep))
    return keep, int(k)


def emit(scene_n, views, pr, keep, active, aoff, tw=TILE, th=TILE):
    _, _, toff = tile_grid(views, tw, th)
    vc = _views_c(views)
    args = [scene_n, len(views), vc, tw, th, _p(active), _p(aoff), _p(toff), _p(pr["vis"]),
            _p(keep), _p(pr["rect"]), _p(pr["depth_bits"])]
    K = lib().or_emit(*args, None, None, 0)
    keys = np.zeros(max(K, 1), np.uint64)
    vals = np.zeros(max(K, 1), np.uint32)
    lib().or_emit(*args, _p(keys), _p(vals), K)
    return keys[:K], vals[:K], toff


def sort_keys(keys, vals):
    k2, v2 = keys.copy(), vals.copy()
    lib().or_sort(k2.shape[0], _p(k2), _p(v2))
    return k2, v2


def ranges(sorted_keys, ntiles):
    r = np.zeros((ntiles, 2), np.int64)
    lib().or_ranges(sorted_keys.shape[0], _p(sorted_keys), ntiles, _p(r))
    return r


EPS_ALPHA = 4e-6      # bound on the relative error of a float32 alpha
EPS_STEP = 3 * 2.0**-24  # relative rounding of one float32 transmittance update


def render(scene, views, tw=TILE, th=TILE, keep_frac=(3, 10), eps_alpha=EPS_ALPHA, eps_step=EPS_STEP,
           nthreads=None, colours=None, blend=True, extra_active=None):
    """The whole tiled pipeline in FP64. Returns every intermediate.
    extra_active: {view index: bool [tiles_y][tiles_x]} tiles added to that
    view's mask before counting (the full-resolution fallback)."""
    act, aoff = tile_masks(views, tw, th)
    if extra_active:
        act = act.copy()
        for v, m in extra_active.items():
            m = np.asarray(m, dtype=bool).reshape(-1)
            a0 = int(aoff[v])
            act[a0:a0 + m.size] |= m.astype(act.dtype)
    pr = project(scene, views, tw, th, act, aoff, nthreads)
    n, nv = scene.n, len(views)
    keep = np.zeros((nv, n), np.uint8)
    kcount = np.zeros(nv, np.int64)
    for v, vw in enumerate(views):
        if vw.select:
            keep[v], kcount[v] = select(pr["vis"][v], pr["score"][v], *keep_frac)
    keys, vals, toff = emit(n, views, pr, keep, act, aoff, tw, th)
    skeys, svals = sort_keys(keys, vals)
    rng = ranges(skeys, int(toff[-1]))
    res = dict(pr, active=act, aoff=aoff, tile_off=toff, keep=keep, kept=kcount, keys=keys, vals=vals,
               sorted_keys=skeys, sorted_vals=svals, ranges=rng)
    if not blend:
        return res
    n_eyes = max(v.eye for v in views) + 1
    if colours is None:
        campos = [None] * n_eyes
        for v in views:
            campos[v.eye] = v.campos
        colours = colour(scene, campos)
    ioff = image_offsets(views)
    npx = int(ioff[-1])
    rgb, T = np.zeros(3 * npx), np.zeros(npx)
    last, amb, pairs = np.zeros(npx, np.int32), np.zeros(npx, np.uint8), np.zeros(npx, np.int64)
    amb_tol = np.zeros(npx)
    vc = _views_c(views)
    op = np.ascontiguousarray(scene.opacity, np.float32)
    lib().or_blend(nv, vc, tw, th, _p(act), _p(aoff), _p(toff), _p(ioff), _p(svals), _p(rng), n,
                   _p(pr["mu"]), _p(pr["cov"]), _p(pr["det"]), _p(op), _p(colours), eps_alpha, eps_step,
                   _p(rgb), _p(T), _p(last), _p(amb), _p(pairs), _p(amb_tol), nthreads or default_threads())
    res.update(colour=colours, img_off=ioff, rgb=rgb, T=T, last=last, amb=amb, pairs=pairs, amb_tol=amb_tol,
               _opac=op)
    res["images"] = split_images(views, ioff, rgb, T, last, amb, pairs, amb_tol)
    return res


def split_images(views, ioff, rgb, T, last, amb, pairs, amb_tol):
    out = []
    for v, vw in enumerate(views):
        a, b = int(ioff[v]), int(ioff[v + 1])
        H, W = vw.height, vw.width
        out.append(dict(rgb=rgb[3 * a:3 * b].reshape(3, H, W), T=T[a:b].reshape(H, W),
                        last=last[a:b].reshape(H, W), amb=amb[a:b].reshape(H, W),
                        amb_tol=amb_tol[a:b].reshape(H, W),
                        pairs=pairs[a:b].reshape(H, W)))
    return out


def render_brute(scene, views, keep=None, colours=None, tw=TILE, th=TILE):
    """The plain definition (no tiles) for small scenes: returns per-view images."""
    pr = project(scene, views, tw, th, None, None, 1)
    n, nv = scene.n, len(views)
    if keep is None:
        keep = np.zeros((nv, n), np.uint8)
    n_eyes = max(v.eye for v in views) + 1
    if colours is None:
        campos = [None] * n_eyes
        for v in views:
            campos[v.eye] = v.campos
        colours = colour(scene, campos)
    ioff = image_offsets(views)
    npx = int(ioff[-1])
    rgb, T = np.zeros(3 * npx), np.zeros(npx)
    vc = _views_c(views)
    op = np.ascontiguousarray(scene.opacity, np.float32)
    lib().or_blend_brute(n, nv, vc, _p(ioff), _p(pr["proj"]), _p(np.ascontiguousarray(keep)),
                         _p(pr["depth_bits"]), _p(pr["mu"]), _p(pr["cov"]), _p(pr["det"]), _p(op),
                         _p(colours), _p(rgb), _p(T))
    imgs = []
    for v, vw in enumerate(views):
        a, b = int(ioff[v]), int(ioff[v + 1])
        imgs.append(dict(rgb=rgb[3 * a:3 * b].reshape(3, vw.height, vw.width), T=T[a:b].reshape(vw.height, vw.width)))
    return imgs


def blend_pixels(scene, views, pr, keep, colours, v, xs, ys, eps_alpha=None, eps_step=None, nthreads=None):
    """Brute-force colours, T, ambiguity flags and ambiguity tolerances (the
    colour change a reversed near-threshold decision causes) of sampled pixels
    (xs, ys) of view v, from the projection arrays of project()."""
    xs = np.ascontiguousarray(xs, np.int32)
    ys = np.ascontiguousarray(ys, np.int32)
    npx = xs.size
    rgb, T, amb, tol = np.zeros((npx, 3)), np.zeros(npx), np.zeros(npx, np.int32), np.zeros(npx)
    vc = _views_c(views)
    op = np.ascontiguousarray(scene.opacity, np.float32)
    lib().or_blend_pixels(scene.n, v, vc, _p(pr["proj"]), _p(None if keep is None else np.ascontiguousarray(keep)),
                          _p(pr["depth_bits"]), _p(pr["mu"]), _p(pr["cov"]), _p(pr["det"]), _p(op),
                          _p(np.ascontiguousarray(colours)), EPS_ALPHA if eps_alpha is None else eps_alpha,
                          EPS_STEP if eps_step is None else eps_step, npx, _p(xs), _p(ys), _p(rgb), _p(T), _p(amb),
                          _p(tol), nthreads or default_threads())
    return rgb, T, amb, tol


def pixel_trace(res, view_index, px, py, tw=TILE, th=TILE, views=None):
    """Transmittance after each entry of the pixel's tile list."""
    vw = views[view_index]
    TX = (vw.width + tw - 1) // tw
    gt = int(res["tile_off"][view_index]) + (int(py) // th) * TX + int(px) // tw
    s, e = res["ranges"][gt]
    lst = np.ascontiguousarray(res["sorted_vals"][s:e])
    tr = np.zeros(max(e - s, 1))
    w = lib().or_pixel_trace(view_index, px + 0.5, py + 0.5, _p(lst), e - s, res["mu"].shape[1],
                             _p(np.ascontiguousarray(res["mu"])), _p(np.ascontiguousarray(res["cov"])),
                             _p(np.ascontiguousarray(res["det"])), _p(res["_opac"]), _p(tr))
    return tr[:w]


def composite(W, H, gaze, radius_px, fovea, mid, periph, mid_scale=2, periph_scale=4, periph_full=None):
    out = np.zeros((3, H, W))
    f = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)
    lib().or_composite(W, H, float(gaze[0]), float(gaze[1]), float(radius_px[0]), float(radius_px[1]),
                       _p(f(fovea)), _p(f(mid)), mid_scale, _p(f(periph)), periph_scale, _p(f(periph_full)), _p(out))
    return out


def region_sse(W, H, gaze, radius_px, a, b):
    sse = np.zeros(3)
    cnt = np.zeros(3, np.int64)
    lib().or_region_sse(W, H, float(gaze[0]), float(gaze[1]), float(radius_px[0]), float(radius_px[1]),
                        _p(np.ascontiguousarray(a, np.float64)), _p(np.ascontiguousarray(b, np.float64)),
                        _p(sse), _p(cnt))
    return sse, cnt


def psnr_from_sse(sse, count_px):
    """PSNR over RGB of images in [0,1]: 10 log10(1 / MSE), MSE over 3 x count."""
    if count_px == 0:
        return float("inf")
    mse = sse / (3.0 * count_px)
    return float("inf") if mse == 0.0 else 10.0 * math.log10(1.0 / mse)


def periphery_psnr(W, H, gaze, radius_px, img, ref):
    """PSNR outside the fovea (mid + periphery regions), and the outer region alone."""
    sse, cnt = region_sse(W, H, gaze, radius_px, img, ref)
    return psnr_from_sse(sse[1] + sse[2], int(cnt[1] + cnt[2])), psnr_from_sse(sse[2], int(cnt[2]))


def render_foveated(scene, cams, gazes, radius_px, keep_frac=(3, 10), nthreads=None, periph_full=None):
    """Foveated stereo frame: three layers per eye, composited to full resolution."""
    views = foveated_views(cams, gazes, radius_px)
    res = render(scene, views, keep_frac=keep_frac, nthreads=nthreads)
    outs = []
    for e, cam in enumerate(cams):
        L = res["images"][3 * e: 3 * e + 3]
        outs.append(composite(cam.width, cam.height, gazes[e], radius_px, L[0]["rgb"], L[1]["rgb"], L[2]["rgb"],
                              periph_full=None if periph_full is None else periph_full[e]))
    res["views"] = views
    res["out"] = np.stack(outs)
    return res


def render_full(scene, cams, nthreads=None):
    views = [full_view(c, e) for e, c in enumerate(cams)]
    res = render(scene, views, nthreads=nthreads)
    res["views"] = views
    res["out"] = np.stack([im["rgb"] for im in res["images"]])
    return res


# ---------------------------------------------------------------------------
# differentiable render (backward pass of the training loop)
# ---------------------------------------------------------------------------
def render_grad(mean, log_scale, quat, logit, sh, view: View, weights, smooth=False, deg=3,
                eps_alpha=EPS_ALPHA, eps_step=EPS_STEP, nthreads=None, window=None):
    """Render one view from the raw parameters and back-propagate dL/dI.

    The forward is the plain definition (every projectable Gaussian in (depth,
    index) order at every pixel; scale = exp(log-scale), opacity =
    sigmoid(logit)); the backward is the analytic chain rule of it, used by the
    optimisation of the Gaussian parameters (Sec. 2.3).  ``weights`` is dL/dI,
    float64 [3][H][W].  ``smooth`` drops the alpha skip, the early stop and the
    clamps so that finite differences can pin the chain.

    Inputs: mean [3][N], log_scale [3][N], quat [4][N] (w,x,y,z), logit [N],
    sh [16][3][N], all float32.  ``window`` = (x0, y0, w, h) restricts the
    rendered and differentiated pixels (default: the whole view).  Returns
    dict(image [3][H][W] f64, amb [H][W] u8, n_proj, grads
    mean/log_scale/quat/logit/sh in the input layouts, f64)."""
    L = lib()
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    mean, log_scale, quat, logit, sh = f32(mean), f32(log_scale), f32(quat), f32(logit), f32(sh)
    n = int(mean.shape[1])
    nk = (deg + 1) ** 2
    assert mean.shape == (3, n) and log_scale.shape == (3, n) and quat.shape == (4, n)
    assert logit.shape == (n,) and sh.shape[1:] == (3, n) and sh.shape[0] >= nk
    sh = np.ascontiguousarray(sh[:nk])
    H, W = view.height, view.width
    w = np.ascontiguousarray(weights, dtype=np.float64)
    assert w.shape == (3, H, W)
    img = np.zeros((3, H, W), np.float64)
    amb = np.zeros((H, W), np.uint8)
    g = dict(mean=np.zeros((3, n)), log_scale=np.zeros((3, n)), quat=np.zeros((4, n)), logit=np.zeros(n),
             sh=np.zeros((nk, 3, n)))
    vc = view.to_c()
    x0, y0, ww, wh = (0, 0, W, H) if window is None else (int(a) for a in window)
    assert 0 <= x0 and 0 <= y0 and ww >= 0 and wh >= 0 and x0 + ww <= W and y0 + wh <= H
    m = L.or_render_grad(n, _p(mean), _p(log_scale), _p(quat), _p(logit), _p(sh), deg, C.byref(vc),
                         1 if smooth else 0, _p(w), eps_alpha, eps_step, x0, y0, ww, wh, _p(img), _p(amb),
                         _p(g["mean"]), _p(g["log_scale"]), _p(g["quat"]), _p(g["logit"]), _p(g["sh"]),
                         nthreads or default_threads())
    return dict(image=img, amb=amb, n_proj=int(m), grads=g)


# ---------------------------------------------------------------------------
# per-tile error estimate of the periphery and full-resolution fallback
# ---------------------------------------------------------------------------
def tile_mass(res, views, pv, tw=TILE, th=TILE):
    """(D, K) [ty][tx] of periphery view pv: for every visible Gaussian, its
    opacity mass 2 pi o sqrt(det) = 2 x score split evenly over the tiles of its
    rectangle, per pixel of a tile; D sums the Gaussians the subset dropped,
    K the kept ones."""
    TX = (views[pv].width + tw - 1) // tw
    TY = (views[pv].height + th - 1) // th
    D, K = np.zeros((TY, TX)), np.zeros((TY, TX))
    for i in np.nonzero(res["count"][pv] > 0)[0]:
        x0, x1, y0, y1 = (int(a) for a in res["rect"][pv][i])
        nt = (x1 - x0 + 1) * (y1 - y0 + 1)
        tgt = K if res["keep"][pv][i] else D
        tgt[y0:y1 + 1, x0:x1 + 1] += 2.0 * res["score"][pv][i] / (nt * tw * th)
    return D, K


def fallback_estimate(D, K, coef, power):
    """coef x (dT^2)^power, dT = exp(-K) - exp(-(K + D)): the rise of the tile's
    transmittance under T ~ exp(-opacity mass per pixel) when the dropped mass
    D is removed."""
    dT = np.exp(-K) - np.exp(-(K + D))
    return np.where(dT > 0, coef * np.power(np.maximum(dT * dT, 1e-300), power), 0.0)


def fallback_flags(D, K, vp, vf, r_mid, thr, coef, power, tw=TILE, th=TILE):
    """Periphery tiles whose estimate reaches thr and that contain a
    full-resolution pixel centre farther than r_mid from the gaze (vf's gaze,
    full-resolution pixels); s = vf.fx / vp.fx full-resolution pixels per
    periphery pixel.  Returns (flags [TY][TX], extra bool mask of vf's tiles)."""
    s = int(round(vf.fx / vp.fx))
    span = tw * s
    est = fallback_estimate(D, K, coef, power)
    TY, TX = D.shape
    flags = np.zeros((TY, TX), bool)
    for ty in range(TY):
        for tx in range(TX):
            x0, x1 = tx * span + 0.5, min((tx + 1) * span, vf.width) - 0.5
            y0, y1 = ty * span + 0.5, min((ty + 1) * span, vf.height) - 0.5
            fx = max(abs(x0 - vf.gx), abs(x1 - vf.gx))
            fy = max(abs(y0 - vf.gy), abs(y1 - vf.gy))
            outer = x0 <= x1 and y0 <= y1 and fx * fx + fy * fy > r_mid * r_mid
            flags[ty, tx] = outer and est[ty, tx] >= thr
    FX = (vf.width + tw - 1) // tw
    FY = (vf.height + th - 1) // th
    extra = np.zeros((FY, FX), bool)
    for ty, tx in zip(*np.nonzero(flags)):
        extra[ty * s:(ty + 1) * s, tx * s:(tx + 1) * s] = True
    return flags, extra


def composite_fallback(out, fovea, flags, W, H, gaze, r_mid, span):
    """Pixels outside r_mid whose periphery tile is flagged take the
    full-resolution layer's value (out, fovea: [3][H][W])."""
    out = out.copy()
    ys, xs = np.mgrid[0:H, 0:W]
    rho2 = (xs + 0.5 - gaze[0]) ** 2 + (ys + 0.5 - gaze[1]) ** 2
    sel = (rho2 > r_mid * r_mid) & flags[ys // span, xs // span]
    out[:, sel] = fovea[:, sel]
    return out
