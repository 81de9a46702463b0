// Projection stage of 3D Gaussian Splatting (paper Sec. 2.3: every ellipsoid
// is projected to a screen ellipse and the tiles it intersects are found), run
// once per frame for every layer of every eye so that later stages reuse it
// (Sec. 3.5).  One thread per (Gaussian, eye): its geometry is loaded with
// coalesced structure-of-arrays reads, its 3D and view-space covariances are
// formed once, and every layer view of that eye is projected from them.  The
// view-dependent colour (SH, 192 B per Gaussian) is evaluated later, only for
// the entries that emit keys (k_entry_colour).
//
// The integer outputs (tile rectangle, active-tile count, depth key, periphery
// score bits) come from a float64 "key path" whose every operation is written
// out below in a fixed order: explicit fma() for each product-sum, IEEE
// division and square root, no contraction (the library is compiled with
// -ffp-contract=off).  The same sequence, evaluated in float64 anywhere,
// yields the same bits.
#include "a3fr_internal.h"

namespace a3fr {

// ------------------------------------------------------------------------
// active-tile masks
// ------------------------------------------------------------------------
__device__ __forceinline__ bool tile_active(const a3fr_view &v, int tx, int ty) {
    if (v.mask == A3FR_MASK_ALL) return true;
    if (v.r_out < 0.0) return false;  // an empty mask
    int xe = (tx + 1) * kTile; if (xe > v.width) xe = v.width;
    int ye = (ty + 1) * kTile; if (ye > v.height) ye = v.height;
    double x0 = (double)(tx * kTile) + 0.5, x1 = (double)xe - 0.5;
    double y0 = (double)(ty * kTile) + 0.5, y1 = (double)ye - 0.5;
    double ddx = fmax(fmax(x0 - v.gx, v.gx - x1), 0.0);
    double ddy = fmax(fmax(y0 - v.gy, v.gy - y1), 0.0);
    double d2 = ddx * ddx + ddy * ddy;
    if (!(d2 <= v.r_out * v.r_out)) return false;
    if (v.mask == A3FR_MASK_ANNULUS && v.r_in > 0.0) {
        double ri2 = v.r_in * v.r_in;
        double ax = x0 - v.gx, bx = x1 - v.gx, ay = y0 - v.gy, by = y1 - v.gy;
        bool inside = (ax * ax + ay * ay <= ri2) && (bx * bx + ay * ay <= ri2) &&
                      (ax * ax + by * by <= ri2) && (bx * bx + by * by <= ri2);
        if (inside) return false;
    }
    return true;
}

// One wavefront per tile row of every view: active flags, and for masked views
// a row prefix count (row_prefix[x] = active tiles in columns < x) and the
// columns of the row's active tiles in order (row_list), built with ballots.
// Incremental rounds: a frozen view has no active tile; a view excluding done
// tiles drops the tiles an earlier round rendered and marks its new ones done.
// The ranges of zero are cleared first, spread over every thread of the grid.
__global__ void __launch_bounds__(256) k_tile_masks(const DevView *views, int64_t rows_total, const int32_t *row_view,
                                                    const int32_t *row_y, uint16_t *row_prefix, uint16_t *row_list,
                                                    uint8_t *active, uint8_t *done, FillSegs zero) {
    if (zero.count > 0) {
        int64_t total = 0;
        for (int k = 0; k < zero.count; ++k) total += zero.n[k];
        for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < total;
             j += (int64_t)gridDim.x * blockDim.x) {
            int64_t q = j;
            int k = 0;
            while (q >= zero.n[k]) q -= zero.n[k++];
            zero.p[k][q] = 0u;
        }
    }
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= rows_total) return;
    const DevView &dv = views[row_view[r]];
    const int ty = row_y[r];
    const int TX = dv.tiles_x;
    uint8_t *act = active + dv.tile_off + (int64_t)ty * TX;
    const bool frozen = (dv.round_flags & kRoundFrozen) != 0;
    const bool excl = done && (dv.round_flags & kRoundExclDone) != 0;
    uint8_t *dn = excl ? done + dv.tile_off + (int64_t)ty * TX : nullptr;
    if (dv.v.mask == A3FR_MASK_ALL) {
        for (int tx = lane; tx < TX; tx += 64) act[tx] = frozen ? 0 : 1;
        return;
    }
    uint16_t *pre = row_prefix + dv.mask_off + (int64_t)ty * (TX + 1);
    uint16_t *lst = row_list + dv.mask_off + (int64_t)ty * (TX + 1);
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    uint32_t c = 0;
    for (int tx0 = 0; tx0 < TX; tx0 += 64) {
        const int tx = tx0 + lane;
        bool a = !frozen && tx < TX && tile_active(dv.v, tx, ty);
        if (excl && a) {
            a = dn[tx] == 0;
            if (a) dn[tx] = 1;
        }
        const uint64_t m = __ballot(a);
        const uint32_t below = (uint32_t)__popcll(m & lt);
        if (tx < TX) {
            pre[tx] = (uint16_t)(c + below);
            act[tx] = a ? 1 : 0;
            if (a) lst[c + below] = (uint16_t)tx;
        }
        c += (uint32_t)__popcll(m);
    }
    if (lane == 0) pre[TX] = (uint16_t)c;
}

void launch_tile_masks(const DevView *views, int nv, int64_t rows_total, const int32_t *row_view,
                       const int32_t *row_y, uint16_t *row_prefix, uint16_t *row_list, uint8_t *active,
                       uint8_t *done, const FillSegs &zero, hipStream_t s) {
    (void)nv;
    if (rows_total == 0) {
        if (zero.count > 0) launch_zero_segs(zero, s);
        return;
    }
    hipLaunchKernelGGL(k_tile_masks, dim3((unsigned)((rows_total + 3) / 4)), dim3(256), 0, s, views, rows_total,
                       row_view, row_y, row_prefix, row_list, active, done, zero);
}

// ------------------------------------------------------------------------
// key path
// ------------------------------------------------------------------------
struct Cov3 { double s00, s01, s02, s11, s12, s22; };

// Sigma3D = (R(q) S)(R(q) S)^T for the normalised quaternion q = (w,x,y,z).
__device__ __forceinline__ bool gaussian_cov3(double qw, double qx, double qy, double qz, double s0, double s1,
                                              double s2, Cov3 &S) {
    double nq = sqrt(fma(qw, qw, fma(qx, qx, fma(qy, qy, qz * qz))));
    if (!(nq > 0.0)) return false;
    double w = qw / nq, x = qx / nq, y = qy / nq, z = qz / nq;
    double xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z;
    double wx = w * x, wy = w * y, wz = w * z;
    // rotation of the unit quaternion, row-major, times diag(s) column-wise
    double m00 = (1.0 - 2.0 * (yy + zz)) * s0, m01 = (2.0 * (xy - wz)) * s1, m02 = (2.0 * (xz + wy)) * s2;
    double m10 = (2.0 * (xy + wz)) * s0, m11 = (1.0 - 2.0 * (xx + zz)) * s1, m12 = (2.0 * (yz - wx)) * s2;
    double m20 = (2.0 * (xz - wy)) * s0, m21 = (2.0 * (yz + wx)) * s1, m22 = (1.0 - 2.0 * (xx + yy)) * s2;
    S.s00 = fma(m00, m00, fma(m01, m01, m02 * m02));
    S.s01 = fma(m00, m10, fma(m01, m11, m02 * m12));
    S.s02 = fma(m00, m20, fma(m01, m21, m02 * m22));
    S.s11 = fma(m10, m10, fma(m11, m11, m12 * m12));
    S.s12 = fma(m10, m20, fma(m11, m21, m12 * m22));
    S.s22 = fma(m20, m20, fma(m21, m21, m22 * m22));
    return true;
}

// Sigma_view = Rw Sigma3D Rw^T, evaluated as A = Rw Sigma3D, then A Rw^T.
__device__ __forceinline__ void view_cov(const double *Rw, const Cov3 &S, Cov3 &V) {
    const double Sm[9] = {S.s00, S.s01, S.s02, S.s01, S.s11, S.s12, S.s02, S.s12, S.s22};
    double A[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            A[3 * r + c] = fma(Rw[3 * r + 0], Sm[0 * 3 + c], fma(Rw[3 * r + 1], Sm[1 * 3 + c], Rw[3 * r + 2] * Sm[2 * 3 + c]));
    auto e = [&](int r, int c) {
        return fma(A[3 * r + 0], Rw[3 * c + 0], fma(A[3 * r + 1], Rw[3 * c + 1], A[3 * r + 2] * Rw[3 * c + 2]));
    };
    V.s00 = e(0, 0); V.s01 = e(0, 1); V.s02 = e(0, 2);
    V.s11 = e(1, 1); V.s12 = e(1, 2); V.s22 = e(2, 2);
}

// Real spherical harmonics up to degree 3 (Condon-Shortley phase, m = -l..l)
// at unit direction (x, y, z); each constant is the closed-form normalisation
// sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) (x sqrt 2 for m != 0) of its polynomial.
__device__ __forceinline__ void sh_basis(float x, float y, float z, float *Y) {
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[0] = 0.28209479177387814f;                    // 1/(2 sqrt(pi))
    const float c1 = 0.4886025119029199f;           // sqrt(3/(4 pi))
    Y[1] = -c1 * y; Y[2] = c1 * z; Y[3] = -c1 * x;
    const float c2a = 1.0925484305920792f;          // sqrt(15/pi)/2
    const float c2b = 0.31539156525252005f;         // sqrt(5/pi)/4
    const float c2c = 0.5462742152960396f;          // sqrt(15/pi)/4
    Y[4] = c2a * x * y; Y[5] = -c2a * y * z; Y[6] = c2b * (2.0f * zz - xx - yy);
    Y[7] = -c2a * x * z; Y[8] = c2c * (xx - yy);
    const float c3a = 0.5900435899266435f;          // sqrt(35/(2 pi))/4
    const float c3b = 2.890611442640554f;           // sqrt(105/pi)/2
    const float c3c = 0.4570457994644658f;          // sqrt(21/(2 pi))/4
    const float c3d = 0.3731763325901154f;          // sqrt(7/pi)/4
    const float c3e = 1.445305721320277f;           // sqrt(105/pi)/4
    Y[9] = -c3a * y * (3.0f * xx - yy);
    Y[10] = c3b * x * y * z;
    Y[11] = -c3c * y * (4.0f * zz - xx - yy);
    Y[12] = c3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
    Y[13] = -c3c * x * (4.0f * zz - xx - yy);
    Y[14] = c3e * z * (xx - yy);
    Y[15] = -c3a * x * (xx - 3.0f * yy);
}

// Footprint bound Q(o) of opacity o: a pixel takes the Gaussian only where
// o exp(-q/2) >= 1/255; the smallest step k/8 with exp(k/16) >= (1.001 x 255) o
// (a lower-bound search over the increasing table exp(k/16), k = 0..kExtentSteps),
// else kExtentQ.
__device__ __forceinline__ double footprint_q(float op, const double *s_exp) {
    double qe = kExtentQ;
    const double t = (1.001 * 255.0) * (double)op;
    int lo = 1, cnt_k = kExtentSteps;
    while (cnt_k > 0) {
        const int half = cnt_k >> 1;
        if (s_exp[lo + half] < t) {
            lo += half + 1;
            cnt_k -= half + 1;
        } else {
            cnt_k = half;
        }
    }
    if (lo <= kExtentSteps) qe = (double)lo / 8.0;
    return qe;
}

// The Gaussian in one eye's camera: view-space centre p and covariance V
// (front: in front of the near plane with a valid rotation).
struct EyeProj {
    double p0, p1, p2, xz, yz;
    Cov3 V;
    bool front;
};

__device__ __forceinline__ void eye_project(const a3fr_view &v0, double mx, double my, double mz, bool cov_ok,
                                            const Cov3 &S, EyeProj &E) {
    const double *Rw = v0.R;
    E.p0 = fma(Rw[0], mx, fma(Rw[1], my, fma(Rw[2], mz, v0.t[0])));
    E.p1 = fma(Rw[3], mx, fma(Rw[4], my, fma(Rw[5], mz, v0.t[1])));
    E.p2 = fma(Rw[6], mx, fma(Rw[7], my, fma(Rw[8], mz, v0.t[2])));
    E.front = E.p2 > kZNear && cov_ok;
    if (E.front) view_cov(Rw, S, E.V);
    E.xz = E.p0 / E.p2;
    E.yz = E.p1 / E.p2;
}

// One layer view: the dilated 2D covariance (a, b, c), its determinant, the
// centre (u, w) and the footprint box's tile rectangle [x0, x1] x [y0, y1]
// (clamped to the grid); visible when the box meets the image.
struct LayerProj {
    double a, b, c, det, u, w;
    int x0, x1, y0, y1;
    bool visible;
};

__device__ __forceinline__ void layer_project(const DevView &dv, const EyeProj &E, double qe, LayerProj &L) {
    const a3fr_view &v = dv.v;
    L.visible = false;
    if (!E.front) return;
    const Cov3 &V = E.V;
    const double limx = dv.limx, limy = dv.limy;  // (1.3 (W/2)) / fx, computed on the host
    const double txc = fmin(fmax(E.xz, -limx), limx);
    const double tyc = fmin(fmax(E.yz, -limy), limy);
    const double j00 = v.fx / E.p2, j02 = -(j00 * txc);
    const double j11 = v.fy / E.p2, j12 = -(j11 * tyc);
    const double B00 = fma(j00, V.s00, j02 * V.s02), B01 = fma(j00, V.s01, j02 * V.s12),
                 B02 = fma(j00, V.s02, j02 * V.s22);
    const double B11 = fma(j11, V.s11, j12 * V.s12), B12 = fma(j11, V.s12, j12 * V.s22);
    L.a = fma(B00, j00, B02 * j02) + kDilate;
    L.b = fma(B01, j11, B02 * j12);
    L.c = fma(B11, j11, B12 * j12) + kDilate;
    L.det = fma(L.a, L.c, -(L.b * L.b));
    if (!(L.det > 0.0)) return;
    L.u = fma(v.fx, E.xz, v.cx);
    L.w = fma(v.fy, E.yz, v.cy);
    const double ex = sqrt(qe * L.a), ey = sqrt(qe * L.c);
    const double lox = L.u - ex, hix = L.u + ex, loy = L.w - ey, hiy = L.w + ey;
    if (!(hix >= 0.5 && lox <= (double)v.width - 0.5 && hiy >= 0.5 && loy <= (double)v.height - 0.5)) return;
    double fx0 = ceil((lox - ((double)kTile - 0.5)) / (double)kTile);
    double fx1 = floor((hix - 0.5) / (double)kTile);
    double fy0 = ceil((loy - ((double)kTile - 0.5)) / (double)kTile);
    double fy1 = floor((hiy - 0.5) / (double)kTile);
    fx0 = fmax(fx0, 0.0); fx1 = fmin(fx1, (double)(dv.tiles_x - 1));
    fy0 = fmax(fy0, 0.0); fy1 = fmin(fy1, (double)(dv.tiles_y - 1));
    if (!(fx0 <= fx1 && fy0 <= fy1)) return;
    L.x0 = (int)fx0; L.x1 = (int)fx1; L.y0 = (int)fy0; L.y1 = (int)fy1;
    L.visible = true;
}

__device__ __forceinline__ uint64_t pack_rect(const LayerProj &L) {
    return (uint64_t)(uint16_t)L.x0 | ((uint64_t)(uint16_t)L.x1 << 16) | ((uint64_t)(uint16_t)L.y0 << 32) |
           ((uint64_t)(uint16_t)L.y1 << 48);
}

// One thread per (Gaussian, group of consecutive views of one eye): the
// Gaussian's geometry is loaded once, its 3D and view-space covariances
// formed once, and each view of the group (the layers of that eye) gets the
// float64 key path: its active-tile count (every slot), its float32 depth bits
// (entries that emit keys, and every visible entry of a view whose mask may
// grow later), its tile rectangle (only in the views that keep rectangles for
// a later recount or mass estimate, rect_slot >= 0) and, in a selecting view,
// its score; a Gaussian visible in a view of the group also gets its packed
// geometry (48 B) written for the record pass.  The blend record of an entry
// is formed later, entry by entry (k_entry_record), once the entries are known.
__global__ void __launch_bounds__(256) k_preprocess(a3fr_scene sc, const DevView *__restrict__ views, int ngroups,
                                                    const int32_t *__restrict__ groups,
                                                    const uint32_t *__restrict__ cum,
                                                    uint32_t *__restrict__ counts, uint32_t *__restrict__ depth,
                                                    uint64_t *__restrict__ rect, double *__restrict__ score,
                                                    GeomPack *__restrict__ pack,
                                                    const double *__restrict__ exp_tab) {
    __shared__ double s_exp[kExtentSteps + 1];
    for (int k = threadIdx.x; k <= kExtentSteps; k += blockDim.x) s_exp[k] = exp_tab[k];
    __syncthreads();
    const int64_t n = sc.n;
    // block b: chunk of 256 Gaussians and eye group, numbered so that the groups of
    // one chunk are 8 blocks apart (blocks go to the 8 XCDs in turn): they run on
    // one XCD at about the same time, and the chunk's geometry comes from HBM once
    const int xl = (int)(blockIdx.x & 7u);
    const int64_t rest = blockIdx.x >> 3;
    const int grp = (int)(rest % ngroups);
    const int64_t chunk = (rest / ngroups) * 8 + xl;
    const int64_t i = chunk * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int v_begin = groups[grp], v_end = groups[grp + 1];
    const float fx = sc.mean_dev[i], fy = sc.mean_dev[n + i], fz = sc.mean_dev[2 * n + i];
    const float qw = sc.quat_dev[i], qx = sc.quat_dev[n + i], qy = sc.quat_dev[2 * n + i], qz = sc.quat_dev[3 * n + i];
    const float sx = sc.scale_dev[i], sy = sc.scale_dev[n + i], sz = sc.scale_dev[2 * n + i];
    const float op = sc.opacity_dev[i];
    const double mx = fx, my = fy, mz = fz;
    Cov3 S;
    const bool cov_ok = gaussian_cov3(qw, qx, qy, qz, sx, sy, sz, S);
    EyeProj E;
    eye_project(views[v_begin].v, mx, my, mz, cov_ok, S, E);
    const double qe = footprint_q(op, s_exp);
    bool seen = false;  // visible in a view of this group
    for (int vi = v_begin; vi < v_end; ++vi) {
        const DevView &dv = views[vi];
        const int64_t slot = (int64_t)vi * n + i;
        LayerProj L;
        layer_project(dv, E, qe, L);
        uint32_t cnt = 0;
        if (L.visible) {
            if (dv.v.mask == A3FR_MASK_ALL) {
                cnt = (uint32_t)((L.x1 - L.x0 + 1) * (L.y1 - L.y0 + 1));
            } else {
                // active tiles in the rectangle from the view's summed-area
                // table (cum[ty][tx]: active tiles in rows < ty, columns < tx),
                // over the part of the rectangle that can hold active tiles
                const int cx0 = max(L.x0, dv.ax0), cx1 = min(L.x1, dv.ax1);
                const int cy0 = max(L.y0, dv.ay0), cy1 = min(L.y1, dv.ay1);
                if (cx0 <= cx1 && cy0 <= cy1) {
                    const uint32_t *C = cum + dv.cum_off;
                    const int64_t st = dv.tiles_x + 1, r0 = (int64_t)cy0 * st, r1 = (int64_t)(cy1 + 1) * st;
                    cnt = (C[r1 + cx1 + 1] - C[r0 + cx1 + 1]) - (C[r1 + cx0] - C[r0 + cx0]);
                }
            }
            // the depth key of entries that emit keys (and of every visible
            // entry of a view whose mask may grow); in the masked layers most
            // visible Gaussians touch no active tile
            if (cnt != 0 || dv.remask) {
                depth[slot] = __float_as_uint((float)E.p2);
                if (dv.v.select) score[(int64_t)dv.sel_slot * n + i] = ((double)op * 3.141592653589793) * sqrt(L.det);
            }
        }
        counts[slot] = cnt;
        if (dv.rect_slot >= 0) rect[(int64_t)dv.rect_slot * n + i] = L.visible ? pack_rect(L) : kEmptyRect;
        seen = seen || L.visible;
    }
    if (seen) {  // the record pass reads the packed geometry of visible Gaussians only (each group
                 // seeing one writes the same values)
        GeomPack g;
        g.a = make_float4(fx, fy, fz, op);
        g.b = make_float4(sx, sy, sz, qw);
        g.c = make_float4(qx, qy, qz, 0.0f);
        pack[i] = g;
    }
}

void launch_preprocess(const a3fr_scene &sc, const DevView *views, int ngroups, const int32_t *groups,
                       const uint32_t *cum, uint32_t *counts, uint32_t *depth, uint64_t *rect, double *score,
                       GeomPack *pack, const double *exp_tab, hipStream_t s) {
    if (sc.n == 0 || ngroups == 0) return;
    const int blk = 256;
    const int64_t chunks = (sc.n + blk - 1) / blk;
    const int64_t grid = (chunks + 7) / 8 * 8 * ngroups;  // see k_preprocess for the numbering
    hipLaunchKernelGGL(k_preprocess, dim3((unsigned)grid), dim3(blk), 0, s, sc, views, ngroups, groups, cum, counts,
                       depth, rect, score, pack, exp_tab);
}

// View-dependent colour (degree <= 3 real SH, float32) of Gaussian i (mean
// m) seen from its view's eye centre, clamped at zero, written into its record.
__device__ __forceinline__ void colour_into(const a3fr_scene &sc, const a3fr_view &vw, int64_t i, const float4 &m,
                                            Record &rr) {
    const float dx = m.x - (float)vw.campos[0], dy = m.y - (float)vw.campos[1], dz = m.z - (float)vw.campos[2];
    const float inv = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
    float Y[16];
    sh_basis(dx * inv, dy * inv, dz * inv, Y);
    const int nk = (sc.sh_degree + 1) * (sc.sh_degree + 1);
    // this Gaussian's coefficients are contiguous: [coef][channel]
    const float *f = sc.sh_dev + i * (int64_t)nk * 3;
    float col[3] = {0.5f, 0.5f, 0.5f};
    if (nk == 16) {
        // degree 3: 48 floats = 12 independent 16-byte loads issued together
        float4 q[12];
        const float4 *f4 = reinterpret_cast<const float4 *>(f);
#pragma unroll
        for (int k = 0; k < 12; ++k) q[k] = f4[k];
        const float *c = reinterpret_cast<const float *>(q);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            col[0] = fmaf(Y[k], c[3 * k + 0], col[0]);
            col[1] = fmaf(Y[k], c[3 * k + 1], col[1]);
            col[2] = fmaf(Y[k], c[3 * k + 2], col[2]);
        }
    } else {
        for (int k = 0; k < nk; ++k) {
            col[0] = fmaf(Y[k], f[3 * k + 0], col[0]);
            col[1] = fmaf(Y[k], f[3 * k + 1], col[1]);
            col[2] = fmaf(Y[k], f[3 * k + 2], col[2]);
        }
    }
    rr.r = fmaxf(col[0], 0.0f);
    rr.g = fmaxf(col[1], 0.0f);
    rr.b = fmaxf(col[2], 0.0f);
}

// The blend record of every entry (Sec. 3.5: formed once and reused by every
// tile and round that draws it): entry j is (view, Gaussian) slot ent[j]; its
// key path is evaluated again with the same float64 operations as in
// k_preprocess (so the rectangle and depth equal the ones its keys were
// counted with), then the record -- centre in float64, inverse covariance in
// LDL^T form for exp2, opacity, the view-dependent colour and the depth bits
// -- and the rectangle are written at j, contiguously, and map[slot] = j.
// Grid-stride over the entries (the device count, bounded by cap, the records'
// capacity; a larger count raises bit 2 of err, when given, and leaves the
// rest unwritten).
__global__ void __launch_bounds__(256) k_entry_record(a3fr_scene sc, const GeomPack *__restrict__ pack,
                                                      const DevView *__restrict__ views,
                                                      const uint32_t *__restrict__ ent, const uint32_t *n_ent,
                                                      int64_t cap, const double *__restrict__ exp_tab,
                                                      Record *__restrict__ rec, uint64_t *__restrict__ rect_e,
                                                      uint32_t *__restrict__ map, uint32_t *err) {
    __shared__ double s_exp[kExtentSteps + 1];
    for (int k = threadIdx.x; k <= kExtentSteps; k += blockDim.x) s_exp[k] = exp_tab[k];
    __syncthreads();
    int64_t E = *n_ent;
    if (E > cap) {
        if (err && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(err, 4u);  // err NULL: the caller checks
        E = cap;
    }
    const int64_t n = sc.n;
    const double kLog2e = 1.4426950408889634;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < E; j += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t slot = ent[j];
        const int v = (int)(slot / (uint64_t)n);
        const int64_t i = (int64_t)slot - (int64_t)v * n;
        const DevView &dv = views[v];
        const GeomPack g = pack[i];
        const double mx = g.a.x, my = g.a.y, mz = g.a.z;
        Cov3 S;
        const bool cov_ok = gaussian_cov3(g.b.w, g.c.x, g.c.y, g.c.z, g.b.x, g.b.y, g.b.z, S);
        EyeProj E3;
        eye_project(dv.v, mx, my, mz, cov_ok, S, E3);
        const float op = g.a.w;
        LayerProj L;
        layer_project(dv, E3, footprint_q(op, s_exp), L);
        // an entry is visible in its view (it was counted so); the inverse
        // covariance in LDL^T form, float64 then rounded once
        const double inv_c = 1.0 / L.c, inv_det = 1.0 / L.det;
        Record R;
        R.u = L.u; R.v = L.w;
        R.a2 = (float)(-0.5 * kLog2e * (L.c * inv_det));
        R.k = (float)(-(L.b * inv_c));
        R.c2 = (float)(-0.5 * kLog2e * inv_c);
        R.o = op;
        colour_into(sc, dv.v, i, g.a, R);
        R.dbits = __float_as_uint((float)E3.p2);
        rec[j] = R;
        rect_e[j] = pack_rect(L);
        map[slot] = (uint32_t)j;
    }
}

void launch_entry_record(const a3fr_scene &sc, const GeomPack *pack, const DevView *views, const uint32_t *ent,
                         const uint32_t *n_ent, int64_t m, int64_t cap, const double *exp_tab, Record *rec,
                         uint64_t *rect_e, uint32_t *map, uint32_t *err, hipStream_t s) {
    const int64_t work = m < cap ? m : cap;
    if (work <= 0) return;
    int64_t blocks = (work + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_entry_record, dim3((unsigned)blocks), dim3(256), 0, s, sc, pack, views, ent, n_ent, cap,
                       exp_tab, rec, rect_e, map, err);
}

}  // namespace a3fr
