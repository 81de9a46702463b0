// Rasterization stage (paper Sec. 2.3: the colour of a pixel is the
// front-to-back volume-rendering sum over the depth-sorted ellipses of its
// tile), the foveated composite (Sec. 2.2: full detail at the gaze, coarser
// around it), and the quality judge.
//
// Blend mapping on CDNA (wave64): one wavefront per 16x16 tile, each lane
// owns four horizontally adjacent pixels of one row (so the row-dependent
// terms of the quadratic form are computed once per Gaussian per lane).  The
// tile's depth-sorted list is consumed in batches of 64: each lane gathers one
// 48-byte record, converts its centre to tile-relative float32 (exact enough
// at any image size because the record keeps the centre in float64) and puts
// it in LDS; then every lane walks the batch with broadcast LDS reads.  The
// wave stops as soon as a ballot finds no live pixel.
#include "a3fr_internal.h"

namespace a3fr {

constexpr int kBatch = 64;

// COUNT: also count evaluated (pixel, Gaussian) pairs -- every list entry a
// pixel evaluates while it is live, the one that stops it included.
template <bool COUNT>
__global__ void __launch_bounds__(64) k_blend(const DevView *__restrict__ views, int nv,
                                              const uint8_t *__restrict__ active, const uint32_t *__restrict__ ranges,
                                              const uint32_t *__restrict__ vals, const Record *__restrict__ rec,
                                              int64_t n, float *__restrict__ rgb, float *__restrict__ Tout,
                                              uint32_t *__restrict__ lastout, unsigned long long *__restrict__ pairs) {
    const int64_t gt = blockIdx.x;
    if (!active[gt]) return;
    // view of this tile: views are ordered by tile offset
    int lo = 0, hi = nv - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].tile_off <= gt) lo = mid; else hi = mid - 1;
    }
    const DevView &dv = views[lo];
    const int64_t lt = gt - dv.tile_off;
    const int tx = (int)(lt % dv.tiles_x), ty = (int)(lt / dv.tiles_x);
    const int W = dv.v.width, H = dv.v.height;
    const int x0 = tx * kTile, y0 = ty * kTile;
    const int lane = threadIdx.x;
    const int py = lane >> 2, px0 = (lane & 3) * 4;
    const float fy = (float)py + 0.5f;
    float fxq[4];
    bool alive[4];
    float T[4], Cr[4], Cg[4], Cb[4];
    uint32_t last[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        fxq[q] = (float)(px0 + q) + 0.5f;
        alive[q] = (x0 + px0 + q < W) && (y0 + py < H);
        T[q] = 1.0f; Cr[q] = Cg[q] = Cb[q] = 0.0f; last[q] = 0;
    }
    const uint32_t start = ranges[2 * gt], end = ranges[2 * gt + 1];
    const Record *R = rec + (int64_t)lo * n;
    __shared__ float s_u[kBatch], s_v[kBatch], s_a[kBatch], s_k[kBatch], s_c[kBatch], s_o[kBatch];
    __shared__ float s_r[kBatch], s_g[kBatch], s_b[kBatch];
    const double dx0 = (double)x0, dy0 = (double)y0;
    uint32_t npairs = 0;

    for (uint32_t b0 = start; b0 < end; b0 += kBatch) {
        if (__ballot(alive[0] || alive[1] || alive[2] || alive[3]) == 0ull) break;
        const uint32_t j = b0 + lane;
        if (j < end) {
            const Record r = R[vals[j]];
            s_u[lane] = (float)(r.u - dx0);
            s_v[lane] = (float)(r.v - dy0);
            s_a[lane] = r.a2; s_k[lane] = r.k; s_c[lane] = r.c2; s_o[lane] = r.o;
            s_r[lane] = r.r; s_g[lane] = r.g; s_b[lane] = r.b;
        }
        __syncthreads();
        const uint32_t cnt = (end - b0) < (uint32_t)kBatch ? (end - b0) : (uint32_t)kBatch;
        for (uint32_t jj = 0; jj < cnt; ++jj) {
            const float mu = s_u[jj], mv = s_v[jj], a2 = s_a[jj], kk = s_k[jj], c2 = s_c[jj], o = s_o[jj];
            const float dy = fy - mv;
            const float kdy = kk * dy;
            const float cdy = c2 * dy * dy;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (COUNT) npairs += alive[q] ? 1u : 0u;
                const float t = (fxq[q] - mu) + kdy;
                const float e = fmaf(a2, t * t, cdy);
                const float al = fminf(kAlphaMax, o * __builtin_amdgcn_exp2f(e));
                if (alive[q] && al >= kAlphaMin) {
                    const float Tn = T[q] * (1.0f - al);
                    if (Tn < kTMin) {
                        alive[q] = false;
                    } else {
                        const float wgt = al * T[q];
                        Cr[q] = fmaf(wgt, s_r[jj], Cr[q]);
                        Cg[q] = fmaf(wgt, s_g[jj], Cg[q]);
                        Cb[q] = fmaf(wgt, s_b[jj], Cb[q]);
                        T[q] = Tn;
                        last[q] = b0 - start + jj + 1;
                    }
                }
            }
        }
        __syncthreads();
    }
    if (COUNT) {
        unsigned long long tot = npairs;
        for (int off = 32; off > 0; off >>= 1) tot += __shfl_down(tot, off, 64);
        if (lane == 0) atomicAdd(pairs, tot);
    }
    const int64_t HW = (int64_t)W * H;
    float *img = rgb + 3 * dv.img_off;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int x = x0 + px0 + q, y = y0 + py;
        if (x < W && y < H) {
            const int64_t pix = (int64_t)y * W + x;
            img[pix] = Cr[q] + T[q] * dv.v.bg[0];
            img[HW + pix] = Cg[q] + T[q] * dv.v.bg[1];
            img[2 * HW + pix] = Cb[q] + T[q] * dv.v.bg[2];
            if (Tout) Tout[dv.img_off + pix] = T[q];
            if (lastout) lastout[dv.img_off + pix] = last[q];
        }
    }
}

void launch_blend(const DevView *views, int nv, int64_t ntiles, const uint8_t *active, const uint32_t *ranges,
                  const uint32_t *vals, const Record *rec, int64_t n, float *rgb, float *T, uint32_t *last,
                  unsigned long long *pairs, hipStream_t s) {
    if (ntiles == 0) return;
    if (pairs)
        hipLaunchKernelGGL(k_blend<true>, dim3((unsigned)ntiles), dim3(64), 0, s, views, nv, active, ranges, vals, rec,
                           n, rgb, T, last, pairs);
    else
        hipLaunchKernelGGL(k_blend<false>, dim3((unsigned)ntiles), dim3(64), 0, s, views, nv, active, ranges, vals,
                           rec, n, rgb, T, last, pairs);
}

// ------------------------------------------------------------------------
// reverse blend
// ------------------------------------------------------------------------
// Same tile mapping as k_blend (one wave per tile, four horizontally adjacent
// pixels per lane, 64-record LDS batches), but the batches are taken from the
// back: each pixel starts at its last blended Gaussian with its final
// transmittance T and S = T (bg . D), D = dL/dC, and for each blended
// Gaussian j (alpha >= 1/255, position < last) going towards the front
//   T_j   = T_{j+1} / (1 - alpha_j)           (transmittance in front of j)
//   dL/dalpha_j = T_j (c_j . D) - S / (1 - alpha_j),   S += (c_j . D) alpha_j T_j,
//   dL/dc_j    += alpha_j T_j D.
// Through alpha = o 2^e (when not clamped at 0.99): dL/do += dL/dalpha 2^e and
// g = dL/de = dL/dalpha alpha ln 2.  With e = a2 t^2 + c2 dy^2, t = dx + k dy,
// the pixel sums kept per Gaussian are
//   [0] sum g t^2, [1] sum g t, [2] sum g t dy, [3] sum g dy^2, [4] sum g dy,
//   [5] dL/do, [6..8] dL/d(r, g, b)
// (a2, k, c2 are constant per Gaussian and are applied in the projection's
// reverse).  The 9 sums are reduced across the wave and added with one atomic
// each into acc[(view * n + index) * 12 + 0..8].
__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__global__ void __launch_bounds__(64) k_blend_bwd(const DevView *__restrict__ views, int nv,
                                                  const uint8_t *__restrict__ active,
                                                  const uint32_t *__restrict__ ranges,
                                                  const uint32_t *__restrict__ vals, const Record *__restrict__ rec,
                                                  int64_t n, const float *__restrict__ dl, const float *__restrict__ Tin,
                                                  const uint32_t *__restrict__ lastin, float *__restrict__ acc) {
    const int64_t gt = blockIdx.x;
    if (!active[gt]) return;
    int lo = 0, hi = nv - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].tile_off <= gt) lo = mid; else hi = mid - 1;
    }
    const DevView &dv = views[lo];
    const int64_t lt = gt - dv.tile_off;
    const int tx = (int)(lt % dv.tiles_x), ty = (int)(lt / dv.tiles_x);
    const int W = dv.v.width, H = dv.v.height;
    const int x0 = tx * kTile, y0 = ty * kTile;
    const int lane = threadIdx.x;
    const int py = lane >> 2, px0 = (lane & 3) * 4;
    const float fy = (float)py + 0.5f;
    const uint32_t start = ranges[2 * gt], end = ranges[2 * gt + 1];
    const uint32_t len = end - start;
    const int64_t HW = (int64_t)W * H;
    const float *dimg = dl + 3 * dv.img_off;
    float fxq[4], T[4], S[4], D0[4], D1[4], D2[4];
    uint32_t last[4];
    uint32_t maxlast = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        fxq[q] = (float)(px0 + q) + 0.5f;
        const int x = x0 + px0 + q, y = y0 + py;
        T[q] = 1.0f; S[q] = 0.0f; D0[q] = D1[q] = D2[q] = 0.0f; last[q] = 0;
        if (x < W && y < H) {
            const int64_t pix = (int64_t)y * W + x;
            T[q] = Tin[dv.img_off + pix];
            last[q] = min(lastin[dv.img_off + pix], len);
            D0[q] = dimg[pix]; D1[q] = dimg[HW + pix]; D2[q] = dimg[2 * HW + pix];
            S[q] = T[q] * (dv.v.bg[0] * D0[q] + dv.v.bg[1] * D1[q] + dv.v.bg[2] * D2[q]);
            maxlast = max(maxlast, last[q]);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) maxlast = max(maxlast, (uint32_t)__shfl_xor((int)maxlast, off, 64));
    const Record *R = rec + (int64_t)lo * n;
    float *A = acc + (int64_t)lo * n * 12;
    __shared__ float s_u[kBatch], s_v[kBatch], s_a[kBatch], s_k[kBatch], s_c[kBatch], s_o[kBatch];
    __shared__ float s_r[kBatch], s_g[kBatch], s_b[kBatch];
    __shared__ uint32_t s_i[kBatch];
    const double dx0 = (double)x0, dy0 = (double)y0;
    const float kLn2 = 0.6931471805599453f;

    for (int64_t bend = maxlast; bend > 0; bend -= kBatch) {
        const uint32_t bstart = bend > kBatch ? (uint32_t)(bend - kBatch) : 0u;
        const uint32_t cnt = (uint32_t)bend - bstart;
        if ((uint32_t)lane < cnt) {
            const uint32_t idx = vals[start + bstart + lane];
            const Record r = R[idx];
            s_u[lane] = (float)(r.u - dx0);
            s_v[lane] = (float)(r.v - dy0);
            s_a[lane] = r.a2; s_k[lane] = r.k; s_c[lane] = r.c2; s_o[lane] = r.o;
            s_r[lane] = r.r; s_g[lane] = r.g; s_b[lane] = r.b;
            s_i[lane] = idx;
        }
        __syncthreads();
        for (int jj = (int)cnt - 1; jj >= 0; --jj) {
            const uint32_t pos = bstart + (uint32_t)jj;
            const float mu = s_u[jj], mv = s_v[jj], a2 = s_a[jj], kk = s_k[jj], c2 = s_c[jj], o = s_o[jj];
            const float cr = s_r[jj], cg = s_g[jj], cb = s_b[jj];
            const float dy = fy - mv;
            const float kdy = kk * dy;
            const float cdy = c2 * dy * dy;
            float g_t2 = 0.f, g_t = 0.f, g_tdy = 0.f, g_dy2 = 0.f, g_dy = 0.f, g_o = 0.f, g_r = 0.f, g_g = 0.f, g_b = 0.f;
            bool hit = false;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float t = (fxq[q] - mu) + kdy;
                const float e = fmaf(a2, t * t, cdy);
                const float ex = __builtin_amdgcn_exp2f(e);
                const float araw = o * ex;
                const float al = fminf(kAlphaMax, araw);
                if (pos < last[q] && al >= kAlphaMin) {
                    hit = true;
                    const float oma = 1.0f - al;
                    const float Tb = T[q] / oma;
                    const float cD = cr * D0[q] + cg * D1[q] + cb * D2[q];
                    const float w = al * Tb;
                    g_r = fmaf(w, D0[q], g_r);
                    g_g = fmaf(w, D1[q], g_g);
                    g_b = fmaf(w, D2[q], g_b);
                    const float dal = Tb * cD - S[q] / oma;
                    S[q] = fmaf(cD, w, S[q]);
                    T[q] = Tb;
                    if (araw < kAlphaMax) {
                        const float g = dal * al * kLn2;
                        const float gt = g * t;
                        g_t2 = fmaf(gt, t, g_t2);
                        g_t += gt;
                        g_tdy = fmaf(gt, dy, g_tdy);
                        const float gdy = g * dy;
                        g_dy2 = fmaf(gdy, dy, g_dy2);
                        g_dy += gdy;
                        g_o = fmaf(dal, ex, g_o);
                    }
                }
            }
            if (__ballot(hit) != 0ull) {
                g_t2 = wave_sum(g_t2); g_t = wave_sum(g_t); g_tdy = wave_sum(g_tdy);
                g_dy2 = wave_sum(g_dy2); g_dy = wave_sum(g_dy); g_o = wave_sum(g_o);
                g_r = wave_sum(g_r); g_g = wave_sum(g_g); g_b = wave_sum(g_b);
                if (lane < 9) {
                    const float val = lane == 0 ? g_t2 : lane == 1 ? g_t : lane == 2 ? g_tdy : lane == 3 ? g_dy2 :
                                      lane == 4 ? g_dy : lane == 5 ? g_o : lane == 6 ? g_r : lane == 7 ? g_g : g_b;
                    atomicAdd(&A[(int64_t)s_i[jj] * 12 + lane], val);
                }
            }
        }
        __syncthreads();
    }
}

void launch_blend_bwd(const DevView *views, int nv, int64_t ntiles, const uint8_t *active, const uint32_t *ranges,
                      const uint32_t *vals, const Record *rec, int64_t n, const float *dl, const float *T,
                      const uint32_t *last, float *acc, hipStream_t s) {
    if (ntiles == 0) return;
    hipLaunchKernelGGL(k_blend_bwd, dim3((unsigned)ntiles), dim3(64), 0, s, views, nv, active, ranges, vals, rec, n,
                       dl, T, last, acc);
}

// ------------------------------------------------------------------------
// composite
// ------------------------------------------------------------------------
__device__ __forceinline__ int region_of(int x, int y, double gx, double gy, double rf, double rm) {
    const double dx = ((double)x + 0.5) - gx, dy = ((double)y + 0.5) - gy;
    const double r2 = dx * dx + dy * dy;
    if (r2 <= rf * rf) return 0;
    if (r2 <= rm * rm) return 1;
    return 2;
}

// bilinear, align_corners = false, clamp to edge; sx = (x + 0.5)/s - 0.5
__device__ __forceinline__ void bilinear_setup(int x, int s, int Wl, int &i0, int &i1, float &w) {
    float sx = ((float)x + 0.5f) / (float)s - 0.5f;
    sx = fminf(fmaxf(sx, 0.0f), (float)(Wl - 1));
    const float f = floorf(sx);
    i0 = (int)f;
    i1 = i0 + 1 < Wl ? i0 + 1 : Wl - 1;
    w = sx - f;
}

__global__ void k_composite(int W, int H, double gx, double gy, double rf, double rm,
                            const float *__restrict__ fovea, const float *__restrict__ mid, int sm,
                            const float *__restrict__ periph, int sp, const float *__restrict__ periph_full,
                            float *__restrict__ out) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= W) return;
    const int64_t HW = (int64_t)W * H, pix = (int64_t)y * W + x;
    const int reg = region_of(x, y, gx, gy, rf, rm);
    if (reg == 0) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) out[ch * HW + pix] = fovea[ch * HW + pix];
        return;
    }
    if (reg == 2 && periph_full) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) out[ch * HW + pix] = periph_full[ch * HW + pix];
        return;
    }
    const int s = reg == 1 ? sm : sp;
    const float *src = reg == 1 ? mid : periph;
    const int Wl = W / s, Hl = H / s;
    int xa, xb, ya, yb;
    float wx, wy;
    bilinear_setup(x, s, Wl, xa, xb, wx);
    bilinear_setup(y, s, Hl, ya, yb, wy);
    const int64_t HWl = (int64_t)Wl * Hl;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const float *p = src + ch * HWl;
        const float top = (1.0f - wx) * p[(int64_t)ya * Wl + xa] + wx * p[(int64_t)ya * Wl + xb];
        const float bot = (1.0f - wx) * p[(int64_t)yb * Wl + xa] + wx * p[(int64_t)yb * Wl + xb];
        out[ch * HW + pix] = (1.0f - wy) * top + wy * bot;
    }
}

void launch_composite(int W, int H, double gx, double gy, double rf, double rm, const float *fovea,
                      const float *mid, int sm, const float *periph, int sp, const float *periph_full,
                      float *out, hipStream_t s) {
    if (W <= 0 || H <= 0) return;
    hipLaunchKernelGGL(k_composite, dim3((unsigned)((W + 255) / 256), (unsigned)H), dim3(256), 0, s, W, H, gx, gy,
                       rf, rm, fovea, mid, sm, periph, sp, periph_full, out);
}

// ------------------------------------------------------------------------
// region squared error (quality judge)
// ------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_region_sse(int W, int H, double gx, double gy, double rf, double rm,
                                                    const float *__restrict__ a, const float *__restrict__ b,
                                                    double *partial, unsigned long long *cnt) {
    const int64_t HW = (int64_t)W * H;
    double acc[3] = {0.0, 0.0, 0.0};
    unsigned long long c[3] = {0, 0, 0};
    for (int64_t pix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pix < HW;
         pix += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(pix % W), y = (int)(pix / W);
        const int reg = region_of(x, y, gx, gy, rf, rm);
        double s = 0.0;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const double u = fmin(fmax((double)a[ch * HW + pix], 0.0), 1.0);
            const double v = fmin(fmax((double)b[ch * HW + pix], 0.0), 1.0);
            s += (u - v) * (u - v);
        }
        acc[0] += reg == 0 ? s : 0.0; acc[1] += reg == 1 ? s : 0.0; acc[2] += reg == 2 ? s : 0.0;
        c[reg] += 1;
    }
    __shared__ double sa[3][256];
    __shared__ unsigned long long sc[3][256];
    for (int r = 0; r < 3; ++r) { sa[r][threadIdx.x] = acc[r]; sc[r][threadIdx.x] = c[r]; }
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            for (int r = 0; r < 3; ++r) {
                sa[r][threadIdx.x] += sa[r][threadIdx.x + off];
                sc[r][threadIdx.x] += sc[r][threadIdx.x + off];
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int r = 0; r < 3; ++r) { partial[3 * blockIdx.x + r] = sa[r][0]; cnt[3 * blockIdx.x + r] = sc[r][0]; }
}

void launch_region_sse(int W, int H, double gx, double gy, double rf, double rm, const float *a, const float *b,
                       double *partial, unsigned long long *cnt, int nblk, hipStream_t s) {
    hipLaunchKernelGGL(k_region_sse, dim3((unsigned)nblk), dim3(256), 0, s, W, H, gx, gy, rf, rm, a, b, partial, cnt);
}

// ------------------------------------------------------------------------
// float64 self-check
// ------------------------------------------------------------------------
__global__ void k_fp64_probe(const double *x, const double *y, double *sq, double *dv, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    sq[i] = sqrt(x[i]);
    dv[i] = x[i] / y[i];
}

void launch_fp64_probe(const double *x, const double *y, double *sq, double *dv, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fp64_probe, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, y, sq, dv, n);
}

}  // namespace a3fr
