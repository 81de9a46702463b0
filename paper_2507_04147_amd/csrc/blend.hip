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

constexpr int kBatch = 64;   // LDS batch of the reverse blend
constexpr float kCullAlpha = 0.95f * kAlphaMin;  // tile bound below which a list entry is dropped

// Whether a list entry can reach alpha >= 1/255 at some pixel centre of its
// tile ((mu, mv): its centre relative to the tile corner).  Over the box of
// centres, the exponent a2 t^2 + c2 dy^2 (a2, c2 <= 0) is at most
// a2 min t^2 + c2 min dy^2, with dy over its interval and t = dx + k dy over
// the sum of intervals; an entry whose bound gives o 2^e below kCullAlpha is
// below the threshold at every pixel (the 5% margin, 0.074 in the exponent,
// is far above the float32 rounding of either side), so dropping it changes
// no pixel and no gradient.
// The same bound over the pixel centres [bx + 0.5, bx + size - 0.5] x
// [by + 0.5, by + size - 0.5] of a square block of the tile.
__device__ __forceinline__ bool box_reach(float a2, float k, float c2, float o, float mu, float mv, float bx, float by,
                                          float size) {
    const float dlo = (by + 0.5f) - mv, dhi = (by + size - 0.5f) - mv;
    const float mdy2 = dlo > 0.0f ? dlo * dlo : (dhi < 0.0f ? dhi * dhi : 0.0f);
    const float k0 = k * dlo, k1 = k * dhi;
    const float tlo = ((bx + 0.5f) - mu) + fminf(k0, k1), thi = ((bx + size - 0.5f) - mu) + fmaxf(k0, k1);
    const float mt2 = tlo > 0.0f ? tlo * tlo : (thi < 0.0f ? thi * thi : 0.0f);
    const float eb = a2 * mt2 + c2 * mdy2;
    return !(a2 <= 0.0f && c2 <= 0.0f) || o * __builtin_amdgcn_exp2f(eb) >= kCullAlpha;
}

__device__ __forceinline__ bool tile_reach(const Record &r, float mu, float mv) {
    return box_reach(r.a2, r.k, r.c2, r.o, mu, mv, 0.0f, 0.0f, (float)kTile);
}

// The exponent at which a Gaussian of opacity o reaches the alpha threshold:
// o 2^e >= 1/255 exactly when e >= -log2(255 o) (o = 0: +inf, never).  Every
// blend (the forward variants, the AMR blend and the reverse blend) takes
// this same float32 decision on the exponent, so that exp2 is evaluated only
// for the entries some pixel of the wave takes; its rounding differs from
// that of o 2^e by far less than the float32 error bound within which the
// oracle flags a decision as ambiguous.
__device__ __forceinline__ float take_exponent(float o) { return -__builtin_amdgcn_logf(255.0f * o); }

// Blend one tile.  BATCH: records staged in LDS per step; ROWS: pixel rows per
// lane (1: four horizontally adjacent pixels, 2: a 2 x 2 block).  Every
// pixel evaluates exactly the same float32 expressions over the same list in
// the same order whatever BATCH, ROWS and the schedule, so all variants give
// bit-identical images.
// COUNT: also count evaluated (pixel, Gaussian) pairs -- every list entry a
// pixel reaches while it is live, the one that stops it included (the
// method's work; entries dropped by the tile bound below count as well).
template <bool COUNT, int BATCH, int ROWS>
__device__ __forceinline__ void blend_tile(int64_t gt, const DevView *__restrict__ views, int nv,
                                           const uint32_t *__restrict__ ranges, const uint32_t *__restrict__ vals,
                                           const Record *__restrict__ rec, int64_t n, float *__restrict__ rgb,
                                           float *__restrict__ Tout, uint32_t *__restrict__ lastout, uint32_t &npairs) {
    constexpr int COLS = 4 / ROWS;
    __shared__ float s_u[BATCH], s_v[BATCH], s_a[BATCH], s_k[BATCH], s_c[BATCH], s_o[BATCH];
    __shared__ float s_r[BATCH], s_g[BATCH], s_b[BATCH], s_e[BATCH];
    __shared__ uint32_t s_j[BATCH];
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
    // lane's pixel block: COLS columns x ROWS rows
    const int py0 = ROWS == 1 ? (lane >> 2) : (lane >> 3) * 2;
    const int px0 = ROWS == 1 ? (lane & 3) * 4 : (lane & 7) * 2;
    float fyr[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) fyr[r] = (float)(py0 + r) + 0.5f;
    float fxq[4];
    // per pixel 0 while it is live, +inf once it has stopped or when it lies
    // outside the image: added to an entry's take exponent, one compare per
    // pair then also carries the live test
    float thr[4];
    float T[4], Cr[4], Cg[4], Cb[4];
    uint32_t last[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int cx = px0 + q % COLS, cy = py0 + q / COLS;
        fxq[q] = (float)cx + 0.5f;
        thr[q] = (x0 + cx < W) && (y0 + cy < H) ? 0.0f : INFINITY;
        T[q] = 1.0f; Cr[q] = Cg[q] = Cb[q] = 0.0f; last[q] = 0;
    }
    const uint32_t start = ranges[2 * gt], end = ranges[2 * gt + 1];
    const Record *R = rec + (int64_t)lo * n;
    const double dx0 = (double)x0, dy0 = (double)y0;
    // software pipeline: the records of the next batch are gathered while the
    // current one is blended (rn: this lane's slots of the batch at b0)
    constexpr int PARTS = (BATCH + 63) / 64;
    Record rn[PARTS];
#pragma unroll
    for (int part = 0; part < PARTS; ++part) {
        const int slot = part * 64 + lane;
        if (slot < BATCH && start + slot < end) rn[part] = R[vals[start + slot]];
    }

    for (uint32_t b0 = start; b0 < end; b0 += BATCH) {
        if (__ballot(fminf(fminf(thr[0], thr[1]), fminf(thr[2], thr[3])) < INFINITY) == 0ull) break;
        // Stage the batch, keeping only the entries that can reach the tile
        // (tile_reach), packed in list order with their positions for the
        // last-blended index.
        uint32_t cnt = 0;
#pragma unroll
        for (int part = 0; part < PARTS; ++part) {
            const int slot = part * 64 + lane;
            const uint32_t j = b0 + slot;
            bool keep = false;
            Record r;
            float mu = 0.0f, mv = 0.0f;
            if (slot < BATCH && j < end) {
                r = rn[part];
                mu = (float)(r.u - dx0);
                mv = (float)(r.v - dy0);
                keep = tile_reach(r, mu, mv);
            }
            const uint64_t km = __ballot(keep);
            if (keep) {
                const int at = (int)cnt + __popcll(km & ((1ull << lane) - 1ull));
                s_u[at] = mu;
                s_v[at] = mv;
                s_a[at] = r.a2; s_k[at] = r.k; s_c[at] = r.c2; s_o[at] = r.o;
                s_r[at] = r.r; s_g[at] = r.g; s_b[at] = r.b;
                s_e[at] = take_exponent(r.o);
                s_j[at] = (uint32_t)slot;
            }
            cnt += (uint32_t)__popcll(km);
        }
        __syncthreads();
#pragma unroll
        for (int part = 0; part < PARTS; ++part) {
            const int slot = part * 64 + lane;
            const uint32_t j = b0 + BATCH + slot;
            if (slot < BATCH && j < end) rn[part] = R[vals[j]];
        }
        // COUNT: a dropped entry is still a pair of every live pixel (nothing
        // changes between kept entries, so the live pixels are those at the next one)
        int prev = -1;
        for (uint32_t jj = 0; jj < cnt; ++jj) {
            const float mu = s_u[jj], mv = s_v[jj], a2 = s_a[jj], kk = s_k[jj], c2 = s_c[jj], o = s_o[jj];
            const float cr = s_r[jj], cg = s_g[jj], cb = s_b[jj];
            const uint32_t idx = b0 - start + s_j[jj] + 1;
            if (COUNT) {
                uint32_t live = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) live += thr[q] < INFINITY ? 1u : 0u;
                npairs += live * (uint32_t)((int)s_j[jj] - prev - 1);
                prev = (int)s_j[jj];
            }
            float kdy[ROWS], cdy[ROWS];
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const float dy = fyr[r] - mv;
                kdy[r] = kk * dy;
                cdy[r] = c2 * dy * dy;
            }
            const float et = s_e[jj];
            float ex[4];
            bool take[4];
            bool any = false;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int rr = q / COLS;
                if (COUNT) npairs += thr[q] < INFINITY ? 1u : 0u;
                const float t = (fxq[q] - mu) + kdy[rr];
                ex[q] = fmaf(a2, t * t, cdy[rr]);
                take[q] = ex[q] >= et + thr[q];
                any = any || take[q];
            }
            // most evaluated pairs fall outside the footprint (alpha < 1/255): skip when the whole wave does
            if (__ballot(any) == 0ull) continue;
            // branch-free: a pixel that does not blend adds fma(0, c, C) = C (colours >= 0)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float al = fminf(kAlphaMax, o * __builtin_amdgcn_exp2f(ex[q]));
                const float Tn = T[q] * (1.0f - al);
                const bool stop = take[q] && Tn < kTMin;
                const bool blend = take[q] && !stop;
                const float wgt = blend ? al * T[q] : 0.0f;
                Cr[q] = fmaf(wgt, cr, Cr[q]);
                Cg[q] = fmaf(wgt, cg, Cg[q]);
                Cb[q] = fmaf(wgt, cb, Cb[q]);
                T[q] = blend ? Tn : T[q];
                last[q] = blend ? idx : last[q];
                thr[q] = stop ? INFINITY : thr[q];
            }
        }
        if (COUNT) {
            const int nb = (int)((end - b0) < (uint32_t)BATCH ? (end - b0) : (uint32_t)BATCH);
            uint32_t live = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) live += thr[q] < INFINITY ? 1u : 0u;
            npairs += live * (uint32_t)(nb - prev - 1);
        }
        __syncthreads();
    }
    const int64_t HW = (int64_t)W * H;
    float *img = rgb + 3 * dv.img_off;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int x = x0 + px0 + q % COLS, y = y0 + py0 + q / COLS;
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

template <bool COUNT>
__device__ __forceinline__ void add_pairs(uint32_t npairs, unsigned long long *pairs) {
    if (COUNT) {
        unsigned long long tot = npairs;
        for (int off = 32; off > 0; off >>= 1) tot += __shfl_down(tot, off, 64);
        if ((threadIdx.x & 63) == 0) atomicAdd(pairs, tot);
    }
}

// ------------------------------------------------------------------------
// AMR levels (Sec. 3.4): each tile is split into 8 x 8 blocks of 2 x 2
// pixels; a tile of level L renders the first L positions of every block
// (top-left, top-right, bottom-left, bottom-right) and the other positions
// inherit the rendered pixel above them, else the top-left one.  Lane l owns
// block (l % 8, l / 8), so a level-L tile costs L pixels per lane.  The
// level follows the distance from the gaze to the tile's pixel-centre
// rectangle: <= r4: 4, <= r3: 3, <= r2: 2, else 1.  Rendered pixels evaluate
// the same float32 expressions over the same list as k_blend.
// ------------------------------------------------------------------------
__device__ __forceinline__ int amr_level(const a3fr_view &v, int tx, int ty, double r4, double r3, double r2) {
    int xe = (tx + 1) * kTile; if (xe > v.width) xe = v.width;
    int ye = (ty + 1) * kTile; if (ye > v.height) ye = v.height;
    const double x0 = (double)(tx * kTile) + 0.5, x1 = (double)xe - 0.5;
    const double y0 = (double)(ty * kTile) + 0.5, y1 = (double)ye - 0.5;
    const double ddx = fmax(fmax(x0 - v.gx, v.gx - x1), 0.0);
    const double ddy = fmax(fmax(y0 - v.gy, v.gy - y1), 0.0);
    const double d2 = ddx * ddx + ddy * ddy;
    return d2 <= r4 * r4 ? 4 : d2 <= r3 * r3 ? 3 : d2 <= r2 * r2 ? 2 : 1;
}

// ---- AMR levels by Gaussian count ------------------------------------------
// A tile's count key orders the tiles of a view by (number of Gaussians
// descending, tile index ascending): (count << 32) | ~local tile index.
__device__ __forceinline__ uint64_t amr_count_key(const uint32_t *ranges, int64_t gt, int64_t t) {
    const uint32_t c = ranges[2 * gt + 1] - ranges[2 * gt];
    return ((uint64_t)c << 32) | (uint64_t)(0xffffffffu - (uint32_t)t);
}

// Number of a view's T tiles that reach the level of fraction f: ceil(f T).
__device__ __forceinline__ int64_t amr_count_k(double f, int64_t T) {
    const int64_t k = (int64_t)ceil(f * (double)T);
    return k < T ? k : T;
}

// One block per view: for each fraction f of (f4, f3, f2), the k-th largest
// count key with k = ceil(f T) (T tiles of the view), by an MSD radix select
// over the 64-bit keys (8-bit digits, a block histogram per digit); a tile
// reaches that level iff its key is at least the threshold (k = 0: none does;
// the threshold is not written).
__global__ void __launch_bounds__(1024) k_amr_thresholds(const DevView *__restrict__ views,
                                                         const uint32_t *__restrict__ ranges, double f4, double f3,
                                                         double f2, uint64_t *__restrict__ thr) {
    __shared__ uint32_t hist[256];
    __shared__ unsigned long long s_prefix;
    __shared__ uint32_t s_krem;
    const DevView &dv = views[blockIdx.x];
    const int64_t T = (int64_t)dv.tiles_x * dv.tiles_y;
    const double fr[3] = {f4, f3, f2};
    for (int q = 0; q < 3; ++q) {
        const int64_t k = amr_count_k(fr[q], T);
        if (k <= 0) continue;  // uniform over the block
        if (threadIdx.x == 0) {
            s_prefix = 0ull;
            s_krem = (uint32_t)k;
        }
        __syncthreads();
        for (int d = 7; d >= 0; --d) {
            for (int b = threadIdx.x; b < 256; b += blockDim.x) hist[b] = 0u;
            __syncthreads();
            const uint64_t prefix = s_prefix;
            for (int64_t t = threadIdx.x; t < T; t += blockDim.x) {
                const uint64_t key = amr_count_key(ranges, dv.tile_off + t, t);
                if (d == 7 || (key >> (8 * (d + 1))) == prefix) atomicAdd(&hist[(key >> (8 * d)) & 255u], 1u);
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                uint32_t above = 0;
                const uint32_t kr = s_krem;
                for (int b = 255; b >= 0; --b) {
                    if (above + hist[b] >= kr) {
                        s_prefix = (prefix << 8) | (uint64_t)b;
                        s_krem = kr - above;
                        break;
                    }
                    above += hist[b];
                }
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) thr[3 * blockIdx.x + q] = s_prefix;
        __syncthreads();
    }
}

// Level of every tile: eccentricity (mode 0), Gaussian count (1) or the
// smaller of the two (2).
__global__ void __launch_bounds__(256) k_amr_levels(const DevView *__restrict__ views, int nv, int64_t ntiles,
                                                    const uint32_t *__restrict__ ranges, double r4, double r3,
                                                    double r2, double f4, double f3, double f2, int mode,
                                                    const uint64_t *__restrict__ thr,
                                                    uint8_t *__restrict__ lv) {
    const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gt >= ntiles) return;
    int lo = 0, hi = nv - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].tile_off <= gt) lo = mid; else hi = mid - 1;
    }
    const DevView &dv = views[lo];
    const int64_t lt = gt - dv.tile_off;
    const int tx = (int)(lt % dv.tiles_x), ty = (int)(lt / dv.tiles_x);
    const int ecc = amr_level(dv.v, tx, ty, r4, r3, r2);
    int cnt = 1;
    if (mode != 0) {
        const uint64_t key = amr_count_key(ranges, gt, lt);
        const int64_t T = (int64_t)dv.tiles_x * dv.tiles_y;
        const double fr[3] = {f4, f3, f2};
#pragma unroll
        for (int q = 0; q < 3; ++q) cnt += amr_count_k(fr[q], T) > 0 && key >= thr[3 * lo + q];
    }
    lv[gt] = (uint8_t)(mode == 0 ? ecc : mode == 1 ? cnt : min(ecc, cnt));
}

template <int NP>
__device__ __forceinline__ void amr_tile(const DevView &dv, int64_t lo, int tx, int ty, uint32_t start, uint32_t end,
                                         const uint32_t *__restrict__ vals, const Record *__restrict__ rec, int64_t n,
                                         float *__restrict__ rgb, bool interp) {
    constexpr int BATCH = 64;
    __shared__ float s_u[BATCH], s_v[BATCH], s_a[BATCH], s_k[BATCH], s_c[BATCH], s_o[BATCH];
    __shared__ float s_r[BATCH], s_g[BATCH], s_b[BATCH], s_e[BATCH];
    const int W = dv.v.width, H = dv.v.height;
    const int x0 = tx * kTile, y0 = ty * kTile;
    const int lane = threadIdx.x;
    const int bx = 2 * (lane & 7), by = 2 * (lane >> 3);  // the lane's 2 x 2 block in the tile
    float fx[NP], fy[NP], T[NP], Cr[NP], Cg[NP], Cb[NP];
    float thr[NP];  // 0 while the pixel is live, +inf once stopped or outside the image
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int cx = bx + (k & 1), cy = by + (k >> 1);
        fx[k] = (float)cx + 0.5f;
        fy[k] = (float)cy + 0.5f;
        thr[k] = (x0 + cx < W) && (y0 + cy < H) ? 0.0f : INFINITY;
        T[k] = 1.0f; Cr[k] = Cg[k] = Cb[k] = 0.0f;
    }
    const Record *R = rec + lo * n;
    const double dx0 = (double)x0, dy0 = (double)y0;
    for (uint32_t b0 = start; b0 < end; b0 += BATCH) {
        bool any_alive = false;
#pragma unroll
        for (int k = 0; k < NP; ++k) any_alive = any_alive || thr[k] < INFINITY;
        if (__ballot(any_alive) == 0ull) break;
        const uint32_t j = b0 + lane;
        bool keep = false;
        Record r;
        float mu = 0.0f, mv = 0.0f;
        if (j < end) {
            r = R[vals[j]];
            mu = (float)(r.u - dx0);
            mv = (float)(r.v - dy0);
            keep = tile_reach(r, mu, mv);
        }
        const uint64_t km = __ballot(keep);
        if (keep) {
            const int at = __popcll(km & ((1ull << lane) - 1ull));
            s_u[at] = mu;
            s_v[at] = mv;
            s_a[at] = r.a2; s_k[at] = r.k; s_c[at] = r.c2; s_o[at] = r.o;
            s_r[at] = r.r; s_g[at] = r.g; s_b[at] = r.b;
            s_e[at] = take_exponent(r.o);
        }
        __syncthreads();
        const uint32_t cnt = (uint32_t)__popcll(km);
        for (uint32_t jj = 0; jj < cnt; ++jj) {
            const float mu = s_u[jj], mv = s_v[jj], a2 = s_a[jj], kk = s_k[jj], c2 = s_c[jj], o = s_o[jj];
            const float et = s_e[jj];
            float ex[NP];
            bool take[NP];
            bool any = false;
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                const float dy = fy[k] - mv;
                const float kdy = kk * dy;
                const float cdy = c2 * dy * dy;
                const float t = (fx[k] - mu) + kdy;
                ex[k] = fmaf(a2, t * t, cdy);
                take[k] = ex[k] >= et + thr[k];
                any = any || take[k];
            }
            if (__ballot(any) == 0ull) continue;
            const float cr = s_r[jj], cg = s_g[jj], cb = s_b[jj];
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                const float al = fminf(kAlphaMax, o * __builtin_amdgcn_exp2f(ex[k]));
                const float Tn = T[k] * (1.0f - al);
                const bool stop = take[k] && Tn < kTMin;
                const bool blend = take[k] && !stop;
                const float wgt = blend ? al * T[k] : 0.0f;
                Cr[k] = fmaf(wgt, cr, Cr[k]);
                Cg[k] = fmaf(wgt, cg, Cg[k]);
                Cb[k] = fmaf(wgt, cb, Cb[k]);
                T[k] = blend ? Tn : T[k];
                thr[k] = stop ? INFINITY : thr[k];
            }
        }
        __syncthreads();
    }
    // rendered positions, then the inherited ones (with interpolation, only the
    // rendered ones: k_amr_interp fills the others from the top-left samples)
    const int64_t HW = (int64_t)W * H;
    float *img = rgb + 3 * dv.img_off;
    float vr[4], vg[4], vb[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int src = k < NP ? k : (k - 2 >= 0 && k - 2 < NP ? k - 2 : 0);
        vr[k] = Cr[src] + T[src] * dv.v.bg[0];
        vg[k] = Cg[src] + T[src] * dv.v.bg[1];
        vb[k] = Cb[src] + T[src] * dv.v.bg[2];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int x = x0 + bx + (k & 1), y = y0 + by + (k >> 1);
        if (x < W && y < H && (k < NP || !interp)) {
            const int64_t pix = (int64_t)y * W + x;
            img[pix] = vr[k];
            img[HW + pix] = vg[k];
            img[2 * HW + pix] = vb[k];
        }
    }
}

__global__ void __launch_bounds__(64) k_blend_amr(const DevView *__restrict__ views, int nv,
                                                  const uint32_t *__restrict__ ranges,
                                                  const uint32_t *__restrict__ vals, const Record *__restrict__ rec,
                                                  int64_t n, const uint8_t *__restrict__ lv, int interp,
                                                  float *__restrict__ rgb) {
    const int64_t gt = blockIdx.x;
    int lo = 0, hi = nv - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].tile_off <= gt) lo = mid; else hi = mid - 1;
    }
    const DevView &dv = views[lo];
    const int64_t lt = gt - dv.tile_off;
    const int tx = (int)(lt % dv.tiles_x), ty = (int)(lt / dv.tiles_x);
    const uint32_t start = ranges[2 * gt], end = ranges[2 * gt + 1];
    const bool ip = interp != 0;
    switch (lv[gt]) {  // wave-uniform
        case 4: amr_tile<4>(dv, lo, tx, ty, start, end, vals, rec, n, rgb, ip); break;
        case 3: amr_tile<3>(dv, lo, tx, ty, start, end, vals, rec, n, rgb, ip); break;
        case 2: amr_tile<2>(dv, lo, tx, ty, start, end, vals, rec, n, rgb, ip); break;
        default: amr_tile<1>(dv, lo, tx, ty, start, end, vals, rec, n, rgb, ip); break;
    }
}

// Interpolation of the unrendered positions of view blockIdx.y: the bilinear
// interpolation of the 2 x 2 blocks' top-left samples (rendered at every level)
// at the pixel's position on that half-resolution grid, clamped at the last
// block: 0.5 (a + b) between two samples, 0.25 ((a + b) + (c + d)) among four.
__global__ void __launch_bounds__(256) k_amr_interp(const DevView *__restrict__ views, const uint8_t *__restrict__ lv,
                                                    float *__restrict__ rgb) {
    const DevView &dv = views[blockIdx.y];
    const int W = dv.v.width, H = dv.v.height;
    const int64_t pix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= (int64_t)W * H) return;
    const int x = (int)(pix % W), y = (int)(pix / W);
    const int k = (x & 1) + 2 * (y & 1);
    if (k < (int)lv[dv.tile_off + (int64_t)(y / kTile) * dv.tiles_x + x / kTile]) return;  // rendered
    const int bx = x >> 1, by = y >> 1, BX = (W + 1) >> 1, BY = (H + 1) >> 1;
    const int x0 = 2 * bx, y0 = 2 * by, x1 = 2 * min(bx + 1, BX - 1), y1 = 2 * min(by + 1, BY - 1);
    const int64_t HW = (int64_t)W * H;
    float *img = rgb + 3 * dv.img_off;
    for (int ch = 0; ch < 3; ++ch) {
        const float *c = img + ch * HW;
        const float a = c[(int64_t)y0 * W + x0];
        float v;
        if ((x & 1) && (y & 1)) {
            const float b = c[(int64_t)y0 * W + x1], cc = c[(int64_t)y1 * W + x0], d = c[(int64_t)y1 * W + x1];
            v = 0.25f * ((a + b) + (cc + d));
        } else if (x & 1) {
            v = 0.5f * (a + c[(int64_t)y0 * W + x1]);
        } else {
            v = 0.5f * (a + c[(int64_t)y1 * W + x0]);
        }
        img[ch * HW + pix] = v;
    }
}

void launch_blend_amr(const DevView *views, int nv, int64_t ntiles, const uint32_t *ranges, const uint32_t *vals,
                      const Record *rec, int64_t n, const AmrLevels &a, uint64_t *thr, uint8_t *lv, float *rgb,
                      int64_t max_pixels, hipStream_t s) {
    if (ntiles == 0) return;
    if (a.mode != 0)
        hipLaunchKernelGGL(k_amr_thresholds, dim3((unsigned)nv), dim3(1024), 0, s, views, ranges, a.f[0], a.f[1],
                           a.f[2], thr);
    hipLaunchKernelGGL(k_amr_levels, dim3((unsigned)((ntiles + 255) / 256)), dim3(256), 0, s, views, nv, ntiles,
                       ranges, a.r[0], a.r[1], a.r[2], a.f[0], a.f[1], a.f[2], a.mode, thr, lv);
    hipLaunchKernelGGL(k_blend_amr, dim3((unsigned)ntiles), dim3(64), 0, s, views, nv, ranges, vals, rec, n, lv,
                       a.interp, rgb);
    if (a.interp && max_pixels > 0)
        hipLaunchKernelGGL(k_amr_interp, dim3((unsigned)((max_pixels + 255) / 256), (unsigned)nv), dim3(256), 0, s,
                           views, lv, rgb);
}

// Quadrant schedule: a block of four waves per tile, wave w owning the 8 x 8
// quadrant (w % 2, w / 2) with one pixel per lane.  The block stages each
// batch of the list in LDS; every wave then keeps the staged entries that can
// reach its quadrant (box_reach over its pixel centres) and walks only those,
// so an entry costs the quadrants it can touch rather than the whole tile.
// Every pixel evaluates the same float32 expressions over the same list in
// the same order as k_blend, so the images are bit-identical.
template <bool COUNT, int BATCH>
__global__ void __launch_bounds__(256) k_blend_quad(const DevView *__restrict__ views, int nv,
                                                   const uint8_t *__restrict__ active,
                                                   const uint32_t *__restrict__ ranges,
                                                   const uint32_t *__restrict__ vals, const Record *__restrict__ rec,
                                                   int64_t n, float *__restrict__ rgb, float *__restrict__ Tout,
                                                   uint32_t *__restrict__ lastout,
                                                   unsigned long long *__restrict__ pairs, TileRanges tr) {
    if ((int64_t)blockIdx.x >= tr.len[blockIdx.y]) return;  // block-uniform
    const int64_t gt = tr.base[blockIdx.y] + blockIdx.x;
    if (!active[gt]) return;  // block-uniform
    __shared__ float s_u[BATCH], s_v[BATCH], s_a[BATCH], s_k[BATCH], s_c[BATCH], s_o[BATCH];
    __shared__ float s_r[BATCH], s_g[BATCH], s_b[BATCH], s_e[BATCH];
    __shared__ uint16_t s_list[4][BATCH];
    __shared__ uint32_t s_live[4];
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
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int qx = (w & 1) * 8, qy = (w >> 1) * 8;
    const int px = qx + (lane & 7), py = qy + (lane >> 3);
    const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
    // 0 while the pixel is live, +inf once it has stopped or when it lies
    // outside the image (added to an entry's take exponent)
    float thr = (x0 + px < W) && (y0 + py < H) ? 0.0f : INFINITY;
    float T = 1.0f, Cr = 0.0f, Cg = 0.0f, Cb = 0.0f;
    uint32_t last = 0, npairs = 0;
    const uint32_t start = ranges[2 * gt], end = ranges[2 * gt + 1];
    const Record *R = rec + (int64_t)lo * n;
    const double dx0 = (double)x0, dy0 = (double)y0;
    const uint64_t ltm = (1ull << lane) - 1ull;

    for (uint32_t b0 = start; b0 < end; b0 += BATCH) {
        const uint64_t live = __ballot(thr < INFINITY);
        if (lane == 0) s_live[w] = live != 0ull ? 1u : 0u;
        for (int slot = tid; slot < BATCH; slot += 256) {
            const uint32_t j = b0 + slot;
            if (j < end) {
                const Record r = R[vals[j]];
                s_u[slot] = (float)(r.u - dx0);
                s_v[slot] = (float)(r.v - dy0);
                s_a[slot] = r.a2; s_k[slot] = r.k; s_c[slot] = r.c2; s_o[slot] = r.o;
                s_r[slot] = r.r; s_g[slot] = r.g; s_b[slot] = r.b;
                s_e[slot] = take_exponent(r.o);
            }
        }
        __syncthreads();
        if ((s_live[0] | s_live[1] | s_live[2] | s_live[3]) == 0u) break;  // block-uniform: every pixel done
        const uint32_t cnt = (end - b0) < (uint32_t)BATCH ? (end - b0) : (uint32_t)BATCH;
        uint32_t wcnt = 0;
        if (live != 0ull) {
            for (uint32_t base = 0; base < cnt; base += 64) {
                const uint32_t jj = base + (uint32_t)lane;
                const bool keep = jj < cnt && box_reach(s_a[jj], s_k[jj], s_c[jj], s_o[jj], s_u[jj], s_v[jj],
                                                        (float)qx, (float)qy, 8.0f);
                const uint64_t km = __ballot(keep);
                if (keep) s_list[w][wcnt + (uint32_t)__popcll(km & ltm)] = (uint16_t)jj;
                wcnt += (uint32_t)__popcll(km);
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        // COUNT: a dropped entry is still a pair of every live pixel
        int prev = -1;
        for (uint32_t q = 0; q < wcnt; ++q) {
            const uint32_t jj = s_list[w][q];
            if (COUNT) {
                npairs += thr < INFINITY ? (uint32_t)((int)jj - prev) : 0u;  // the dropped ones before it, and itself
                prev = (int)jj;
            }
            const float mu = s_u[jj], mv = s_v[jj], a2 = s_a[jj], kk = s_k[jj], c2 = s_c[jj], o = s_o[jj];
            const float dy = fy - mv;
            const float kdy = kk * dy;
            const float cdy = c2 * dy * dy;
            const float t = (fx - mu) + kdy;
            const float e = fmaf(a2, t * t, cdy);
            const bool take = e >= s_e[jj] + thr;
            if (__ballot(take) == 0ull) continue;
            const float al = fminf(kAlphaMax, o * __builtin_amdgcn_exp2f(e));
            const float cr = s_r[jj], cg = s_g[jj], cb = s_b[jj];
            const float Tn = T * (1.0f - al);
            const bool stop = take && Tn < kTMin;
            const bool blend = take && !stop;
            const float wgt = blend ? al * T : 0.0f;
            Cr = fmaf(wgt, cr, Cr);
            Cg = fmaf(wgt, cg, Cg);
            Cb = fmaf(wgt, cb, Cb);
            T = blend ? Tn : T;
            last = blend ? b0 - start + jj + 1 : last;
            thr = stop ? INFINITY : thr;
        }
        if (COUNT) npairs += thr < INFINITY ? (uint32_t)((int)cnt - 1 - prev) : 0u;
        __syncthreads();  // the staging is reused by the next batch
    }
    const int x = x0 + px, y = y0 + py;
    if (x < W && y < H) {
        const int64_t HW = (int64_t)W * H;
        float *img = rgb + 3 * dv.img_off;
        const int64_t pix = (int64_t)y * W + x;
        img[pix] = Cr + T * dv.v.bg[0];
        img[HW + pix] = Cg + T * dv.v.bg[1];
        img[2 * HW + pix] = Cb + T * dv.v.bg[2];
        if (Tout) Tout[dv.img_off + pix] = T;
        if (lastout) lastout[dv.img_off + pix] = last;
    }
    add_pairs<COUNT>(npairs, pairs);
}

// grid schedule: one wave per tile, in tile order
template <bool COUNT, int BATCH, int ROWS>
__global__ void __launch_bounds__(64) k_blend(const DevView *__restrict__ views, int nv,
                                              const uint8_t *__restrict__ active, const uint32_t *__restrict__ ranges,
                                              const uint32_t *__restrict__ vals, const Record *__restrict__ rec,
                                              int64_t n, float *__restrict__ rgb, float *__restrict__ Tout,
                                              uint32_t *__restrict__ lastout, unsigned long long *__restrict__ pairs,
                                              TileRanges tr) {
    if ((int64_t)blockIdx.x >= tr.len[blockIdx.y]) return;  // block-uniform
    const int64_t gt = tr.base[blockIdx.y] + blockIdx.x;
    if (!active[gt]) return;
    uint32_t npairs = 0;
    blend_tile<COUNT, BATCH, ROWS>(gt, views, nv, ranges, vals, rec, n, rgb, Tout, lastout, npairs);
    add_pairs<COUNT>(npairs, pairs);
}

// queue schedule: persistent waves pull active tiles, longest lists first
template <bool COUNT, int BATCH, int ROWS>
__global__ void __launch_bounds__(64) k_blend_queue(const DevView *__restrict__ views, int nv,
                                                    const uint32_t *__restrict__ order, const uint32_t *n_order,
                                                    uint32_t *counter, const uint32_t *__restrict__ ranges,
                                                    const uint32_t *__restrict__ vals, const Record *__restrict__ rec,
                                                    int64_t n, float *__restrict__ rgb, float *__restrict__ Tout,
                                                    uint32_t *__restrict__ lastout,
                                                    unsigned long long *__restrict__ pairs) {
    const uint32_t total = *n_order;
    uint32_t npairs = 0;
    for (;;) {
        uint32_t t = 0;
        if (threadIdx.x == 0) t = atomicAdd(counter, 1u);
        t = __shfl(t, 0, 64);
        if (t >= total) break;
        blend_tile<COUNT, BATCH, ROWS>((int64_t)order[t], views, nv, ranges, vals, rec, n, rgb, Tout, lastout, npairs);
    }
    add_pairs<COUNT>(npairs, pairs);
}

// Longest-first order of the active tiles: bucket b = bit length of the list
// length (0 for an empty list), buckets in descending order (an O(n) counting
// sort; within a bucket the order is arbitrary, which changes no pixel).
// ws: [0..33) histogram, [33..66) running offsets, [66] active count, [67] queue counter.
__global__ void k_len_hist(const uint8_t *__restrict__ active, const uint32_t *__restrict__ ranges, int64_t ntiles,
                           uint32_t *__restrict__ ws) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles || !active[t]) return;
    const uint32_t len = ranges[2 * t + 1] - ranges[2 * t];
    const int b = len ? 32 - __clz(len) : 0;
    atomicAdd(&ws[b], 1u);
}

__global__ void k_len_scan(uint32_t *ws) {
    if (threadIdx.x != 0) return;
    uint32_t acc = 0;
    for (int b = 32; b >= 0; --b) {
        ws[33 + b] = acc;
        acc += ws[b];
    }
    ws[66] = acc;
    ws[67] = 0;
}

__global__ void k_len_scatter(const uint8_t *__restrict__ active, const uint32_t *__restrict__ ranges, int64_t ntiles,
                              uint32_t *__restrict__ ws, uint32_t *__restrict__ order) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles || !active[t]) return;
    const uint32_t len = ranges[2 * t + 1] - ranges[2 * t];
    const int b = len ? 32 - __clz(len) : 0;
    order[atomicAdd(&ws[33 + b], 1u)] = (uint32_t)t;
}

template <int BATCH, int ROWS>
static void launch_variant(const BlendArgs &a, const TileRanges &tr, int64_t longest, bool queue, hipStream_t s) {
    if (!queue) {
        const dim3 g((unsigned)longest, (unsigned)tr.count);
        if (a.pairs)
            hipLaunchKernelGGL((k_blend<true, BATCH, ROWS>), g, dim3(64), 0, s, a.views, a.nv, a.active, a.ranges,
                               a.vals, a.rec, a.n, a.rgb, a.T, a.last, a.pairs, tr);
        else
            hipLaunchKernelGGL((k_blend<false, BATCH, ROWS>), g, dim3(64), 0, s, a.views, a.nv, a.active, a.ranges,
                               a.vals, a.rec, a.n, a.rgb, a.T, a.last, a.pairs, tr);
        return;
    }
    const unsigned grid = (unsigned)(a.ntiles < a.queue_waves ? a.ntiles : a.queue_waves);
    if (a.pairs)
        hipLaunchKernelGGL((k_blend_queue<true, BATCH, ROWS>), dim3(grid), dim3(64), 0, s, a.views, a.nv, a.order,
                           a.ws + 66, a.ws + 67, a.ranges, a.vals, a.rec, a.n, a.rgb, a.T, a.last, a.pairs);
    else
        hipLaunchKernelGGL((k_blend_queue<false, BATCH, ROWS>), dim3(grid), dim3(64), 0, s, a.views, a.nv, a.order,
                           a.ws + 66, a.ws + 67, a.ranges, a.vals, a.rec, a.n, a.rgb, a.T, a.last, a.pairs);
}

void launch_blend_order(const uint8_t *active, const uint32_t *ranges, int64_t ntiles, uint32_t *ws, uint32_t *order,
                        hipStream_t s) {
    launch_fill_u32(ws, 0u, kBlendWsWords, s);
    if (ntiles == 0) return;
    const unsigned g = (unsigned)((ntiles + 255) / 256);
    hipLaunchKernelGGL(k_len_hist, dim3(g), dim3(256), 0, s, active, ranges, ntiles, ws);
    hipLaunchKernelGGL(k_len_scan, dim3(1), dim3(64), 0, s, ws);
    hipLaunchKernelGGL(k_len_scatter, dim3(g), dim3(256), 0, s, active, ranges, ntiles, ws, order);
}

void launch_blend(const BlendArgs &a, int variant, hipStream_t s) {
    if (a.ntiles == 0) return;
    const BlendVariant v = blend_variant(variant);
    TileRanges tr = a.tr;
    if (tr.count <= 0) {
        tr.count = 1;
        tr.base[0] = 0;
        tr.len[0] = a.ntiles;
    }
    int64_t longest = 0;
    for (int k = 0; k < tr.count; ++k) longest = tr.len[k] > longest ? tr.len[k] : longest;
    if (longest == 0) return;
    if (v.quad) {
        const dim3 g((unsigned)longest, (unsigned)tr.count), b(256);
        switch (v.batch) {
            case 64:
                if (a.pairs) hipLaunchKernelGGL((k_blend_quad<true, 64>), g, b, 0, s, a.views, a.nv, a.active, a.ranges,
                                                a.vals, a.rec, a.n, a.rgb, a.T, a.last, a.pairs, tr);
                else hipLaunchKernelGGL((k_blend_quad<false, 64>), g, b, 0, s, a.views, a.nv, a.active, a.ranges,
                                        a.vals, a.rec, a.n, a.rgb, a.T, a.last, a.pairs, tr);
                break;
            case 128:
                if (a.pairs) hipLaunchKernelGGL((k_blend_quad<true, 128>), g, b, 0, s, a.views, a.nv, a.active, a.ranges,
                                                a.vals, a.rec, a.n, a.rgb, a.T, a.last, a.pairs, tr);
                else hipLaunchKernelGGL((k_blend_quad<false, 128>), g, b, 0, s, a.views, a.nv, a.active, a.ranges,
                                        a.vals, a.rec, a.n, a.rgb, a.T, a.last, a.pairs, tr);
                break;
            default:
                if (a.pairs) hipLaunchKernelGGL((k_blend_quad<true, 256>), g, b, 0, s, a.views, a.nv, a.active, a.ranges,
                                                a.vals, a.rec, a.n, a.rgb, a.T, a.last, a.pairs, tr);
                else hipLaunchKernelGGL((k_blend_quad<false, 256>), g, b, 0, s, a.views, a.nv, a.active, a.ranges,
                                        a.vals, a.rec, a.n, a.rgb, a.T, a.last, a.pairs, tr);
                break;
        }
        return;
    }
    if (v.queue) {  // every tile (the callers pass no ranges with a queue variant)
        launch_blend_order(a.active, a.ranges, a.ntiles, a.ws, a.order, s);
        launch_fill_u32(a.ws + 67, 0u, 1, s);
    }
    switch (v.batch * 10 + v.rows) {
        case 321: launch_variant<32, 1>(a, tr, longest, v.queue, s); break;
        case 322: launch_variant<32, 2>(a, tr, longest, v.queue, s); break;
        case 641: launch_variant<64, 1>(a, tr, longest, v.queue, s); break;
        case 642: launch_variant<64, 2>(a, tr, longest, v.queue, s); break;
        case 1281: launch_variant<128, 1>(a, tr, longest, v.queue, s); break;
        default: launch_variant<128, 2>(a, tr, longest, v.queue, s); break;
    }
}

BlendVariant blend_variant(int k) {
    static const int batches[3] = {32, 64, 128}, quad_batches[3] = {64, 128, 256};
    BlendVariant v;
    k = k < 0 ? 0 : (k >= kBlendVariants ? kBlendVariants - 1 : k);
    if (k >= 12) {  // four waves per tile, an 8 x 8 quadrant each
        v.batch = quad_batches[k - 12];
        v.rows = 1;
        v.queue = false;
        v.quad = true;
        return v;
    }
    v.batch = batches[k % 3];
    v.rows = 1 + (k / 3) % 2;
    v.queue = k / 6 != 0;
    v.quad = false;
    return v;
}

// ------------------------------------------------------------------------
// reverse blend
// ------------------------------------------------------------------------
// Same tile mapping as k_blend (one wave per tile, four horizontally adjacent
// pixels per lane, 64-record LDS batches), but the batches are taken from the
// back: each pixel starts at its last blended Gaussian with its final
// transmittance T and S = T (bg . D), D = dL/dC, and for each blended
// Gaussian j (alpha >= 1/255, position < last) going towards the front
//   T_j   = T_{j+1} / (1 - alpha_j)           (transmittance in front of j;
//           times the hardware reciprocal, 1 ulp, instead of a divide)
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

// Wave sums of eight values at once.  At offset 32 a lane keeps the half of
// its values selected by lane bit 5 and receives the same half from its
// partner (4 shuffles), at 16 the half of those by bit 4 (2), at 8 by bit 3
// (1); after three plain steps (4, 2, 1) lane l holds the sum over the wave of
// value l >> 3.
__device__ __forceinline__ float wave_multi_sum8(const float (&v)[8], int lane) {
    const bool b5 = (lane >> 5) & 1, b4 = (lane >> 4) & 1, b3 = (lane >> 3) & 1;
    float h4[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float keep = b5 ? v[4 + i] : v[i], give = b5 ? v[i] : v[4 + i];
        h4[i] = keep + __shfl_xor(give, 32, 64);
    }
    float h2[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const float keep = b4 ? h4[2 + i] : h4[i], give = b4 ? h4[i] : h4[2 + i];
        h2[i] = keep + __shfl_xor(give, 16, 64);
    }
    float x;
    {
        const float keep = b3 ? h2[1] : h2[0], give = b3 ? h2[0] : h2[1];
        x = keep + __shfl_xor(give, 8, 64);
    }
#pragma unroll
    for (int off = 4; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// Wave sums of V values at once (V = 32 or 64), the same halving as above run
// to the end: at each exchange step a lane keeps the half of its values
// selected by one lane bit and receives that half from its partner, so after
// log2 V steps (V - 1 shuffles) lane l holds the sum over the wave of value
// l >> (6 - log2 V); with V = 32 a last plain step at offset 1 completes it.
template <int V>
__device__ __forceinline__ float wave_multi_sum(const float (&v)[V], int lane) {
    static_assert(V == 32 || V == 64, "32 or 64 values");
    float c[V];
#pragma unroll
    for (int i = 0; i < V; ++i) c[i] = v[i];
#pragma unroll
    for (int off = 32, n = V; n > 1; off >>= 1, n >>= 1) {
        const bool b = (lane & off) != 0;
#pragma unroll
        for (int i = 0; i < n / 2; ++i) {
            const float keep = b ? c[n / 2 + i] : c[i], give = b ? c[i] : c[n / 2 + i];
            c[i] = keep + __shfl_xor(give, off, 64);
        }
    }
    float x = c[0];
    if (V == 32) x += __shfl_xor(x, 1, 64);
    return x;
}

// entries of the list whose nine sums are reduced together (9 x 7 = 63 of
// the 64 lanes: one shuffle tree per seven entries instead of one per entry)
constexpr int kBwdGroup = 7;
constexpr int kBwdVals = 64;

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
    __shared__ float s_r[kBatch], s_g[kBatch], s_b[kBatch], s_e[kBatch];
    __shared__ uint32_t s_i[kBatch], s_p[kBatch];
    const double dx0 = (double)x0, dy0 = (double)y0;
    const float kLn2 = 0.6931471805599453f;

    for (int64_t bend = maxlast; bend > 0; bend -= kBatch) {
        const uint32_t bstart = bend > kBatch ? (uint32_t)(bend - kBatch) : 0u;
        const uint32_t cnt = (uint32_t)bend - bstart;
        // the batch's entries that can reach the tile (tile_reach), packed in list order
        bool keep = false;
        Record r;
        uint32_t idx = 0;
        float mu = 0.0f, mv = 0.0f;
        if ((uint32_t)lane < cnt) {
            idx = vals[start + bstart + lane];
            r = R[idx];
            mu = (float)(r.u - dx0);
            mv = (float)(r.v - dy0);
            keep = tile_reach(r, mu, mv);
        }
        const uint64_t km = __ballot(keep);
        if (keep) {
            const int at = __popcll(km & ((1ull << lane) - 1ull));
            s_u[at] = mu;
            s_v[at] = mv;
            s_a[at] = r.a2; s_k[at] = r.k; s_c[at] = r.c2; s_o[at] = r.o;
            s_r[at] = r.r; s_g[at] = r.g; s_b[at] = r.b;
            s_e[at] = take_exponent(r.o);
            s_i[at] = idx;
            s_p[at] = bstart + (uint32_t)lane;
        }
        __syncthreads();
        for (int jb = __popcll(km) - 1; jb >= 0; jb -= kBwdGroup) {  // groups of entries, back to front
            float vsum[kBwdVals];
#pragma unroll
            for (int i = 0; i < kBwdVals; ++i) vsum[i] = 0.0f;
            uint32_t hitm = 0;
#pragma unroll
            for (int u = 0; u < kBwdGroup; ++u) {
                const int jj = jb - u;
                if (jj < 0) break;  // wave-uniform
                const uint32_t pos = s_p[jj];
                const float mu = s_u[jj], mv = s_v[jj], a2 = s_a[jj], kk = s_k[jj], c2 = s_c[jj], o = s_o[jj];
                const float cr = s_r[jj], cg = s_g[jj], cb = s_b[jj], et = s_e[jj];
                const float dy = fy - mv;
                const float kdy = kk * dy;
                const float cdy = c2 * dy * dy;
                float g_t2 = 0.f, g_t = 0.f, g_tdy = 0.f, g_dy2 = 0.f, g_dy = 0.f, g_o = 0.f, g_r = 0.f, g_g = 0.f,
                      g_b = 0.f;
                bool hit = false;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float t = (fxq[q] - mu) + kdy;
                    const float e = fmaf(a2, t * t, cdy);
                    const float ex = __builtin_amdgcn_exp2f(e);
                    const float araw = o * ex;
                    const float al = fminf(kAlphaMax, araw);
                    if (pos < last[q] && e >= et) {  // blended in the forward (the same decision)
                        hit = true;
                        const float oma = 1.0f - al;
                        const float inv = __builtin_amdgcn_rcpf(oma);  // 1 ulp; 1 - alpha in [0.01, 1]
                        const float Tb = T[q] * inv;
                        const float cD = cr * D0[q] + cg * D1[q] + cb * D2[q];
                        const float w = al * Tb;
                        g_r = fmaf(w, D0[q], g_r);
                        g_g = fmaf(w, D1[q], g_g);
                        g_b = fmaf(w, D2[q], g_b);
                        const float dal = Tb * cD - S[q] * inv;
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
                if (__ballot(hit) != 0ull) hitm |= 1u << u;
                vsum[9 * u + 0] = g_t2; vsum[9 * u + 1] = g_t; vsum[9 * u + 2] = g_tdy;
                vsum[9 * u + 3] = g_dy2; vsum[9 * u + 4] = g_dy; vsum[9 * u + 5] = g_o;
                vsum[9 * u + 6] = g_r; vsum[9 * u + 7] = g_g; vsum[9 * u + 8] = g_b;
            }
            if (hitm != 0u) {  // wave-uniform
                // lane l: sum l % 9 of the group's entry l / 9
                const float sum = wave_multi_sum<kBwdVals>(vsum, lane);
                const int u = lane / 9, k = lane - 9 * (lane / 9);
                if (u < kBwdGroup && ((hitm >> u) & 1u))
                    atomicAdd(&A[(int64_t)s_i[jb - u] * 12 + k], sum);
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

// One output pixel (x, y): fovea inside r_f, bilinear mid layer inside r_mid,
// then the periphery: a flagged periphery tile from the full-resolution layer,
// else nothing when the network already wrote it, else the given
// full-resolution periphery or the bilinear periphery layer.
__device__ __forceinline__ void composite_px(int x, int y, int W, int H, double gx, double gy, double rf, double rm,
                                             const float *__restrict__ fovea, const float *__restrict__ mid, int sm,
                                             const float *__restrict__ periph, int sp,
                                             const float *__restrict__ periph_full, int periph_done,
                                             const uint8_t *__restrict__ fb_flags, int fb_tiles_x,
                                             float *__restrict__ out) {
    const int64_t HW = (int64_t)W * H, pix = (int64_t)y * W + x;
    const int reg = region_of(x, y, gx, gy, rf, rm);
    if (reg == 0) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) out[ch * HW + pix] = fovea[ch * HW + pix];
        return;
    }
    // periphery tiles flagged for the full-resolution fallback come from the full-resolution layer
    if (reg == 2 && fb_flags && fb_flags[(int64_t)(y / (kTile * sp)) * fb_tiles_x + x / (kTile * sp)]) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) out[ch * HW + pix] = fovea[ch * HW + pix];
        return;
    }
    if (reg == 2 && periph_done) return;  // already written by the upsampler
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
        // vertical interpolation in columns xa and xb, then horizontal (the upsampler's
        // residual takes the same steps, so a network with zero weights gives these bits)
        const float va = (1.0f - wy) * p[(int64_t)ya * Wl + xa] + wy * p[(int64_t)yb * Wl + xa];
        const float vb = (1.0f - wy) * p[(int64_t)ya * Wl + xb] + wy * p[(int64_t)yb * Wl + xb];
        out[ch * HW + pix] = (1.0f - wx) * va + wx * vb;
    }
}

__global__ void k_composite(int W, int H, double gx, double gy, double rf, double rm,
                            const float *__restrict__ fovea, const float *__restrict__ mid, int sm,
                            const float *__restrict__ periph, int sp, const float *__restrict__ periph_full,
                            int periph_done,
                            const uint8_t *__restrict__ fb_flags, int fb_tiles_x, const DevView *gaze_view,
                            float *__restrict__ out) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (gaze_view) {  // the gaze of this frame, from the device view table
        gx = gaze_view->v.gx;
        gy = gaze_view->v.gy;
    }
    const int y = blockIdx.y;
    if (x >= W) return;
    composite_px(x, y, W, H, gx, gy, rf, rm, fovea, mid, sm, periph, sp, periph_full, periph_done, fb_flags,
                 fb_tiles_x, out);
}

void launch_composite(int W, int H, double gx, double gy, double rf, double rm, const float *fovea,
                      const float *mid, int sm, const float *periph, int sp, const float *periph_full, bool periph_done,
                      const uint8_t *fb_flags, int fb_tiles_x, const DevView *gaze_view, float *out, hipStream_t s) {
    if (W <= 0 || H <= 0) return;
    hipLaunchKernelGGL(k_composite, dim3((unsigned)((W + 255) / 256), (unsigned)H), dim3(256), 0, s, W, H, gx, gy,
                       rf, rm, fovea, mid, sm, periph, sp, periph_full, (int)periph_done, fb_flags, fb_tiles_x, gaze_view,
                       out);
}

// Every eye of a frame (all W x H) in one launch: blockIdx.z = eye, a block
// covers 64 x 16 pixels (a wave per row, each thread four rows at a stride of
// four).  Eye e's gaze, layers and fallback flags come from its views in the
// device view table: fovea 3e, mid 3e + 1, periphery 3e + 2; its output is
// out + 3 W H e.  When the network has written the periphery, a block whose
// pixel centre nearest the gaze lies outside r_mid holds periphery pixels
// only (the distances of the others are at least as large, also after
// rounding), so it has nothing to write unless the one periphery tile that
// holds it is flagged.
constexpr int kCompW = 64, kCompH = 16;

__global__ void __launch_bounds__(256) k_composite_eyes(int W, int H, double rf, double rm, int sm, int sp,
                                                        const DevView *__restrict__ views,
                                                        const float *__restrict__ layers, int periph_done,
                                                        const uint8_t *__restrict__ fb_flags,
                                                        float *__restrict__ out) {
    const int e = blockIdx.z;
    const DevView &d0 = views[3 * e], &d1 = views[3 * e + 1], &d2 = views[3 * e + 2];
    const double gx = d0.v.gx, gy = d0.v.gy;
    const int x0 = blockIdx.x * kCompW, y0 = blockIdx.y * kCompH;
    const int xe = x0 + kCompW - 1 < W ? x0 + kCompW - 1 : W - 1;
    const int ye = y0 + kCompH - 1 < H ? y0 + kCompH - 1 : H - 1;
    const uint8_t *flags = fb_flags ? fb_flags + d2.tile_off : nullptr;
    if (periph_done) {
        const int xn = (int)fmin(fmax(floor(gx), (double)x0), (double)xe);
        const int yn = (int)fmin(fmax(floor(gy), (double)y0), (double)ye);
        if (region_of(xn, yn, gx, gy, rf, rm) == 2) {
            if (!flags) return;
            const int pt = kTile * sp;
            if (x0 / pt == xe / pt && y0 / pt == ye / pt && !flags[(int64_t)(y0 / pt) * d2.tiles_x + x0 / pt]) return;
        }
    }
    const int64_t HW = (int64_t)W * H;
    const float *fov = layers + 3 * d0.img_off, *mid = layers + 3 * d1.img_off, *per = layers + 3 * d2.img_off;
    float *o = out + (int64_t)e * 3 * HW;
    const int x = x0 + (int)(threadIdx.x & 63);
    if (x >= W) return;
#pragma unroll
    for (int k = 0; k < kCompH / 4; ++k) {
        const int y = y0 + (int)(threadIdx.x >> 6) + 4 * k;
        if (y < H)
            composite_px(x, y, W, H, gx, gy, rf, rm, fov, mid, sm, per, sp, nullptr, periph_done, flags, d2.tiles_x,
                         o);
    }
}

void launch_composite_eyes(int n_eyes, int W, int H, double rf, double rm, int sm, int sp, const DevView *views,
                           const float *layers, bool periph_done, const uint8_t *fb_flags, float *out,
                           hipStream_t s) {
    if (n_eyes <= 0 || W <= 0 || H <= 0) return;
    hipLaunchKernelGGL(k_composite_eyes, dim3((unsigned)((W + kCompW - 1) / kCompW),
                                              (unsigned)((H + kCompH - 1) / kCompH), (unsigned)n_eyes),
                       dim3(256), 0, s, W, H, rf, rm, sm, sp, views, layers, (int)periph_done, fb_flags, out);
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

// Sums of the per-block partials of k_region_sse, on the device: one lane per
// region adds the blocks' values in block order, as a3fr_region_sse's host loop
// does, so both give the same bits.
__global__ void k_region_sse_sum(const double *__restrict__ partial, const unsigned long long *__restrict__ cnt,
                                 int nblk, double *sse3, int64_t *count3) {
    const int r = threadIdx.x;
    if (r >= 3) return;
    double s = 0.0;
    unsigned long long k = 0;
    for (int j = 0; j < nblk; ++j) {
        s += partial[3 * j + r];
        k += cnt[3 * j + r];
    }
    sse3[r] = s;
    count3[r] = (int64_t)k;
}

void launch_region_sse_sum(const double *partial, const unsigned long long *cnt, int nblk, double *sse3,
                           int64_t *count3, hipStream_t s) {
    hipLaunchKernelGGL(k_region_sse_sum, dim3(1), dim3(64), 0, s, partial, cnt, nblk, sse3, count3);
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
