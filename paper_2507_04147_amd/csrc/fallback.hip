// Per-tile error estimate of the periphery and full-resolution fallback.
//
// The periphery layer draws only the Gaussians of largest opacity x
// projected area (the coarse, cheaper rendering of the regions away from the
// gaze, Sec. 2.2).  Dropping Gaussians changes a tile most where the tile is
// not saturated (background or far content shows through): with D_t and K_t
// the opacity mass per pixel of the dropped and of the kept visible Gaussians
// over periphery tile t (each Gaussian's 2 pi o sqrt(det Sigma2D), the
// integral of o exp(-q/2), spread evenly over the tiles of its rectangle),
// the transmittance model T ~ exp(-mass) gives the rise of the tile's
// transmittance dT = exp(-K) - exp(-(K + D)) caused by the subset, and the
// squared-error estimate coef x (dT^2)^power (calibrated on rendered frames).
// Tiles whose estimate reaches the threshold and that reach outside the
// mid-layer radius are added to the eye's full-resolution layer (same
// projection, all Gaussians): its tile mask grows, its rows and per-Gaussian
// tile counts are rebuilt, and the composite takes those pixels from it.
#include "a3fr_internal.h"

namespace a3fr {

// Every kernel below handles all eyes of the frame in one launch: pair k of
// the batch (a periphery view and its eye's full-resolution view) is
// blockIdx.y.

// Each visible Gaussian of the periphery view adds its per-pixel share to the
// four corners of its tile rectangle in a 2D difference array (float64,
// [2][TY+1][TX+1]: dropped, kept), so the cost per Gaussian does not depend
// on its size; a prefix sum over the tile grid then gives D and K.
__device__ __forceinline__ void drop_share(double *d, int64_t plane, int S, uint64_t r, double score, bool kept) {
    const int x0 = (int)(r & 0xffff), x1 = (int)((r >> 16) & 0xffff), y0 = (int)((r >> 32) & 0xffff),
              y1 = (int)(r >> 48);
    const int nt = (x1 - x0 + 1) * (y1 - y0 + 1);
    const double share = 2.0 * score / ((double)nt * (double)(kTile * kTile));
    d += kept ? plane : 0;
    atomicAdd(&d[(int64_t)y0 * S + x0], share);
    atomicAdd(&d[(int64_t)y0 * S + x1 + 1], -share);
    atomicAdd(&d[(int64_t)(y1 + 1) * S + x0], -share);
    atomicAdd(&d[(int64_t)(y1 + 1) * S + x1 + 1], share);
}

__global__ void __launch_bounds__(256) k_drop_energy(const DevView *__restrict__ views, FbBatch b, int64_t n,
                                                     const uint32_t *__restrict__ counts,
                                                     const uint8_t *__restrict__ keep,
                                                     const uint64_t *__restrict__ rect,
                                                     const double *__restrict__ score, double *__restrict__ diff) {
    const int k = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int pv = b.pv[k];
    const int64_t slot = (int64_t)pv * n + i;
    if (counts[slot] == 0) return;
    const DevView &dv = views[pv];
    const int S = dv.tiles_x + 1;
    drop_share(diff + b.doff[k], (int64_t)(dv.tiles_y + 1) * S, S, rect[(int64_t)dv.rect_slot * n + i],
               score[(int64_t)dv.sel_slot * n + i], keep[slot] != 0);
}

// Contention-free variant for grids that fit in LDS: persistent blocks add
// into a block-local difference array (LDS atomics), write it out as one
// partial each ([pair][block][cells], cells = b.max_cells apart), and
// k_drop_reduce sums the partials; device-scope atomics on a few hundred
// addresses from every XCD would serialise.
constexpr int kDropUnroll = 8;
__global__ void __launch_bounds__(256) k_drop_energy_lds(const DevView *__restrict__ views, FbBatch b, int64_t n,
                                                         const uint32_t *__restrict__ counts,
                                                         const uint8_t *__restrict__ keep,
                                                         const uint64_t *__restrict__ rect,
                                                         const double *__restrict__ score,
                                                         double *__restrict__ partials) {
    extern __shared__ double sh[];
    const int k = blockIdx.y, pv = b.pv[k];
    const DevView &dv = views[pv];
    const int S = dv.tiles_x + 1;
    const int64_t plane = (int64_t)(dv.tiles_y + 1) * S;
    const int cells = (int)(2 * plane);
    for (int c = threadIdx.x; c < cells; c += blockDim.x) sh[c] = 0.0;
    __syncthreads();
    const uint64_t *rv = rect + (int64_t)dv.rect_slot * n;
    const double *sv = score + (int64_t)dv.sel_slot * n;
    const uint32_t *cv = counts + (int64_t)pv * n;
    const uint8_t *kv = keep + (int64_t)pv * n;
    // kDropUnroll Gaussians per step, their loads unconditional (indices past
    // n read the last Gaussian and are dropped) and issued together, so a
    // thread waits for one round trip per step rather than two per Gaussian
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < n; i0 += kDropUnroll * stride) {
        uint32_t c[kDropUnroll];
        uint64_t r[kDropUnroll];
        double sc[kDropUnroll];
        uint8_t kp[kDropUnroll];
#pragma unroll
        for (int u = 0; u < kDropUnroll; ++u) {
            const int64_t i = i0 + u * stride, ic = i < n ? i : n - 1;
            c[u] = cv[ic];
            r[u] = rv[ic];
            sc[u] = sv[ic];
            kp[u] = kv[ic];
        }
#pragma unroll
        for (int u = 0; u < kDropUnroll; ++u)
            if (i0 + u * stride < n && c[u] != 0) drop_share(sh, plane, S, r[u], sc[u], kp[u] != 0);
    }
    __syncthreads();
    double *out = partials + ((int64_t)k * gridDim.x + blockIdx.x) * b.max_cells;
    for (int c = threadIdx.x; c < cells; c += blockDim.x) out[c] = sh[c];
}

// 256 threads per 16 cells of one pair: sixteen slices of the partials per
// cell, each summed by one thread (independent loads, no dependent chain),
// then the slices summed in LDS.
__global__ void __launch_bounds__(256) k_drop_reduce(const DevView *__restrict__ views, FbBatch b,
                                                     const double *__restrict__ partials, int nparts,
                                                     double *__restrict__ diff) {
    __shared__ double red[16][16];
    const int kp = blockIdx.y;
    const DevView &dv = views[b.pv[kp]];
    const int cells = 2 * (dv.tiles_y + 1) * (dv.tiles_x + 1);
    const int c = threadIdx.x & 15, slice = threadIdx.x >> 4;
    const int k = blockIdx.x * 16 + c;
    const double *part = partials + (int64_t)kp * nparts * b.max_cells;
    double acc = 0.0;
    if (k < cells) {
#pragma unroll 8
        for (int g = slice; g < nparts; g += 16) acc += part[(int64_t)g * b.max_cells + k];
    }
    red[slice][c] = acc;
    __syncthreads();
    if (slice == 0 && k < cells) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < 16; ++q) t += red[q][c];
        diff[b.doff[kp] + k] = t;
    }
}

// Flag of periphery tile t of pair k: set when the tile's estimate reaches the
// threshold and one of the full-resolution pixel centres it covers lies
// outside r_mid (the composite's periphery region); a flagged tile activates
// the tiles it covers in the full-resolution layer fv (s = full-resolution
// pixels per periphery pixel).
__device__ __forceinline__ void fallback_flag_tile(const DevView &dp, const DevView &df, double r_mid, int64_t t,
                                                   const float *energy, int64_t ntiles, double threshold, double coef,
                                                   double power, uint8_t *flags, uint8_t *active,
                                                   uint32_t *n_flagged) {
    const int tx = (int)(t % dp.tiles_x), ty = (int)(t / dp.tiles_x);
    const int s = (int)llround(df.v.fx / dp.v.fx);
    const int span = kTile * s;  // full-resolution pixels per periphery tile, per axis
    const double x0 = (double)tx * span + 0.5, x1 = fmin((double)(tx + 1) * span, (double)df.v.width) - 0.5;
    const double y0 = (double)ty * span + 0.5, y1 = fmin((double)(ty + 1) * span, (double)df.v.height) - 0.5;
    const double gx = df.v.gx, gy = df.v.gy;
    const double fx = fmax(fabs(x0 - gx), fabs(x1 - gx)), fy = fmax(fabs(y0 - gy), fabs(y1 - gy));
    const bool outer = x0 <= x1 && y0 <= y1 && fx * fx + fy * fy > r_mid * r_mid;
    // Beer-Lambert: transmittance ~ exp(-mass per pixel); dropping raises it by dT
    const double D = energy[dp.tile_off + t], K = energy[ntiles + dp.tile_off + t];
    const double dT = exp(-K) - exp(-(K + D));
    const double est = dT > 0.0 ? coef * pow(dT * dT, power) : 0.0;
    const bool flag = outer && est >= threshold;
    flags[dp.tile_off + t] = flag ? 1 : 0;
    if (!flag) return;
    atomicAdd(n_flagged, 1u);
    for (int yy = ty * s; yy < (ty + 1) * s && yy < df.tiles_y; ++yy)
        for (int xx = tx * s; xx < (tx + 1) * s && xx < df.tiles_x; ++xx)
            active[df.tile_off + (int64_t)yy * df.tiles_x + xx] = 1;
}

// One block per pair: 2D inclusive prefix sum of its two difference planes
// (in place: first along each row, then down each column, one thread per row
// or column, so a thread's chain of dependent loads is one row or column
// long), written as float32 into energy [2][ntiles] at the view's tiles; then
// the same block flags the pair's periphery tiles (fallback_flag_tile).
__global__ void __launch_bounds__(1024) k_drop_prefix(const DevView *__restrict__ views, FbBatch b, double *diff,
                                                      int64_t ntiles, float *__restrict__ energy, double threshold,
                                                      double coef, double power, uint8_t *__restrict__ flags,
                                                      uint8_t *__restrict__ active, uint32_t *__restrict__ n_flagged) {
    extern __shared__ double pre[];  // the two planes when they fit (dynamic size, else unused)
    const int kp = blockIdx.x;
    const DevView &dv = views[b.pv[kp]];
    const int TX = dv.tiles_x, TY = dv.tiles_y, S = TX + 1;
    const int64_t plane = (int64_t)(TY + 1) * S;
    const bool lds = 2 * plane * (int64_t)sizeof(double) <= kFbLdsBytes;
    double *d = diff + b.doff[kp];
    if (lds) {
        for (int64_t k = threadIdx.x; k < 2 * plane; k += blockDim.x) pre[k] = d[k];
        __syncthreads();
        d = pre;
    }
    for (int r = threadIdx.x; r < 2 * TY; r += blockDim.x) {
        double *row = d + (r / TY) * plane + (int64_t)(r % TY) * S;
        double acc = 0.0;
        for (int x = 0; x < TX; ++x) {
            acc += row[x];
            row[x] = acc;
        }
    }
    __syncthreads();
    for (int cidx = threadIdx.x; cidx < 2 * TX; cidx += blockDim.x) {
        const int pl = cidx / TX, x = cidx % TX;
        const double *col = d + pl * plane + x;
        float *E = energy + (int64_t)pl * ntiles + dv.tile_off + x;
        double acc = 0.0;
        for (int y = 0; y < TY; ++y) {
            acc += col[(int64_t)y * S];
            E[(int64_t)y * TX] = (float)acc;
        }
    }
    __syncthreads();  // the block's energies are in memory
    const DevView &df = views[b.fv[kp]];
    for (int64_t t = threadIdx.x; t < (int64_t)TX * TY; t += blockDim.x)
        fallback_flag_tile(dv, df, b.r_mid[kp], t, energy, ntiles, threshold, coef, power, flags, active, n_flagged);
}

// Persistent blocks of the mass maps: one per compute unit of the MI355X per
// pair, so each thread visits a few Gaussians and the dependent loads overlap.
int drop_energy_parts() { return 256; }

void launch_drop_energy(const DevView *views, const FbBatch &b, int64_t n, const uint32_t *counts,
                        const uint8_t *keep, const uint64_t *rect, const double *score, double *diff,
                        double *partials, int64_t ntiles, float *energy, double threshold, double coef, double power,
                        uint8_t *flags, uint8_t *active, uint32_t *n_flagged, hipStream_t s) {
    if (b.count == 0) return;
    const size_t lds = sizeof(double) * (size_t)b.max_cells;
    const bool fits = lds <= (size_t)kFbLdsBytes;
    if (n > 0 && partials && fits) {
        const int parts = drop_energy_parts();
        hipLaunchKernelGGL(k_drop_energy_lds, dim3(parts, b.count), dim3(256), lds, s, views, b, n, counts, keep, rect,
                           score, partials);
        hipLaunchKernelGGL(k_drop_reduce, dim3((b.max_cells + 15) / 16, b.count), dim3(256), 0, s, views, b, partials,
                           parts, diff);
    } else if (n > 0) {
        hipLaunchKernelGGL(k_drop_energy, dim3((unsigned)((n + 255) / 256), b.count), dim3(256), 0, s, views, b, n,
                           counts, keep, rect, score, diff);
    }
    hipLaunchKernelGGL(k_drop_prefix, dim3(b.count), dim3(1024), fits ? lds : 0, s, views, b, diff, ntiles, energy,
                       threshold, coef, power, flags, active, n_flagged);
}

// Row prefix and active-column list of the remasked views' rows from their
// active flags (wave per row, ballot prefix).
__global__ void __launch_bounds__(256) k_rows_from_active(const DevView *views, int64_t rows_total,
                                                          const int32_t *row_view, const int32_t *row_y,
                                                          const uint8_t *active, uint16_t *row_prefix,
                                                          uint16_t *row_list, const uint32_t *n_flagged) {
    if (*n_flagged == 0) return;  // no tile joined any mask: rows unchanged
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= rows_total) return;
    const DevView &dv = views[row_view[r]];
    if (!dv.remask || dv.v.mask == A3FR_MASK_ALL) return;
    const int ty = row_y[r];
    const int TX = dv.tiles_x;
    const uint8_t *act = active + dv.tile_off + (int64_t)ty * TX;
    uint16_t *pre = row_prefix + dv.mask_off + (int64_t)ty * (TX + 1);
    uint16_t *lst = row_list + dv.mask_off + (int64_t)ty * (TX + 1);
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    uint32_t c = 0;
    for (int tx0 = 0; tx0 < TX; tx0 += 64) {
        const int tx = tx0 + lane;
        const bool a = tx < TX && act[tx] != 0;
        const uint64_t m = __ballot(a);
        const uint32_t below = (uint32_t)__popcll(m & lt);
        if (tx < TX) {
            pre[tx] = (uint16_t)(c + below);
            if (a) lst[c + below] = (uint16_t)tx;
        }
        c += (uint32_t)__popcll(m);
    }
    if (lane == 0) pre[TX] = (uint16_t)c;
}

void launch_rows_from_active(const DevView *views, int64_t rows_total, const int32_t *row_view, const int32_t *row_y,
                             const uint8_t *active, uint16_t *row_prefix, uint16_t *row_list,
                             const uint32_t *n_flagged, hipStream_t s) {
    if (rows_total == 0) return;
    hipLaunchKernelGGL(k_rows_from_active, dim3((unsigned)((rows_total + 3) / 4)), dim3(256), 0, s, views, rows_total,
                       row_view, row_y, active, row_prefix, row_list, n_flagged);
}

// Active tiles covered by each visible Gaussian's rectangle in the
// full-resolution view of pair blockIdx.y, from the rebuilt row prefixes.
__global__ void __launch_bounds__(256) k_recount(const DevView *__restrict__ views, FbBatch b, int64_t n,
                                                 const uint64_t *__restrict__ rect,
                                                 const uint16_t *__restrict__ row_prefix, uint32_t *__restrict__ counts,
                                                 const uint32_t *n_flagged) {
    if (n_flagged && *n_flagged == 0) return;  // masks unchanged: the counts of the projection stand
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int fv = b.fv[blockIdx.y];
    const DevView &dv = views[fv];
    const int64_t slot = (int64_t)fv * n + i;
    const uint64_t r = rect[(int64_t)dv.rect_slot * n + i];  // the view keeps every slot's rectangle
    const int x0 = (int)(r & 0xffff), x1 = (int)((r >> 16) & 0xffff), y0 = (int)((r >> 32) & 0xffff),
              y1 = (int)(r >> 48);
    if (x0 > x1 || y0 > y1) return;  // not visible: count stays 0
    const uint16_t *pre = row_prefix + dv.mask_off;
    uint32_t cnt = 0;
    for (int ty = y0; ty <= y1; ++ty) {
        const uint16_t *rp = pre + (int64_t)ty * (dv.tiles_x + 1);
        cnt += (uint32_t)(rp[x1 + 1] - rp[x0]);
    }
    counts[slot] = cnt;
}

void launch_recount(const DevView *views, const FbBatch &b, int64_t n, const uint64_t *rect,
                    const uint16_t *row_prefix, uint32_t *counts, const uint32_t *n_flagged, hipStream_t s) {
    if (n == 0 || b.count == 0) return;
    hipLaunchKernelGGL(k_recount, dim3((unsigned)((n + 255) / 256), b.count), dim3(256), 0, s, views, b, n, rect,
                       row_prefix, counts, n_flagged);
}

}  // namespace a3fr
