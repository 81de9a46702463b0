// Periphery subset, key-count scan and tile-key emission.
//
// The periphery layer draws only the visible Gaussians with the largest
// opacity x projected area: the top ceil(num/den x N_vis) by the 96-bit key
// (score bits, ~index), i.e. score descending, index ascending.  It is found
// by an MSD radix select over 8-bit digits: a histogram pass over the
// candidates that still match the chosen prefix, then a one-block decision
// that picks the digit holding the k-th largest key.  Keys are unique, so the
// select ends (usually after 3-4 of the 12 possible passes) as soon as the
// chosen bucket is kept whole; later passes exit at once.
//
// Keys (paper Sec. 2.3: the tiles each ellipse intersects, then per-tile depth
// order): the visible (view, Gaussian) entries are compacted in (view, index)
// order, sorted by depth (sort.hip), prefix-summed in that order, and then each
// entry writes one 32-bit key (its global tile id) per active tile of its
// rectangle, row by row, with the Gaussian index as value.  A stable sort of
// these keys by tile id leaves every tile's list in (depth, index) order.
#include "a3fr_internal.h"

namespace a3fr {

// ------------------------------------------------------------------------
// periphery select
// ------------------------------------------------------------------------
struct SelState {
    uint32_t n_vis, k, k_rem, done;   // done: 0 running, 1 finished
    uint32_t mode;                    // 0: compare digits, 1: keep all visible, 2: keep none
    uint32_t npass;                   // digits[0..npass) define the kept prefix
    uint32_t pad[2];
    uint32_t digit[12];
};

__device__ __forceinline__ uint32_t sel_digit(double score, uint32_t idx, int pass) {
    const uint64_t sb = (uint64_t)__double_as_longlong(score);
    if (pass < 8) return (uint32_t)(sb >> (56 - 8 * pass)) & 255u;
    return ((~idx) >> (24 - 8 * (pass - 8))) & 255u;
}

__global__ void k_sel_init(SelState *st, uint32_t *hist, int nsel) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nsel * (int)(sizeof(SelState) / 4)) reinterpret_cast<uint32_t *>(st)[t] = 0;
    for (int j = t; j < nsel * 12 * 256; j += gridDim.x * blockDim.x) hist[j] = 0;
}

__global__ void __launch_bounds__(256) k_sel_hist(const int32_t *sel_views, const uint32_t *__restrict__ counts,
                                                  const double *__restrict__ score, int64_t n, int pass,
                                                  const SelState *st, uint32_t *hist) {
    const int slot = blockIdx.y;
    if (st[slot].done) return;
    __shared__ uint32_t h[256];
    __shared__ uint32_t dig[12];
    h[threadIdx.x] = 0;
    if (threadIdx.x < 12) dig[threadIdx.x] = st[slot].digit[threadIdx.x];
    __syncthreads();
    const int64_t base = (int64_t)sel_views[slot] * n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (counts[base + i] == 0) continue;
        const double sc = score[base + i];
        bool match = true;
        for (int p = 0; p < pass; ++p)
            if (sel_digit(sc, (uint32_t)i, p) != dig[p]) { match = false; break; }
        if (match) atomicAdd(&h[sel_digit(sc, (uint32_t)i, pass)], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[((int64_t)slot * 12 + pass) * 256 + threadIdx.x], h[threadIdx.x]);
}

__global__ void __launch_bounds__(256) k_sel_decide(int pass, int keep_num, int keep_den, SelState *st,
                                                    const uint32_t *hist) {
    const int slot = blockIdx.x;
    SelState &S = st[slot];
    if (S.done) return;
    const int d = threadIdx.x;
    __shared__ uint32_t suf[257];
    const uint32_t h = hist[((int64_t)slot * 12 + pass) * 256 + d];
    suf[d] = h;
    if (d == 0) suf[256] = 0;
    __syncthreads();
    // inclusive suffix sums suf[d] = sum_{d' >= d} h[d'] (Hillis-Steele over 256)
    for (int off = 1; off < 256; off <<= 1) {
        uint32_t add = (d + off < 256) ? suf[d + off] : 0u;
        __syncthreads();
        suf[d] += add;
        __syncthreads();
    }
    __shared__ uint32_t s_krem, s_done;
    if (d == 0) {
        uint32_t done = 0;
        if (pass == 0) {
            const uint32_t nvis = suf[0];
            const uint64_t k = ((uint64_t)keep_num * nvis + (uint64_t)keep_den - 1) / (uint64_t)keep_den;
            S.n_vis = nvis;
            S.k = (uint32_t)k;
            S.k_rem = (uint32_t)k;
            if (k == 0) { S.mode = 2; done = 1; }
            else if (k >= nvis) { S.mode = 1; done = 1; }
            if (done) S.done = 1;
        }
        s_krem = S.k_rem;
        s_done = done;
    }
    __syncthreads();
    if (s_done) return;
    const uint32_t krem = s_krem;
    const uint32_t above = suf[d + 1];
    if (suf[d] >= krem && above < krem) {
        const uint32_t k2 = krem - above;
        S.digit[pass] = (uint32_t)d;
        S.k_rem = k2;
        S.npass = (uint32_t)pass + 1;
        if (h == k2 || pass == 11) S.done = 1;
    }
}

__global__ void __launch_bounds__(256) k_sel_mark(const int32_t *sel_views, const uint32_t *__restrict__ counts,
                                                  const double *__restrict__ score, int64_t n, const SelState *st,
                                                  uint8_t *keep) {
    const int slot = blockIdx.y;
    __shared__ uint32_t dig[12];
    if (threadIdx.x < 12) dig[threadIdx.x] = st[slot].digit[threadIdx.x];
    __syncthreads();
    const uint32_t mode = st[slot].mode, npass = st[slot].npass;
    const int64_t base = (int64_t)sel_views[slot] * n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint8_t kp = 0;
        if (counts[base + i] != 0) {
            if (mode == 1) kp = 1;
            else if (mode == 0) {
                const double sc = score[base + i];
                kp = 1;  // equal through the decided prefix: the bucket is kept whole
                for (uint32_t p = 0; p < npass; ++p) {
                    const uint32_t dg = sel_digit(sc, (uint32_t)i, (int)p);
                    if (dg != dig[p]) { kp = dg > dig[p] ? 1 : 0; break; }
                }
            }
        }
        keep[base + i] = kp;
    }
}

void launch_select(const DevView *views, int nv, const int32_t *sel_views, int nsel, int64_t n,
                   const uint32_t *counts, const double *score, int keep_num, int keep_den,
                   uint32_t *sel_hist, uint8_t *keep, hipStream_t s) {
    (void)views; (void)nv;
    if (nsel == 0 || n == 0) return;
    // state lives right after the histograms
    SelState *st = reinterpret_cast<SelState *>(sel_hist + (int64_t)nsel * 12 * 256);
    hipLaunchKernelGGL(k_sel_init, dim3(64), dim3(256), 0, s, st, sel_hist, nsel);
    int64_t blocks = (n + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    for (int pass = 0; pass < 12; ++pass) {
        hipLaunchKernelGGL(k_sel_hist, dim3((unsigned)blocks, (unsigned)nsel), dim3(256), 0, s, sel_views, counts,
                           score, n, pass, st, sel_hist);
        hipLaunchKernelGGL(k_sel_decide, dim3((unsigned)nsel), dim3(256), 0, s, pass, keep_num, keep_den, st,
                           sel_hist);
    }
    hipLaunchKernelGGL(k_sel_mark, dim3((unsigned)blocks, (unsigned)nsel), dim3(256), 0, s, sel_views, counts,
                       score, n, st, keep);
}

// ------------------------------------------------------------------------
// scans: compaction of the visible entries, then key offsets in depth order
// ------------------------------------------------------------------------
constexpr int kScanItems = 16;
constexpr int kScanBlock = 256;
constexpr int kScanTile = kScanItems * kScanBlock;  // 4096 entries per block

// Entry e = view * n + index contributes keys iff it is visible in its view and,
// for a selecting view, kept.
struct EntryFlags {
    const uint32_t *counts;
    const uint8_t *keep;
    const DevView *views;
    int64_t n;
    __device__ __forceinline__ uint32_t operator()(int64_t e, int64_t m) const {
        if (e >= m) return 0;
        if (counts[e] == 0) return 0;
        const int v = (int)(e / n);
        if (views[v].v.select && !keep[e]) return 0;
        return 1;
    }
};

// Key count of the j-th entry in depth order.
struct SortedCounts {
    const uint32_t *counts;
    const uint32_t *ent;
    const uint32_t *n_ent;
    __device__ __forceinline__ uint32_t operator()(int64_t j, int64_t) const {
        return j < (int64_t)*n_ent ? counts[ent[j]] : 0u;
    }
};

// wave-level inclusive scan of a 64-bit value (wave64 via shuffles)
__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint64_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}

// block-wide exclusive scan of one 64-bit value per thread (256 threads)
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t x, uint64_t *total) {
    __shared__ uint64_t wsum[kScanBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint64_t inc = wave_incl_scan(x);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint64_t wpre = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kScanBlock / 64; ++k) {
        if (k < w) wpre += wsum[k];
        tot += wsum[k];
    }
    __syncthreads();
    *total = tot;
    return wpre + inc - x;
}

template <class F>
__global__ void __launch_bounds__(kScanBlock) k_scan_reduce(F f, int64_t m, uint64_t *block_sums) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint64_t acc = 0;
#pragma unroll 4
    for (int j = 0; j < kScanItems; ++j) acc += f(base + (int64_t)j * kScanBlock + threadIdx.x, m);
    uint64_t tot;
    block_excl_scan(acc, &tot);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// one block: exclusive scan of nb block sums in chunks of 1024; writes the
// grand total as u64 and (clamped) u32
__global__ void __launch_bounds__(1024) k_scan_blocks(uint64_t *block_sums, int64_t nb, uint64_t *total,
                                                      uint32_t *total32) {
    __shared__ uint64_t wsum[16];
    __shared__ uint64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int64_t c0 = 0; c0 < nb; c0 += 1024) {
        const int64_t j = c0 + threadIdx.x;
        const uint64_t x = j < nb ? block_sums[j] : 0;
        const uint64_t inc = wave_incl_scan(x);
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        uint64_t wpre = 0, tot = 0;
        for (int k = 0; k < 16; ++k) {
            if (k < w) wpre += wsum[k];
            tot += wsum[k];
        }
        const uint64_t base = carry;
        if (j < nb) block_sums[j] = base + wpre + inc - x;
        __syncthreads();
        if (threadIdx.x == 0) carry = base + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *total = carry;
        *total32 = carry > 0xffffffffull ? 0xffffffffu : (uint32_t)carry;
    }
}

// Compaction: entry e with flag 1 goes to slot (its exclusive prefix), with
// its depth bits as sort key.  Thread t owns 16 consecutive entries (blocked),
// so the running sum inside a thread follows entry order.
__global__ void __launch_bounds__(kScanBlock) k_compact_down(EntryFlags f, int64_t m, const uint64_t *block_pre,
                                                             const uint32_t *__restrict__ depth,
                                                             uint32_t *__restrict__ ent, uint32_t *__restrict__ dkey) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t flags = 0, cnt = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const uint32_t fl = f(base + j, m);
        flags |= fl << j;
        cnt += fl;
    }
    uint64_t tot;
    uint64_t run = block_pre[blockIdx.x] + block_excl_scan(cnt, &tot);
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        if ((flags >> j) & 1u) {
            const int64_t e = base + j;
            ent[run] = (uint32_t)e;
            dkey[run] = depth[e];
            ++run;
        }
    }
}

// Offsets of the keys of the entries in depth order; offsets[E] = K.
__global__ void __launch_bounds__(kScanBlock) k_offsets_down(SortedCounts f, int64_t m, const uint64_t *block_pre,
                                                             const uint64_t *total, uint32_t *offsets) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    const int64_t E = *f.n_ent;
    uint32_t c[kScanItems];
    uint64_t acc = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        c[j] = f(base + j, m);
        acc += c[j];
    }
    uint64_t tot;
    uint64_t run = block_pre[blockIdx.x] + block_excl_scan(acc, &tot);
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t e = base + j;
        if (e < E) offsets[e] = (uint32_t)run;
        run += c[j];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) offsets[E] = (uint32_t)*total;
}

void launch_compact_entries(const uint32_t *counts, const uint8_t *keep, const DevView *views, int nv, int64_t n,
                            const uint32_t *depth, uint32_t *ent, uint32_t *dkey, uint64_t *block_sums,
                            uint64_t *total, uint32_t *n_ent, hipStream_t s) {
    const int64_t m = (int64_t)nv * n;
    const int64_t nb = (m + kScanTile - 1) / kScanTile;
    EntryFlags f{counts, keep, views, n};
    if (nb > 0) hipLaunchKernelGGL(k_scan_reduce<EntryFlags>, dim3((unsigned)nb), dim3(kScanBlock), 0, s, f, m, block_sums);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, block_sums, nb, total, n_ent);
    if (nb > 0)
        hipLaunchKernelGGL(k_compact_down, dim3((unsigned)nb), dim3(kScanBlock), 0, s, f, m, block_sums, depth, ent, dkey);
}

void launch_key_offsets(const uint32_t *counts, const uint32_t *ent, const uint32_t *n_ent, int64_t m,
                        uint32_t *offsets, uint64_t *block_sums, uint64_t *total, uint32_t *total32, hipStream_t s) {
    const int64_t nb = (m + kScanTile - 1) / kScanTile;
    SortedCounts f{counts, ent, n_ent};
    if (nb > 0) hipLaunchKernelGGL(k_scan_reduce<SortedCounts>, dim3((unsigned)nb), dim3(kScanBlock), 0, s, f, m, block_sums);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, block_sums, nb, total, total32);
    hipLaunchKernelGGL(k_offsets_down, dim3((unsigned)(nb > 0 ? nb : 1)), dim3(kScanBlock), 0, s, f, m, block_sums,
                       total, offsets);
}

// ------------------------------------------------------------------------
// key emission (entries in depth order)
// ------------------------------------------------------------------------
constexpr uint32_t kBigKeys = 48;  // entries with more keys go to the cooperative path

__device__ __forceinline__ void unpack_rect(uint64_t r, int &x0, int &x1, int &y0, int &y1) {
    x0 = (int)(r & 0xffff); x1 = (int)((r >> 16) & 0xffff);
    y0 = (int)((r >> 32) & 0xffff); y1 = (int)((r >> 48) & 0xffff);
}

__global__ void __launch_bounds__(256) k_emit(const DevView *__restrict__ views, int64_t n,
                                              const uint32_t *__restrict__ ent, const uint32_t *n_ent,
                                              const uint32_t *__restrict__ offsets, const uint64_t *__restrict__ rect,
                                              const uint16_t *__restrict__ row_prefix,
                                              const uint16_t *__restrict__ row_list, uint32_t *__restrict__ keys,
                                              uint32_t *__restrict__ vals, uint32_t *big_list, uint32_t *big_count) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= (int64_t)*n_ent) return;
    const uint32_t off = offsets[j];
    const uint32_t cnt = offsets[j + 1] - off;
    if (cnt == 0) return;
    if (cnt > kBigKeys) {
        big_list[atomicAdd(big_count, 1u)] = (uint32_t)j;
        return;
    }
    const int64_t e = ent[j];
    const int v = (int)(e / n);
    const DevView &dv = views[v];
    const uint32_t i = (uint32_t)(e - (int64_t)v * n);
    int x0, x1, y0, y1;
    unpack_rect(rect[e], x0, x1, y0, y1);
    const int TX = dv.tiles_x;
    const uint32_t tbase = (uint32_t)dv.tile_off;
    uint32_t w = off;
    const uint32_t wend = off + cnt;  // never write past this entry's slots
    if (dv.v.mask == A3FR_MASK_ALL) {
        for (int ty = y0; ty <= y1; ++ty)
            for (int tx = x0; tx <= x1 && w < wend; ++tx) {
                keys[w] = tbase + (uint32_t)(ty * TX + tx);
                vals[w] = i;
                ++w;
            }
    } else {
        for (int ty = y0; ty <= y1; ++ty) {
            const uint16_t *rp = row_prefix + dv.mask_off + (int64_t)ty * (TX + 1);
            const uint16_t *rl = row_list + dv.mask_off + (int64_t)ty * (TX + 1);
            for (int p = rp[x0]; p < rp[x1 + 1] && w < wend; ++p) {
                keys[w] = tbase + (uint32_t)(ty * TX + rl[p]);
                vals[w] = i;
                ++w;
            }
        }
    }
}

// One block per entry with many keys; threads write consecutive keys.
__global__ void __launch_bounds__(256) k_emit_big(const DevView *__restrict__ views, int64_t n,
                                                  const uint32_t *__restrict__ ent,
                                                  const uint32_t *__restrict__ offsets, const uint64_t *__restrict__ rect,
                                                  const uint16_t *__restrict__ row_prefix,
                                                  const uint16_t *__restrict__ row_list, uint32_t *__restrict__ keys,
                                                  uint32_t *__restrict__ vals, const uint32_t *big_list,
                                                  const uint32_t *big_count) {
    const uint32_t nbig = *big_count;
    for (uint32_t b = blockIdx.x; b < nbig; b += gridDim.x) {
        const int64_t j = big_list[b];
        const int64_t e = ent[j];
        const int v = (int)(e / n);
        const DevView &dv = views[v];
        const uint32_t i = (uint32_t)(e - (int64_t)v * n);
        const uint32_t off = offsets[j];
        const uint32_t cnt_e = offsets[j + 1] - off;
        int x0, x1, y0, y1;
        unpack_rect(rect[e], x0, x1, y0, y1);
        const int TX = dv.tiles_x;
        const uint32_t tbase = (uint32_t)dv.tile_off;
        if (dv.v.mask == A3FR_MASK_ALL) {
            const uint32_t wdt = (uint32_t)(x1 - x0 + 1);
            uint32_t cnt = wdt * (uint32_t)(y1 - y0 + 1);
            if (cnt > cnt_e) cnt = cnt_e;
            for (uint32_t q = threadIdx.x; q < cnt; q += blockDim.x) {
                const int ty = y0 + (int)(q / wdt), tx = x0 + (int)(q % wdt);
                keys[off + q] = tbase + (uint32_t)(ty * TX + tx);
                vals[off + q] = i;
            }
        } else {
            uint32_t run = off;
            for (int ty = y0; ty <= y1; ++ty) {
                const uint16_t *rp = row_prefix + dv.mask_off + (int64_t)ty * (TX + 1);
                const uint16_t *rl = row_list + dv.mask_off + (int64_t)ty * (TX + 1);
                const int p0 = rp[x0];
                int rc = rp[x1 + 1] - p0;
                if (run + (uint32_t)rc > off + cnt_e) rc = (int)(off + cnt_e - run);
                for (int q = threadIdx.x; q < rc; q += blockDim.x) {
                    keys[run + q] = tbase + (uint32_t)(ty * TX + rl[p0 + q]);
                    vals[run + q] = i;
                }
                run += (uint32_t)rc;
            }
        }
    }
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        p[j] = v;
}

void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
}

void launch_emit(const DevView *views, int64_t n, int64_t m, const uint32_t *ent, const uint32_t *n_ent,
                 const uint32_t *offsets, const uint64_t *rect, const uint16_t *row_prefix, const uint16_t *row_list,
                 uint32_t *keys, uint32_t *vals, uint32_t *big_list, uint32_t *big_count, hipStream_t s) {
    if (m == 0) return;
    launch_fill_u32(big_count, 0u, 1, s);
    hipLaunchKernelGGL(k_emit, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, views, n, ent, n_ent, offsets, rect,
                       row_prefix, row_list, keys, vals, big_list, big_count);
    hipLaunchKernelGGL(k_emit_big, dim3(2048), dim3(256), 0, s, views, n, ent, offsets, rect, row_prefix, row_list,
                       keys, vals, big_list, big_count);
}

// ------------------------------------------------------------------------
// inspection: 64-bit (tile << 32 | depth bits) keys from tile ids and values
// ------------------------------------------------------------------------
__global__ void k_make_keys64(const DevView *__restrict__ views, int nv, int64_t n, const uint32_t *__restrict__ tiles,
                              const uint32_t *__restrict__ vals, int64_t K, const uint32_t *__restrict__ depth,
                              uint64_t *__restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= K) return;
    const uint32_t t = tiles[j];
    int lo = 0, hi = nv - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].tile_off <= (int64_t)t) lo = mid; else hi = mid - 1;
    }
    const uint32_t i = vals[j] < (uint32_t)n ? vals[j] : 0u;
    out[j] = ((uint64_t)t << 32) | (uint64_t)depth[(int64_t)lo * n + i];
}

void launch_make_keys64(const DevView *views, int nv, int64_t n, const uint32_t *tiles, const uint32_t *vals,
                        int64_t K, const uint32_t *depth, uint64_t *out, hipStream_t s) {
    if (K == 0) return;
    hipLaunchKernelGGL(k_make_keys64, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, s, views, nv, n, tiles, vals, K,
                       depth, out);
}

}  // namespace a3fr
