// Per-tile depth sort (paper Sec. 2.3: the ellipses of each tile are sorted by
// depth, near to far).
//
// The order required is (tile, depth, Gaussian index).  It is produced in two
// stable radix sorts of 32-bit keys instead of one sort of 64-bit
// (tile, depth) keys:
//   1. the visible (view, Gaussian) entries -- about one per visible Gaussian
//      and layer, far fewer than keys -- are sorted by their float32 depth bits
//      (positive floats order like their bit patterns), starting from
//      (view, index) order so that equal depths stay in index order;
//   2. the keys, emitted entry by entry in that depth order, are sorted by
//      tile id alone; stability keeps each tile's keys in (depth, index) order.
//
// Both use the same onesweep LSD kernel for gfx950 (8-bit digits):
//  * one coalesced pass builds the digit histograms of every pass;
//  * one kernel per digit: a block takes the next partition id from an atomic
//    counter (so it only waits on partitions that have already started), loads
//    its keys wave-striped (lane-consecutive, coalesced), ranks them stably
//    inside each wave with 8 ballots (lanes sharing a digit) and a popcount of
//    the lower lanes, publishes its per-digit counts, resolves its global
//    digit offsets by decoupled look-back over the preceding partitions, and
//    scatters through LDS so that consecutive threads write consecutive
//    addresses of each digit run.
// The element count is read from device memory, so a launch may be sized by
// an upper bound; blocks past the last partition exit at once.
#include "a3fr_internal.h"

namespace a3fr {

constexpr int kSortThreads = 512;
constexpr int kSortWaves = kSortThreads / kWave;      // 8
// keys per thread (kSortItemsLarge / kSortItemsSmall): the entry depth sort's
// few hundred thousand keys in 8192-key partitions would leave most compute
// units idle with one long partition each, so it runs 2048-key partitions
constexpr int kRadix = 256;
constexpr int kDigitWaves = kRadix / kWave;           // waves holding one digit per lane
constexpr int kMaxPasses = 4;                         // 32-bit keys

int sort_partitions(int64_t n, int items) {
    const int64_t part = (int64_t)kSortThreads * items;
    return (int)((n + part - 1) / part);
}

// Histograms of the npass low digits of n keys (n read from *n_dev).  Each
// wave keeps its own LDS histograms; the block adds them to the global ones.
// Keys come four to a lane (16-byte loads).  Neighbouring keys often share a
// digit (tile ids of one Gaussian's rectangle, depths of one depth range),
// and LDS atomics of a wave on one address serialise: when every valid key of
// the wave's step has the same digit, one lane adds the count.
constexpr int kHistThreads = 512;
constexpr int kHistWaves = kHistThreads / kWave;
__device__ __forceinline__ void hist_add(uint32_t (*h)[kRadix], int npass, uint32_t k, bool valid, int lane) {
    const uint64_t vm = __ballot(valid);
    const int first = __ffsll((unsigned long long)vm) - 1;  // a valid lane (vm != 0 for the callers)
    for (int p = 0; p < npass; ++p) {
        const uint32_t d = (k >> (8 * p)) & 255u;
        const uint32_t d0 = __shfl(d, first, 64);
        const uint64_t same = __ballot(valid && d == d0);
        if (same == vm) {
            if (lane == first) atomicAdd(&h[p][d0], (uint32_t)__popcll(vm));
        } else if (valid) {
            atomicAdd(&h[p][d], 1u);
        }
    }
}

// The kernel also clears the look-back status words (64-bit) of the
// partitions the passes will use (those of n keys, not of the n_max the
// workspace is sized for): pass p's words start at status + p x parts_max x
// kRadix.
__global__ void __launch_bounds__(kHistThreads) k_sort_hist(const uint32_t *__restrict__ keys, const uint32_t *n_dev,
                                                            int npass, uint32_t *__restrict__ hist, int items,
                                                            int64_t parts_max) {
    __shared__ uint32_t h[kHistWaves][kMaxPasses][kRadix];
    for (int j = threadIdx.x; j < kHistWaves * kMaxPasses * kRadix; j += blockDim.x) (&h[0][0][0])[j] = 0;
    const int64_t n = *n_dev;
    {
        // status = hist + npass x kRadix + 8 (u32 words): 16-byte aligned with the workspace, and so is each
        // pass's part; kRadix 64-bit words per partition = kRadix / 2 uint4
        uint4 *status = reinterpret_cast<uint4 *>(hist + (int64_t)npass * kRadix + 8);
        const int64_t parts = (n + (int64_t)kSortThreads * items - 1) / ((int64_t)kSortThreads * items);
        const int64_t per = parts * (kRadix / 2), stride = parts_max * (kRadix / 2);
        const uint4 z = {0u, 0u, 0u, 0u};
        for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < npass * per;
             j += (int64_t)gridDim.x * blockDim.x) {
            const int64_t p = j / per;
            status[p * stride + (j - p * per)] = z;
        }
    }
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // wave-uniform loop over 256-key steps (64 lanes x 4 keys)
    const int64_t nwaves = (int64_t)gridDim.x * kHistWaves;
    for (int64_t base = ((int64_t)blockIdx.x * kHistWaves + w) * 256; base < n; base += nwaves * 256) {
        const int64_t j = base + 4 * lane;
        uint4 k4 = {0u, 0u, 0u, 0u};
        if (j + 3 < n) {
            k4 = *reinterpret_cast<const uint4 *>(keys + j);
        } else {
            if (j < n) k4.x = keys[j];
            if (j + 1 < n) k4.y = keys[j + 1];
            if (j + 2 < n) k4.z = keys[j + 2];
        }
        hist_add(h[w], npass, k4.x, j < n, lane);
        if (base + 1 < n) hist_add(h[w], npass, k4.y, j + 1 < n, lane);
        if (base + 2 < n) hist_add(h[w], npass, k4.z, j + 2 < n, lane);
        if (base + 3 < n) hist_add(h[w], npass, k4.w, j + 3 < n, lane);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < npass * kRadix; j += blockDim.x) {
        uint32_t c = 0;
#pragma unroll
        for (int q = 0; q < kHistWaves; ++q) c += (&h[q][0][0])[j];
        if (c) atomicAdd(&hist[j], c);
    }
}

// Look-back status word of a (partition, digit): [63:62] flag (1 aggregate,
// 2 inclusive prefix), [61:0] count; 64-bit so that counts up to 2^32 - 1 keys fit.
constexpr uint64_t kSt64Agg = 1ull << 62, kSt64Inc = 2ull << 62, kSt64Val = (1ull << 62) - 1;
__device__ __forceinline__ uint64_t ld_status(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_status(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One stable pass over digit (key >> shift) & 255.  Persistent: each block
// takes partition ids from the pass counter until they run out, so a launch
// sized by an upper bound costs nothing for the partitions that do not exist.
// err: sticky flag set if a look-back wait exceeds its bound (never expected:
// predecessors always publish; the bound turns a logic error into a report
// instead of a hang).
template <int kSortItems>
__global__ void __launch_bounds__(kSortThreads, 4) k_onesweep(const uint32_t *__restrict__ kin,
                                                           const uint32_t *__restrict__ vin,
                                                           uint32_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                           const uint32_t *n_dev, int shift,
                                                           const uint32_t *__restrict__ ghist, uint64_t *status,
                                                           uint32_t *counter, uint32_t *err) {
    constexpr int kSortPart = kSortThreads * kSortItems;
    __shared__ uint32_t s_part;
    __shared__ uint32_t s_wh[kSortWaves][kRadix];
    __shared__ uint32_t s_lstart[kRadix];
    __shared__ uint32_t s_gbase[kRadix];
    __shared__ uint32_t s_gexcl[kRadix];
    __shared__ uint32_t s_wsum[kDigitWaves];
    __shared__ uint32_t s_k[kSortPart];
    __shared__ uint32_t s_v[kSortPart];

    const int64_t K = *n_dev;
    const int nparts = (int)((K + kSortPart - 1) / kSortPart);
    // the grid is sized for the largest count; blocks beyond the partitions of
    // this count leave without touching the shared partition counter (every
    // partition is still taken: the lower blocks keep pulling until none is left)
    if ((int)blockIdx.x >= nparts) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    // exclusive scan of the global digit counts, once per block
    if (tid < kRadix) {
        const uint32_t g = ghist[tid];
        uint32_t inc = g;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(inc, off, 64);
            if (lane >= off) inc += y;
        }
        if (lane == 63) s_wsum[w] = inc;
    }
    __syncthreads();
    if (tid < kRadix) {
        uint32_t pre = 0;
#pragma unroll
        for (int q = 0; q < kDigitWaves; ++q) if (q < w) pre += s_wsum[q];
        const uint32_t g = ghist[tid];
        // recompute the inclusive value (cheap) rather than keep it live across the barrier
        uint32_t inc = g;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(inc, off, 64);
            if (lane >= off) inc += y;
        }
        s_gexcl[tid] = pre + inc - g;
    }

    for (;;) {
        __syncthreads();  // previous partition done with the LDS
        if (tid == 0) s_part = atomicAdd(counter, 1u);
        for (int j = tid; j < kSortWaves * kRadix; j += kSortThreads) (&s_wh[0][0])[j] = 0;
        __syncthreads();
        const uint32_t part = s_part;
        if ((int)part >= nparts) break;
        const int64_t base = (int64_t)part * kSortPart;

        uint32_t key[kSortItems], rk[kSortItems];
#pragma unroll
        for (int it = 0; it < kSortItems; ++it) {
            const int64_t pos = base + w * (kSortItems * kWave) + it * kWave + lane;
            key[it] = pos < K ? kin[pos] : 0u;
        }
#pragma unroll
        for (int it = 0; it < kSortItems; ++it) {
            const int64_t pos = base + w * (kSortItems * kWave) + it * kWave + lane;
            const bool valid = pos < K;
            const uint32_t d = (key[it] >> shift) & 255u;
            uint64_t m = __ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t bb = __ballot(bit);
                m &= bit ? bb : ~bb;
            }
            const uint32_t below = (uint32_t)__popcll(m & lt_mask);
            uint32_t prior = 0;
            if (valid) prior = s_wh[w][d];
            rk[it] = prior + below;
            if (valid && below == 0) s_wh[w][d] = prior + (uint32_t)__popcll(m);
        }
        // the values are loaded now, so that their round trip overlaps the
        // digit bookkeeping and the look-back (they were not live during the ranking)
        uint32_t val[kSortItems];
#pragma unroll
        for (int it = 0; it < kSortItems; ++it) {
            const int64_t pos = base + w * (kSortItems * kWave) + it * kWave + lane;
            val[it] = pos < K ? vin[pos] : 0u;
        }
        __syncthreads();

        // threads 0..255 = digits: totals, per-wave exclusive offsets, publication, look-back
        uint32_t tot = 0;
        if (tid < kRadix) {
            const int d = tid;
            uint32_t c[kSortWaves];
#pragma unroll
            for (int q = 0; q < kSortWaves; ++q) { c[q] = s_wh[q][d]; tot += c[q]; }
            st_status(&status[(int64_t)part * kRadix + d], (part == 0 ? kSt64Inc : kSt64Agg) | (uint64_t)tot);
            uint32_t run = 0;
#pragma unroll
            for (int q = 0; q < kSortWaves; ++q) { s_wh[q][d] = run; run += c[q]; }
            // block-local exclusive scan over digits (waves 0..3)
            uint32_t inc = tot;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t y = __shfl_up(inc, off, 64);
                if (lane >= off) inc += y;
            }
            if (lane == 63) s_wsum[w] = inc;
            s_lstart[d] = inc - tot;  // wave-local part; the waves' offsets are added below
        }
        __syncthreads();
        if (tid < kRadix) {
            uint32_t pre = 0;
#pragma unroll
            for (int q = 0; q < kDigitWaves; ++q) if (q < w) pre += s_wsum[q];
            s_lstart[tid] += pre;
        }
        __syncthreads();
        // local scatter into LDS (positions within the partition are known
        // before the look-back), then the digit threads look back
#pragma unroll
        for (int it = 0; it < kSortItems; ++it) {
            const int64_t pos = base + w * (kSortItems * kWave) + it * kWave + lane;
            if (pos < K) {
                const uint32_t dg = (key[it] >> shift) & 255u;
                const uint32_t lp = s_lstart[dg] + s_wh[w][dg] + rk[it];
                s_k[lp] = key[it];
                s_v[lp] = val[it];
            }
        }
        if (tid < kRadix) {
            const int d = tid;
            uint64_t excl = 0;
            if (part > 0) {
                // look back over a window of kWin predecessors at a time: the
                // window's loads are independent, so one round trip to the
                // coherence point covers up to kWin partitions
                constexpr int kWin = 8;
                int64_t p = (int64_t)part - 1;
                uint32_t spins = 0;
                bool found = false;
                while (!found && p >= 0) {
                    uint64_t st[kWin];
#pragma unroll
                    for (int q = 0; q < kWin; ++q)
                        st[q] = (p - q >= 0) ? ld_status(&status[(p - q) * kRadix + d]) : kSt64Inc;
                    int used = 0;
#pragma unroll
                    for (int q = 0; q < kWin; ++q) {
                        if (found || used < q) continue;  // stopped earlier in this window
                        const uint32_t flag = (uint32_t)(st[q] >> 62);
                        if (flag == 0) continue;           // not published yet: reload from here
                        excl += st[q] & kSt64Val;
                        used = q + 1;
                        if (flag == 2) found = true;
                    }
                    p -= used;
                    if (!found && used == 0 && ++spins > (1u << 24)) { atomicOr(err, 1u); break; }
                }
                st_status(&status[(int64_t)part * kRadix + d], kSt64Inc | (excl + tot));
            }
            s_gbase[d] = s_gexcl[d] + (uint32_t)excl;
        }
        __syncthreads();
        const int64_t rem = K - base;
        const int nvalid = rem < kSortPart ? (int)rem : kSortPart;
        for (int j = tid; j < nvalid; j += kSortThreads) {
            const uint32_t kk = s_k[j];
            const uint32_t dg = (kk >> shift) & 255u;
            const uint32_t g = s_gbase[dg] + ((uint32_t)j - s_lstart[dg]);
            if ((int64_t)g < K) {
                kout[g] = kk;
                vout[g] = s_v[j];
            }
        }
    }
}

// ws (u32 words): one workspace [hist npass x 256 | counters 8 | status npass x partitions x 256 (u64)]
// cleared by one fill, then the digit histograms of all passes.
int64_t sort_workspace_words(int64_t n_max, int npass, int items) {
    return sort_zero_words(npass) + 2 * (int64_t)npass * sort_partitions(n_max, items) * kRadix;
}

int64_t sort_zero_words(int npass) { return (int64_t)npass * kRadix + 8; }

void launch_sort_prepare(const uint32_t *keys, const uint32_t *n_dev, int64_t n_max, int npass, int items,
                         uint32_t *ws, hipStream_t s, bool zeroed) {
    const int nparts = sort_partitions(n_max, items);
    if (!zeroed) launch_fill_u32(ws, 0u, sort_zero_words(npass), s);
    if (nparts == 0) return;
    int hblocks = (int)((n_max + kHistThreads * 16 - 1) / (kHistThreads * 16));
    if (hblocks > 512) hblocks = 512;
    hipLaunchKernelGGL(k_sort_hist, dim3((unsigned)hblocks), dim3(kHistThreads), 0, s, keys, n_dev, npass, ws, items,
                       (int64_t)nparts);
}

void launch_sort_pass(const uint32_t *ki, const uint32_t *vi, uint32_t *ko, uint32_t *vo, const uint32_t *n_dev,
                      int64_t n_max, int npass, int items, int p, uint32_t *ws, uint32_t *err, hipStream_t s) {
    const int nparts = sort_partitions(n_max, items);
    if (nparts == 0) return;
    uint32_t *hist = ws, *ctr = ws + (int64_t)npass * kRadix;
    uint64_t *status = reinterpret_cast<uint64_t *>(ctr + 8);  // 8-byte aligned: npass x 1 KiB + 32 B in
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    // persistent blocks: LDS per block ~74 KB (16 items) or ~26 KB (4 items)
    const int resident = cus * (items == kSortItemsSmall ? 4 : 2);
    const int grid = nparts < resident ? nparts : resident;
    if (items == kSortItemsSmall)
        hipLaunchKernelGGL(k_onesweep<kSortItemsSmall>, dim3((unsigned)grid), dim3(kSortThreads), 0, s, ki, vi, ko, vo,
                           n_dev, 8 * p, hist + (int64_t)p * kRadix, status + (int64_t)p * nparts * kRadix, ctr + p,
                           err);
    else
        hipLaunchKernelGGL(k_onesweep<kSortItemsLarge>, dim3((unsigned)grid), dim3(kSortThreads), 0, s, ki, vi, ko, vo,
                           n_dev, 8 * p, hist + (int64_t)p * kRadix, status + (int64_t)p * nparts * kRadix, ctr + p,
                           err);
}

// ------------------------------------------------------------------------
// tile ranges from the sorted tile ids
// ------------------------------------------------------------------------
// One thread per tile: its range [start, end) in the sorted tile ids by two
// binary searches (lower bounds of t and t + 1); an empty tile gets (0, 0).
// Threads of a wave search neighbouring tiles, so the upper levels of the
// searches hit the same cache lines.
__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t *__restrict__ a, uint32_t n, uint32_t v) {
    uint32_t lo = 0, len = n;
    while (len > 0) {
        const uint32_t half = len >> 1;
        if (a[lo + half] < v) {
            lo += half + 1;
            len -= half + 1;
        } else {
            len = half;
        }
    }
    return lo;
}

__global__ void __launch_bounds__(256) k_ranges(const uint32_t *__restrict__ tiles, int64_t K, const uint32_t *K_dev,
                                                int64_t ntiles, uint32_t *__restrict__ ranges) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    if (K_dev && (int64_t)*K_dev < K) K = *K_dev;  // capacity mode
    const uint32_t n = (uint32_t)K;
    const uint32_t s0 = lower_bound_u32(tiles, n, (uint32_t)t);
    const uint32_t s1 = lower_bound_u32(tiles, n, (uint32_t)t + 1u);
    ranges[2 * t] = s0 == s1 ? 0u : s0;
    ranges[2 * t + 1] = s0 == s1 ? 0u : s1;
}

void launch_ranges(const uint32_t *tiles, int64_t K, const uint32_t *K_dev, int64_t ntiles, uint32_t *ranges,
                   hipStream_t s) {
    if (ntiles == 0) return;
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)((ntiles + 255) / 256)), dim3(256), 0, s, tiles, K, K_dev, ntiles,
                       ranges);
}

}  // namespace a3fr
