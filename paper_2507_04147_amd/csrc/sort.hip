// Per-tile depth sort (paper Sec. 2.3: the ellipses of each tile are sorted by
// depth, near to far) as one stable LSD radix sort of the 64-bit
// (tile << 32 | depth bits) keys with their Gaussian-index values.
//
// Onesweep structure for gfx950:
//  * one pass over the keys builds the digit histograms of every 8-bit pass;
//  * then one kernel per pass.  A block takes the next partition id from an
//    atomic counter (so it only ever waits on partitions that have already
//    started), loads 4096 keys wave-striped (lane-consecutive, coalesced), ranks
//    them stably inside each wave with ballots (8 ballots give the lanes that
//    share a digit; popcount below the lane gives the rank), publishes its
//    digit counts, and finds its global digit offsets by decoupled look-back
//    over the preceding partitions' published counts;
//  * keys are first scattered into LDS in sorted order and then written out,
//    so that consecutive threads write consecutive addresses of each digit run.
// Stability: within a partition the wave-striped processing order (item, lane)
// equals memory order, and waves / partitions are combined in order.
#include "a3fr_internal.h"

namespace a3fr {

constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / kWave;
constexpr int kSortItems = 16;
constexpr int kSortPart = kSortThreads * kSortItems;  // 4096 keys per partition
constexpr int kRadix = 256;
constexpr int kMaxPasses = 8;

int sort_passes_for_bits(int bits) { return (bits + 7) / 8; }

__global__ void __launch_bounds__(256) k_sort_hist(const uint64_t *__restrict__ keys, int64_t K, int npass,
                                                   uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[kMaxPasses][kRadix];
    for (int j = threadIdx.x; j < kMaxPasses * kRadix; j += blockDim.x) (&h[0][0])[j] = 0;
    __syncthreads();
    // each thread walks a contiguous run of keys and flushes a digit's count
    // only when the digit changes (keys of one Gaussian share most digits)
    const int64_t per_thread = 16;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x * per_thread;
    for (int64_t b0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * per_thread; b0 < K; b0 += stride) {
        const int64_t b1 = b0 + per_thread < K ? b0 + per_thread : K;
        for (int p = 0; p < npass; ++p) {
            uint32_t cur = 0xffffffffu, run = 0;
            for (int64_t j = b0; j < b1; ++j) {
                const uint32_t d = (uint32_t)(keys[j] >> (8 * p)) & 255u;
                if (d != cur) {
                    if (run) atomicAdd(&h[p][cur], run);
                    cur = d;
                    run = 0;
                }
                ++run;
            }
            if (run) atomicAdd(&h[p][cur], run);
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < npass * kRadix; j += blockDim.x) {
        const uint32_t c = (&h[0][0])[j];
        if (c) atomicAdd(&hist[j], c);
    }
}

__device__ __forceinline__ uint32_t ld_status(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_status(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void __launch_bounds__(kSortThreads) k_onesweep(const uint64_t *__restrict__ kin,
                                                           const uint32_t *__restrict__ vin,
                                                           uint64_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                           int64_t K, int shift, const uint32_t *__restrict__ ghist,
                                                           uint32_t *status, uint32_t *counter) {
    __shared__ uint32_t s_part;
    __shared__ uint32_t s_wh[kSortWaves][kRadix];
    __shared__ uint32_t s_lstart[kRadix];
    __shared__ uint32_t s_gbase[kRadix];
    __shared__ uint32_t s_wsum[kSortWaves];
    __shared__ uint64_t s_k[kSortPart];
    __shared__ uint32_t s_v[kSortPart];

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) s_part = atomicAdd(counter, 1u);
    for (int j = tid; j < kSortWaves * kRadix; j += kSortThreads) (&s_wh[0][0])[j] = 0;
    __syncthreads();
    const uint32_t part = s_part;
    const int64_t base = (int64_t)part * kSortPart;

    uint64_t key[kSortItems];
    uint32_t val[kSortItems];
    uint32_t rk[kSortItems];
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t pos = base + w * (kSortItems * kWave) + it * kWave + lane;
        const bool valid = pos < K;
        key[it] = valid ? kin[pos] : 0ull;
        val[it] = valid ? vin[pos] : 0u;
    }
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t pos = base + w * (kSortItems * kWave) + it * kWave + lane;
        const bool valid = pos < K;
        const uint32_t d = (uint32_t)(key[it] >> shift) & 255u;
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
    __syncthreads();

    // per-digit totals and per-wave exclusive offsets (thread = digit)
    const int d = tid;
    uint32_t c[kSortWaves];
    uint32_t tot = 0;
#pragma unroll
    for (int q = 0; q < kSortWaves; ++q) { c[q] = s_wh[q][d]; tot += c[q]; }
    // publish this partition's count of digit d
    st_status(&status[(int64_t)part * kRadix + d], (part == 0 ? kFlagInc : kFlagAgg) | tot);
    {
        uint32_t run = 0;
#pragma unroll
        for (int q = 0; q < kSortWaves; ++q) { s_wh[q][d] = run; run += c[q]; }
    }
    // block-local exclusive scan over digits
    {
        uint32_t inc = tot;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(inc, off, 64);
            if (lane >= off) inc += y;
        }
        if (lane == 63) s_wsum[w] = inc;
        __syncthreads();
        uint32_t pre = 0;
#pragma unroll
        for (int q = 0; q < kSortWaves; ++q) if (q < w) pre += s_wsum[q];
        s_lstart[d] = pre + inc - tot;
    }
    // global base of digit d: digits below it over all keys, then this digit in earlier partitions
    uint32_t gexcl;
    {
        const uint32_t g = ghist[d];
        uint32_t inc = g;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(inc, off, 64);
            if (lane >= off) inc += y;
        }
        __syncthreads();
        if (lane == 63) s_wsum[w] = inc;
        __syncthreads();
        uint32_t pre = 0;
#pragma unroll
        for (int q = 0; q < kSortWaves; ++q) if (q < w) pre += s_wsum[q];
        gexcl = pre + inc - g;
    }
    uint32_t excl = 0;
    if (part > 0) {
        int64_t p = (int64_t)part - 1;
        uint32_t spins = 0;
        while (p >= 0) {
            const uint32_t st = ld_status(&status[p * kRadix + d]);
            const uint32_t flag = st >> 30;
            if (flag == 0) {
                // predecessors always publish; the bound only turns a logic
                // error into a reported failure instead of a hang
                if (++spins > (1u << 26)) { atomicOr(counter - (shift / 8) + kMaxPasses, 1u); break; }
                continue;
            }
            excl += st & kValMask;
            if (flag == 2) break;
            --p;
        }
        st_status(&status[(int64_t)part * kRadix + d], kFlagInc | (excl + tot));
    }
    s_gbase[d] = gexcl + excl;
    __syncthreads();

#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t pos = base + w * (kSortItems * kWave) + it * kWave + lane;
        if (pos < K) {
            const uint32_t dg = (uint32_t)(key[it] >> shift) & 255u;
            const uint32_t lp = s_lstart[dg] + s_wh[w][dg] + rk[it];
            s_k[lp] = key[it];
            s_v[lp] = val[it];
        }
    }
    __syncthreads();
    const int64_t rem = K - base;
    const int nvalid = rem < kSortPart ? (int)rem : kSortPart;
    for (int j = tid; j < nvalid; j += kSortThreads) {
        const uint64_t kk = s_k[j];
        const uint32_t dg = (uint32_t)(kk >> shift) & 255u;
        const uint32_t g = s_gbase[dg] + ((uint32_t)j - s_lstart[dg]);
        if ((int64_t)g < K) {
            kout[g] = kk;
            vout[g] = s_v[j];
        }
    }
}

// Digit histograms of all npass passes (and cleared look-back state).
// status must hold npass x ceil(K/4096) x 256 words; counters holds npass words
// plus, at index kMaxPasses, a sticky error flag (look-back gave up waiting)
// that the owner clears once.
void launch_sort_hist(const uint64_t *keys, int64_t K, int npass, uint32_t *hist, uint32_t *status,
                      uint32_t *counters, hipStream_t s) {
    const int64_t nparts = (K + kSortPart - 1) / kSortPart;
    launch_fill_u32(hist, 0u, (int64_t)npass * kRadix, s);
    launch_fill_u32(status, 0u, (int64_t)npass * nparts * kRadix, s);
    launch_fill_u32(counters, 0u, npass, s);
    int64_t hblocks = (K + 256 * 16 - 1) / (256 * 16);
    if (hblocks > 4096) hblocks = 4096;
    if (K > 0) hipLaunchKernelGGL(k_sort_hist, dim3((unsigned)hblocks), dim3(256), 0, s, keys, K, npass, hist);
}

// One onesweep pass over digit p (bits 8p .. 8p+7): (ki, vi) -> (ko, vo).
void launch_sort_pass(const uint64_t *ki, const uint32_t *vi, uint64_t *ko, uint32_t *vo, int64_t K, int p,
                      const uint32_t *hist, uint32_t *status, uint32_t *counters, hipStream_t s) {
    const int64_t nparts = (K + kSortPart - 1) / kSortPart;
    if (nparts == 0) return;
    hipLaunchKernelGGL(k_onesweep, dim3((unsigned)nparts), dim3(kSortThreads), 0, s, ki, vi, ko, vo, K, 8 * p,
                       hist + (int64_t)p * kRadix, status + (int64_t)p * nparts * kRadix, counters + p);
}

// ------------------------------------------------------------------------
// tile ranges
// ------------------------------------------------------------------------
__global__ void k_ranges(const uint64_t *__restrict__ keys, int64_t K, int64_t ntiles, uint32_t *__restrict__ ranges) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= K) return;
    const uint64_t t = keys[j] >> 32;
    if ((int64_t)t >= ntiles) return;
    if (j == 0 || (keys[j - 1] >> 32) != t) ranges[2 * t] = (uint32_t)j;
    if (j == K - 1 || (keys[j + 1] >> 32) != t) ranges[2 * t + 1] = (uint32_t)(j + 1);
}

void launch_ranges(const uint64_t *keys, int64_t K, int64_t ntiles, uint32_t *ranges, hipStream_t s) {
    launch_fill_u32(ranges, 0u, 2 * ntiles, s);
    if (K == 0) return;
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, s, keys, K, ntiles, ranges);
}

}  // namespace a3fr
