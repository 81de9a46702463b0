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
// Both are LSD radix sorts with 8-bit digits whose blocks rank their keys
// stably inside each wave with 8 ballots (lanes sharing a digit) and a
// popcount of the lower lanes, and scatter them through LDS so that
// consecutive threads write consecutive addresses of each digit run.  They
// differ in how a partition learns where its digits start, chosen by size:
//  * the entry sort (a hundred or more 4096-key partitions): onesweep, one kernel
//    per digit after one histogram pass; a block takes the next partition id
//    from an atomic counter, publishes its digit counts and resolves its
//    offsets by decoupled look-back over the preceding partitions;
//  * the tile-id sort (a thousand and more 8192-key partitions): there the
//    look-back's chain of inclusive prefixes -- a device-coherent round trip
//    per window of predecessors, with every resident block waiting on it --
//    costs more than a second read of the keys, so each pass is reduce, then
//    scan, then scatter: a count kernel writes every partition's digit counts,
//    a scan kernel sums them by groups of partitions and its last block turns
//    the group sums into the start of every (group, digit), and the scatter
//    kernel adds the counts of the earlier partitions of its group
//    (independent loads, issued while its keys load).  No block waits for
//    another.  (Summing the groups with device-scope atomics in the count
//    kernel instead is several times slower than the scan kernel.)
// The key count is read from device memory, so every launch may be sized by
// an upper bound.
#include <algorithm>

#include "a3fr_internal.h"

namespace a3fr {

constexpr int kSortThreads = 512;
constexpr int kSortWaves = kSortThreads / kWave;      // 8
constexpr int kOsThreads = 1024;                      // the entry sort's blocks (16 waves: 4096-key partitions)
constexpr int kOsWaves = kOsThreads / kWave;
constexpr int kRadix = 256;
constexpr int kDigitWaves = kRadix / kWave;           // waves holding one digit per lane
constexpr int kMaxPasses = 4;                         // 32-bit keys
constexpr int kGroup = 32;                            // partitions per scan group (tile-id sort)
constexpr int kScanBatch = 64;                        // independent loads per round trip in the scan

static int sort_cus() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    return cus;
}

// ==========================================================================
// entry depth sort: onesweep
// ==========================================================================
static int onesweep_partitions(int64_t n, int items) {
    const int64_t part = (int64_t)kOsThreads * items;
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
        const int64_t parts = (n + (int64_t)kOsThreads * items - 1) / ((int64_t)kOsThreads * items);
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
__global__ void __launch_bounds__(kOsThreads) k_onesweep(const uint32_t *__restrict__ kin,
                                                           const uint32_t *__restrict__ vin,
                                                           uint32_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                           const uint32_t *n_dev, int shift,
                                                           const uint32_t *__restrict__ ghist, uint64_t *status,
                                                           uint32_t *counter, uint32_t *err) {
    constexpr int kSortPart = kOsThreads * kSortItems;
    __shared__ uint32_t s_part;
    __shared__ uint32_t s_wh[kOsWaves][kRadix];
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
        for (int j = tid; j < kOsWaves * kRadix; j += kOsThreads) (&s_wh[0][0])[j] = 0;
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
            uint32_t c[kOsWaves];
#pragma unroll
            for (int q = 0; q < kOsWaves; ++q) { c[q] = s_wh[q][d]; tot += c[q]; }
            st_status(&status[(int64_t)part * kRadix + d], (part == 0 ? kSt64Inc : kSt64Agg) | (uint64_t)tot);
            uint32_t run = 0;
#pragma unroll
            for (int q = 0; q < kOsWaves; ++q) { s_wh[q][d] = run; run += c[q]; }
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
        for (int j = tid; j < nvalid; j += kOsThreads) {
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
int64_t onesweep_workspace_words(int64_t n_max, int npass) {
    return onesweep_zero_words(npass) + 2 * (int64_t)npass * onesweep_partitions(n_max, kSortItemsSmall) * kRadix;
}

int64_t onesweep_zero_words(int npass) { return (int64_t)npass * kRadix + 8; }

void launch_onesweep_prepare(const uint32_t *keys, const uint32_t *n_dev, int64_t n_max, int npass, uint32_t *ws,
                             hipStream_t s, bool zeroed) {
    constexpr int items = kSortItemsSmall;
    const int nparts = onesweep_partitions(n_max, items);
    if (!zeroed) launch_fill_u32(ws, 0u, onesweep_zero_words(npass), s);
    if (nparts == 0) return;
    int hblocks = (int)((n_max + kHistThreads * 16 - 1) / (kHistThreads * 16));
    if (hblocks > 512) hblocks = 512;
    hipLaunchKernelGGL(k_sort_hist, dim3((unsigned)hblocks), dim3(kHistThreads), 0, s, keys, n_dev, npass, ws, items,
                       (int64_t)nparts);
}

void launch_onesweep_pass(const uint32_t *ki, const uint32_t *vi, uint32_t *ko, uint32_t *vo, const uint32_t *n_dev,
                          int64_t n_max, int npass, int p, uint32_t *ws, uint32_t *err, hipStream_t s) {
    constexpr int items = kSortItemsSmall;
    const int nparts = onesweep_partitions(n_max, items);
    if (nparts == 0) return;
    uint32_t *hist = ws, *ctr = ws + (int64_t)npass * kRadix;
    uint64_t *status = reinterpret_cast<uint64_t *>(ctr + 8);  // 8-byte aligned: npass x 1 KiB + 32 B in
    // persistent blocks: LDS per block ~52 KB
    const int resident = sort_cus();  // one 16-wave block per compute unit at its register count
    const int grid = nparts < resident ? nparts : resident;
    hipLaunchKernelGGL(k_onesweep<items>, dim3((unsigned)grid), dim3(kOsThreads), 0, s, ki, vi, ko, vo, n_dev,
                       8 * p, hist + (int64_t)p * kRadix, status + (int64_t)p * nparts * kRadix, ctr + p, err);
}


// ==========================================================================
// tile-id sort: count (with the scan in its last block), scatter
// ==========================================================================
static int64_t tile_sort_parts(int64_t n) { return (n + kSortThreads * kSortItemsLarge - 1) / (kSortThreads * kSortItemsLarge); }
static int64_t tile_sort_groups(int64_t parts) { return (parts + kGroup - 1) / kGroup; }

// workspace (u32 words): [tickets 8 | cnt parts x 256 | gsum groups x 256 | base groups x 256];
// the tickets start at zero and every pass leaves them so
int64_t sort_zero_words(int64_t /*n_max*/) { return 8; }
int64_t sort_workspace_words(int64_t n_max) {
    const int64_t parts = tile_sort_parts(n_max);
    return 8 + (parts + 2 * tile_sort_groups(parts)) * kRadix;
}

// ---- count -------------------------------------------------------------------
// Neighbouring keys often share a digit (tile ids of one Gaussian's rectangle,
// depths of one depth range), and LDS atomics of a wave on one address
// serialise: when every valid key of a wave's step has the same digit, one lane
// adds the count.
template <int I>
__global__ void __launch_bounds__(kSortThreads) k_sort_count(const uint32_t *__restrict__ keys,
                                                             const uint32_t *n_dev, int shift,
                                                             uint32_t *__restrict__ cnt) {
    constexpr int kPart = kSortThreads * I;
    static_assert(I % 4 == 0, "four keys per load");
    __shared__ uint32_t h[kSortWaves][kRadix];
    const int64_t K = *n_dev;
    const int64_t P = (K + kPart - 1) / kPart;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int64_t part = blockIdx.x; part < P; part += gridDim.x) {
        __syncthreads();  // the previous partition's totals are read
        for (int j = threadIdx.x; j < kSortWaves * kRadix; j += kSortThreads) (&h[0][0])[j] = 0;
        __syncthreads();
        const int64_t base = part * kPart;
#pragma unroll
        for (int it = 0; it < I / 4; ++it) {
            const int64_t j = base + ((int64_t)it * kSortThreads + threadIdx.x) * 4;
            uint4 k4 = {0u, 0u, 0u, 0u};
            if (j + 3 < K) {
                k4 = *reinterpret_cast<const uint4 *>(keys + j);
            } else {
                if (j < K) k4.x = keys[j];
                if (j + 1 < K) k4.y = keys[j + 1];
                if (j + 2 < K) k4.z = keys[j + 2];
            }
            const uint32_t kk[4] = {k4.x, k4.y, k4.z, k4.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool valid = j + q < K;
                const uint64_t vm = __ballot(valid);
                if (vm == 0) continue;  // wave-uniform
                const uint32_t d = (kk[q] >> shift) & 255u;
                const int first = __ffsll((unsigned long long)vm) - 1;
                const uint32_t d0 = __shfl(d, first, 64);
                const uint64_t same = __ballot(valid && d == d0);
                if (same == vm) {
                    if (lane == first) atomicAdd(&h[w][d0], (uint32_t)__popcll(vm));
                } else if (valid) {
                    atomicAdd(&h[w][d], 1u);
                }
            }
        }
        __syncthreads();
        for (int d = threadIdx.x; d < kRadix; d += kSortThreads) {
            uint32_t c = 0;
#pragma unroll
            for (int q = 0; q < kSortWaves; ++q) c += h[q][d];
            cnt[part * kRadix + d] = c;
        }
    }
}

// ---- scan --------------------------------------------------------------------
// Block g (256 threads, one per digit) of a grid of at least one block per
// group; every block takes a ticket, the last one writes
// base[g][d] = sum over digits d' < d of the totals + sum over groups g' < g of gsum[g'][d].
// The group sums pass between blocks through device-coherent stores and loads.
__global__ void __launch_bounds__(256) k_sort_scan(const uint32_t *__restrict__ cnt, const uint32_t *n_dev,
                                                   int part_keys, uint32_t *gsum, uint32_t *__restrict__ base,
                                                   uint32_t *ticket) {
    const int64_t K = *n_dev;
    const int64_t P = (K + part_keys - 1) / part_keys;
    const int64_t G = (P + kGroup - 1) / kGroup;
    const int d = threadIdx.x;
    for (int64_t g = blockIdx.x; g < G; g += gridDim.x) {
        uint32_t c[kGroup];
#pragma unroll
        for (int q = 0; q < kGroup; ++q) c[q] = cnt[min(g * kGroup + q, P - 1) * kRadix + d];
        uint32_t s = 0;
#pragma unroll
        for (int q = 0; q < kGroup; ++q) s += (g * kGroup + q < P) ? c[q] : 0u;
        __hip_atomic_store(&gsum[g * kRadix + d], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __threadfence();
    __shared__ uint32_t s_last;
    __syncthreads();
    if (d == 0)
        s_last = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
    __syncthreads();
    if (!s_last || G == 0) return;
    __threadfence();
    // totals of every digit, kScanBatch independent loads per round trip; the
    // last batch stays in v for the second pass (with G <= kScanBatch, the
    // usual case, the group sums are read once)
    uint32_t tot = 0;
    uint32_t v[kScanBatch];
    for (int64_t q0 = 0; q0 < G; q0 += kScanBatch) {
#pragma unroll
        for (int q = 0; q < kScanBatch; ++q)
            v[q] = __hip_atomic_load(&gsum[min(q0 + q, G - 1) * kRadix + d], __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
        for (int q = 0; q < kScanBatch; ++q) tot += (q0 + q < G) ? v[q] : 0u;
    }
    // exclusive scan over the digits
    __shared__ uint32_t s_ws[kDigitWaves];
    const int lane = d & 63, w = d >> 6;
    uint32_t inc = tot;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(inc, off, 64);
        if (lane >= off) inc += y;
    }
    if (lane == 63) s_ws[w] = inc;
    __syncthreads();
    uint32_t run = inc - tot;
    for (int q = 0; q < w; ++q) run += s_ws[q];
    for (int64_t q0 = 0; q0 < G; q0 += kScanBatch) {
        if (G > kScanBatch) {  // block-uniform: more than one batch, reloaded in order
#pragma unroll
            for (int q = 0; q < kScanBatch; ++q)
                v[q] = __hip_atomic_load(&gsum[min(q0 + q, G - 1) * kRadix + d], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
        }
#pragma unroll
        for (int q = 0; q < kScanBatch; ++q)
            if (q0 + q < G) {
                base[(q0 + q) * kRadix + d] = run;
                run += v[q];
            }
    }
    if (d == 0) *ticket = 0u;  // every block has taken its ticket: ready for the next use
}

// ---- scatter -----------------------------------------------------------------
// at least 4 waves per SIMD (<= 128 VGPRs): two 8-wave blocks per compute unit
template <int I>
__global__ void __launch_bounds__(kSortThreads, 4) k_sort_scatter(const uint32_t *__restrict__ kin,
                                                                  const uint32_t *__restrict__ vin,
                                                                  uint32_t *__restrict__ kout,
                                                                  uint32_t *__restrict__ vout, const uint32_t *n_dev,
                                                                  int shift, const uint32_t *__restrict__ cnt,
                                                                  const uint32_t *__restrict__ base) {
    constexpr int kPart = kSortThreads * I;
    __shared__ uint32_t s_wh[kSortWaves][kRadix];
    __shared__ uint32_t s_lstart[kRadix];
    __shared__ uint32_t s_gbase[kRadix];
    __shared__ uint32_t s_wsum[kDigitWaves];
    __shared__ uint32_t s_k[kPart];
    __shared__ uint32_t s_v[kPart];
    const uint32_t K = *n_dev;
    const int P = (int)(((int64_t)K + kPart - 1) / kPart);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int part = blockIdx.x; part < P; part += gridDim.x) {
        __syncthreads();  // the previous partition is done with the LDS
        for (int j = tid; j < kSortWaves * kRadix; j += kSortThreads) (&s_wh[0][0])[j] = 0;
        // positions in 32 bits: b0 + l for a local index l < rem = K - b0 (no overflow near 2^32 keys)
        const uint32_t b0 = (uint32_t)part * kPart, rem = K - b0;
        // global start of this partition's digits: its group's start plus the
        // earlier partitions of the group (independent of the keys)
        if (tid < kRadix) {
            const int p0 = part / kGroup * kGroup;
            uint32_t c[kGroup];
#pragma unroll
            for (int q = 0; q < kGroup; ++q) c[q] = cnt[(int64_t)min(p0 + q, part) * kRadix + tid];
            uint32_t o = base[(int64_t)(part / kGroup) * kRadix + tid];
#pragma unroll
            for (int q = 0; q < kGroup; ++q) o += (p0 + q < part) ? c[q] : 0u;
            s_gbase[tid] = o;
        }
        const uint32_t l0 = (uint32_t)(w * (I * kWave) + lane);  // local index of item 0; item it adds it x 64
        uint32_t key[I], rk[I], val[I];
#pragma unroll
        for (int it = 0; it < I; ++it) key[it] = l0 + it * kWave < rem ? kin[b0 + l0 + it * kWave] : 0u;
        __syncthreads();
        // stable rank inside each wave: lanes with the same digit, then the
        // wave's running count of that digit
#pragma unroll
        for (int it = 0; it < I; ++it) {
            const bool valid = l0 + it * kWave < rem;
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
        // the values are loaded now: their round trip overlaps the digit
        // bookkeeping, and they are not live during the ranking
#pragma unroll
        for (int it = 0; it < I; ++it) val[it] = l0 + it * kWave < rem ? vin[b0 + l0 + it * kWave] : 0u;
        __syncthreads();
        // threads 0..255 = digits: per-wave exclusive offsets, block-local digit starts
        if (tid < kRadix) {
            const int d = tid;
            uint32_t c[kSortWaves], tot = 0;
#pragma unroll
            for (int q = 0; q < kSortWaves; ++q) { c[q] = s_wh[q][d]; tot += c[q]; }
            uint32_t run = 0;
#pragma unroll
            for (int q = 0; q < kSortWaves; ++q) { s_wh[q][d] = run; run += c[q]; }
            uint32_t inc = tot;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t y = __shfl_up(inc, off, 64);
                if (lane >= off) inc += y;
            }
            if (lane == 63) s_wsum[w] = inc;
            s_lstart[d] = inc - tot;
        }
        __syncthreads();
        if (tid < kRadix) {
            uint32_t pre = 0;
#pragma unroll
            for (int q = 0; q < kDigitWaves; ++q) if (q < w) pre += s_wsum[q];
            s_lstart[tid] += pre;
            s_gbase[tid] -= s_lstart[tid];  // global position = s_gbase[d] + local position (mod 2^32)
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < I; ++it) {
            if (l0 + it * kWave < rem) {
                const uint32_t dg = (key[it] >> shift) & 255u;
                const uint32_t lp = s_lstart[dg] + s_wh[w][dg] + rk[it];
                s_k[lp] = key[it];
                s_v[lp] = val[it];
            }
        }
        __syncthreads();
        const int nvalid = rem < (uint32_t)kPart ? (int)rem : kPart;
        for (int j = tid; j < nvalid; j += kSortThreads) {
            const uint32_t kk = s_k[j];
            const uint32_t g = s_gbase[(kk >> shift) & 255u] + (uint32_t)j;
            if (g < K) {
                kout[g] = kk;
                vout[g] = s_v[j];
            }
        }
    }
}

void launch_sort_count(const uint32_t *ki, const uint32_t *n_dev, int64_t n_max, int p, uint32_t *ws, hipStream_t s) {
    const int64_t parts = tile_sort_parts(n_max);
    if (parts == 0) return;
    const int64_t groups = tile_sort_groups(parts);
    uint32_t *cnt = ws + 8, *gsum = cnt + parts * kRadix, *base = gsum + groups * kRadix;
    const int grid = (int)std::min<int64_t>(parts, 16 * sort_cus());
    hipLaunchKernelGGL(k_sort_count<kSortItemsLarge>, dim3(grid), dim3(kSortThreads), 0, s, ki, n_dev, 8 * p, cnt);
    const int sgrid = (int)std::min<int64_t>(groups, 4096);
    hipLaunchKernelGGL(k_sort_scan, dim3(sgrid), dim3(kRadix), 0, s, cnt, n_dev, kSortThreads * kSortItemsLarge, gsum,
                       base, ws + p);
}

void launch_sort_scatter(const uint32_t *ki, const uint32_t *vi, uint32_t *ko, uint32_t *vo, const uint32_t *n_dev,
                         int64_t n_max, int p, const uint32_t *ws, hipStream_t s) {
    const int64_t parts = tile_sort_parts(n_max);
    if (parts == 0) return;
    const int64_t groups = tile_sort_groups(parts);
    const uint32_t *cnt = ws + 8, *base = cnt + (parts + groups) * kRadix;
    const int grid = (int)std::min<int64_t>(parts, 16 * sort_cus());
    hipLaunchKernelGGL(k_sort_scatter<kSortItemsLarge>, dim3(grid), dim3(kSortThreads), 0, s, ki, vi, ko, vo, n_dev,
                       8 * p, cnt, base);
}

// ------------------------------------------------------------------------
// tile ranges from the sorted tile ids
// ------------------------------------------------------------------------
// One thread per tile: its range [start, end) in the sorted tile ids by two
// binary searches (lower bounds of t and t + 1); an empty tile gets (0, 0).
// Threads of a wave search neighbouring tiles, so the upper levels of the
// searches hit the same cache lines.

// Lower bounds of v0 and v1 in the sorted a[0, n), n >= 1, found together so
// that their two chains of dependent loads overlap.  Branch-free halving: the
// lower bound stays in [b, b + len] (everything before b is below the value),
// and the steps depend only on n, the same for every lane.
__device__ __forceinline__ void lower_bounds2_u32(const uint32_t *__restrict__ a, uint32_t n, uint32_t v0,
                                                  uint32_t v1, uint32_t &r0, uint32_t &r1) {
    uint32_t b0 = 0, b1 = 0, len = n;
    while (len > 1) {
        const uint32_t half = len >> 1;
        const uint32_t x0 = a[b0 + half - 1], x1 = a[b1 + half - 1];
        b0 += x0 < v0 ? half : 0u;
        b1 += x1 < v1 ? half : 0u;
        len -= half;
    }
    r0 = b0 + (a[b0] < v0 ? 1u : 0u);
    r1 = b1 + (a[b1] < v1 ? 1u : 0u);
}

__global__ void __launch_bounds__(256) k_ranges(const uint32_t *__restrict__ tiles, int64_t K, const uint32_t *K_dev,
                                                int64_t ntiles, uint32_t *__restrict__ ranges) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    if (K_dev && (int64_t)*K_dev < K) K = *K_dev;  // capacity mode
    const uint32_t n = (uint32_t)K;
    uint32_t s0 = 0, s1 = 0;
    if (n > 0) lower_bounds2_u32(tiles, n, (uint32_t)t, (uint32_t)t + 1u, s0, s1);
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
