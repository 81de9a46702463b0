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
// Selection key of visible Gaussian i: the 96-bit (score bits, ~i) -- score
// descending, index ascending.  Scores are non-negative doubles, so their bit
// patterns order like the values and bit 63 is 0.
//   1. two histogram levels of 12 bits each (score bits 62..51, then 50..39 of
//      the Gaussians in the chosen level-1 bucket), per block in LDS; the
//      blocks of the next kernel each pick the bucket holding the k-th largest
//      key from it;
//   2. every visible Gaussian outside the chosen 24-bit bucket is decided at
//      once, those inside are listed as candidates (usually a handful);
//   3. one block per view runs an MSD radix select over the candidates'
//      remaining 71 key bits (score bits 38..0, ~index) and marks the kept ones.
constexpr int kSelBits = 12;
constexpr int kSelBuckets = 1 << kSelBits;
constexpr int kSelLow = 63 - 2 * kSelBits;      // 39 score bits below the two levels
constexpr int kSelKeyBits = kSelLow + 32;       // candidate key bits
constexpr int kSelDigits = (kSelKeyBits + 7) / 8;

struct SelState {
    uint32_t n_vis, k, k_rem, mode;  // mode 0: select, 1: keep all visible, 2: keep none
    uint32_t b0, b1, ncand, pad;     // chosen level buckets
};

__device__ __forceinline__ uint32_t sel_level(uint64_t bits, int level) {
    return (uint32_t)(bits >> (63 - kSelBits * (level + 1))) & (uint32_t)(kSelBuckets - 1);
}

// The bucket of one level holding the k-th largest key, found by a whole
// block of 256 threads: thread t owns kSelBuckets/256 consecutive buckets,
// the highest first.  Every block of the kernel that needs it repeats this
// (16 KB of histogram from L2) instead of a separate one-block launch.
// k: ceil(keep_num x total / keep_den) for the first level (total = visible
// count), else k_fixed.  out->bucket and out->krem are set when 0 < k <= total.
struct PickOut {
    uint32_t total, k, bucket, krem;
};
__device__ void pick_bucket(const uint32_t *h, bool first_level, uint32_t k_fixed, int keep_num, int keep_den,
                            PickOut *out) {
    constexpr int kPer = kSelBuckets / 256;
    __shared__ uint32_t wsum[4];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int hi = kSelBuckets - kPer * t;
    uint32_t c[kPer];
    uint32_t loc = 0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        c[q] = h[hi - 1 - q];
        loc += c[q];
    }
    uint32_t inc = loc;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(inc, off, 64);
        if (lane >= off) inc += y;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (q < w) pre += wsum[q];
        tot += wsum[q];
    }
    const uint64_t k = first_level ? ((uint64_t)keep_num * tot + (uint64_t)keep_den - 1) / (uint64_t)keep_den
                                   : (uint64_t)k_fixed;
    if (t == 0) {
        out->total = tot;
        out->k = (uint32_t)k;
    }
    uint32_t above = pre + inc - loc;
    if (k > 0 && above < k && above + loc >= k) {
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            if (above + c[q] >= k) {
                out->bucket = (uint32_t)(hi - 1 - q);
                out->krem = (uint32_t)(k - above);
                break;
            }
            above += c[q];
        }
    }
    __syncthreads();
}

// First-level decision of a view from its level-0 histogram: mode 0 select,
// 1 keep every visible Gaussian, 2 keep none.
__device__ __forceinline__ uint32_t pick_mode(const PickOut &p) {
    return p.k == 0 ? 2u : (p.k >= p.total ? 1u : 0u);
}

// Adds one to bucket d of the wave's lanes with valid set: lanes sharing the
// first valid lane's bucket (often most of them: scores of similar size share
// their top bits) add with a single LDS atomic.
__device__ __forceinline__ void sel_count(uint32_t *lh, uint32_t d, bool valid) {
    const uint64_t vm = __ballot(valid);
    if (vm == 0) return;
    const int lane = threadIdx.x & 63;
    const int first = __ffsll((unsigned long long)vm) - 1;
    const uint32_t d0 = __shfl(d, first, 64);
    const uint64_t same = __ballot(valid && d == d0);
    if (lane == first) atomicAdd(&lh[d0], (uint32_t)__popcll(same));
    if (valid && d != d0) atomicAdd(&lh[d], 1u);
}

constexpr int kSelUnroll = 8;
// Level histograms; a level-1 block first takes the level-0 decision (block
// 0 of the view stores it in the state for the later kernels).
__global__ void __launch_bounds__(256) k_sel_hist(const int32_t *sel_views, const uint32_t *__restrict__ counts,
                                                  const double *__restrict__ score, int64_t n, int level,
                                                  SelState *st, uint32_t *hist, int keep_num, int keep_den) {
    const int slot = blockIdx.y;
    __shared__ uint32_t lh[kSelBuckets];
    __shared__ PickOut p0;
    uint32_t b0 = 0;
    if (level > 0) {
        pick_bucket(hist + (int64_t)slot * 2 * kSelBuckets, true, 0u, keep_num, keep_den, &p0);
        const uint32_t mode = pick_mode(p0);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            SelState &S = st[slot];
            S.n_vis = p0.total;
            S.k = p0.k;
            S.mode = mode;
            S.ncand = 0;
            S.b0 = p0.bucket;
            S.k_rem = p0.krem;
        }
        if (mode != 0) return;  // block-uniform
        b0 = p0.bucket;
    }
    for (int b = threadIdx.x; b < kSelBuckets; b += blockDim.x) lh[b] = 0;
    __syncthreads();
    const int64_t base = (int64_t)sel_views[slot] * n, sbase = (int64_t)slot * n;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // block-uniform trip count (the ballots need whole waves); the step's
    // loads are unconditional (indices past n read the last Gaussian and are
    // dropped), so that they issue together and are waited for once
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < n; i0 += kSelUnroll * stride) {
        uint32_t cv[kSelUnroll];
        uint64_t bits[kSelUnroll];
#pragma unroll
        for (int u = 0; u < kSelUnroll; ++u) {
            const int64_t i = i0 + u * stride + threadIdx.x, ic = i < n ? i : n - 1;
            cv[u] = counts[base + ic];
            bits[u] = (uint64_t)__double_as_longlong(score[sbase + ic]);
        }
#pragma unroll
        for (int u = 0; u < kSelUnroll; ++u) {
            const int64_t i = i0 + u * stride + threadIdx.x;
            const bool valid = i < n && cv[u] != 0 && (level == 0 || sel_level(bits[u], 0) == b0);
            sel_count(lh, sel_level(bits[u], level), valid);
        }
    }
    __syncthreads();
    uint32_t *h = hist + ((int64_t)slot * 2 + level) * kSelBuckets;
    for (int b = threadIdx.x; b < kSelBuckets; b += blockDim.x)
        if (lh[b]) atomicAdd(&h[b], lh[b]);
}

// Decides every visible Gaussian outside the chosen 24-bit bucket and lists
// those inside as candidates; every block takes both level decisions from the
// histograms (block 0 of the view stores the second in the state).
__global__ void __launch_bounds__(256) k_sel_gather(const int32_t *sel_views, const uint32_t *__restrict__ counts,
                                                    const double *__restrict__ score, int64_t n, SelState *st,
                                                    const uint32_t *hist, int keep_num, int keep_den,
                                                    uint64_t *cand_key, uint32_t *cand_idx, uint8_t *keep) {
    const int slot = blockIdx.y;
    const int64_t base = (int64_t)sel_views[slot] * n, sbase = (int64_t)slot * n;
    __shared__ PickOut p0, p1;
    pick_bucket(hist + (int64_t)slot * 2 * kSelBuckets, true, 0u, keep_num, keep_den, &p0);
    const uint32_t mode = pick_mode(p0);
    uint32_t top = 0;  // chosen 24-bit prefix
    if (mode == 0) {
        pick_bucket(hist + ((int64_t)slot * 2 + 1) * kSelBuckets, false, p0.krem, keep_num, keep_den, &p1);
        top = (p0.bucket << kSelBits) | p1.bucket;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st[slot].b1 = p1.bucket;
            st[slot].k_rem = p1.krem;
        }
    }
    const int lane = threadIdx.x & 63;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // block-uniform trip count; each step's loads are unconditional (indices
    // past n read the last Gaussian and are dropped), issued together
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < n; i0 += kSelUnroll * stride) {
        uint32_t cv[kSelUnroll];
        uint64_t bits[kSelUnroll];
#pragma unroll
        for (int u = 0; u < kSelUnroll; ++u) {
            const int64_t i = i0 + u * stride + threadIdx.x, ic = i < n ? i : n - 1;
            cv[u] = counts[base + ic];
            bits[u] = (uint64_t)__double_as_longlong(score[sbase + ic]);
        }
#pragma unroll
        for (int u = 0; u < kSelUnroll; ++u) {
            const int64_t i = i0 + u * stride + threadIdx.x;
            uint8_t kp = 0;
            bool cand = false;
            if (i < n && cv[u] != 0) {
                if (mode == 1) {
                    kp = 1;
                } else if (mode == 0) {
                    const uint32_t tb = (uint32_t)(bits[u] >> kSelLow);
                    kp = tb > top ? 1 : 0;
                    cand = tb == top;
                }
            }
            const uint64_t m = __ballot(cand);  // one atomic per wave for its candidates
            if (m) {
                uint32_t first = 0;
                const int leader = __ffsll((unsigned long long)m) - 1;
                if (lane == leader) first = atomicAdd(&st[slot].ncand, (uint32_t)__popcll(m));
                first = __shfl(first, leader, 64);
                if (cand) {
                    const uint32_t c = first + (uint32_t)__popcll(m & lt);
                    cand_key[(int64_t)slot * n + c] = bits[u] & ((1ull << kSelLow) - 1);
                    cand_idx[(int64_t)slot * n + c] = (uint32_t)i;
                }
            }
            if (i < n) keep[base + i] = kp;
        }
    }
}

constexpr uint32_t kSelDirect = 1024;  // candidates ranked by direct comparison (one block)

// Candidate key (score low bits, ~index) as a 128-bit integer: larger is kept first.
__device__ __forceinline__ unsigned __int128 sel_ckey(uint64_t lo, uint32_t idx) {
    return ((unsigned __int128)lo << 32) | (unsigned __int128)(~idx);
}

__global__ void __launch_bounds__(1024) k_sel_final(const int32_t *sel_views, int64_t n, const SelState *st,
                                                    const uint64_t *cand_key, const uint32_t *cand_idx,
                                                    uint8_t *keep) {
    const int slot = blockIdx.x, t = threadIdx.x;
    if (st[slot].mode != 0) return;
    const uint32_t nc = st[slot].ncand;
    const uint64_t *ck = cand_key + (int64_t)slot * n;
    const uint32_t *ci = cand_idx + (int64_t)slot * n;
    const int64_t base = (int64_t)sel_views[slot] * n;
    __shared__ uint32_t hist[256];
    __shared__ uint32_t s_krem, s_done, s_np;
    __shared__ unsigned long long s_pre_hi, s_pre_lo;  // chosen key prefix (digits so far), 128-bit
    if (nc <= kSelDirect) {
        // few candidates (the usual case): each is kept iff fewer than k_rem
        // candidates have a larger key (keys are unique), one comparison pass in LDS
        __shared__ uint64_t s_ck[kSelDirect];
        __shared__ uint32_t s_ci[kSelDirect];
        for (uint32_t c = t; c < nc; c += blockDim.x) { s_ck[c] = ck[c]; s_ci[c] = ci[c]; }
        __syncthreads();
        const uint32_t krem = st[slot].k_rem;
        for (uint32_t c = t; c < nc; c += blockDim.x) {
            const unsigned __int128 key = sel_ckey(s_ck[c], s_ci[c]);
            uint32_t above = 0;
            for (uint32_t d = 0; d < nc; ++d) above += sel_ckey(s_ck[d], s_ci[d]) > key ? 1u : 0u;
            keep[base + s_ci[c]] = above < krem ? 1 : 0;
        }
        return;
    }
    if (t == 0) { s_krem = st[slot].k_rem; s_done = 0; s_np = 0; s_pre_hi = 0; s_pre_lo = 0; }
    __syncthreads();
    for (int p = 0; p < kSelDigits; ++p) {
        const int sh = kSelDigits * 8 - 8 * (p + 1);  // shift of digit p in the zero-padded key
        if (t < 256) hist[t] = 0;
        __syncthreads();
        const unsigned __int128 pre = ((unsigned __int128)s_pre_hi << 64) | s_pre_lo;
        for (uint32_t c = t; c < nc; c += blockDim.x) {
            const unsigned __int128 key = sel_ckey(ck[c], ci[c]) << (kSelDigits * 8 - kSelKeyBits);
            if (p == 0 || (key >> (sh + 8)) == pre) atomicAdd(&hist[(uint32_t)(key >> sh) & 255u], 1u);
        }
        __syncthreads();
        if (t == 0) {
            uint32_t above = 0;
            const uint32_t kr = s_krem;
            for (int d = 255; d >= 0; --d) {
                const uint32_t c = hist[d];
                if (above + c >= kr) {
                    const unsigned __int128 np = (pre << 8) | (unsigned __int128)d;
                    s_pre_hi = (unsigned long long)(np >> 64);
                    s_pre_lo = (unsigned long long)np;
                    s_krem = kr - above;
                    s_np = (uint32_t)p + 1;
                    if (c == kr - above) s_done = 1;
                    break;
                }
                above += c;
            }
        }
        __syncthreads();
        if (s_done) break;
    }
    // kept: candidates whose key prefix (s_np digits) is >= the chosen prefix
    const int sh = kSelDigits * 8 - 8 * (int)s_np;
    const unsigned __int128 pre = ((unsigned __int128)s_pre_hi << 64) | s_pre_lo;
    for (uint32_t c = t; c < nc; c += blockDim.x) {
        const unsigned __int128 key = sel_ckey(ck[c], ci[c]) << (kSelDigits * 8 - kSelKeyBits);
        keep[base + ci[c]] = (key >> sh) >= pre ? 1 : 0;
    }
}

void launch_select(const DevView *views, int nv, const int32_t *sel_views, int nsel, int64_t n,
                   const uint32_t *counts, const double *score, int keep_num, int keep_den,
                   uint32_t *sel_ws, uint8_t *keep, hipStream_t s, bool zeroed) {
    (void)views; (void)nv;
    if (nsel == 0 || n == 0) return;
    // workspace: hist [nsel][2][4096] u32 | state [nsel] (8 words) | cand_key [nsel][n] u64 | cand_idx [nsel][n] u32
    uint32_t *hist = sel_ws;
    SelState *st = reinterpret_cast<SelState *>(sel_ws + (int64_t)nsel * 2 * kSelBuckets);
    uint64_t *ck = reinterpret_cast<uint64_t *>(sel_ws + (int64_t)nsel * 2 * kSelBuckets + (int64_t)nsel * 8);
    uint32_t *ci = reinterpret_cast<uint32_t *>(ck + (int64_t)nsel * n);
    if (!zeroed) launch_fill_u32(hist, 0u, select_hist_words(nsel), s);
    int64_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    const unsigned hb = (unsigned)(blocks < 256 ? blocks : 256);
    for (int level = 0; level < 2; ++level)
        hipLaunchKernelGGL(k_sel_hist, dim3(hb, (unsigned)nsel), dim3(256), 0, s, sel_views, counts, score, n, level, st,
                           hist, keep_num, keep_den);
    hipLaunchKernelGGL(k_sel_gather, dim3(hb, (unsigned)nsel), dim3(256), 0, s, sel_views, counts, score, n, st, hist,
                       keep_num, keep_den, ck, ci, keep);
    hipLaunchKernelGGL(k_sel_final, dim3((unsigned)nsel), dim3(1024), 0, s, sel_views, n, st, ck, ci, keep);
}

// words of the level histograms at the start of the select workspace (cleared before each select)
int64_t select_hist_words(int nsel) { return (int64_t)nsel * 2 * kSelBuckets; }

// words of select workspace (hist, state, candidates) for nsel views of n Gaussians
int64_t select_workspace_words(int nsel, int64_t n) {
    return (int64_t)nsel * 2 * kSelBuckets + (int64_t)nsel * 8 + (int64_t)nsel * n * 3 + 4;
}

// ------------------------------------------------------------------------
// scans: compaction of the visible entries, then key offsets in depth order
// ------------------------------------------------------------------------
constexpr int kScanItems = 16;
constexpr int kScanBlock = 128;
constexpr int kScanTile = kScanItems * kScanBlock;  // 2048 entries per block (key offsets)
// the compaction's partitions: 12 waves of 1024 slots (two blocks per CU at
// its register count, so that a stereo frame of a million Gaussians, 6M slots,
// is in flight at once; fewer, larger partitions take fewer tickets, which
// are serialised on one device-coherent counter)
constexpr int kCompactItems = 16;
constexpr int kCompactBlock = 768;
constexpr int kCompactTile = kCompactItems * kCompactBlock;

// Slot e = view * n + index is an entry iff it has keys (a count) and, in a
// selecting view, is kept; in a view with keep_visible, iff its rectangle
// (kept for that view) is not empty, keys or not.
struct EntryFlags {
    const uint32_t *counts;
    const uint8_t *keep;
    const uint64_t *rect;
    const DevView *views;
    int64_t n;
};

// Key counts of the entries in depth order: the j-th is ecnt[order[j]]
// (order: entry indices sorted by depth; ecnt: the entries' key counts in
// entry order, written by the compaction, so that the gather reads a compact
// array rather than the slots).
struct SortedCounts {
    const uint32_t *ecnt;
    const uint32_t *order;
    const uint32_t *n_ent;
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

// Single-pass scans with decoupled look-back (lookback_prefix).  Each block
// takes its partition (consecutive items) from a ticket counter, so a
// partition's predecessors are already held by running blocks (or done).
// Status words are 64-bit: flag in the top two bits, value in the low 62,
// zeroed before the launch.  Workspace (uint64): [0] compaction ticket, [1]
// offsets ticket, then the compaction partitions' words, then the offsets
// partitions' words.
constexpr uint64_t kStAgg = 1ull << 62, kStInc = 2ull << 62, kStVal = (1ull << 62) - 1;
constexpr uint32_t kPrefixSpins = 1u << 22;  // bound on a wait (never expected: a report, not a hang)

__device__ __forceinline__ uint64_t ld_st64(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_st64(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t wave_sum64(uint64_t x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// Called by all 64 lanes of one wave of the block: the exclusive prefix of
// partition part, whose own total is tot.  It publishes the total (flag AGG;
// partition 0 publishes its inclusive prefix at once), then walks back over
// the predecessors' words, the nearest first, kPrefixWindows windows of 64
// per round of device-coherent loads, adding totals until it meets an
// inclusive prefix (flag INC), and publishes its own inclusive prefix.  So a
// block reads a few windows however many partitions precede it (a sum of
// every predecessor's total instead costs a read per predecessor and block:
// 20% slower on 64 frames of 3M Gaussians, 94k partitions).  One window per
// round trip measured as fast as two and eight on a frame's 489 partitions.
constexpr int kPrefixWindows = 1;
__device__ uint64_t lookback_prefix(uint64_t *status, int64_t part, uint64_t tot, uint32_t *err) {
    const int lane = threadIdx.x & 63;
    if (lane == 0) st_st64(&status[part], (part == 0 ? kStInc : kStAgg) | tot);
    uint64_t excl = 0;
    uint32_t spins = 0;
    bool done = part == 0;
    for (int64_t top = part - 1; !done; top -= kPrefixWindows * 64) {
        uint64_t st[kPrefixWindows];
#pragma unroll
        for (int u = 0; u < kPrefixWindows; ++u) {
            const int64_t q = top - u * 64 - lane;
            st[u] = q >= 0 ? ld_st64(&status[q]) : kStInc;  // below partition 0: an inclusive prefix of 0
        }
#pragma unroll
        for (int u = 0; u < kPrefixWindows; ++u) {
            if (done) break;  // wave-uniform
            const int64_t q = top - u * 64 - lane;
            while (__ballot((st[u] >> 62) == 0) != 0) {
                if (++spins > kPrefixSpins) {
                    if (lane == 0) atomicOr(err, 1u);
                    st[u] = (st[u] >> 62) == 0 ? kStInc : st[u];
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                if ((st[u] >> 62) == 0) st[u] = ld_st64(&status[q]);
            }
            const uint64_t inc = __ballot((st[u] >> 62) == 2);
            if (inc) {
                const int first = __ffsll((unsigned long long)inc) - 1;  // the nearest inclusive prefix
                excl += wave_sum64(lane <= first ? (st[u] & kStVal) : 0ull);
                done = true;
            } else {
                excl += wave_sum64(st[u] & kStVal);
            }
        }
    }
    if (lane == 0 && part > 0) st_st64(&status[part], kStInc | (excl + tot));
    return excl;
}

// Barrier of the block that orders its LDS accesses only: global loads in
// flight stay in flight across it (a plain __syncthreads waits for them).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Loads of slots e0 + 64 r, r < kCompactItems, issued back to back and waited
// for once (a load under a branch is waited for before the branch's other side
// writes its register, so there is none): the counts and, where keep is given
// (it then holds a byte for every slot), the keep bytes; the depths.  kClamp:
// indices past the last slot read the last slot (the caller drops them).
template <bool kClamp>
__device__ __forceinline__ void compact_loads(const EntryFlags &f, int64_t e0, int64_t m, uint32_t (&cv)[kCompactItems],
                                              uint8_t (&kv)[kCompactItems]) {
#pragma unroll
    for (int r = 0; r < kCompactItems; ++r) {
        const int64_t e = e0 + r * 64;
        cv[r] = f.counts[kClamp && e >= m ? m - 1 : e];
    }
    if (f.keep) {
#pragma unroll
        for (int r = 0; r < kCompactItems; ++r) {
            const int64_t e = e0 + r * 64;
            kv[r] = f.keep[kClamp && e >= m ? m - 1 : e];
        }
    }
}
template <bool kClamp>
__device__ __forceinline__ void depth_loads(const uint32_t *__restrict__ depth, int64_t e0, int64_t m,
                                            uint32_t (&dv)[kCompactItems]) {
#pragma unroll
    for (int r = 0; r < kCompactItems; ++r) {
        const int64_t e = e0 + r * 64;
        dv[r] = depth[kClamp && e >= m ? m - 1 : e];
    }
}

// Compaction: slot e with flag 1 becomes entry j (its exclusive prefix):
// ent[j] = e, with its depth bits as sort key dkey[j] and j itself as sort
// value dval[j].  Each wave takes 1024 consecutive slots in 16 rounds of 64
// (coalesced), packing the flagged ones with a ballot per round; the waves of
// a block are combined in LDS and the blocks by the look-back.  The
// loads are few round trips: the views' flags, the counts and the keep bytes
// together; the depths (read for every slot and dropped where there is no
// entry: the entries are spread over most cache lines of the array anyway)
// issued before the prefix and in flight while it is formed; only the
// rectangles of keep_visible views wait for the counts.  keep: NULL when no
// view selects.
__global__ void __launch_bounds__(kCompactBlock) k_compact(EntryFlags f, int64_t m, int64_t nb, uint64_t *ws,
                                                        const uint32_t *__restrict__ depth, uint32_t *__restrict__ ent,
                                                        uint32_t *__restrict__ dkey, uint32_t *__restrict__ dval,
                                                        uint32_t *__restrict__ ecnt, uint64_t *total,
                                                        uint32_t *total32, uint32_t *err) {
    __shared__ uint32_t s_part;
    __shared__ uint64_t s_w[kCompactBlock / 64];
    __shared__ uint64_t s_excl;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x == 0) s_part = atomicAdd(reinterpret_cast<uint32_t *>(&ws[0]), 1u);
    __syncthreads();
    const int64_t part = s_part;
    const int64_t wbase = part * kCompactTile + (int64_t)w * 64 * kCompactItems;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const bool full = wbase + 64 * kCompactItems <= m;  // wave-uniform: no slot past the last
    // views of the block's slots: at most two when n >= kCompactTile
    const bool per_elem = f.n < kCompactTile;
    const int64_t v0 = (part * kCompactTile) / f.n, b1 = (v0 + 1) * f.n;
    const int64_t v1 = b1 < m ? v0 + 1 : v0;
    uint32_t cv[kCompactItems];
    uint8_t kv[kCompactItems];
    if (full)
        compact_loads<false>(f, wbase + lane, m, cv, kv);
    else
        compact_loads<true>(f, wbase + lane, m, cv, kv);
    const int32_t s0 = f.views[v0].v.select, s1 = f.views[v1].v.select;
    const int32_t k0 = f.views[v0].keep_visible, k1 = f.views[v1].keep_visible;
    const bool sel0 = f.keep && s0 != 0, sel1 = f.keep && b1 < m && s1 != 0;
    // keep_visible views count as such only when the rectangles are given
    const bool vis0 = f.rect && k0 != 0, vis1 = f.rect && b1 < m && k1 != 0;
    if (per_elem) {
#pragma unroll
        for (int r = 0; r < kCompactItems; ++r) {
            const int64_t e = wbase + r * 64 + lane;
            if (e >= m) cv[r] = 0;
            else if (cv[r] != 0 && f.keep && f.views[e / f.n].v.select != 0 && kv[r] == 0) cv[r] = 0;
        }
    } else {
#pragma unroll
        for (int r = 0; r < kCompactItems; ++r) {
            const int64_t e = wbase + r * 64 + lane;
            if (e >= m || ((e < b1 ? sel0 : sel1) && kv[r] == 0)) cv[r] = 0;
        }
    }
    // every visible slot of a keep_visible view is an entry, keys or not (bit r of vbits)
    uint32_t vbits = 0u;
    if (f.rect && (per_elem || vis0 || vis1)) {
        bool vv[kCompactItems];
#pragma unroll
        for (int r = 0; r < kCompactItems; ++r) {
            const int64_t e = wbase + r * 64 + lane;
            vv[r] = false;
            if (e < m && cv[r] == 0) {
                const int64_t v = per_elem ? e / f.n : (e < b1 ? v0 : v0 + 1);
                const DevView &dvw = f.views[v];
                if (dvw.keep_visible && dvw.rect_slot >= 0 &&
                    f.rect[(int64_t)dvw.rect_slot * f.n + (e - v * f.n)] != kEmptyRect)
                    vv[r] = true;
            }
        }
#pragma unroll
        for (int r = 0; r < kCompactItems; ++r) vbits |= (uint32_t)vv[r] << r;
    }
    uint32_t cnt = 0;
#pragma unroll
    for (int r = 0; r < kCompactItems; ++r) cnt += (uint32_t)__popcll(__ballot(cv[r] != 0 || ((vbits >> r) & 1u)));
    if (lane == 0) s_w[w] = cnt;
    uint32_t dv[kCompactItems];
    if (full)
        depth_loads<false>(depth, wbase + lane, m, dv);
    else
        depth_loads<true>(depth, wbase + lane, m, dv);
    lds_barrier();  // the depths stay in flight while the prefix is formed
    if (w == 0) {
        uint64_t tot = 0;
#pragma unroll
        for (int q = 0; q < kCompactBlock / 64; ++q) tot += s_w[q];
        const uint64_t excl = lookback_prefix(ws + 2, part, tot, err);
        if (lane == 0) {
            s_excl = excl;
            if (part == nb - 1) {
                *total = excl + tot;
                *total32 = excl + tot > 0xffffffffull ? 0xffffffffu : (uint32_t)(excl + tot);
            }
        }
    }
    lds_barrier();
    uint64_t run = s_excl;
    for (int q = 0; q < w; ++q) run += s_w[q];
#pragma unroll
    for (int r = 0; r < kCompactItems; ++r) {
        const bool flag = cv[r] != 0 || ((vbits >> r) & 1u);
        const uint64_t mk = __ballot(flag);
        if (flag) {
            const uint64_t pos = run + (uint64_t)__popcll(mk & lt);
            ent[pos] = (uint32_t)(wbase + r * 64 + lane);
            dkey[pos] = dv[r];
            dval[pos] = (uint32_t)pos;
            if (ecnt) ecnt[pos] = cv[r];
        }
        run += (uint64_t)__popcll(mk);
    }
}

// Offsets of the keys of the entries in depth order; offsets[E] = K.  The
// grid is sized for the largest entry count; blocks past the partitions of
// the device count leave without a ticket.  Each wave takes 1024 consecutive
// entries in 16 rounds of 64 (coalesced loads of the order, gathers of the
// counts, coalesced stores), with a wave scan per round; the waves of a block
// are combined in LDS and the blocks by the look-back.
__host__ __device__ inline int64_t compact_parts(int64_t m) { return (m + kCompactTile - 1) / kCompactTile; }

// Totals for the host (sig != NULL, host-coherent memory): E, K, then the
// sequence number seq, released after them at system scope.
__device__ __forceinline__ void totals_to_host(uint64_t *sig, uint64_t seq, uint64_t E, uint64_t K) {
    if (!sig) return;
    __hip_atomic_store(&sig[0], E, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&sig[1], K, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&sig[2], seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ void __launch_bounds__(kScanBlock) k_offsets(SortedCounts f, int64_t m, uint64_t *ws,
                                                        uint64_t *total, uint32_t *total32, uint32_t *offsets,
                                                        uint32_t *err, uint64_t *sig, uint64_t seq) {
    __shared__ uint32_t s_part;
    __shared__ uint64_t s_w[kScanBlock / 64];
    __shared__ uint64_t s_excl;
    const int64_t E = *f.n_ent;
    const int64_t nparts = (E + kScanTile - 1) / kScanTile;
    if (E == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            offsets[0] = 0;
            *total = 0;
            *total32 = 0;
            totals_to_host(sig, seq, 0, 0);
        }
        return;
    }
    if ((int64_t)blockIdx.x >= nparts) return;  // block-uniform
    if (threadIdx.x == 0) s_part = atomicAdd(reinterpret_cast<uint32_t *>(&ws[1]), 1u);
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t part = s_part;
    const int64_t wbase = part * kScanTile + (int64_t)w * 64 * kScanItems;
    // unconditional loads at clamped indices (issued back to back), then the
    // counts past E dropped
    const int64_t lastE = E - 1;
    uint32_t c[kScanItems];
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        const int64_t j = wbase + r * 64 + lane;
        c[r] = f.order[j < E ? j : lastE];
    }
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) c[r] = f.ecnt[c[r]];
    uint64_t acc = 0;
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        if (wbase + r * 64 + lane >= E) c[r] = 0;
        acc += c[r];
    }
    acc = wave_sum64(acc);
    if (lane == 0) s_w[w] = acc;
    __syncthreads();
    if (w == 0) {
        uint64_t tot = 0;
#pragma unroll
        for (int q = 0; q < kScanBlock / 64; ++q) tot += s_w[q];
        const uint64_t excl = lookback_prefix(ws + 2 + compact_parts(m), part, tot, err);
        if (lane == 0) {
            s_excl = excl;
            if (part == nparts - 1) {
                const uint64_t K = excl + tot;
                offsets[E] = (uint32_t)K;
                *total = K;
                *total32 = K > 0xffffffffull ? 0xffffffffu : (uint32_t)K;
                totals_to_host(sig, seq, (uint64_t)E, K);
            }
        }
    }
    __syncthreads();
    uint64_t run = s_excl;
    for (int q = 0; q < w; ++q) run += s_w[q];
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        const int64_t e = wbase + r * 64 + lane;
        const uint64_t inc = wave_incl_scan((uint64_t)c[r]);
        if (e < E) offsets[e] = (uint32_t)(run + inc - c[r]);
        run += __shfl(inc, 63, 64);
    }
}

int64_t scan_workspace_words(int64_t m) { return 2 + compact_parts(m) + (m + kScanTile - 1) / kScanTile; }

void launch_compact_entries(const uint32_t *counts, const uint8_t *keep, const uint64_t *rect, const DevView *views,
                            int nv, int64_t n, const uint32_t *depth, uint32_t *ent, uint32_t *dkey, uint32_t *dval,
                            uint32_t *ecnt, uint64_t *ws, uint64_t *total, uint32_t *n_ent, uint32_t *err,
                            hipStream_t s, bool zeroed) {
    const int64_t m = (int64_t)nv * n;
    const int64_t nb = compact_parts(m);
    // both scans' tickets and status words
    if (!zeroed) launch_fill_u32(reinterpret_cast<uint32_t *>(ws), 0u, 2 * scan_workspace_words(m), s);
    if (nb == 0) {
        FillSegs z{};
        z.p[0] = reinterpret_cast<uint32_t *>(total), z.n[0] = 2;
        z.p[1] = n_ent, z.n[1] = 1;
        z.count = 2;
        launch_zero_segs(z, s);
        return;
    }
    EntryFlags f{counts, keep, rect, views, n};
    hipLaunchKernelGGL(k_compact, dim3((unsigned)nb), dim3(kCompactBlock), 0, s, f, m, nb, ws, depth, ent, dkey, dval,
                       ecnt, total, n_ent, err);
}

void launch_key_offsets(const uint32_t *ecnt, const uint32_t *order, const uint32_t *n_ent, int64_t m,
                        uint32_t *offsets, uint64_t *ws, uint64_t *total, uint32_t *total32, uint32_t *err,
                        uint64_t *sig, uint64_t seq, hipStream_t s) {
    const int64_t nb = (m + kScanTile - 1) / kScanTile;
    SortedCounts f{ecnt, order, n_ent};
    hipLaunchKernelGGL(k_offsets, dim3((unsigned)(nb > 0 ? nb : 1)), dim3(kScanBlock), 0, s, f, m, ws, total,
                       total32, offsets, err, sig, seq);
}

// ------------------------------------------------------------------------
// key emission (entries in depth order)
// ------------------------------------------------------------------------
// Key-parallel, so every wavefront writes 64 consecutive keys (coalesced)
// whatever the sizes of the entries.  A first kernel records, for every chunk
// of kEmitChunk keys, the entry holding its first key; the chunk's keys then
// belong to at most kEmitChunk consecutive entries, which the block stages in
// LDS.  Within its entry a key's tile is found directly (row-major division of
// the rectangle) when every tile of the rectangle is active; otherwise (a
// masked view) by a binary search over rows of the view's 2D prefix table of
// active tiles (cum[ty][tx] = active tiles in rows < ty, columns < tx), then
// the row's list of active columns.

__device__ __forceinline__ void unpack_rect(uint64_t r, int &x0, int &x1, int &y0, int &y1) {
    x0 = (int)(r & 0xffff); x1 = (int)((r >> 16) & 0xffff);
    y0 = (int)((r >> 32) & 0xffff); y1 = (int)((r >> 48) & 0xffff);
}

// Key chunks of kEmitChunk consecutive keys: chunk c starts inside the entry
// (depth order) whose key range holds key c * kEmitChunk.
constexpr int kEmitChunk = 1024;
constexpr int kEmitBlock = 512;

// Thread per entry j (depth order: entry order[j] of this pass, slot
// ent[order[j]], record r = map[slot] when the records belong to an earlier
// pass, else order[j]): the chunks whose first key lies in its key range start
// at j; and its slot, record index and rectangle (rect_e[r]) are copied to
// esort[j], rsort[j] and rect_s[j], so the emission reads them next to the
// offsets instead of through the indices.  Block 0 also clears
// zero[0, zero_words) (the key sort's tickets and group sums).
__global__ void __launch_bounds__(256) k_chunk_starts(const uint32_t *n_ent, const uint32_t *__restrict__ offsets,
                                                      const uint32_t *__restrict__ order,
                                                      const uint32_t *__restrict__ ent,
                                                      const uint32_t *__restrict__ map,
                                                      const uint64_t *__restrict__ rect_e,
                                                      uint64_t *__restrict__ rect_s, uint32_t *__restrict__ esort,
                                                      uint32_t *__restrict__ rsort,
                                                      uint32_t *__restrict__ chunk_start, int64_t nchunks,
                                                      int64_t cap, uint32_t *__restrict__ zero, int zero_words) {
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < zero_words; i += blockDim.x) zero[i] = 0u;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= (int64_t)*n_ent || j >= cap) return;  // entries past the capacity emit no key (k_clamp_keys)
    const uint64_t lo = offsets[j], hi = offsets[j + 1];
    const uint32_t e = order[j];
    if (map) {  // records of an earlier pass: found through the slot
        const uint32_t slot = ent[e];
        const uint32_t r = map[slot];
        rect_s[j] = rect_e[r];
        esort[j] = slot;
        rsort[j] = r;
    } else {    // the record is the entry: its rectangle loads beside the slot
        // (read as two words, so that the compiler does not merge this load
        // with the other branch's behind a common wait for the slot)
        const uint2 rw = reinterpret_cast<const uint2 *>(rect_e)[e];
        const uint32_t slot = ent[e];
        const uint64_t rc = ((uint64_t)rw.y << 32) | rw.x;
        rect_s[j] = rc;
        esort[j] = slot;
        rsort[j] = e;
    }
    for (uint64_t c = (lo + kEmitChunk - 1) / kEmitChunk; c * kEmitChunk < hi && (int64_t)c < nchunks; ++c)
        chunk_start[c] = (uint32_t)j;
}

// One block per chunk of kEmitChunk keys, kEmitChunk / kEmitBlock keys per
// thread at a stride of kEmitBlock (coalesced stores).  The chunk's keys
// belong to at most kEmitChunk consecutive entries (each entry has at least
// one key); their key offsets, Gaussian indices, views and rectangles are
// staged in LDS first (all loads of the block in flight together).  A key then
// finds its entry by bisection in LDS and its tile as the r-th tile of the
// entry's rectangle, row-major: directly when every tile of the rectangle is
// active (a view with all tiles active, or a rectangle inside the mask), else
// by bisection over the rows with the view's 2D active-tile prefix and the
// row's list of active columns.  The keys of a thread advance through each
// bisection step together, so their dependent loads overlap; two keys per
// thread keep the registers low enough for eight blocks per compute unit (the
// LDS limit), which hides the latency of the chains better than more keys
// per thread.
constexpr int kEmitPer = kEmitChunk / kEmitBlock;

// per-view fields the emission needs, staged in LDS
struct EmitView {
    uint32_t tile_off;
    int32_t tiles_x;
    int32_t cum_off;   // -1: every tile active
    int32_t mask_off;
};
constexpr int kEmitMaxViews = kMaxViews;

__global__ void __launch_bounds__(kEmitBlock) k_emit(const DevView *__restrict__ views, int nv, int64_t n,
                                                     const uint32_t *__restrict__ esort,
                                                     const uint32_t *__restrict__ rsort, const uint32_t *n_ent,
                                                     const uint32_t *__restrict__ offsets,
                                                     const uint32_t *__restrict__ chunk_start,
                                                     const uint64_t *__restrict__ rect_s,
                                                     const uint16_t *__restrict__ row_prefix,
                                                     const uint16_t *__restrict__ row_list,
                                                     const uint32_t *__restrict__ cum, uint32_t *__restrict__ keys,
                                                     uint32_t *__restrict__ vals, int64_t K, const uint32_t *K_dev) {
    __shared__ uint32_t s_off[kEmitChunk + 1];
    __shared__ uint32_t s_i[kEmitChunk];
    __shared__ uint32_t s_v[kEmitChunk];
    __shared__ uint64_t s_rect[kEmitChunk];
    __shared__ EmitView s_view[kEmitMaxViews];
    const int tid = threadIdx.x;
    const int64_t q0 = (int64_t)blockIdx.x * kEmitChunk;
    if (K_dev && (int64_t)*K_dev < K) K = *K_dev;  // capacity mode: the device count, clamped
    if (q0 >= K) return;                           // block-uniform
    const int64_t E = *n_ent;
    if (E == 0) return;  // no entry, no key (block-uniform)
    const int64_t j0 = chunk_start[blockIdx.x];
    const int64_t qend = q0 + kEmitChunk < K ? q0 + kEmitChunk : K;
    // s_off[t] = offsets[j0 + t] (offsets[E], the key total, past the last entry):
    // s_off[0] <= q0 and s_off[kEmitChunk] > q0 + kEmitChunk - 1.  A thread's
    // loads are issued together, the views' fields with them (every field
    // loaded, then selected: no load waits on another).
    uint32_t oo[kEmitPer];
#pragma unroll
    for (int u = 0; u < kEmitPer; ++u) {
        const int64_t ja = j0 + tid + u * kEmitBlock;
        oo[u] = offsets[ja < E ? ja : E];
    }
    const int64_t jc = j0 + kEmitChunk;
    const uint32_t oc = offsets[jc < E ? jc : E];
    for (int v = tid; v < nv; v += kEmitBlock) {
        const DevView &dv = views[v];
        const int32_t mask = dv.v.mask, coff = (int32_t)dv.cum_off, moff = (int32_t)dv.mask_off;
        const uint32_t toff = (uint32_t)dv.tile_off;
        const int32_t tx = dv.tiles_x;
        const bool all = mask == A3FR_MASK_ALL;
        s_view[v] = EmitView{toff, tx, all ? -1 : coff, all ? -1 : moff};
    }
#pragma unroll
    for (int u = 0; u < kEmitPer; ++u) s_off[tid + u * kEmitBlock] = oo[u];
    if (tid == 0) s_off[kEmitChunk] = oc;
    __syncthreads();
    // the entries with keys in [q0, qend): t < kEmitChunk with s_off[t] < qend (then j0 + t < E);
    // their record index (the keys' value), view and rectangle
    // (loaded unconditionally, both of a thread's entries together; a slot
    // whose entry holds no key of the chunk reads entry j0, the chunk's first,
    // so that it costs no memory traffic)
    const uint32_t nn = (uint32_t)n;
    {
        uint64_t rc[kEmitPer];
        uint32_t es[kEmitPer], rs[kEmitPer];
#pragma unroll
        for (int u = 0; u < kEmitPer; ++u) {
            const int t = tid + u * kEmitBlock;
            const int64_t jc = (int64_t)s_off[t] < qend ? j0 + t : j0;
            rc[u] = rect_s[jc];
            es[u] = esort[jc];
            rs[u] = rsort[jc];
        }
#pragma unroll
        for (int u = 0; u < kEmitPer; ++u) {
            const int t = tid + u * kEmitBlock;
            if ((int64_t)s_off[t] < qend) {
                s_rect[t] = rc[u];
                s_v[t] = es[u] / nn;
                s_i[t] = rs[u];
            }
        }
    }
    __syncthreads();
    int lo[kEmitPer], hi[kEmitPer];
    int64_t q[kEmitPer];
#pragma unroll
    for (int k = 0; k < kEmitPer; ++k) {
        q[k] = q0 + (int64_t)k * kEmitBlock + tid;
        lo[k] = 0;
        hi[k] = kEmitChunk;
    }
    // largest t with s_off[t] <= q (kEmitChunk is a power of two: exact after log2 steps)
#pragma unroll
    for (int step = kEmitChunk; step > 1; step >>= 1) {
#pragma unroll
        for (int k = 0; k < kEmitPer; ++k) {
            const int mid = (lo[k] + hi[k]) >> 1;
            if ((int64_t)s_off[mid] <= q[k]) lo[k] = mid; else hi[k] = mid;
        }
    }
    // keys past qend (last chunk, capacity mode) take entry 0, which is staged; nothing is stored for them
#pragma unroll
    for (int k = 0; k < kEmitPer; ++k)
        if (q[k] >= qend) lo[k] = 0;
    // per key: entry fields, and the row search state for partially active rectangles
    uint32_t r[kEmitPer], base[kEmitPer];
    int x0[kEmitPer], x1[kEmitPer], y0[kEmitPer], y1[kEmitPer], ra[kEmitPer], rb[kEmitPer];
    int tx[kEmitPer], ty[kEmitPer], TX[kEmitPer];
    bool search[kEmitPer];
    const uint32_t *cm[kEmitPer];
#pragma unroll
    for (int k = 0; k < kEmitPer; ++k) {
        const int t = lo[k];
        r[k] = (uint32_t)(q[k] - s_off[t]);
        unpack_rect(s_rect[t], x0[k], x1[k], y0[k], y1[k]);
        const EmitView &ev = s_view[s_v[t]];
        TX[k] = ev.tiles_x;
        const uint32_t w = (uint32_t)(x1[k] - x0[k] + 1);
        const uint32_t cnt = s_off[t + 1] - s_off[t];
        search[k] = q[k] < qend && ev.cum_off >= 0 && cnt != w * (uint32_t)(y1[k] - y0[k] + 1);
        ty[k] = y0[k] + (int)(r[k] / w);
        tx[k] = x0[k] + (int)(r[k] % w);
        cm[k] = cum + (search[k] ? ev.cum_off : 0);
        ra[k] = y0[k];
        rb[k] = y1[k] + 1;
        base[k] = 0;
    }
    // row ty: largest y in [y0, y1] with (keys of the entry in rows < y) <= r; bra keeps
    // that count for row ra (0 for y0), so the row's count needs no second load, and the
    // prefix of row y0 (base) is loaded with the first bisection step's
    uint32_t bra[kEmitPer];
#pragma unroll
    for (int k = 0; k < kEmitPer; ++k) bra[k] = 0;
    bool more = true, first = true;
    while (more) {
        more = false;
#pragma unroll
        for (int k = 0; k < kEmitPer; ++k)
            if (search[k] && rb[k] - ra[k] > 1) {
                const int64_t st = TX[k] + 1;
                const int mid = (ra[k] + rb[k]) >> 1;
                const uint32_t cmid = cm[k][(int64_t)mid * st + x1[k] + 1] - cm[k][(int64_t)mid * st + x0[k]];
                if (first) base[k] = cm[k][(int64_t)y0[k] * st + x1[k] + 1] - cm[k][(int64_t)y0[k] * st + x0[k]];
                const uint32_t before = cmid - base[k];
                if (before <= r[k]) {
                    ra[k] = mid;
                    bra[k] = before;
                } else {
                    rb[k] = mid;
                }
                more |= rb[k] - ra[k] > 1;
            }
        first = false;
    }
#pragma unroll
    for (int k = 0; k < kEmitPer; ++k)
        if (search[k]) {
            const int64_t st = TX[k] + 1;
            const int t = lo[k];
            const EmitView &ev = s_view[s_v[t]];
            ty[k] = ra[k];
            const uint32_t before = bra[k];
            const uint16_t *rp = row_prefix + ev.mask_off + (int64_t)ty[k] * st;
            const uint16_t *rl = row_list + ev.mask_off + (int64_t)ty[k] * st;
            tx[k] = rl[rp[x0[k]] + (r[k] - before)];
        }
#pragma unroll
    for (int k = 0; k < kEmitPer; ++k)
        if (q[k] < qend) {
            const int t = lo[k];
            keys[q[k]] = s_view[s_v[t]].tile_off + (uint32_t)(ty[k] * TX[k] + tx[k]);
            vals[q[k]] = s_i[t];
        }
}

// cum[v][ty][tx] for masked views: active tiles in rows < ty and columns < tx.
// One wavefront per (view, column): a wave-wide scan down the rows.
__global__ void __launch_bounds__(256) k_mask_cum(const DevView *__restrict__ views,
                                                  const uint16_t *__restrict__ row_prefix, uint32_t *__restrict__ cum,
                                                  const uint32_t *skip_if_zero) {
    if (skip_if_zero && *skip_if_zero == 0) return;
    const DevView &dv = views[blockIdx.y];
    if (dv.v.mask == A3FR_MASK_ALL) return;
    const int TX = dv.tiles_x, TY = dv.tiles_y, stride = TX + 1;
    const int tx = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (tx > TX) return;
    uint32_t *cm = cum + dv.cum_off;
    const uint16_t *rp = row_prefix + dv.mask_off;
    if (lane == 0) cm[tx] = 0;
    uint32_t carry = 0;
    for (int r0 = 0; r0 < TY; r0 += 64) {
        const int ty = r0 + lane;
        uint32_t x = ty < TY ? (uint32_t)rp[(int64_t)ty * stride + tx] : 0u;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (ty < TY) cm[(int64_t)(ty + 1) * stride + tx] = carry + x;
        carry += __shfl(x, 63, 64);
    }
}

void launch_mask_cum(const DevView *views, int nv, int max_tiles_x, const uint16_t *row_prefix, uint32_t *cum,
                     hipStream_t s, const uint32_t *skip_if_zero) {
    if (nv == 0) return;
    hipLaunchKernelGGL(k_mask_cum, dim3((unsigned)((max_tiles_x + 1 + 3) / 4), (unsigned)nv), dim3(256), 0, s, views,
                       row_prefix, cum, skip_if_zero);
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

// Zeroes up to kFillSegs buffers in one launch (the segments are walked as one
// concatenated range).
__global__ void k_zero_segs(FillSegs f) {
    int64_t total = 0;
    for (int k = 0; k < f.count; ++k) total += f.n[k];
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < total; j += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = j;
        int k = 0;
        while (r >= f.n[k]) r -= f.n[k++];
        f.p[k][r] = 0u;
    }
}

void launch_zero_segs(const FillSegs &f, hipStream_t s) {
    int64_t total = 0;
    for (int k = 0; k < f.count; ++k) total += f.n[k];
    if (total <= 0) return;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_zero_segs, dim3((unsigned)blocks), dim3(256), 0, s, f);
}

int64_t emit_chunks(int64_t K) { return (K + kEmitChunk - 1) / kEmitChunk; }

void launch_emit(const DevView *views, int nv, int64_t n, int64_t m, const EmitEntries &ee, const uint32_t *n_ent,
                 const uint32_t *offsets, const uint16_t *row_prefix, const uint16_t *row_list, const uint32_t *cum,
                 uint32_t *chunk_start, uint32_t *keys, uint32_t *vals, int64_t K, const uint32_t *K_dev,
                 uint32_t *zero, int zero_words, hipStream_t s) {
    if (m == 0 || K == 0) return;
    const int64_t nchunks = emit_chunks(K);
    const int64_t work = ee.cap < m ? ee.cap : m;
    hipLaunchKernelGGL(k_chunk_starts, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s, n_ent, offsets, ee.order,
                       ee.ent, ee.map, ee.rect_e, ee.rect_s, ee.esort, ee.rsort, chunk_start, nchunks, ee.cap, zero,
                       zero_words);
    hipLaunchKernelGGL(k_emit, dim3((unsigned)nchunks), dim3(kEmitBlock), 0, s, views, nv, n, ee.esort, ee.rsort,
                       n_ent, offsets, chunk_start, ee.rect_s, row_prefix, row_list, cum, keys, vals, K, K_dev);
}

// capacity mode: the sort count is min(key total, key capacity), and when the
// entries exceed the entry capacity, no more than the keys of the entries
// within it; an overflow raises bit 1 of the error word
__global__ void k_clamp_keys(const uint64_t *total, uint64_t cap, const uint32_t *n_ent, const uint32_t *offsets,
                             uint64_t ecap, uint32_t *n32, uint32_t *err) {
    uint64_t t = *total;
    bool over = t > cap;
    if ((uint64_t)*n_ent > ecap) {
        const uint64_t te = offsets[ecap];
        if (te < t) t = te;
        over = true;
    }
    *n32 = (uint32_t)(t < cap ? t : cap);
    if (over) atomicOr(err, 2u);
}

void launch_clamp_keys(const uint64_t *total, int64_t cap, const uint32_t *n_ent, const uint32_t *offsets,
                       int64_t ecap, uint32_t *n32, uint32_t *err, hipStream_t s) {
    hipLaunchKernelGGL(k_clamp_keys, dim3(1), dim3(1), 0, s, total, (uint64_t)cap, n_ent, offsets, (uint64_t)ecap,
                       n32, err);
}

// ------------------------------------------------------------------------
// inspection: 64-bit (tile << 32 | depth bits) keys from tile ids and values
// ------------------------------------------------------------------------
__global__ void k_make_keys64(const uint32_t *__restrict__ tiles, const uint32_t *__restrict__ vals, int64_t K,
                              const Record *__restrict__ rec, int64_t n_rec, uint64_t *__restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= K) return;
    const uint32_t r = vals[j];
    out[j] = ((uint64_t)tiles[j] << 32) | (uint64_t)((int64_t)r < n_rec ? rec[r].dbits : 0u);
}

void launch_make_keys64(const uint32_t *tiles, const uint32_t *vals, int64_t K, const Record *rec, int64_t n_rec,
                        uint64_t *out, hipStream_t s) {
    if (K == 0) return;
    hipLaunchKernelGGL(k_make_keys64, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, s, tiles, vals, K, rec, n_rec,
                       out);
}

// inspection: key values (record indices) as Gaussian indices: the record's slot modulo n
__global__ void k_vals_to_index(const uint32_t *__restrict__ vals, int64_t K, const uint32_t *__restrict__ rent,
                                int64_t n_rec, int64_t n, uint32_t *__restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= K) return;
    const uint32_t r = vals[j];
    out[j] = (int64_t)r < n_rec ? (uint32_t)((uint64_t)rent[r] % (uint64_t)n) : 0xffffffffu;
}

void launch_vals_to_index(const uint32_t *vals, int64_t K, const uint32_t *rent, int64_t n_rec, int64_t n,
                          uint32_t *out, hipStream_t s) {
    if (K == 0) return;
    hipLaunchKernelGGL(k_vals_to_index, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, s, vals, K, rent, n_rec, n,
                       out);
}

// inspection: out[j] = src[idx[j]] (u32), or a dense [m] array from per-entry
// values: out[ent[j]] = src[j] (64-bit or record words) after a fill
__global__ void k_gather_u32(const uint32_t *__restrict__ src, const uint32_t *__restrict__ idx, int64_t cnt,
                             uint32_t *__restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < cnt) out[j] = src[idx[j]];
}

void launch_gather_u32(const uint32_t *src, const uint32_t *idx, int64_t cnt, uint32_t *out, hipStream_t s) {
    if (cnt <= 0) return;
    hipLaunchKernelGGL(k_gather_u32, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, src, idx, cnt, out);
}

template <typename T>
__global__ void k_scatter_dense(const T *__restrict__ src, const uint32_t *__restrict__ ent, int64_t cnt,
                                T *__restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < cnt) out[ent[j]] = src[j];
}

void launch_scatter_dense_u64(const uint64_t *src, const uint32_t *ent, int64_t cnt, uint64_t *out, hipStream_t s) {
    if (cnt <= 0) return;
    hipLaunchKernelGGL(k_scatter_dense<uint64_t>, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, src, ent, cnt,
                       out);
}

void launch_scatter_dense_rec(const Record *src, const uint32_t *ent, int64_t cnt, Record *out, hipStream_t s) {
    if (cnt <= 0) return;
    hipLaunchKernelGGL(k_scatter_dense<Record>, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, src, ent, cnt,
                       out);
}

}  // namespace a3fr
