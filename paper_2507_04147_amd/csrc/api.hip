// Host side of the C ABI (include/a3fr.h): argument checks, the context's
// growable device workspace, and the order of launches of one frame.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdint>
#include <mutex>
#include <new>
#include <utility>
#include <string>
#include <vector>

#include "a3fr_internal.h"

using namespace a3fr;

namespace {

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

// Region sums of the PSNR judge: per-block partials [kSseParts][3] float64,
// then [kSseParts][3] uint64 pixel counts.
constexpr int kSseParts = 1024;
constexpr size_t kSseScratchBytes = (size_t)kSseParts * 3 * (sizeof(double) + sizeof(unsigned long long));

}  // namespace

// Scratch of a3fr_region_sse_noalloc: a static device array (one copy per GPU,
// kept until the process ends), so that entry point allocates nothing.  In host
// code the name stands for a host-side handle, not a device address: kernels
// and copies take the address hipGetSymbolAddress returns for each device.
static __device__ __align__(256) unsigned char scratch[kSseScratchBytes];

namespace {

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchDevices] = {};

// Device address of scratch on device dev, looked up once per device with that
// device current (it is made current for the lookup and restored after).
hipError_t scratch_on_device(int dev, void **out) {
    *out = nullptr;
    if (dev < 0 || dev >= kScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

struct a3fr_ctx {
    hipStream_t stream = nullptr;
    std::string err;
    // frame description
    int nv = 0;
    int64_t n = 0;
    int64_t ntiles = 0;
    int64_t npix = 0;
    int nsel = 0;
    int64_t rows_total = 0;
    int64_t mask_entries = 0;
    int64_t cum_entries = 0;
    int max_tiles_x = 1;
    std::vector<DevView> hviews;
    std::vector<int32_t> hrow_view, hrow_y, hsel_views, hgroups;
    // pinned staging for uploads and small readbacks
    void *pinned = nullptr;
    size_t pinned_cap = 0;
    hipEvent_t upload_done = nullptr;
    uint64_t *h_total = nullptr;
    hipEvent_t total_ready = nullptr;  // the key total has reached h_total
    // host-coherent words the key-offsets kernel writes the entry and key
    // totals and a sequence number into ([0] E, [1] K, [2] seq), so that the
    // host reads them without a copy or an event in the stream (h_sig: host
    // address, d_sig: device address; NULL when unavailable); sig_seq: the
    // number of the last frame that asked for them, sig_pending: this frame's
    // totals come that way
    uint64_t *h_sig = nullptr, *d_sig = nullptr;
    uint64_t sig_seq = 0;
    bool sig_pending = false;
    // a3fr_set_host_wait(1): host waits sleep on blocking-sync events instead of polling
    bool block_wait = false;
    hipEvent_t total_ready_block = nullptr, sync_block = nullptr;
    // second stream of a foveated frame: the fovea and mid layers are blended
    // on it while the main stream blends the periphery and runs the network
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // the records of a frame's entries are formed in a3fr_bin_sort, where they
    // are computed while the host waits for the key total
    bool records_pending = false;
    a3fr_scene rec_scene{};
    // device workspace.  Per (view, Gaussian) slot: counts, depth, keep, map
    // (slot -> record), the compaction and depth-sort arrays, offsets; rect only
    // for views that keep every slot's rectangle (rect_slot), score only for
    // selecting views (sel_slot).  Per record (entry): rec, rect_e.  Per
    // depth-ordered entry of an emission: rect_s, esort, rsort.
    DevBuf views, row_view, row_y, row_prefix, row_list, active;
    DevBuf counts, depth, rect, score, keep, sel_views, sel, map;
    DevBuf rec, rect_e, rect_s, esort, rsort;
    DevBuf offsets, block_sums, scalars;
    DevBuf ent_a, ent_b, dkey_a, dkey_b, dval_a, dval_b;  // entries (records' / a round's), depth sort
    DevBuf ecnt;               // key count of each entry, in entry order
    DevBuf gpack;              // packed geometry of every Gaussian, written by the projection
    DevBuf keys_a, keys_b, vals_a, vals_b;
    DevBuf sort_status, ranges;
    DevBuf grad_acc;           // reverse blend sums, [records][12] float
    int nrect = 0;             // views keeping every slot's rectangle
    int64_t n_rec = 0;         // records of the last record pass (exact mode)
    int64_t n_ent_pass = 0;    // entries of the last emission (exact mode)
    bool map_mode = false;     // the last emission's records belong to an earlier pass (incremental rounds)
    bool inc_round0 = false;   // layouts made now: the first round of an incremental frame (keep_visible)
    int64_t ecap = 0;          // graph mode: entry (and record) capacity
    // upsampler workspace: packed weights, activations (NHWC + channel-major copies), gradients
    DevBuf net_pk, net_x0, net_x0c, net_a1, net_a1c, net_a2, net_a2c, net_g3, net_g3c, net_g2, net_g2c, net_g1c,
        net_sse;
    int net_B = 0, net_h = 0, net_w = 0;   // geometry of the channel-major copies (zero borders valid)
    const float *net_theta = nullptr;      // a3fr_set_upsampler
    // full-resolution fallback of the periphery (a3fr_set_fallback)
    double fb_thr = INFINITY, fb_coef = 0.0, fb_pow = 1.0;
    struct FbPair { int pv, fv; double r_mid; };
    std::vector<FbPair> fb_plan;           // set by a3fr_render_foveated for its a3fr_preprocess
    bool fb_last = false;                  // the last preprocess ran the fallback steps
    bool amr_last = false;                 // the last frame was a3fr_render_amr (tile levels in amr_lv)
    // incremental foveal rounds (a3fr_incremental_*)
    bool inc_mode = false;                 // layouts made now: remask fovea and mid layers, apply inc_flags
    std::vector<int32_t> inc_flags;        // round flags per view of the next layout
    bool inc_ready = false;                // a3fr_incremental_begin done, frame not finished
    int inc_eyes = 0;
    int64_t inc_n = 0, inc_ntiles = 0, inc_npix = 0;
    std::vector<a3fr_camera> inc_cams;
    a3fr_fovea inc_fovea{};
    DevBuf inc_done;                       // [tiles] rendered by an earlier round
    DevBuf inc_periph;                     // upsampled periphery of each eye [eyes][3][H][W] (network set)
    bool inc_net = false;                  // the periphery of the incremental frame went through the network
    DevBuf fb_energy, fb_flags, fb_diff, fb_part, fb_count;
    bool net_trained_fwd = false;          // the last forward kept activations for a backward
    DevBuf layers, sse_part, sse_cnt, cum, chunk_start;
    DevBuf keys_e, vals_e;     // emission-order copy (debug option)
    bool keep_emission = false;
    // per-stage event timing
    bool profiling = false;
    bool count_pairs = false;              // profiling mode 1 also counts blend pairs
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<int, size_t>> ev_marks;  // (stage, index of the start event)
    int64_t prof_sort_keys = 0, prof_sort_passes = 0;
    DevBuf pair_count;          // evaluated blend pairs while profiling
    bool pairs_armed = false;
    // state
    bool preprocessed = false;
    bool sorted = false;
    bool sorted_in_b = false;
    bool blend_bwd_done = false;
    int blend_variant = kBlendDefault;     // a3fr_set_blend_variant / a3fr_autotune_blend
    // graph mode: key buffers sized to a capacity, counts stay on the device
    int64_t capacity = 0;                  // 0: exact mode (bin_sort reads the key count)
    bool capturing = false;                // inside a3fr_graph_capture's stream capture
    const int32_t *d_row_view = nullptr, *d_row_y = nullptr, *d_sel_views = nullptr, *d_groups = nullptr;
    const double *d_exp_tab = nullptr;
    hipStream_t own_stream = nullptr;      // capture stream when the caller's is the null stream
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int g_eyes = 0;
    std::vector<a3fr_camera> g_cams;
    a3fr_fovea g_fovea{};
    int n_cus = 256;
    DevBuf blend_ws, blend_order, tune_img;
    DevBuf amr_thr, amr_lv;    // AMR count thresholds [views][3], tile levels [tiles]
    int sh_degree = 0;
    int64_t K = 0;
};

namespace {

a3fr_status fail(a3fr_ctx *c, a3fr_status s, const std::string &msg) {
    if (c) c->err = msg;
    return s;
}

#define HIPCHECK(ctx, expr)                                                                    \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail((ctx), A3FR_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

a3fr_status ensure(a3fr_ctx *c, DevBuf &b, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (b.cap >= bytes) return A3FR_OK;
    if (c->capturing)
        return fail(c, A3FR_ECAPACITY, "a buffer would grow during graph capture (the warm-up frame sized it smaller)");
    if (c->gexec)  // the captured graph holds this buffer's address
        return fail(c, A3FR_ECAPACITY, "the workspace is frozen while a graph is held (a3fr_graph_destroy first)");
    if (b.p) {
        // the old buffer may still be read by queued work
        HIPCHECK(c, hipStreamSynchronize(c->stream));
        HIPCHECK(c, hipFree(b.p));
        b.p = nullptr;
        b.cap = 0;
    }
    size_t want = bytes + bytes / 4;
    want = (want + 255) & ~size_t(255);
    if (hipMalloc(&b.p, want) != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return fail(c, A3FR_ENOMEM, "hipMalloc of " + std::to_string(want) + " bytes failed");
    }
    b.cap = want;
    return A3FR_OK;
}

template <class T>
T *P(DevBuf &b) { return reinterpret_cast<T *>(b.p); }

// Device scalars of one frame (the scalars buffer, 64 bytes):
//   u64 [0] entries total, u64 [1] keys total, u32 [4] entries (sort count),
//   u32 [5] keys (sort count), u32 [6] sticky sort error flag.
uint64_t *sc_ent_total(DevBuf &b) { return reinterpret_cast<uint64_t *>(b.p); }
uint64_t *sc_key_total(DevBuf &b) { return reinterpret_cast<uint64_t *>(b.p) + 1; }
uint32_t *sc_n_ent(DevBuf &b) { return reinterpret_cast<uint32_t *>(b.p) + 4; }
uint32_t *sc_n_keys(DevBuf &b) { return reinterpret_cast<uint32_t *>(b.p) + 5; }
uint32_t *sc_err(DevBuf &b) { return reinterpret_cast<uint32_t *>(b.p) + 6; }

#define TRY(expr)                           \
    do {                                    \
        a3fr_status s_ = (expr);            \
        if (s_ != A3FR_OK) return s_;       \
    } while (0)

a3fr_status check_launch(a3fr_ctx *c, const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, A3FR_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return A3FR_OK;
}

a3fr_status ensure_pinned(a3fr_ctx *c, size_t bytes) {
    if (c->upload_done) HIPCHECK(c, hipEventSynchronize(c->upload_done));
    if (c->pinned_cap >= bytes) return A3FR_OK;
    if (c->pinned) HIPCHECK(c, hipHostFree(c->pinned));
    c->pinned = nullptr;
    size_t want = bytes + bytes / 2 + 4096;
    if (hipHostMalloc(&c->pinned, want, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        c->pinned_cap = 0;
        return fail(c, A3FR_ENOMEM, "hipHostMalloc failed");
    }
    c->pinned_cap = want;
    return A3FR_OK;
}

bool is_fin(double x) { return std::isfinite(x); }

// Stage timing: a pair of events around each timed interval.
a3fr_status stage_begin(a3fr_ctx *c, int stage, size_t *slot) {
    *slot = SIZE_MAX;
    if (!c->profiling) return A3FR_OK;
    while (c->ev_pool.size() < c->ev_used + 2) {
        hipEvent_t e;
        HIPCHECK(c, hipEventCreate(&e));
        c->ev_pool.push_back(e);
    }
    *slot = c->ev_used;
    c->ev_used += 2;
    c->ev_marks.emplace_back(stage, *slot);
    HIPCHECK(c, hipEventRecord(c->ev_pool[*slot], c->stream));
    return A3FR_OK;
}

a3fr_status stage_end(a3fr_ctx *c, size_t slot) {
    if (slot == SIZE_MAX) return A3FR_OK;
    HIPCHECK(c, hipEventRecord(c->ev_pool[slot + 1], c->stream));
    return A3FR_OK;
}

struct StageTimer {
    a3fr_ctx *c;
    size_t slot;
    a3fr_status st;
    StageTimer(a3fr_ctx *cc, int stage) : c(cc), slot(SIZE_MAX) { st = stage_begin(c, stage, &slot); }
    ~StageTimer() { (void)stage_end(c, slot); }
};

a3fr_status check_scene(a3fr_ctx *c, const a3fr_scene *s) {
    if (!s) return fail(c, A3FR_EINVAL, "scene is NULL");
    if (s->n < 0 || s->n >= (int64_t(1) << 31)) return fail(c, A3FR_EINVAL, "scene.n must be in [0, 2^31)");
    if (s->sh_degree < 0 || s->sh_degree > 3) return fail(c, A3FR_EINVAL, "scene.sh_degree must be 0..3");
    if (s->n > 0 && (!s->mean_dev || !s->scale_dev || !s->quat_dev || !s->opacity_dev || !s->sh_dev))
        return fail(c, A3FR_EINVAL, "scene arrays must not be NULL");
    return A3FR_OK;
}

a3fr_status check_view(a3fr_ctx *c, const a3fr_view &v, int k) {
    std::string w = "view " + std::to_string(k) + ": ";
    if (v.width <= 0 || v.height <= 0) return fail(c, A3FR_EINVAL, w + "width and height must be positive");
    if ((v.width + kTile - 1) / kTile > 65535 || (v.height + kTile - 1) / kTile > 65535)
        return fail(c, A3FR_EINVAL, w + "more than 65535 tiles per axis");
    if ((int64_t)v.width * v.height > (int64_t(1) << 31)) return fail(c, A3FR_EINVAL, w + "image too large");
    if (v.eye < 0 || v.eye >= kMaxEyes) return fail(c, A3FR_EINVAL, w + "eye must be 0..127");
    if (v.mask < 0 || v.mask > 2) return fail(c, A3FR_EINVAL, w + "mask must be 0, 1 or 2");
    if (v.select != 0 && v.select != 1) return fail(c, A3FR_EINVAL, w + "select must be 0 or 1");
    if (!(v.fx > 0.0) || !(v.fy > 0.0) || !is_fin(v.fx) || !is_fin(v.fy) || !is_fin(v.cx) || !is_fin(v.cy))
        return fail(c, A3FR_EINVAL, w + "focal lengths must be positive and finite");
    for (int j = 0; j < 9; ++j) if (!is_fin(v.R[j])) return fail(c, A3FR_EINVAL, w + "R not finite");
    for (int j = 0; j < 3; ++j)
        if (!is_fin(v.t[j]) || !is_fin(v.campos[j])) return fail(c, A3FR_EINVAL, w + "t/campos not finite");
    if (v.mask != A3FR_MASK_ALL && (!is_fin(v.gx) || !is_fin(v.gy) || !is_fin(v.r_out) || !is_fin(v.r_in)))
        return fail(c, A3FR_EINVAL, w + "gaze and radii must be finite");
    return A3FR_OK;
}

}  // namespace

static void graph_release(a3fr_ctx *c);

extern "C" {

const char *a3fr_status_str(a3fr_status s) {
    switch (s) {
        case A3FR_OK: return "ok";
        case A3FR_EINVAL: return "invalid argument";
        case A3FR_ENOMEM: return "out of device memory";
        case A3FR_ECAPACITY: return "capacity exceeded";
        case A3FR_EDEVICE: return "device error";
        case A3FR_ENOTREADY: return "call order violated";
    }
    return "unknown status";
}

const char *a3fr_last_error(const a3fr_ctx *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

a3fr_status a3fr_create(a3fr_ctx **out, void *hip_stream) {
    if (!out) return A3FR_EINVAL;
    *out = nullptr;
    a3fr_ctx *c = new (std::nothrow) a3fr_ctx();
    if (!c) return A3FR_ENOMEM;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    if (hipEventCreateWithFlags(&c->upload_done, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return A3FR_EDEVICE;
    }
    if (hipEventCreateWithFlags(&c->total_ready, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipEventDestroy(c->upload_done);
        delete c;
        return A3FR_EDEVICE;
    }
    if (hipHostMalloc(reinterpret_cast<void **>(&c->h_total), 64, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipEventDestroy(c->upload_done);
        delete c;
        return A3FR_ENOMEM;
    }
    {   // optional: without it the totals are read back by a copy
        void *hs = nullptr, *ds = nullptr;
        if (hipHostMalloc(&hs, 64, hipHostMallocCoherent | hipHostMallocMapped) == hipSuccess &&
            hipHostGetDevicePointer(&ds, hs, 0) == hipSuccess) {
            c->h_sig = static_cast<uint64_t *>(hs);
            c->d_sig = static_cast<uint64_t *>(ds);
            std::memset(hs, 0, 64);
        } else {
            if (hs) (void)hipHostFree(hs);
            (void)hipGetLastError();
        }
    }
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
        c->n_cus = cus;
    (void)hipGetLastError();
    {   // the scratch of the allocation-free entry point on the context's device
        hipDevice_t sdev = 0;
        void *p = nullptr;
        if (hipStreamGetDevice(c->stream, &sdev) != hipSuccess || scratch_on_device((int)sdev, &p) != hipSuccess) {
            (void)hipGetLastError();  // a later call of that entry point retries and reports
        }
    }
    *out = c;
    return A3FR_OK;
}

void a3fr_destroy(a3fr_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    graph_release(c);
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    DevBuf *bufs[] = {&c->views, &c->row_view, &c->row_y, &c->row_prefix, &c->row_list, &c->active,
                      &c->counts, &c->depth, &c->rect, &c->rect_s, &c->rec, &c->score, &c->keep, &c->sel_views,
                      &c->sel, &c->map, &c->rect_e, &c->esort, &c->rsort, &c->dval_a, &c->dval_b,
                      &c->offsets, &c->block_sums, &c->scalars, &c->ent_a, &c->ent_b, &c->ecnt, &c->gpack, &c->dkey_a,
                      &c->dkey_b, &c->keys_a, &c->keys_b,
                      &c->vals_a, &c->vals_b, &c->grad_acc, &c->net_pk, &c->net_x0, &c->net_x0c, &c->net_a1,
                      &c->net_a1c, &c->net_a2, &c->net_a2c, &c->net_g3, &c->net_g3c, &c->net_g2, &c->net_g2c,
                      &c->net_g1c, &c->net_sse, &c->fb_energy, &c->fb_flags, &c->fb_diff, &c->fb_part, &c->inc_periph, &c->inc_done, &c->fb_count, &c->blend_ws,
                      &c->blend_order, &c->tune_img, &c->amr_thr, &c->amr_lv,
                      &c->sort_status, &c->ranges, &c->layers, &c->sse_part,
                      &c->sse_cnt, &c->keys_e, &c->vals_e, &c->pair_count, &c->cum, &c->chunk_start};
    for (DevBuf *b : bufs)
        if (b->p) (void)hipFree(b->p);
    if (c->pinned) (void)hipHostFree(c->pinned);
    if (c->h_total) (void)hipHostFree(c->h_total);
    if (c->h_sig) (void)hipHostFree(c->h_sig);
    if (c->upload_done) (void)hipEventDestroy(c->upload_done);
    if (c->total_ready) (void)hipEventDestroy(c->total_ready);
    if (c->total_ready_block) (void)hipEventDestroy(c->total_ready_block);
    if (c->sync_block) (void)hipEventDestroy(c->sync_block);
    if (c->side) {
        (void)hipStreamSynchronize(c->side);
        (void)hipStreamDestroy(c->side);
    }
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    delete c;
}

a3fr_status a3fr_set_stream(a3fr_ctx *c, void *hip_stream) {
    if (!c) return A3FR_EINVAL;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    return A3FR_OK;
}

a3fr_status a3fr_set_debug(a3fr_ctx *c, int32_t keep_emission_order) {
    if (!c) return A3FR_EINVAL;
    c->keep_emission = keep_emission_order != 0;
    return A3FR_OK;
}

a3fr_status a3fr_set_profiling(a3fr_ctx *c, int32_t enable) {
    if (!c) return A3FR_EINVAL;
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    c->profiling = enable != 0;
    c->count_pairs = enable == 1;
    c->ev_used = 0;
    c->ev_marks.clear();
    c->prof_sort_keys = c->prof_sort_passes = 0;
    return A3FR_OK;
}

a3fr_status a3fr_get_profile(a3fr_ctx *c, a3fr_profile *out) {
    if (!c || !out) return A3FR_EINVAL;
    std::memset(out, 0, sizeof(*out));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    for (auto &m : c->ev_marks) {
        float ms = 0.0f;
        HIPCHECK(c, hipEventElapsedTime(&ms, c->ev_pool[m.second], c->ev_pool[m.second + 1]));
        out->ms[m.first] += ms;
        out->launches[m.first] += 1;
    }
    out->sort_keys = c->prof_sort_keys;
    out->sort_passes = c->prof_sort_passes;
    if (c->pairs_armed) {
        unsigned long long pc = 0;
        HIPCHECK(c, hipMemcpy(&pc, c->pair_count.p, sizeof(pc), hipMemcpyDeviceToHost));
        out->blend_pairs = (int64_t)pc;
        c->pairs_armed = false;
    }
    c->ev_used = 0;
    c->ev_marks.clear();
    c->prof_sort_keys = c->prof_sort_passes = 0;
    return A3FR_OK;
}

a3fr_status a3fr_set_host_wait(a3fr_ctx *c, int32_t blocking) {
    if (!c) return A3FR_EINVAL;
    if (blocking != 0 && blocking != 1) return fail(c, A3FR_EINVAL, "set_host_wait: blocking must be 0 or 1");
    if (blocking) {
        const unsigned fl = hipEventBlockingSync | hipEventDisableTiming;
        if (!c->total_ready_block) HIPCHECK(c, hipEventCreateWithFlags(&c->total_ready_block, fl));
        if (!c->sync_block) HIPCHECK(c, hipEventCreateWithFlags(&c->sync_block, fl));
    }
    c->block_wait = blocking != 0;
    return A3FR_OK;
}

a3fr_status a3fr_sync(a3fr_ctx *c) {
    if (!c) return A3FR_EINVAL;
    if (c->block_wait) {
        HIPCHECK(c, hipEventRecord(c->sync_block, c->stream));
        HIPCHECK(c, hipEventSynchronize(c->sync_block));
    }
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    HIPCHECK(c, hipGetLastError());
    if (c->scalars.p) {
        uint32_t flag = 0;
        HIPCHECK(c, hipMemcpy(&flag, sc_err(c->scalars), sizeof(uint32_t), hipMemcpyDeviceToHost));
        if (flag & 6u) {
            launch_fill_u32(sc_err(c->scalars), 0u, 1, c->stream);
            HIPCHECK(c, hipStreamSynchronize(c->stream));
            return fail(c, A3FR_ECAPACITY, "key or entry count exceeded the graph's capacity (frame incomplete)");
        }
        if (flag & 1u) return fail(c, A3FR_EDEVICE, "a scan's look-back gave up waiting (internal error)");
    }
    return A3FR_OK;
}

static a3fr_status preprocess_layout(a3fr_ctx *c, int64_t n, const a3fr_view *views, int32_t nv);
static a3fr_status preprocess_kernels(a3fr_ctx *c, const a3fr_scene *scene, int32_t keep_num, int32_t keep_den);
static a3fr_status entry_stages(a3fr_ctx *c, const a3fr_scene *scene, bool zeroed = false, bool map_mode = false);

a3fr_status a3fr_preprocess(a3fr_ctx *c, const a3fr_scene *scene, const a3fr_view *views, int32_t nv,
                            int32_t keep_num, int32_t keep_den) {
    if (!c) return A3FR_EINVAL;
    TRY(check_scene(c, scene));
    if (!views || nv < 1 || nv > kMaxViews) return fail(c, A3FR_EINVAL, "n_views must be in [1, 384]");
    bool any_sel = false;
    for (int k = 0; k < nv; ++k) {
        TRY(check_view(c, views[k], k));
        any_sel |= views[k].select != 0;
    }
    if (any_sel && (keep_den <= 0 || keep_num < 0 || keep_num > keep_den))
        return fail(c, A3FR_EINVAL, "keep fraction must satisfy 0 <= keep_num <= keep_den, keep_den > 0");
    // views of one eye share pose
    for (int k = 0; k < nv; ++k)
        for (int j = 0; j < k; ++j)
            if (views[j].eye == views[k].eye &&
                (std::memcmp(views[j].R, views[k].R, sizeof(views[k].R)) != 0 ||
                 std::memcmp(views[j].t, views[k].t, sizeof(views[k].t)) != 0 ||
                 std::memcmp(views[j].campos, views[k].campos, sizeof(views[k].campos)) != 0))
                return fail(c, A3FR_EINVAL, "views with the same eye must share R, t and campos");
    const int64_t n = scene->n;
    if (!c->inc_mode) c->inc_ready = false;  // another frame reuses the buffers of the rounds
    c->records_pending = false;
    if (c->capturing) {
        // the view table of each replay is uploaded by a3fr_graph_launch; the layout is the warm-up's
        if (nv != c->nv || n != c->n) return fail(c, A3FR_EINVAL, "graph capture: frame layout changed");
    } else {
        TRY(preprocess_layout(c, n, views, nv));
    }
    return preprocess_kernels(c, scene, keep_num, keep_den);
}

static a3fr_status preprocess_layout(a3fr_ctx *c, int64_t n, const a3fr_view *views, int32_t nv) {
    // ---- frame layout
    c->hviews.resize(nv);
    c->hrow_view.clear();
    c->hrow_y.clear();
    c->hsel_views.clear();
    c->hgroups.clear();
    for (int k = 0; k < nv; ++k)
        if (k == 0 || views[k].eye != views[k - 1].eye) c->hgroups.push_back(k);
    c->hgroups.push_back(nv);
    int64_t toff = 0, ioff = 0, moff = 0, coff = 0;
    int max_tx = 1, nrect = 0;
    for (int k = 0; k < nv; ++k) {
        DevView &d = c->hviews[k];
        std::memset(&d, 0, sizeof(d));
        d.v = views[k];
        d.tiles_x = (views[k].width + kTile - 1) / kTile;
        // float64, same operations as the key path's definition (no contraction in this file)
        d.limx = (1.3 * (0.5 * (double)views[k].width)) / views[k].fx;
        d.limy = (1.3 * (0.5 * (double)views[k].height)) / views[k].fy;
        d.tiles_y = (views[k].height + kTile - 1) / kTile;
        d.ax0 = 0; d.ax1 = d.tiles_x - 1; d.ay0 = 0; d.ay1 = d.tiles_y - 1;
        if (views[k].mask != A3FR_MASK_ALL) {
            // an active tile's pixel-centre rectangle comes within r_out of the gaze
            const double r = views[k].r_out, gx = views[k].gx, gy = views[k].gy, t = (double)kTile;
            if (!(r >= 0.0)) {
                d.ax0 = 1; d.ax1 = 0;
            } else {
                // clamped in float64 to [-1, tiles] before the conversion
                const auto cl = [](double v, int hi) { return (int32_t)std::min(std::max(v, -1.0), (double)hi); };
                d.ax0 = std::max(0, cl(std::floor((gx - r - (t - 0.5)) / t) - 1.0, d.tiles_x));
                d.ax1 = std::min(d.tiles_x - 1, cl(std::floor((gx + r - 0.5) / t) + 1.0, d.tiles_x));
                d.ay0 = std::max(0, cl(std::floor((gy - r - (t - 0.5)) / t) - 1.0, d.tiles_y));
                d.ay1 = std::min(d.tiles_y - 1, cl(std::floor((gy + r - 0.5) / t) + 1.0, d.tiles_y));
            }
        }
        d.tile_off = toff;
        d.img_off = ioff;
        d.mask_off = views[k].mask == A3FR_MASK_ALL ? -1 : moff;
        d.cum_off = views[k].mask == A3FR_MASK_ALL ? -1 : coff;
        if (views[k].mask != A3FR_MASK_ALL) coff += (int64_t)(d.tiles_y + 1) * (d.tiles_x + 1);
        if (d.tiles_x > max_tx) max_tx = d.tiles_x;
        d.sel_slot = views[k].select ? (int32_t)c->hsel_views.size() : -1;
        bool fb_periph = false;
        for (const auto &fp : c->fb_plan) {
            if (fp.fv == k) d.remask = 1;
            if (fp.pv == k) fb_periph = true;
        }
        if (c->inc_mode) {
            if (k % 3 != 2) d.remask = 1;  // fovea and mid layers: their masks change between rounds
            d.round_flags = k < (int)c->inc_flags.size() ? c->inc_flags[k] : 0;
            d.keep_visible = c->inc_round0 && d.remask ? 1 : 0;
        }
        // rectangles of every slot: views recounted after the projection, and the
        // fallback's periphery views (their mass maps)
        d.rect_slot = d.remask || fb_periph ? nrect++ : -1;
        if (views[k].select) c->hsel_views.push_back(k);
        if (views[k].mask != A3FR_MASK_ALL) moff += (int64_t)d.tiles_y * (d.tiles_x + 1);
        for (int ty = 0; ty < d.tiles_y; ++ty) {
            c->hrow_view.push_back(k);
            c->hrow_y.push_back(ty);
        }
        toff += (int64_t)d.tiles_x * d.tiles_y;
        ioff += (int64_t)views[k].width * views[k].height;
    }
    if (toff >= (int64_t(1) << 31)) return fail(c, A3FR_ECAPACITY, "more than 2^31 tiles in one frame");
    c->nv = nv;
    c->n = n;
    c->ntiles = toff;
    c->npix = ioff;
    c->nsel = (int)c->hsel_views.size();
    c->rows_total = (int64_t)c->hrow_view.size();
    c->mask_entries = moff;
    c->cum_entries = coff;
    c->max_tiles_x = max_tx;
    c->nrect = nrect;
    c->preprocessed = false;
    c->sorted = false;
    c->blend_bwd_done = false;

    // ---- workspace
    const int64_t m = (int64_t)nv * n;
    if (m >= (int64_t(1) << 32)) return fail(c, A3FR_ECAPACITY, "more than 2^32 - 1 (view, Gaussian) slots");
    TRY(ensure(c, c->row_prefix, sizeof(uint16_t) * moff));
    TRY(ensure(c, c->row_list, sizeof(uint16_t) * moff));
    TRY(ensure(c, c->cum, sizeof(uint32_t) * coff));
    TRY(ensure(c, c->active, (size_t)toff));
    TRY(ensure(c, c->counts, sizeof(uint32_t) * m));
    TRY(ensure(c, c->depth, sizeof(uint32_t) * m));
    TRY(ensure(c, c->map, sizeof(uint32_t) * m));
    TRY(ensure(c, c->rect, sizeof(uint64_t) * (size_t)nrect * n));
    TRY(ensure(c, c->score, sizeof(double) * (size_t)c->nsel * n));
    TRY(ensure(c, c->keep, c->nsel ? (size_t)m : 16));
    TRY(ensure(c, c->sel, sizeof(uint32_t) * (size_t)select_workspace_words(c->nsel, n)));
    TRY(ensure(c, c->offsets, sizeof(uint32_t) * (m + 1)));
    TRY(ensure(c, c->block_sums, sizeof(uint64_t) * (size_t)scan_workspace_words(m)));
    if (!c->scalars.p) {
        TRY(ensure(c, c->scalars, 64));
        launch_fill_u32(P<uint32_t>(c->scalars), 0u, 16, c->stream);
    }
    TRY(ensure(c, c->ent_a, sizeof(uint32_t) * m));
    TRY(ensure(c, c->ecnt, sizeof(uint32_t) * m));
    TRY(ensure(c, c->gpack, sizeof(GeomPack) * (size_t)n));
    if (c->inc_mode) TRY(ensure(c, c->ent_b, sizeof(uint32_t) * m));
    TRY(ensure(c, c->dkey_a, sizeof(uint32_t) * m));
    TRY(ensure(c, c->dkey_b, sizeof(uint32_t) * m));
    TRY(ensure(c, c->dval_a, sizeof(uint32_t) * m));
    TRY(ensure(c, c->dval_b, sizeof(uint32_t) * m));
    TRY(ensure(c, c->sort_status, sizeof(uint32_t) * (size_t)onesweep_workspace_words(m, 4)));

    // ---- one upload through pinned staging:
    // [views | row views | row ys | selecting views | groups | exp(k/16) table of the footprint bound]
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t bytes_v = sizeof(DevView) * nv, bytes_r = sizeof(int32_t) * c->rows_total,
                 bytes_s = sizeof(int32_t) * (c->nsel + 1), bytes_g = sizeof(int32_t) * c->hgroups.size(),
                 bytes_e = sizeof(double) * (kExtentSteps + 1);
    const size_t o_rv = al(bytes_v), o_ry = o_rv + al(bytes_r), o_sv = o_ry + al(bytes_r), o_gr = o_sv + al(bytes_s),
                 o_ex = o_gr + al(bytes_g), total = o_ex + al(bytes_e);
    TRY(ensure(c, c->views, total));
    TRY(ensure_pinned(c, total));
    char *pin = static_cast<char *>(c->pinned);
    std::memcpy(pin, c->hviews.data(), bytes_v);
    std::memcpy(pin + o_rv, c->hrow_view.data(), bytes_r);
    std::memcpy(pin + o_ry, c->hrow_y.data(), bytes_r);
    if (c->nsel) std::memcpy(pin + o_sv, c->hsel_views.data(), sizeof(int32_t) * c->nsel);
    std::memcpy(pin + o_gr, c->hgroups.data(), bytes_g);
    double *ex_tab = reinterpret_cast<double *>(pin + o_ex);
    for (int k = 0; k <= kExtentSteps; ++k) ex_tab[k] = std::exp((double)k / 16.0);
    HIPCHECK(c, hipMemcpyAsync(c->views.p, pin, total, hipMemcpyHostToDevice, c->stream));
    HIPCHECK(c, hipEventRecord(c->upload_done, c->stream));
    char *frame = static_cast<char *>(c->views.p);
    c->d_row_view = reinterpret_cast<const int32_t *>(frame + o_rv);
    c->d_row_y = reinterpret_cast<const int32_t *>(frame + o_ry);
    c->d_sel_views = reinterpret_cast<const int32_t *>(frame + o_sv);
    c->d_groups = reinterpret_cast<const int32_t *>(frame + o_gr);
    c->d_exp_tab = reinterpret_cast<const double *>(frame + o_ex);
    return A3FR_OK;
}

static a3fr_status preprocess_kernels(a3fr_ctx *c, const a3fr_scene *scene, int32_t keep_num, int32_t keep_den) {
    const int64_t n = c->n;
    const int nv = c->nv;
    const int64_t toff = c->ntiles;
    const int32_t *d_row_view = c->d_row_view, *d_row_y = c->d_row_y, *d_sel_views = c->d_sel_views,
                  *d_groups = c->d_groups;
    c->preprocessed = false;
    c->sorted = false;
    c->blend_bwd_done = false;
    c->sh_degree = scene->sh_degree;

    // the fallback pairs (periphery view, its eye's full-resolution view); their
    // difference planes [2][tiles_y + 1][tiles_x + 1] (doubles) go in batches of
    // up to kFbMax per launch
    const bool do_fb = !c->fb_plan.empty() && c->nsel;
    std::vector<FbBatch> fbs;
    int64_t dwords = 0, max_part = 0;
    if (do_fb) {
        for (const auto &fp : c->fb_plan) {
            if (fbs.empty() || fbs.back().count == kFbMax) fbs.push_back(FbBatch{});
            FbBatch &fb = fbs.back();
            const DevView &hp = c->hviews[fp.pv];
            const int cells = 2 * (hp.tiles_y + 1) * (hp.tiles_x + 1);
            fb.pv[fb.count] = fp.pv;
            fb.fv[fb.count] = fp.fv;
            fb.r_mid[fb.count] = fp.r_mid;
            fb.doff[fb.count] = dwords;
            fb.max_cells = std::max(fb.max_cells, cells);
            ++fb.count;
            dwords += cells;
            max_part = std::max<int64_t>(max_part, (int64_t)fb.count * fb.max_cells);
        }
        TRY(ensure(c, c->fb_energy, sizeof(float) * 2 * (size_t)toff));
        TRY(ensure(c, c->fb_flags, (size_t)toff));
        TRY(ensure(c, c->fb_diff, sizeof(double) * (size_t)dwords));
        TRY(ensure(c, c->fb_part, sizeof(double) * (size_t)drop_energy_parts() * (size_t)max_part));
        TRY(ensure(c, c->fb_count, 16));
    }
    // what the later stages accumulate into, cleared by the tile-mask launch:
    // the select histograms, the fallback's counters and planes, the scans'
    // tickets and status words, the depth sort's digit counts and pass
    // counters (its histogram kernel clears the status words of the
    // partitions in use)
    FillSegs z{};
    {
        const int64_t m = (int64_t)nv * n;
        const auto add = [&z](void *p, int64_t words) {
            z.p[z.count] = reinterpret_cast<uint32_t *>(p);
            z.n[z.count] = words;
            ++z.count;
        };
        if (c->nsel) add(c->sel.p, select_hist_words(c->nsel));
        if (do_fb) {
            add(c->fb_count.p, 1);
            add(c->fb_energy.p, 2 * toff);
            add(c->fb_diff.p, 2 * dwords);
        }
        add(c->block_sums.p, 2 * scan_workspace_words(m));
        add(c->sort_status.p, onesweep_zero_words(4));
    }

    // ---- kernels
    const DevView *dv = P<DevView>(c->views);
    { StageTimer t_(c, A3FR_STAGE_MASKS);
    launch_tile_masks(dv, nv, c->rows_total, d_row_view, d_row_y,
                      P<uint16_t>(c->row_prefix), P<uint16_t>(c->row_list), P<uint8_t>(c->active), nullptr, z,
                      c->stream);
      if (c->cum_entries) launch_mask_cum(dv, nv, c->max_tiles_x, P<uint16_t>(c->row_prefix), P<uint32_t>(c->cum), c->stream); }
    { StageTimer t_(c, A3FR_STAGE_PREPROCESS);
    launch_preprocess(*scene, dv, (int)c->hgroups.size() - 1, d_groups, P<uint32_t>(c->cum), P<uint32_t>(c->counts),
                      P<uint32_t>(c->depth), P<uint64_t>(c->rect), P<double>(c->score), P<GeomPack>(c->gpack),
                      c->d_exp_tab, c->stream); }
    if (c->nsel) { StageTimer t_(c, A3FR_STAGE_SELECT);
        launch_select(dv, nv, d_sel_views, c->nsel, n, P<uint32_t>(c->counts), P<double>(c->score),
                      keep_num, keep_den, P<uint32_t>(c->sel), P<uint8_t>(c->keep), c->stream, true); }
    c->fb_last = false;
    c->amr_last = false;
    if (do_fb) {
        // periphery error estimate; flagged tiles join the full-resolution layer's mask; recount it
        StageTimer t_(c, A3FR_STAGE_FALLBACK);
        for (const FbBatch &fb : fbs) {
            launch_drop_energy(dv, fb, n, P<uint32_t>(c->counts), P<uint8_t>(c->keep), P<uint64_t>(c->rect),
                               P<double>(c->score), P<double>(c->fb_diff), P<double>(c->fb_part), toff,
                               P<float>(c->fb_energy), c->fb_thr, c->fb_coef, c->fb_pow, P<uint8_t>(c->fb_flags),
                               P<uint8_t>(c->active), P<uint32_t>(c->fb_count), c->stream);
        }
        launch_rows_from_active(dv, c->rows_total, d_row_view, d_row_y, P<uint8_t>(c->active),
                                P<uint16_t>(c->row_prefix), P<uint16_t>(c->row_list), P<uint32_t>(c->fb_count),
                                c->stream);
        if (c->cum_entries)
            launch_mask_cum(dv, nv, c->max_tiles_x, P<uint16_t>(c->row_prefix), P<uint32_t>(c->cum), c->stream,
                            P<uint32_t>(c->fb_count));
        for (const FbBatch &fb : fbs)
            launch_recount(dv, fb, n, P<uint64_t>(c->rect), P<uint16_t>(c->row_prefix), P<uint32_t>(c->counts),
                           P<uint32_t>(c->fb_count), c->stream);
        c->fb_last = true;
    }
    return entry_stages(c, scene, true);
}

// The record pass: records and rectangles of the entries ent_a[0 .. E) (E on
// the device, at most cap of them written; a larger E is reported by bit 2 of
// the error word) and the slot -> record map.
static void launch_records(a3fr_ctx *c, const a3fr_scene &scene, int64_t cap) {
    StageTimer t_(c, A3FR_STAGE_COLOUR);
    launch_entry_record(scene, P<GeomPack>(c->gpack), P<DevView>(c->views), P<uint32_t>(c->ent_a),
                        sc_n_ent(c->scalars), (int64_t)c->nv * c->n, cap, c->d_exp_tab, P<Record>(c->rec),
                        P<uint64_t>(c->rect_e), P<uint32_t>(c->map), sc_err(c->scalars), c->stream);
}

// Sizes the record arrays for cap records.
static a3fr_status ensure_records(a3fr_ctx *c, int64_t cap) {
    TRY(ensure(c, c->rec, sizeof(Record) * (size_t)cap));
    TRY(ensure(c, c->rect_e, sizeof(uint64_t) * (size_t)cap));
    return A3FR_OK;
}

// Records held by the record arrays (without growing them).
static int64_t record_capacity(const a3fr_ctx *c) {
    return (int64_t)std::min(c->rec.cap / sizeof(Record), c->rect_e.cap / sizeof(uint64_t));
}

// The entries of one emission: compaction of the slots that have keys (kept)
// into ent (ent_a when this pass makes the records, ent_b when the records come
// from an earlier pass: map_mode), their stable sort by depth, and their key
// offsets in depth order.  With scene set the records are formed for these
// entries in a3fr_bin_sort.  zeroed: the scan and depth-sort workspaces were
// cleared by the frame's first clearing launch.  visible_pass: before that, a
// compaction keeping every visible slot of the keep_visible views, whose
// records are formed at once (the first round of an incremental frame).
static a3fr_status entry_stages(a3fr_ctx *c, const a3fr_scene *scene, bool zeroed, bool map_mode) {
    const int64_t n = c->n;
    const int nv = c->nv;
    const int64_t m = (int64_t)nv * n;
    const DevView *dv = P<DevView>(c->views);
    c->records_pending = false;
    c->map_mode = map_mode;
    const bool visible_pass = c->inc_round0;
    if (visible_pass) {
        // every visible entry of the fovea and mid layers gets its record now, for the later rounds
        {
            StageTimer t_(c, A3FR_STAGE_SCAN);
            launch_compact_entries(P<uint32_t>(c->counts), c->nsel ? P<uint8_t>(c->keep) : nullptr,
                                   P<uint64_t>(c->rect), dv, nv, n, P<uint32_t>(c->depth), P<uint32_t>(c->ent_a),
                                   P<uint32_t>(c->dkey_b),
                                   P<uint32_t>(c->dval_b), nullptr, P<uint64_t>(c->block_sums), sc_ent_total(c->scalars),
                                   sc_n_ent(c->scalars), sc_err(c->scalars), c->stream, zeroed);
        }
        uint32_t E = 0;
        HIPCHECK(c, hipMemcpyAsync(&E, sc_n_ent(c->scalars), 4, hipMemcpyDeviceToHost, c->stream));
        HIPCHECK(c, hipStreamSynchronize(c->stream));
        TRY(ensure_records(c, E));
        launch_records(c, *scene, E);
        c->n_rec = E;
        // the compaction below reuses the scan workspace
        launch_fill_u32(reinterpret_cast<uint32_t *>(c->block_sums.p), 0u, 2 * scan_workspace_words(m), c->stream);
        zeroed = true;
        scene = nullptr;
        map_mode = c->map_mode = true;
    }
    DevBuf &ent = map_mode ? c->ent_b : c->ent_a;
    {
        StageTimer t_(c, A3FR_STAGE_SCAN);
        // (keep_visible views count as such only in the visible pass)
        launch_compact_entries(P<uint32_t>(c->counts), c->nsel ? P<uint8_t>(c->keep) : nullptr,
                               visible_pass ? nullptr : P<uint64_t>(c->rect),
                               dv, nv, n, P<uint32_t>(c->depth), P<uint32_t>(ent), P<uint32_t>(c->dkey_a),
                               P<uint32_t>(c->dval_a), P<uint32_t>(c->ecnt), P<uint64_t>(c->block_sums),
                               sc_ent_total(c->scalars),
                               sc_n_ent(c->scalars), sc_err(c->scalars), c->stream, zeroed);
    }
    if (scene) {
        c->rec_scene = *scene;
        c->records_pending = true;
    }
    {   // stable sort of the entries by depth (4 passes: even, ends in the "a" buffers)
        StageTimer t_(c, A3FR_STAGE_DEPTH_SORT);
        launch_onesweep_prepare(P<uint32_t>(c->dkey_a), sc_n_ent(c->scalars), m, 4, P<uint32_t>(c->sort_status),
                                c->stream, zeroed);
        uint32_t *ki = P<uint32_t>(c->dkey_a), *ko = P<uint32_t>(c->dkey_b);
        uint32_t *vi = P<uint32_t>(c->dval_a), *vo = P<uint32_t>(c->dval_b);
        for (int p = 0; p < 4; ++p) {
            launch_onesweep_pass(ki, vi, ko, vo, sc_n_ent(c->scalars), m, 4, p, P<uint32_t>(c->sort_status),
                                 sc_err(c->scalars), c->stream);
            std::swap(ki, ko);
            std::swap(vi, vo);
        }
    }
    {
        StageTimer t_(c, A3FR_STAGE_SCAN);
        // outside graph mode (no host read-back there) and blocking host waits
        // (they sleep on an event), the totals go straight to the host
        c->sig_pending = c->d_sig && c->capacity <= 0 && !c->block_wait;
        if (c->sig_pending) ++c->sig_seq;
        launch_key_offsets(P<uint32_t>(c->ecnt), P<uint32_t>(c->dval_a), sc_n_ent(c->scalars), m,
                           P<uint32_t>(c->offsets), P<uint64_t>(c->block_sums), sc_key_total(c->scalars),
                           sc_n_keys(c->scalars), sc_err(c->scalars), c->sig_pending ? c->d_sig : nullptr,
                           c->sig_seq, c->stream);
    }
    TRY(check_launch(c, "preprocess"));
    c->preprocessed = true;
    return A3FR_OK;
}

// Waits (polling) until the key-offsets kernel of this frame has written the
// totals and their sequence number to host-coherent memory.  The stream is
// queried every few thousand polls: when it has completed (or failed) the
// words are there (or never will be), so the wait always ends.
static a3fr_status wait_sig(a3fr_ctx *c, uint64_t *E, uint64_t *K) {
    volatile uint64_t *h = c->h_sig;
    for (uint32_t it = 1;; ++it) {
        if (h[2] == c->sig_seq) break;
        if ((it & 4095u) == 0) {
            const hipError_t q = hipStreamQuery(c->stream);
            if (q == hipSuccess) {
                if (h[2] == c->sig_seq) break;
                return fail(c, A3FR_EDEVICE, "the key totals did not reach the host");
            }
            if (q != hipErrorNotReady) {
                (void)hipGetLastError();
                return fail(c, A3FR_EDEVICE, std::string("waiting for the key totals: ") + hipGetErrorString(q));
            }
        }
        __builtin_ia32_pause();
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    *E = h[0];
    *K = h[1];
    return A3FR_OK;
}

a3fr_status a3fr_bin_sort(a3fr_ctx *c, int64_t *n_keys_out) {
    if (!c) return A3FR_EINVAL;
    if (!c->preprocessed) return fail(c, A3FR_ENOTREADY, "a3fr_bin_sort before a3fr_preprocess");
    uint64_t K = 0, E = 0;
    const bool cap_mode = c->capacity > 0;
    const bool recs = c->records_pending;
    c->records_pending = false;
    if (cap_mode) {
        // graph mode: no host read-back; buffers sized to the capacities, counts clamped on the device
        K = (uint64_t)c->capacity;
        E = (uint64_t)c->ecap;
        if (recs) {
            TRY(ensure_records(c, (int64_t)E));
            launch_records(c, c->rec_scene, (int64_t)E);
            c->n_rec = -1;
        }
        if (n_keys_out) *n_keys_out = -1;
    } else {
        // the entry and key totals: written to host-coherent memory by the
        // key-offsets kernel (sig_pending), else read back by a copy (scalars
        // [0], [1]) and an event; the records are formed meanwhile into the
        // arrays as they are (formed again after the wait if they turn out too
        // small)
        const bool sig = c->sig_pending;
        c->sig_pending = false;
        hipEvent_t ready = c->block_wait ? c->total_ready_block : c->total_ready;
        if (!sig) {
            HIPCHECK(c, hipMemcpyAsync(c->h_total, sc_ent_total(c->scalars), 2 * sizeof(uint64_t),
                                       hipMemcpyDeviceToHost, c->stream));
            HIPCHECK(c, hipEventRecord(ready, c->stream));
        }
        const int64_t cap0 = recs ? record_capacity(c) : 0;
        if (cap0 > 0) {
            StageTimer t_(c, A3FR_STAGE_COLOUR);
            launch_entry_record(c->rec_scene, P<GeomPack>(c->gpack), P<DevView>(c->views), P<uint32_t>(c->ent_a),
                                sc_n_ent(c->scalars), (int64_t)c->nv * c->n, cap0, c->d_exp_tab, P<Record>(c->rec),
                                P<uint64_t>(c->rect_e), P<uint32_t>(c->map), nullptr, c->stream);
        }
        if (sig) {
            TRY(wait_sig(c, &E, &K));
        } else {
            HIPCHECK(c, hipEventSynchronize(ready));
            E = c->h_total[0];
            K = c->h_total[1];
        }
        if (recs) {
            if ((int64_t)E > cap0) {
                TRY(ensure_records(c, (int64_t)E));
                launch_records(c, c->rec_scene, (int64_t)E);
            }
            c->n_rec = (int64_t)E;
        }
        c->n_ent_pass = (int64_t)E;
        if (n_keys_out) *n_keys_out = (int64_t)K;
        if (K >= (uint64_t(1) << 32))
            return fail(c, A3FR_ECAPACITY, "key count reached 2^32: " + std::to_string(K));
    }
    TRY(ensure(c, c->rect_s, sizeof(uint64_t) * (size_t)E));
    TRY(ensure(c, c->esort, sizeof(uint32_t) * (size_t)E));
    TRY(ensure(c, c->rsort, sizeof(uint32_t) * (size_t)E));
    const int64_t m = (int64_t)c->nv * c->n;
    TRY(ensure(c, c->keys_a, sizeof(uint32_t) * K));
    TRY(ensure(c, c->keys_b, sizeof(uint32_t) * K));
    TRY(ensure(c, c->vals_a, sizeof(uint32_t) * K));
    TRY(ensure(c, c->vals_b, sizeof(uint32_t) * K));
    TRY(ensure(c, c->chunk_start, sizeof(uint32_t) * (emit_chunks((int64_t)K) + 1)));
    int tile_bits = 1;
    while ((int64_t(1) << tile_bits) < c->ntiles) ++tile_bits;
    const int npass = (tile_bits + 7) / 8;
    TRY(ensure(c, c->sort_status, sizeof(uint32_t) * (size_t)sort_workspace_words((int64_t)K)));
    TRY(ensure(c, c->ranges, sizeof(uint32_t) * 2 * c->ntiles));
    const DevView *dv = P<DevView>(c->views);
    if (cap_mode)
        launch_clamp_keys(sc_key_total(c->scalars), c->capacity, sc_n_ent(c->scalars), P<uint32_t>(c->offsets),
                          c->ecap, sc_n_keys(c->scalars), sc_err(c->scalars), c->stream);
    {
        StageTimer t_(c, A3FR_STAGE_EMIT);
        EmitEntries ee{};
        ee.order = P<uint32_t>(c->dval_a);
        ee.ent = c->map_mode ? P<uint32_t>(c->ent_b) : P<uint32_t>(c->ent_a);
        ee.map = c->map_mode ? P<uint32_t>(c->map) : nullptr;
        ee.rect_e = P<uint64_t>(c->rect_e);
        ee.rect_s = P<uint64_t>(c->rect_s);
        ee.esort = P<uint32_t>(c->esort);
        ee.rsort = P<uint32_t>(c->rsort);
        ee.cap = (int64_t)E;
        launch_emit(dv, c->nv, c->n, m, ee, sc_n_ent(c->scalars), P<uint32_t>(c->offsets), P<uint16_t>(c->row_prefix),
                    P<uint16_t>(c->row_list), P<uint32_t>(c->cum), P<uint32_t>(c->chunk_start),
                    P<uint32_t>(c->keys_a), P<uint32_t>(c->vals_a), (int64_t)K,
                    cap_mode ? sc_n_keys(c->scalars) : nullptr, P<uint32_t>(c->sort_status),
                    (int)sort_zero_words((int64_t)K), c->stream);
    }
    if (c->keep_emission && !cap_mode) {
        TRY(ensure(c, c->keys_e, sizeof(uint32_t) * K));
        TRY(ensure(c, c->vals_e, sizeof(uint32_t) * K));
        HIPCHECK(c, hipMemcpyAsync(c->keys_e.p, c->keys_a.p, sizeof(uint32_t) * K, hipMemcpyDeviceToDevice, c->stream));
        HIPCHECK(c, hipMemcpyAsync(c->vals_e.p, c->vals_a.p, sizeof(uint32_t) * K, hipMemcpyDeviceToDevice, c->stream));
    }
    uint32_t *ki = P<uint32_t>(c->keys_a), *ko = P<uint32_t>(c->keys_b);
    uint32_t *vi = P<uint32_t>(c->vals_a), *vo = P<uint32_t>(c->vals_b);
    bool in_b = false;
    if (K > 1) {
        // the tickets and group sums were cleared by the emission's first kernel
        for (int p = 0; p < npass; ++p) {
            {
                StageTimer t_(c, A3FR_STAGE_SORT_HIST);
                launch_sort_count(ki, sc_n_keys(c->scalars), (int64_t)K, p, P<uint32_t>(c->sort_status), c->stream);
            }
            {
                StageTimer t_(c, A3FR_STAGE_SORT_PASS);
                launch_sort_scatter(ki, vi, ko, vo, sc_n_keys(c->scalars), (int64_t)K, p, P<uint32_t>(c->sort_status),
                                    c->stream);
            }
            std::swap(ki, ko);
            std::swap(vi, vo);
            in_b = !in_b;
        }
        if (c->profiling && !cap_mode) { c->prof_sort_keys += (int64_t)K; c->prof_sort_passes += npass; }
    }
    c->sorted_in_b = in_b;
    c->K = cap_mode ? -1 : (int64_t)K;
    {
        StageTimer t_(c, A3FR_STAGE_RANGES);
        launch_ranges(in_b ? P<uint32_t>(c->keys_b) : P<uint32_t>(c->keys_a), (int64_t)K,
                      cap_mode ? sc_n_keys(c->scalars) : nullptr, c->ntiles,
                      P<uint32_t>(c->ranges), c->stream);
    }
    TRY(check_launch(c, "bin_sort"));
    c->sorted = true;
    c->blend_bwd_done = false;
    return A3FR_OK;
}

}  // extern "C"

namespace {
const uint32_t *sorted_tiles(a3fr_ctx *c) {
    return c->sorted_in_b ? P<uint32_t>(c->keys_b) : P<uint32_t>(c->keys_a);
}
const uint32_t *sorted_vals(a3fr_ctx *c) {
    return c->sorted_in_b ? P<uint32_t>(c->vals_b) : P<uint32_t>(c->vals_a);
}
}  // namespace

extern "C" {

static a3fr_status blend_with(a3fr_ctx *c, int variant, float *rgb, float *T, uint32_t *last,
                              unsigned long long *pairs, hipStream_t stream, const TileRanges *tr = nullptr) {
    TRY(ensure(c, c->blend_ws, sizeof(uint32_t) * kBlendWsWords));
    TRY(ensure(c, c->blend_order, sizeof(uint32_t) * (size_t)c->ntiles));
    BlendArgs a{};
    a.views = P<DevView>(c->views);
    a.nv = c->nv;
    a.ntiles = c->ntiles;
    a.active = P<uint8_t>(c->active);
    a.ranges = P<uint32_t>(c->ranges);
    a.vals = sorted_vals(c);
    a.rec = P<Record>(c->rec);
    a.n = 0;  // key values are record indices
    a.rgb = rgb; a.T = T; a.last = last; a.pairs = pairs;
    a.ws = P<uint32_t>(c->blend_ws);
    a.order = P<uint32_t>(c->blend_order);
    a.queue_waves = (int64_t)c->n_cus * 24;
    if (tr) a.tr = *tr;
    launch_blend(a, variant, stream);
    return check_launch(c, "blend");
}

a3fr_status a3fr_blend(a3fr_ctx *c, float *rgb, float *T, uint32_t *last) {
    if (!c) return A3FR_EINVAL;
    if (!c->sorted) return fail(c, A3FR_ENOTREADY, "a3fr_blend before a3fr_bin_sort");
    if (!rgb) return fail(c, A3FR_EINVAL, "rgb_dev is NULL");
    unsigned long long *pairs = nullptr;
    if (c->profiling && c->count_pairs) {
        TRY(ensure(c, c->pair_count, 16));
        pairs = P<unsigned long long>(c->pair_count);
        if (!c->pairs_armed) {
            launch_fill_u32(P<uint32_t>(c->pair_count), 0u, 2, c->stream);
            c->pairs_armed = true;
        }
    }
    StageTimer t_(c, A3FR_STAGE_BLEND);
    return blend_with(c, c->blend_variant, rgb, T, last, pairs, c->stream);
}

a3fr_status a3fr_set_blend_variant(a3fr_ctx *c, int32_t variant) {
    if (!c) return A3FR_EINVAL;
    if (variant < 0 || variant >= kBlendVariants) return fail(c, A3FR_EINVAL, "blend variant out of range");
    c->blend_variant = variant;
    return A3FR_OK;
}

a3fr_status a3fr_autotune_blend(a3fr_ctx *c, int32_t reps, double *ms_out, int32_t *best_out) {
    if (!c) return A3FR_EINVAL;
    if (!c->sorted) return fail(c, A3FR_ENOTREADY, "a3fr_autotune_blend needs a sorted frame (a3fr_bin_sort)");
    if (reps < 1 || reps > 1000) return fail(c, A3FR_EINVAL, "reps must be in [1, 1000]");
    TRY(ensure(c, c->tune_img, sizeof(float) * 3 * (size_t)(c->npix > 0 ? c->npix : 1)));
    hipEvent_t e0, e1;
    HIPCHECK(c, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(c, A3FR_EDEVICE, "hipEventCreate failed");
    }
    double best_ms = 1e300;
    int best = c->blend_variant;
    a3fr_status st = A3FR_OK;
    for (int k = 0; k < kBlendVariants && st == A3FR_OK; ++k) {
        st = blend_with(c, k, P<float>(c->tune_img), nullptr, nullptr, nullptr, c->stream);  // warm-up
        if (st != A3FR_OK) break;
        if (hipEventRecord(e0, c->stream) != hipSuccess) { st = fail(c, A3FR_EDEVICE, "hipEventRecord"); break; }
        for (int r = 0; r < reps && st == A3FR_OK; ++r)
            st = blend_with(c, k, P<float>(c->tune_img), nullptr, nullptr, nullptr, c->stream);
        if (st != A3FR_OK) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            st = fail(c, A3FR_EDEVICE, "event timing failed");
            break;
        }
        const double per = (double)ms / reps;
        if (ms_out) ms_out[k] = per;
        if (per < best_ms) { best_ms = per; best = k; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    TRY(st);
    c->blend_variant = best;
    if (best_out) *best_out = best;
    return A3FR_OK;
}

static void view_from_camera(const a3fr_camera &cam, int eye, a3fr_view &v) {
    std::memset(&v, 0, sizeof(v));
    std::memcpy(v.R, cam.R, sizeof(v.R));
    std::memcpy(v.t, cam.t, sizeof(v.t));
    std::memcpy(v.campos, cam.campos, sizeof(v.campos));
    v.fx = cam.fx; v.fy = cam.fy; v.cx = cam.cx; v.cy = cam.cy;
    v.width = cam.width; v.height = cam.height;
    v.eye = eye;
    v.mask = A3FR_MASK_ALL;
    v.select = 0;
    std::memcpy(v.bg, cam.bg, sizeof(v.bg));
}

a3fr_status a3fr_render_full(a3fr_ctx *c, const a3fr_scene *scene, const a3fr_camera *cams, int32_t n_cams,
                             float *out) {
    if (!c) return A3FR_EINVAL;
    if (!cams || n_cams < 1 || n_cams > kMaxEyes) return fail(c, A3FR_EINVAL, "n_cams must be in [1, 128]");
    if (!out) return fail(c, A3FR_EINVAL, "out_dev is NULL");
    std::vector<a3fr_view> v(n_cams);
    for (int e = 0; e < n_cams; ++e) view_from_camera(cams[e], e, v[e]);
    const a3fr_status st = a3fr_preprocess(c, scene, v.data(), n_cams, 1, 1);
    TRY(st);
    TRY(a3fr_bin_sort(c, nullptr));
    return a3fr_blend(c, out, nullptr, nullptr);
}

a3fr_status a3fr_render_amr(a3fr_ctx *c, const a3fr_scene *scene, const a3fr_camera *cams, const a3fr_gaze *gaze,
                            int32_t n_eyes, const a3fr_amr *amr, float *out) {
    if (!c) return A3FR_EINVAL;
    if (!cams || !gaze || !amr || !out || n_eyes < 1 || n_eyes > kMaxEyes)
        return fail(c, A3FR_EINVAL, "render_amr: bad arguments");
    const double *r = amr->r_level, *f = amr->count_frac;
    if (amr->level_mode < 0 || amr->level_mode > 2) return fail(c, A3FR_EINVAL, "render_amr: level_mode must be 0, 1 or 2");
    if (amr->fill < 0 || amr->fill > 1) return fail(c, A3FR_EINVAL, "render_amr: fill must be 0 or 1");
    if (amr->level_mode != 1 && (!(r[0] >= 0.0) || !(r[1] >= r[0]) || !(r[2] >= r[1]) || !is_fin(r[2])))
        return fail(c, A3FR_EINVAL, "render_amr: radii must satisfy 0 <= r_level[0] <= r_level[1] <= r_level[2]");
    if (amr->level_mode != 0 && (!(f[0] >= 0.0) || !(f[1] >= f[0]) || !(f[2] >= f[1]) || !(f[2] <= 1.0)))
        return fail(c, A3FR_EINVAL,
                    "render_amr: fractions must satisfy 0 <= count_frac[0] <= count_frac[1] <= count_frac[2] <= 1");
    std::vector<a3fr_view> v(n_eyes);
    for (int e = 0; e < n_eyes; ++e) {
        view_from_camera(cams[e], e, v[e]);
        v[e].gx = gaze[e].x;
        v[e].gy = gaze[e].y;
        if (!is_fin(gaze[e].x) || !is_fin(gaze[e].y)) return fail(c, A3FR_EINVAL, "render_amr: gaze not finite");
    }
    const a3fr_status st = a3fr_preprocess(c, scene, v.data(), n_eyes, 1, 1);
    TRY(st);
    TRY(a3fr_bin_sort(c, nullptr));
    TRY(ensure(c, c->amr_thr, sizeof(uint64_t) * 3 * (size_t)c->nv));
    TRY(ensure(c, c->amr_lv, (size_t)c->ntiles));
    int64_t max_pixels = 0;
    for (int e = 0; e < n_eyes; ++e) max_pixels = std::max(max_pixels, (int64_t)cams[e].width * cams[e].height);
    AmrLevels a{};
    const bool ecc = amr->level_mode != 1;  // radii unused by the count levels
    for (int q = 0; q < 3; ++q) {
        a.r[q] = ecc ? r[q] : 0.0;
        a.f[q] = f[q];
    }
    a.mode = amr->level_mode;
    a.interp = amr->fill;
    StageTimer t_(c, A3FR_STAGE_BLEND);
    launch_blend_amr(P<DevView>(c->views), c->nv, c->ntiles, P<uint32_t>(c->ranges), sorted_vals(c), P<Record>(c->rec),
                     0, a, P<uint64_t>(c->amr_thr), P<uint8_t>(c->amr_lv), out, max_pixels, c->stream);
    c->amr_last = true;
    return check_launch(c, "render_amr");
}

a3fr_status a3fr_make_foveated_views(const a3fr_camera *cams, const a3fr_gaze *gaze, int32_t n_eyes,
                                     const a3fr_fovea *f, a3fr_view *out) {
    if (!cams || !gaze || !f || !out || n_eyes < 1 || n_eyes > kMaxEyes) return A3FR_EINVAL;
    if (f->scale_mid < 1 || f->scale_periph < 1 || !(f->r_fovea >= 0.0) || !(f->r_mid >= f->r_fovea) ||
        !is_fin(f->r_mid) || !is_fin(f->margin) || f->keep_den <= 0 || f->keep_num < 0 || f->keep_num > f->keep_den)
        return A3FR_EINVAL;
    const int scales[3] = {1, f->scale_mid, f->scale_periph};
    for (int e = 0; e < n_eyes; ++e) {
        for (int l = 0; l < 3; ++l) {
            const double s = (double)scales[l];
            a3fr_view &v = out[3 * e + l];
            view_from_camera(cams[e], e, v);
            v.fx = cams[e].fx / s; v.fy = cams[e].fy / s;
            v.cx = cams[e].cx / s; v.cy = cams[e].cy / s;
            v.width = cams[e].width / scales[l];
            v.height = cams[e].height / scales[l];
            v.gx = gaze[e].x / s; v.gy = gaze[e].y / s;
            if (l == 0) {
                v.mask = A3FR_MASK_DISC;
                v.r_out = f->r_fovea / s;
            } else if (l == 1) {
                v.mask = A3FR_MASK_ANNULUS;
                v.r_in = f->r_fovea / s - f->margin;
                v.r_out = f->r_mid / s + f->margin;
            } else {
                v.select = 1;
            }
        }
    }
    return A3FR_OK;
}

a3fr_status a3fr_composite(a3fr_ctx *c, int32_t W, int32_t H, a3fr_gaze g, const a3fr_fovea *f, const float *fov,
                           const float *mid, const float *per, const float *per_full, float *out) {
    if (!c) return A3FR_EINVAL;
    if (!f || W <= 0 || H <= 0 || !fov || !mid || !out || (!per && !per_full))
        return fail(c, A3FR_EINVAL, "composite: bad arguments");
    if (f->scale_mid < 1 || f->scale_periph < 1 || W / f->scale_mid < 1 || H / f->scale_mid < 1 ||
        W / f->scale_periph < 1 || H / f->scale_periph < 1)
        return fail(c, A3FR_EINVAL, "composite: layer scales too large for the image");
    StageTimer t_(c, A3FR_STAGE_COMPOSITE);
    launch_composite(W, H, g.x, g.y, f->r_fovea, f->r_mid, fov, mid, f->scale_mid, per, f->scale_periph, per_full,
                     false, nullptr, 0, nullptr, out, c->stream);
    return check_launch(c, "composite");
}

static NetPacked net_packed(a3fr_ctx *c);
static a3fr_status net_check_geom(a3fr_ctx *c, int B, int h, int w);

// Inference forward of the upsampler: one fused launch runs all three layers
// tile by tile with the weights and activations in LDS (gv: frame mode, see
// NetConvArgs).
static void net_infer(a3fr_ctx *c, const float *theta, const float *in, int64_t in_stride, int B, int h, int w,
                      float *out, int64_t out_stride, const DevView *gv, double rm) {
    NetFusedArgs a{};
    a.img_in = in; a.img_bstride = in_stride;
    a.theta = theta;
    a.img_out = out; a.out_bstride = out_stride;
    a.B = B; a.h = h; a.w = w;
    a.gv = gv; a.gv_stride = 3; a.rm = rm;
    launch_net_fused(a, c->stream);
}

// The upsampler on the periphery layers of a foveated frame, all eyes in one
// batch (frame mode): layer images of eye e sit at a constant distance from
// eye 0's (every eye has the same layer sizes); tiles and units whose
// receptive field lies within r_mid are skipped and only pixels outside r_mid
// are written to out, where the composite leaves them (whole: every pixel is
// computed and written, for a periphery whose gaze comes later).
static a3fr_status net_frame_forward(a3fr_ctx *c, const a3fr_camera *cams, int n_eyes, double r_mid, const float *L,
                                     float *out, bool whole = false) {
    const int W = cams[0].width, H = cams[0].height;
    for (int e = 1; e < n_eyes; ++e)
        if (cams[e].width != W || cams[e].height != H)
            return fail(c, A3FR_EINVAL, "render_foveated: the upsampler needs every eye at the same image size");
    const int h = H / 4, w = W / 4;
    TRY(net_check_geom(c, n_eyes, h, w));
    const int64_t in_stride = n_eyes > 1 ? 3 * (c->hviews[5].img_off - c->hviews[2].img_off) : 3 * (int64_t)h * w;
    c->net_trained_fwd = false;
    net_infer(c, c->net_theta, L + 3 * c->hviews[2].img_off, in_stride, n_eyes, h, w, out, 3 * (int64_t)W * H,
              whole ? nullptr : P<DevView>(c->views), r_mid);
    return check_launch(c, "upsampler");
}

a3fr_status a3fr_render_foveated(a3fr_ctx *c, const a3fr_scene *scene, const a3fr_camera *cams,
                                 const a3fr_gaze *gaze, int32_t n_eyes, const a3fr_fovea *f, float *out) {
    if (!c) return A3FR_EINVAL;
    if (!cams || !gaze || !f || !out || n_eyes < 1 || n_eyes > kMaxEyes)
        return fail(c, A3FR_EINVAL, "render_foveated: bad arguments");
    std::vector<a3fr_view> v(3 * n_eyes);
    if (a3fr_make_foveated_views(cams, gaze, n_eyes, f, v.data()) != A3FR_OK)
        return fail(c, A3FR_EINVAL, "render_foveated: bad fovea parameters");
    if (c->net_theta) {
        if (f->scale_periph != 4) return fail(c, A3FR_EINVAL, "render_foveated: the upsampler needs scale_periph = 4");
        for (int e = 0; e < n_eyes; ++e)
            if (cams[e].width % 4 || cams[e].height % 4)
                return fail(c, A3FR_EINVAL, "render_foveated: the upsampler needs W and H divisible by 4");
    }
    const bool fb = std::isfinite(c->fb_thr);
    c->fb_plan.clear();
    if (fb)
        for (int e = 0; e < n_eyes; ++e) c->fb_plan.push_back({3 * e + 2, 3 * e, f->r_mid});
    a3fr_status st = a3fr_preprocess(c, scene, v.data(), 3 * n_eyes, f->keep_num, f->keep_den);
    c->fb_plan.clear();
    TRY(st);
    TRY(a3fr_bin_sort(c, nullptr));
    TRY(ensure(c, c->layers, sizeof(float) * 3 * (size_t)c->npix));
    float *L = P<float>(c->layers);
    const bool net = c->net_theta != nullptr;
    // Overlap: the main stream blends the periphery layers and runs them
    // through the network while the side stream blends the fovea and mid
    // layers (different layers, different pixels; the composite waits for both).
    // Profiled frames keep one stream, so that each stage is timed alone.  A
    // graph capture records the same fork and join (the side stream joins the
    // capture through the fork event).
    const bool overlap = net && !c->profiling && n_eyes <= kMaxTileRanges && !blend_variant(c->blend_variant).queue;
    if (overlap) {
        if (!c->side) HIPCHECK(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
        if (!c->ev_fork) HIPCHECK(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
        if (!c->ev_join) HIPCHECK(c, hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
        TileRanges per{}, fm{};
        per.count = fm.count = n_eyes;
        for (int e = 0; e < n_eyes; ++e) {
            const DevView &d0 = c->hviews[3 * e], &d2 = c->hviews[3 * e + 2];
            per.base[e] = d2.tile_off;
            per.len[e] = (int64_t)d2.tiles_x * d2.tiles_y;
            fm.base[e] = d0.tile_off;  // fovea and mid views: the tiles before the periphery's
            fm.len[e] = d2.tile_off - d0.tile_off;
        }
        // the periphery's waves are queued first (on the main stream, no
        // cross-stream wait before them), so they are not left behind the
        // far more numerous fovea and mid waves
        // the periphery's few long-list tiles take four waves each (8 x 8
        // quadrant blocks), so that the network can start sooner
        constexpr int kPeriphVariant = 12;
        HIPCHECK(c, hipEventRecord(c->ev_fork, c->stream));
        TRY(blend_with(c, kPeriphVariant, L, nullptr, nullptr, nullptr, c->stream, &per));
        HIPCHECK(c, hipStreamWaitEvent(c->side, c->ev_fork, 0));
        TRY(blend_with(c, c->blend_variant, L, nullptr, nullptr, nullptr, c->side, &fm));
        HIPCHECK(c, hipEventRecord(c->ev_join, c->side));
        TRY(net_frame_forward(c, cams, n_eyes, f->r_mid, L, out));
        HIPCHECK(c, hipStreamWaitEvent(c->stream, c->ev_join, 0));
    } else {
        TRY(a3fr_blend(c, L, nullptr, nullptr));
        if (net) {
            // the network writes the periphery (outside r_mid) of every eye straight into out
            StageTimer t_(c, A3FR_STAGE_NET);
            TRY(net_frame_forward(c, cams, n_eyes, f->r_mid, L, out));
        }
    }
    bool same_size = true;
    for (int e = 1; e < n_eyes; ++e)
        same_size = same_size && cams[e].width == cams[0].width && cams[e].height == cams[0].height;
    if (same_size) {  // every eye in one launch
        StageTimer t_(c, A3FR_STAGE_COMPOSITE);
        launch_composite_eyes(n_eyes, cams[0].width, cams[0].height, f->r_fovea, f->r_mid, f->scale_mid,
                              f->scale_periph, P<DevView>(c->views), L, net,
                              c->fb_last ? P<uint8_t>(c->fb_flags) : nullptr, out, c->stream);
        return check_launch(c, "composite");
    }
    int64_t o_off = 0;
    for (int e = 0; e < n_eyes; ++e) {
        const DevView &d0 = c->hviews[3 * e], &d1 = c->hviews[3 * e + 1], &d2 = c->hviews[3 * e + 2];
        const int W = cams[e].width, H = cams[e].height;
        StageTimer t_(c, A3FR_STAGE_COMPOSITE);
        launch_composite(W, H, gaze[e].x, gaze[e].y, f->r_fovea, f->r_mid, L + 3 * d0.img_off, L + 3 * d1.img_off,
                         f->scale_mid, L + 3 * d2.img_off, f->scale_periph, nullptr, net,
                         c->fb_last ? P<uint8_t>(c->fb_flags) + d2.tile_off : nullptr, d2.tiles_x,
                         P<DevView>(c->views) + 3 * e, out + o_off, c->stream);
        TRY(check_launch(c, "composite"));
        o_off += 3 * (int64_t)W * H;
    }
    return A3FR_OK;
}

a3fr_status a3fr_render_batch(a3fr_ctx *c, const a3fr_scene *scene, const a3fr_camera *cams, const a3fr_gaze *gaze,
                              int32_t n_frames, const a3fr_fovea *f, float *out) {
    if (!c) return A3FR_EINVAL;
    if (n_frames < 1 || 2 * n_frames > kMaxEyes) return fail(c, A3FR_EINVAL, "render_batch: n_frames must be in [1, 64]");
    return a3fr_render_foveated(c, scene, cams, gaze, 2 * n_frames, f, out);
}

// ---- incremental foveal rounds ------------------------------------------------

static a3fr_status inc_check(a3fr_ctx *c, const a3fr_camera *cams, const a3fr_gaze *gaze, int32_t n_eyes,
                             const a3fr_fovea *f, const char *who) {
    if (!cams || !gaze || !f || n_eyes < 1 || n_eyes > kMaxEyes)
        return fail(c, A3FR_EINVAL, std::string(who) + ": bad arguments");
    if (c->gexec) return fail(c, A3FR_EINVAL, std::string(who) + ": release the captured graph first");
    return A3FR_OK;
}

// One round on the buffered projection: the fovea layer's tiles within radius
// of each eye's gaze that no earlier round rendered (and, in the final round,
// the mid layer's annulus around the final gaze) get counts from the stored
// rectangles, are binned and sorted, and are blended into the persistent
// layer images; no other tile is touched and the scene is not read.
static a3fr_status inc_round(a3fr_ctx *c, const a3fr_gaze *gaze, double radius, bool final_round) {
    const int ne = c->inc_eyes;
    std::vector<a3fr_view> v(3 * ne);
    if (a3fr_make_foveated_views(c->inc_cams.data(), gaze, ne, &c->inc_fovea, v.data()) != A3FR_OK)
        return fail(c, A3FR_EINVAL, "incremental round: bad gaze");
    const a3fr_fovea *f = &c->inc_fovea;
    for (int e = 0; e < ne; ++e) {
        if (final_round) continue;  // fovea disc r_f and mid annulus around the final gaze
        v[3 * e].r_out = radius > 0.0 ? radius : -1.0;  // the fovea layer is at full resolution
        // the mid layer: a disc whose radius is offset from its final outer radius
        // as the fovea's is (r_mid - E for Eq. 4, r_mid + E for Eq. 5)
        const double rmid = radius + (f->r_mid - f->r_fovea);
        v[3 * e + 1].mask = A3FR_MASK_DISC;
        v[3 * e + 1].r_in = 0.0;
        v[3 * e + 1].r_out = rmid > 0.0 ? rmid / f->scale_mid + f->margin : -1.0;
    }
    c->inc_flags.assign(3 * ne, 0);
    for (int e = 0; e < ne; ++e) {
        c->inc_flags[3 * e] = kRoundExclDone;
        c->inc_flags[3 * e + 1] = kRoundExclDone;
        c->inc_flags[3 * e + 2] = kRoundFrozen;  // the periphery was rendered by a3fr_incremental_begin
    }
    c->inc_mode = true;
    a3fr_status st = preprocess_layout(c, c->inc_n, v.data(), 3 * ne);
    c->inc_mode = false;
    TRY(st);
    if (c->ntiles != c->inc_ntiles || c->npix != c->inc_npix)
        return fail(c, A3FR_EINVAL, "incremental round: frame layout changed");
    const DevView *dv = P<DevView>(c->views);
    {
        StageTimer t_(c, A3FR_STAGE_MASKS);
        launch_tile_masks(dv, c->nv, c->rows_total, c->d_row_view, c->d_row_y, P<uint16_t>(c->row_prefix),
                          P<uint16_t>(c->row_list), P<uint8_t>(c->active), P<uint8_t>(c->inc_done), FillSegs{},
                          c->stream);
        if (c->cum_entries)
            launch_mask_cum(dv, c->nv, c->max_tiles_x, P<uint16_t>(c->row_prefix), P<uint32_t>(c->cum), c->stream);
        // fovea and mid layers of every eye, up to kFbMax views per launch
        FbBatch rb{};
        for (int e = 0; e < ne; ++e)
            for (int k = 0; k < 2; ++k) {
                rb.fv[rb.count++] = 3 * e + k;
                if (rb.count == kFbMax || (e == ne - 1 && k == 1)) {
                    launch_recount(dv, rb, c->n, P<uint64_t>(c->rect), P<uint16_t>(c->row_prefix),
                                   P<uint32_t>(c->counts), nullptr, c->stream);
                    rb.count = 0;
                }
            }
    }
    c->fb_last = false;
    TRY(entry_stages(c, nullptr, false, true));  // the records of round 0, through the slot -> record map
    TRY(a3fr_bin_sort(c, nullptr));
    StageTimer t_(c, A3FR_STAGE_BLEND);
    return blend_with(c, c->blend_variant, P<float>(c->layers), nullptr, nullptr, nullptr, c->stream);
}

a3fr_status a3fr_incremental_begin(a3fr_ctx *c, const a3fr_scene *scene, const a3fr_camera *cams, int32_t n_eyes,
                                   const a3fr_fovea *f) {
    if (!c) return A3FR_EINVAL;
    c->inc_ready = false;
    std::vector<a3fr_gaze> centre(n_eyes > 0 && n_eyes <= kMaxEyes ? n_eyes : 1);
    for (int e = 0; cams && e < (int)centre.size(); ++e) centre[e] = a3fr_gaze{cams[e].cx, cams[e].cy};
    TRY(inc_check(c, cams, centre.data(), n_eyes, f, "incremental_begin"));
    std::vector<a3fr_view> v(3 * n_eyes);
    if (a3fr_make_foveated_views(cams, centre.data(), n_eyes, f, v.data()) != A3FR_OK)
        return fail(c, A3FR_EINVAL, "incremental_begin: bad fovea parameters");
    if (c->net_theta) {
        if (f->scale_periph != 4) return fail(c, A3FR_EINVAL, "incremental_begin: the upsampler needs scale_periph = 4");
        for (int e = 0; e < n_eyes; ++e)
            if (cams[e].width % 4 || cams[e].height % 4)
                return fail(c, A3FR_EINVAL, "incremental_begin: the upsampler needs W and H divisible by 4");
    }
    // round 0: every layer projected once (the fovea and mid layers with empty
    // masks, keeping every visible entry's rectangle and record), the periphery
    // subset selected and the periphery layer rendered: it needs no gaze
    for (int e = 0; e < n_eyes; ++e) {
        v[3 * e].r_out = -1.0;
        v[3 * e + 1].r_out = -1.0;
    }
    c->fb_plan.clear();
    c->inc_flags.assign(3 * n_eyes, 0);
    c->inc_mode = true;
    c->inc_round0 = true;  // every visible fovea and mid entry gets its record now
    a3fr_status st = a3fr_preprocess(c, scene, v.data(), 3 * n_eyes, f->keep_num, f->keep_den);
    c->inc_mode = false;
    c->inc_round0 = false;
    TRY(st);
    TRY(a3fr_bin_sort(c, nullptr));
    TRY(ensure(c, c->layers, sizeof(float) * 3 * (size_t)c->npix));
    TRY(a3fr_blend(c, P<float>(c->layers), nullptr, nullptr));
    if (c->net_theta) {  // the periphery needs no gaze: upsample all of it now
        int64_t tot = 0;
        for (int e = 0; e < n_eyes; ++e) tot += 3 * (int64_t)cams[e].width * cams[e].height;
        TRY(ensure(c, c->inc_periph, sizeof(float) * (size_t)tot));
        StageTimer t_(c, A3FR_STAGE_NET);
        TRY(net_frame_forward(c, cams, n_eyes, f->r_mid, P<float>(c->layers), P<float>(c->inc_periph), true));
    }
    // the periphery's entries are done: later rounds compact only fovea and mid entries
    for (int e = 0; e < n_eyes; ++e)
        launch_fill_u32(P<uint32_t>(c->counts) + (int64_t)(3 * e + 2) * c->n, 0u, c->n, c->stream);
    const int64_t done_words = ((int64_t)c->ntiles + 3) / 4;
    TRY(ensure(c, c->inc_done, sizeof(uint32_t) * (size_t)done_words));
    launch_fill_u32(P<uint32_t>(c->inc_done), 0u, done_words, c->stream);
    TRY(check_launch(c, "incremental_begin"));
    c->inc_eyes = n_eyes;
    c->inc_n = c->n;
    c->inc_ntiles = c->ntiles;
    c->inc_npix = c->npix;
    c->inc_cams.assign(cams, cams + n_eyes);
    c->inc_fovea = *f;
    c->inc_net = c->net_theta != nullptr;
    c->inc_ready = true;
    return A3FR_OK;
}

a3fr_status a3fr_incremental_round(a3fr_ctx *c, const a3fr_gaze *gaze, double radius) {
    if (!c) return A3FR_EINVAL;
    if (!c->inc_ready) return fail(c, A3FR_ENOTREADY, "a3fr_incremental_round before a3fr_incremental_begin");
    if (!gaze) return fail(c, A3FR_EINVAL, "incremental_round: gaze is NULL");
    if (!(radius >= 0.0) || !is_fin(radius)) return fail(c, A3FR_EINVAL, "incremental_round: radius must be >= 0");
    TRY(inc_check(c, c->inc_cams.data(), gaze, c->inc_eyes, &c->inc_fovea, "incremental_round"));
    a3fr_status st = inc_round(c, gaze, radius, false);
    if (st != A3FR_OK) c->inc_ready = false;
    return st;
}

a3fr_status a3fr_incremental_finish(a3fr_ctx *c, const a3fr_gaze *gaze, float *out) {
    if (!c) return A3FR_EINVAL;
    if (!c->inc_ready) return fail(c, A3FR_ENOTREADY, "a3fr_incremental_finish before a3fr_incremental_begin");
    if (!gaze || !out) return fail(c, A3FR_EINVAL, "incremental_finish: NULL gaze or out");
    TRY(inc_check(c, c->inc_cams.data(), gaze, c->inc_eyes, &c->inc_fovea, "incremental_finish"));
    c->inc_ready = false;
    const a3fr_fovea *f = &c->inc_fovea;
    const int ne = c->inc_eyes;
    TRY(inc_round(c, gaze, f->r_fovea, true));
    float *L = P<float>(c->layers);
    int64_t o_off = 0;
    for (int e = 0; e < ne; ++e) {
        const DevView &d0 = c->hviews[3 * e], &d1 = c->hviews[3 * e + 1], &d2 = c->hviews[3 * e + 2];
        const int W = c->inc_cams[e].width, H = c->inc_cams[e].height;
        StageTimer t_(c, A3FR_STAGE_COMPOSITE);
        launch_composite(W, H, gaze[e].x, gaze[e].y, f->r_fovea, f->r_mid, L + 3 * d0.img_off, L + 3 * d1.img_off,
                         f->scale_mid, L + 3 * d2.img_off, f->scale_periph,
                         c->inc_net ? P<float>(c->inc_periph) + o_off : nullptr, false, nullptr, d2.tiles_x,
                         P<DevView>(c->views) + 3 * e, out + o_off, c->stream);
        TRY(check_launch(c, "composite"));
        o_off += 3 * (int64_t)W * H;
    }
    return A3FR_OK;
}

a3fr_status a3fr_set_upsampler(a3fr_ctx *c, const float *theta) {
    if (!c) return A3FR_EINVAL;
    c->net_theta = theta;
    return A3FR_OK;
}

a3fr_status a3fr_set_fallback(a3fr_ctx *c, double thr, double coef, double power) {
    if (!c) return A3FR_EINVAL;
    if (!(thr >= 0.0) || !(coef >= 0.0) || !is_fin(coef) || !(power > 0.0) || !is_fin(power))
        return fail(c, A3FR_EINVAL, "set_fallback: mse_threshold >= 0, coef >= 0 and power > 0, finite");
    c->fb_thr = thr;
    c->fb_coef = coef;
    c->fb_pow = power;
    return A3FR_OK;
}

static a3fr_status check_params(a3fr_ctx *c, const a3fr_params *p) {
    if (!p) return fail(c, A3FR_EINVAL, "params is NULL");
    if (p->n < 0 || p->n >= (int64_t(1) << 31)) return fail(c, A3FR_EINVAL, "params.n must be in [0, 2^31)");
    if (p->sh_degree < 0 || p->sh_degree > 3) return fail(c, A3FR_EINVAL, "params.sh_degree must be 0..3");
    if (p->n > 0 && (!p->mean_dev || !p->log_scale_dev || !p->quat_dev || !p->logit_dev || !p->sh_dev))
        return fail(c, A3FR_EINVAL, "params arrays must not be NULL");
    return A3FR_OK;
}

a3fr_status a3fr_activate(a3fr_ctx *c, const a3fr_params *p, float *scale, float *opacity) {
    if (!c) return A3FR_EINVAL;
    TRY(check_params(c, p));
    if (p->n > 0 && (!scale || !opacity)) return fail(c, A3FR_EINVAL, "activate: output arrays must not be NULL");
    StageTimer t_(c, A3FR_STAGE_ACTIVATE);
    launch_activate(*p, scale, opacity, c->stream);
    return check_launch(c, "activate");
}

a3fr_status a3fr_blend_backward(a3fr_ctx *c, const float *dl, const float *T, const uint32_t *last) {
    if (!c) return A3FR_EINVAL;
    if (!c->sorted) return fail(c, A3FR_ENOTREADY, "a3fr_blend_backward before a3fr_bin_sort");
    if (!dl || !T || !last) return fail(c, A3FR_EINVAL, "blend_backward: dl_drgb, T and last must not be NULL");
    if (c->map_mode) return fail(c, A3FR_EINVAL, "blend_backward: not for the rounds of an incremental frame");
    // the reverse blend's sums per record (the key values)
    const int64_t nr = c->n_rec >= 0 ? c->n_rec : record_capacity(c);
    TRY(ensure(c, c->grad_acc, sizeof(float) * 12 * (size_t)nr));
    StageTimer t_(c, A3FR_STAGE_BLEND_BWD);
    launch_fill_u32(P<uint32_t>(c->grad_acc), 0u, 12 * nr, c->stream);
    launch_blend_bwd(P<DevView>(c->views), c->nv, c->ntiles, P<uint8_t>(c->active), P<uint32_t>(c->ranges),
                     sorted_vals(c), P<Record>(c->rec), 0, dl, T, last, P<float>(c->grad_acc), c->stream);
    TRY(check_launch(c, "blend_backward"));
    c->blend_bwd_done = true;
    return A3FR_OK;
}

a3fr_status a3fr_preprocess_backward(a3fr_ctx *c, const a3fr_params *p, const a3fr_grads *g) {
    if (!c) return A3FR_EINVAL;
    TRY(check_params(c, p));
    if (!c->blend_bwd_done) return fail(c, A3FR_ENOTREADY, "a3fr_preprocess_backward before a3fr_blend_backward");
    if (p->n != c->n || p->sh_degree != c->sh_degree)
        return fail(c, A3FR_EINVAL, "preprocess_backward: params differ in n or sh_degree from the rendered scene");
    if (!g || (p->n > 0 && (!g->mean_dev || !g->log_scale_dev || !g->quat_dev || !g->logit_dev || !g->sh_dev)))
        return fail(c, A3FR_EINVAL, "preprocess_backward: gradient arrays must not be NULL");
    StageTimer t_(c, A3FR_STAGE_PREPROCESS_BWD);
    launch_preprocess_bwd(*p, P<DevView>(c->views), c->nv, P<uint32_t>(c->counts), P<uint8_t>(c->keep),
                          P<uint32_t>(c->map), P<float>(c->grad_acc), P<Record>(c->rec), *g, c->stream);
    return check_launch(c, "preprocess_backward");
}

// ---- upsampler ------------------------------------------------------------
static NetPacked net_packed(a3fr_ctx *c) {
    uint16_t *p = P<uint16_t>(c->net_pk);
    NetPacked pk;
    pk.f1 = p;
    pk.f2 = pk.f1 + 9 * 32 * 8;
    pk.d2 = pk.f2 + 9 * 32 * 32;
    pk.f3 = pk.d2 + 9 * 32 * 32;
    pk.d3 = pk.f3 + 9 * 48 * 32;
    return pk;
}

static a3fr_status net_check_geom(a3fr_ctx *c, int B, int h, int w) {
    if (B < 1 || h < 1 || w < 1) return fail(c, A3FR_EINVAL, "net: batch, height and width must be positive");
    if ((int64_t)B * h * w > (int64_t(1) << 28) || h > 65535 * 8 || w > 65535 * 64 || B > 65535)
        return fail(c, A3FR_EINVAL, "net: input too large");
    return A3FR_OK;
}

a3fr_status a3fr_net_forward(a3fr_ctx *c, const float *theta, const float *in, int32_t B, int32_t h, int32_t w,
                             float *out, int32_t for_training) {
    if (!c) return A3FR_EINVAL;
    TRY(net_check_geom(c, B, h, w));
    if (!theta || !in || !out) return fail(c, A3FR_EINVAL, "net_forward: NULL pointer");
    const int64_t px = (int64_t)B * h * w;
    const int WS = net_chw_stride(w);
    const int64_t plane = (int64_t)(h + 2) * WS;
    const bool train = for_training != 0;
    if (!train) {  // inference: one fused launch, no activations in memory
        c->net_trained_fwd = false;
        net_infer(c, theta, in, 0, B, h, w, out, 0, nullptr, 0.0);
        return check_launch(c, "net_forward");
    }
    TRY(ensure(c, c->net_pk, sizeof(uint16_t) * kNetPackedElems));
    TRY(ensure(c, c->net_x0, sizeof(uint16_t) * 8 * px));
    TRY(ensure(c, c->net_a1, sizeof(uint16_t) * 32 * px));
    TRY(ensure(c, c->net_a2, sizeof(uint16_t) * 32 * px));
    if (train) {
        DevBuf *chw[] = {&c->net_x0c, &c->net_a1c, &c->net_a2c, &c->net_g3c, &c->net_g2c, &c->net_g1c};
        const int chans[] = {8, 32, 32, 48, 32, 32};
        const bool regeom = c->net_B != B || c->net_h != h || c->net_w != w;
        for (int k = 0; k < 6; ++k) {
            const size_t bytes = sizeof(uint16_t) * (size_t)B * chans[k] * plane;
            const bool grow = chw[k]->cap < bytes;
            TRY(ensure(c, *chw[k], bytes));
            // zero borders (and padding columns) hold for a geometry until it changes
            if (grow || regeom) launch_fill_u32(P<uint32_t>(*chw[k]), 0u, (int64_t)(bytes / 4), c->stream);
        }
        TRY(ensure(c, c->net_g3, sizeof(uint16_t) * 48 * px));
        TRY(ensure(c, c->net_g2, sizeof(uint16_t) * 32 * px));
        TRY(ensure(c, c->net_sse, 16));
        c->net_B = B; c->net_h = h; c->net_w = w;
    }
    c->net_trained_fwd = false;
    const NetPacked pk = net_packed(c);
    launch_net_prep(theta, pk, in, 0, B, h, w, P<uint16_t>(c->net_x0), train ? P<uint16_t>(c->net_x0c) : nullptr,
                    c->stream);
    NetConvArgs a{};
    a.B = B; a.h = h; a.w = w;
    a.in = P<uint16_t>(c->net_x0); a.wpk = pk.f1; a.bias = theta + kNetB1;
    a.out = P<uint16_t>(c->net_a1); a.out_chw = train ? P<uint16_t>(c->net_a1c) : nullptr;
    launch_net_conv(1, false, a, c->stream);
    a.in = P<uint16_t>(c->net_a1); a.wpk = pk.f2; a.bias = theta + kNetB2;
    a.out = P<uint16_t>(c->net_a2); a.out_chw = train ? P<uint16_t>(c->net_a2c) : nullptr;
    launch_net_conv(2, false, a, c->stream);
    a.in = P<uint16_t>(c->net_a2); a.wpk = pk.f3; a.bias = theta + kNetB3;
    a.out = nullptr; a.out_chw = nullptr; a.img_in = in; a.img_out = out;
    launch_net_conv(3, false, a, c->stream);
    TRY(check_launch(c, "net_forward"));
    c->net_trained_fwd = train;
    return A3FR_OK;
}

a3fr_status a3fr_net_backward(a3fr_ctx *c, const float *theta, const float *out, const float *target, float *grad,
                              float *loss) {
    if (!c) return A3FR_EINVAL;
    if (!c->net_trained_fwd) return fail(c, A3FR_ENOTREADY, "net_backward needs a net_forward with for_training = 1");
    if (!theta || !out || !target || !grad) return fail(c, A3FR_EINVAL, "net_backward: NULL pointer");
    if ((reinterpret_cast<uintptr_t>(out) | reinterpret_cast<uintptr_t>(target)) & 15u)
        return fail(c, A3FR_EINVAL, "net_backward: out and target must be 16-byte aligned");
    const int B = c->net_B, h = c->net_h, w = c->net_w;
    const NetPacked pk = net_packed(c);
    launch_fill_u32(reinterpret_cast<uint32_t *>(grad), 0u, kNetParams, c->stream);
    launch_fill_u32(P<uint32_t>(c->net_sse), 0u, 2, c->stream);
    launch_net_mse(out, target, B, h, w, P<uint16_t>(c->net_g3), P<uint16_t>(c->net_g3c), P<double>(c->net_sse), loss,
                   c->stream);
    // input gradients: g2 = (g3 * W3') masked by a2 > 0; g1 = (g2 * W2') masked by a1 > 0
    NetConvArgs a{};
    a.B = B; a.h = h; a.w = w;
    a.in = P<uint16_t>(c->net_g3); a.wpk = pk.d3; a.mask = P<uint16_t>(c->net_a2);
    a.out = P<uint16_t>(c->net_g2); a.out_chw = P<uint16_t>(c->net_g2c);
    launch_net_conv(3, true, a, c->stream);
    a.in = P<uint16_t>(c->net_g2); a.wpk = pk.d2; a.mask = P<uint16_t>(c->net_a1);
    a.out = nullptr; a.out_chw = P<uint16_t>(c->net_g1c);
    launch_net_conv(2, true, a, c->stream);
    // weight gradients
    const int64_t chunks = (int64_t)B * h * ((w + 31) / 32);
    const int slabs = (int)std::min<int64_t>(chunks, 96);
    NetWgradArgs wg{};
    wg.B = B; wg.h = h; wg.w = w; wg.grad = grad;
    wg.g = P<uint16_t>(c->net_g3c); wg.in = P<uint16_t>(c->net_a2c); wg.off_w = kNetW3; wg.off_b = kNetB3;
    launch_net_wgrad(3, wg, slabs, c->stream);
    wg.g = P<uint16_t>(c->net_g2c); wg.in = P<uint16_t>(c->net_a1c); wg.off_w = kNetW2; wg.off_b = kNetB2;
    launch_net_wgrad(2, wg, slabs, c->stream);
    wg.g = P<uint16_t>(c->net_g1c); wg.in = P<uint16_t>(c->net_x0c); wg.off_w = kNetW1; wg.off_b = kNetB1;
    launch_net_wgrad(1, wg, slabs, c->stream);
    (void)theta;
    return check_launch(c, "net_backward");
}

a3fr_status a3fr_net_adam(a3fr_ctx *c, float *theta, const float *grad, float *m, float *v, int32_t step, float lr,
                          float beta1, float beta2, float eps) {
    if (!c) return A3FR_EINVAL;
    if (!theta || !grad || !m || !v) return fail(c, A3FR_EINVAL, "net_adam: NULL pointer");
    if (step < 1 || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps > 0.0f))
        return fail(c, A3FR_EINVAL, "net_adam: step >= 1, lr >= 0, 0 <= beta < 1, eps > 0");
    const float bc1 = (float)(1.0 - std::pow((double)beta1, (double)step));
    const float bc2 = (float)(1.0 - std::pow((double)beta2, (double)step));
    launch_net_adam(theta, grad, m, v, kNetParams, lr, beta1, beta2, eps, bc1, bc2, c->stream);
    return check_launch(c, "net_adam");
}

// ---- graph mode ---------------------------------------------------------------
static void graph_release(a3fr_ctx *c) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    c->capacity = 0;
    c->ecap = 0;
    c->g_eyes = 0;
}

a3fr_status a3fr_graph_destroy(a3fr_ctx *c) {
    if (!c) return A3FR_EINVAL;
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    graph_release(c);
    return A3FR_OK;
}

a3fr_status a3fr_graph_capture(a3fr_ctx *c, const a3fr_scene *scene, const a3fr_camera *cams, const a3fr_gaze *gaze,
                               int32_t n_eyes, const a3fr_fovea *f, float *out, int64_t max_keys) {
    if (!c) return A3FR_EINVAL;
    if (max_keys < 1 || max_keys >= (int64_t(1) << 32)) return fail(c, A3FR_EINVAL, "max_keys must be in [1, 2^32)");
    if (c->profiling) return fail(c, A3FR_ENOTREADY, "turn profiling off before capturing a graph");
    if (!cams || !gaze || !f || !out || n_eyes < 1 || n_eyes > kMaxEyes)
        return fail(c, A3FR_EINVAL, "graph_capture: bad arguments");
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    graph_release(c);
    if (!c->stream) {
        // stream capture needs a stream other than the null stream
        if (!c->own_stream) HIPCHECK(c, hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking));
        c->stream = c->own_stream;
    }
    // an exact frame gives this layout's key and entry counts; the entry (and
    // record) capacity keeps the same headroom over the entries as max_keys
    // over the keys
    a3fr_status st = a3fr_render_foveated(c, scene, cams, gaze, n_eyes, f, out);
    if (st == A3FR_OK) st = a3fr_sync(c);
    if (st != A3FR_OK) return st;
    const int64_t K0 = c->K, E0 = c->n_ent_pass;
    if (K0 > max_keys)
        return fail(c, A3FR_ECAPACITY, "max_keys " + std::to_string(max_keys) + " is below the warm-up frame's " +
                                           std::to_string(K0) + " keys");
    const double head = K0 > 0 ? (double)max_keys / (double)K0 : 1.0;
    c->ecap = std::min<int64_t>((int64_t)c->nv * c->n,
                                std::max<int64_t>(E0, (int64_t)std::ceil((double)E0 * head)) + 1024);
    c->capacity = max_keys;
    // warm-up frame in capacity mode: sizes every buffer for this layout
    st = a3fr_render_foveated(c, scene, cams, gaze, n_eyes, f, out);
    if (st == A3FR_OK) st = a3fr_sync(c);
    if (st != A3FR_OK) {
        c->capacity = 0;
        c->ecap = 0;
        return st;
    }
    if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        c->capacity = 0;
        c->ecap = 0;
        return fail(c, A3FR_EDEVICE, "hipStreamBeginCapture failed");
    }
    c->capturing = true;
    st = a3fr_render_foveated(c, scene, cams, gaze, n_eyes, f, out);
    c->capturing = false;
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(c->stream, &g);
    if (st != A3FR_OK || ee != hipSuccess) {
        (void)hipGetLastError();
        if (g) (void)hipGraphDestroy(g);
        c->capacity = 0;
        c->ecap = 0;
        return st != A3FR_OK ? st : fail(c, A3FR_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ee));
    }
    hipGraphExec_t x = nullptr;
    if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipGraphDestroy(g);
        c->capacity = 0;
        c->ecap = 0;
        return fail(c, A3FR_EDEVICE, "hipGraphInstantiate failed");
    }
    c->graph = g;
    c->gexec = x;
    c->g_eyes = n_eyes;
    c->g_cams.assign(cams, cams + n_eyes);
    c->g_fovea = *f;
    return A3FR_OK;
}

a3fr_status a3fr_graph_launch(a3fr_ctx *c, const a3fr_camera *cams, const a3fr_gaze *gaze) {
    if (!c) return A3FR_EINVAL;
    if (!c->gexec) return fail(c, A3FR_ENOTREADY, "no captured graph");
    if (!cams || !gaze) return fail(c, A3FR_EINVAL, "graph_launch: NULL cameras or gaze");
    const int ne = c->g_eyes;
    for (int e = 0; e < ne; ++e)
        if (cams[e].width != c->g_cams[e].width || cams[e].height != c->g_cams[e].height)
            return fail(c, A3FR_EINVAL, "graph_launch: image sizes differ from the captured frame");
    std::vector<a3fr_view> v(3 * ne);
    if (a3fr_make_foveated_views(cams, gaze, ne, &c->g_fovea, v.data()) != A3FR_OK)
        return fail(c, A3FR_EINVAL, "graph_launch: bad cameras");
    for (int k = 0; k < 3 * ne; ++k) TRY(check_view(c, v[k], k));
    // the fallback plan frozen at capture marks the same views for remasking
    c->fb_plan.clear();
    if (c->fb_last)
        for (int e = 0; e < ne; ++e) c->fb_plan.push_back({3 * e + 2, 3 * e, c->g_fovea.r_mid});
    const int64_t nt = c->ntiles, np = c->npix, rt = c->rows_total;
    a3fr_status st = preprocess_layout(c, c->n, v.data(), 3 * ne);
    c->fb_plan.clear();
    TRY(st);
    if (c->ntiles != nt || c->npix != np || c->rows_total != rt)
        return fail(c, A3FR_EINVAL, "graph_launch: frame layout differs from the captured one");
    HIPCHECK(c, hipGraphLaunch(c->gexec, c->stream));
    c->preprocessed = c->sorted = true;
    c->K = -1;
    return A3FR_OK;
}

a3fr_status a3fr_region_sse(a3fr_ctx *c, int32_t W, int32_t H, a3fr_gaze g, double rf, double rm, const float *a,
                            const float *b, double *sse3, int64_t *count3) {
    if (!c) return A3FR_EINVAL;
    if (W <= 0 || H <= 0 || !a || !b || !sse3 || !count3) return fail(c, A3FR_EINVAL, "region_sse: bad arguments");
    const int nblk = kSseParts;
    TRY(ensure(c, c->sse_part, sizeof(double) * 3 * nblk));
    TRY(ensure(c, c->sse_cnt, sizeof(unsigned long long) * 3 * nblk));
    launch_region_sse(W, H, g.x, g.y, rf, rm, a, b, P<double>(c->sse_part), P<unsigned long long>(c->sse_cnt), nblk,
                      c->stream);
    TRY(check_launch(c, "region_sse"));
    std::vector<double> part(3 * nblk);
    std::vector<unsigned long long> cnt(3 * nblk);
    HIPCHECK(c, hipMemcpyAsync(part.data(), c->sse_part.p, sizeof(double) * 3 * nblk, hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipMemcpyAsync(cnt.data(), c->sse_cnt.p, sizeof(unsigned long long) * 3 * nblk, hipMemcpyDeviceToHost,
                               c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    for (int r = 0; r < 3; ++r) {
        double s = 0.0;
        int64_t k = 0;
        for (int j = 0; j < nblk; ++j) { s += part[3 * j + r]; k += (int64_t)cnt[3 * j + r]; }
        sse3[r] = s;
        count3[r] = k;
    }
    return A3FR_OK;
}

a3fr_status a3fr_region_sse_noalloc(a3fr_ctx *c, int32_t W, int32_t H, a3fr_gaze g, double rf, double rm,
                                    const float *a, const float *b, double *sse3_dev, int64_t *count3_dev) {
    if (!c) return A3FR_EINVAL;
    if (W <= 0 || H <= 0 || !a || !b || !sse3_dev || !count3_dev)
        return fail(c, A3FR_EINVAL, "region_sse_noalloc: bad arguments");
    if ((int64_t)W * H > (int64_t)A3FR_NOALLOC_MAX_PIXELS)
        return fail(c, A3FR_EINVAL, "region_sse_noalloc: W x H = " + std::to_string((int64_t)W * H) +
                                        " exceeds the maximum of " + std::to_string((int64_t)A3FR_NOALLOC_MAX_PIXELS) +
                                        " pixels");
    hipDevice_t dev = 0;
    HIPCHECK(c, hipStreamGetDevice(c->stream, &dev));
    void *p = nullptr;
    HIPCHECK(c, scratch_on_device((int)dev, &p));
    double *part = static_cast<double *>(p);
    unsigned long long *cnt = reinterpret_cast<unsigned long long *>(part + 3 * kSseParts);
    // every block writes its own partial slot: nothing to clear
    launch_region_sse(W, H, g.x, g.y, rf, rm, a, b, part, cnt, kSseParts, c->stream);
    launch_region_sse_sum(part, cnt, kSseParts, sse3_dev, count3_dev, c->stream);
    return check_launch(c, "region_sse_noalloc");
}

// Keys of the last bin_sort: known on the host in exact mode, read from the
// device (the clamped sort count) in capacity mode.
static a3fr_status key_count(a3fr_ctx *c, int64_t *K) {
    if (c->K >= 0 || !c->scalars.p) {
        *K = c->K < 0 ? 0 : c->K;
        return A3FR_OK;
    }
    uint32_t k = 0;
    HIPCHECK(c, hipMemcpyAsync(&k, sc_n_keys(c->scalars), 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    *K = (int64_t)k;
    return A3FR_OK;
}

a3fr_status a3fr_get_counts(a3fr_ctx *c, a3fr_counts *out) {
    if (!c || !out) return A3FR_EINVAL;
    std::memset(out, 0, sizeof(*out));
    if (c->sorted) TRY(key_count(c, &out->n_keys));
    out->n_tiles = c->ntiles;
    if (!c->preprocessed) return A3FR_OK;
    std::vector<uint8_t> act(c->ntiles > 0 ? c->ntiles : 1);
    HIPCHECK(c, hipMemcpyAsync(act.data(), c->active.p, (size_t)c->ntiles, hipMemcpyDeviceToHost, c->stream));
    // SelState (bin.hip): {n_vis, k, k_rem, mode, b0, b1, ncand, pad} = 8 words per slot, after the
    // two 4096-bucket histogram levels
    constexpr int kSelWords = 8;
    std::vector<uint32_t> st((size_t)c->nsel * kSelWords + 1);
    if (c->nsel)
        HIPCHECK(c, hipMemcpyAsync(st.data(), P<uint32_t>(c->sel) + (size_t)c->nsel * 2 * 4096,
                                   sizeof(uint32_t) * kSelWords * c->nsel, hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    for (int64_t t = 0; t < c->ntiles; ++t) out->n_active_tiles += act[t];
    if (c->fb_last) {
        std::vector<uint8_t> fl(c->ntiles);
        HIPCHECK(c, hipMemcpy(fl.data(), c->fb_flags.p, (size_t)c->ntiles, hipMemcpyDeviceToHost));
        for (int k = 0; k < c->nv; ++k)
            if (c->hviews[k].v.select) {
                const DevView &d = c->hviews[k];
                for (int64_t t = 0; t < (int64_t)d.tiles_x * d.tiles_y; ++t) out->n_fallback_tiles += fl[d.tile_off + t];
            }
    }
    for (int s = 0; s < c->nsel; ++s) {
        const int v = c->hsel_views[s];
        if (v < 16) out->n_kept[v] = st[(size_t)kSelWords * s + 1];  // SelState.k
    }
    return A3FR_OK;
}

a3fr_status a3fr_inspect(a3fr_ctx *c, a3fr_buffer which, void *dst, int64_t max_bytes, int64_t *bytes_out) {
    if (!c) return A3FR_EINVAL;
    const bool net_buf = which >= A3FR_BUF_NET_X0 && which <= A3FR_BUF_NET_G1;
    if (!net_buf && !c->preprocessed) return fail(c, A3FR_ENOTREADY, "nothing preprocessed");
    if (net_buf && !c->net_trained_fwd) return fail(c, A3FR_ENOTREADY, "no training forward of the net");
    const int64_t m = (int64_t)c->nv * c->n;
    const int64_t npx = (int64_t)c->net_B * c->net_h * c->net_w;
    const int64_t nplane = (int64_t)c->net_B * (c->net_h + 2) * (c->net_w > 0 ? net_chw_stride(c->net_w) : 0);
    const void *src = nullptr;
    int64_t bytes = 0;
    int make64 = 0;  // 1: emission-order keys, 2: sorted keys (rebuilt as tile << 32 | depth)
    int conv = 0;    // 1: key values as Gaussian indices (emission order), 2: the same, sorted;
                     // 3: rectangles, 4: records, scattered to their slots; 5: entry slots in depth order
    uint32_t n_ent = 0;
    if (which == A3FR_BUF_OFFSETS || which == A3FR_BUF_DEPTH_ORDER) {
        HIPCHECK(c, hipMemcpyAsync(&n_ent, sc_n_ent(c->scalars), 4, hipMemcpyDeviceToHost, c->stream));
        HIPCHECK(c, hipStreamSynchronize(c->stream));
    }
    const bool need_sort = which == A3FR_BUF_KEYS || which == A3FR_BUF_VALS || which == A3FR_BUF_SORTED_KEYS ||
                           which == A3FR_BUF_SORTED_VALS || which == A3FR_BUF_RANGES;
    if (need_sort && !c->sorted) return fail(c, A3FR_ENOTREADY, "keys not sorted yet");
    int64_t Kc = 0;
    if (need_sort) TRY(key_count(c, &Kc));
    if ((which == A3FR_BUF_KEYS || which == A3FR_BUF_VALS) && !c->keep_emission)
        return fail(c, A3FR_ENOTREADY, "emission order kept only with a3fr_set_debug(ctx, 1)");
    const bool need_records = which == A3FR_BUF_RECT || which == A3FR_BUF_RECORDS || make64 || need_sort;
    if (need_records && c->records_pending)
        return fail(c, A3FR_ENOTREADY, "the entries' records are formed by a3fr_bin_sort");
    const int64_t nrec = c->n_rec >= 0 ? c->n_rec : record_capacity(c);
    switch (which) {
        case A3FR_BUF_COUNTS: src = c->counts.p; bytes = 4 * m; break;
        case A3FR_BUF_DEPTH: src = c->depth.p; bytes = 4 * m; break;
        case A3FR_BUF_RECT: conv = 3; bytes = 8 * m; break;
        case A3FR_BUF_OFFSETS: src = c->offsets.p; bytes = 4 * ((int64_t)n_ent + 1); break;
        case A3FR_BUF_KEYS: make64 = 1; bytes = 8 * Kc; break;
        case A3FR_BUF_VALS: conv = 1; bytes = 4 * Kc; break;
        case A3FR_BUF_SORTED_KEYS: make64 = 2; bytes = 8 * Kc; break;
        case A3FR_BUF_SORTED_VALS: conv = 2; bytes = 4 * Kc; break;
        case A3FR_BUF_RANGES: src = c->ranges.p; bytes = 8 * c->ntiles; break;
        case A3FR_BUF_ACTIVE: src = c->active.p; bytes = c->ntiles; break;
        case A3FR_BUF_KEEP: src = c->keep.p; bytes = c->nsel ? m : 0; break;
        case A3FR_BUF_RECORDS: conv = 4; bytes = (int64_t)sizeof(Record) * m; break;
        case A3FR_BUF_DEPTH_ORDER: conv = 5; bytes = 4 * (int64_t)n_ent; break;
        case A3FR_BUF_NET_X0: src = c->net_x0.p; bytes = 2 * 8 * npx; break;
        case A3FR_BUF_NET_A1: src = c->net_a1.p; bytes = 2 * 32 * npx; break;
        case A3FR_BUF_NET_A2: src = c->net_a2.p; bytes = 2 * 32 * npx; break;
        case A3FR_BUF_NET_G3: src = c->net_g3.p; bytes = 2 * 48 * npx; break;
        case A3FR_BUF_NET_G2: src = c->net_g2.p; bytes = 2 * 32 * npx; break;
        case A3FR_BUF_NET_G1: src = c->net_g1c.p; bytes = 2 * 32 * nplane; break;
        case A3FR_BUF_FB_ENERGY:
            if (!c->fb_last) return fail(c, A3FR_ENOTREADY, "no fallback in the last frame");
            src = c->fb_energy.p; bytes = 8 * c->ntiles; break;
        case A3FR_BUF_FB_FLAGS:
            if (!c->fb_last) return fail(c, A3FR_ENOTREADY, "no fallback in the last frame");
            src = c->fb_flags.p; bytes = c->ntiles; break;
        case A3FR_BUF_AMR_LEVELS:
            if (!c->amr_last) return fail(c, A3FR_ENOTREADY, "the last frame was not an AMR frame");
            src = c->amr_lv.p; bytes = c->ntiles; break;
        case A3FR_BUF_SEL_STATE:
            src = P<uint32_t>(c->sel) + select_hist_words(c->nsel); bytes = 32 * (int64_t)c->nsel; break;
        default: return fail(c, A3FR_EINVAL, "unknown buffer");
    }
    if (bytes_out) *bytes_out = bytes;
    if (!dst || bytes == 0) return A3FR_OK;
    if (bytes > max_bytes) return fail(c, A3FR_EINVAL, "destination too small");
    if (make64) {
        const uint32_t *t = make64 == 1 ? P<uint32_t>(c->keys_e) : sorted_tiles(c);
        const uint32_t *v = make64 == 1 ? P<uint32_t>(c->vals_e) : sorted_vals(c);
        launch_make_keys64(t, v, Kc, P<Record>(c->rec), nrec, reinterpret_cast<uint64_t *>(dst), c->stream);
        return check_launch(c, "inspect");
    }
    // the records' slots: the compaction that formed them
    const uint32_t *rent = P<uint32_t>(c->ent_a);
    switch (conv) {
        case 1:
        case 2:
            launch_vals_to_index(conv == 1 ? P<uint32_t>(c->vals_e) : sorted_vals(c), Kc, rent, nrec, c->n,
                                 static_cast<uint32_t *>(dst), c->stream);
            return check_launch(c, "inspect");
        case 3:  // rectangles of the slots with records; x0 = 1, x1 = 0, y0 = 1, y1 = 0 elsewhere
            launch_fill_u32(static_cast<uint32_t *>(dst), 1u, 2 * m, c->stream);
            launch_scatter_dense_u64(P<uint64_t>(c->rect_e), rent, nrec, static_cast<uint64_t *>(dst), c->stream);
            return check_launch(c, "inspect");
        case 4:
            launch_fill_u32(static_cast<uint32_t *>(dst), 0u, (int64_t)(sizeof(Record) / 4) * m, c->stream);
            launch_scatter_dense_rec(P<Record>(c->rec), rent, nrec, static_cast<Record *>(dst), c->stream);
            return check_launch(c, "inspect");
        case 5:
            launch_gather_u32(c->map_mode ? P<uint32_t>(c->ent_b) : rent, P<uint32_t>(c->dval_a), n_ent,
                              static_cast<uint32_t *>(dst), c->stream);
            return check_launch(c, "inspect");
        default: break;
    }
    HIPCHECK(c, hipMemcpyAsync(dst, src, (size_t)bytes, hipMemcpyDeviceToDevice, c->stream));
    return A3FR_OK;
}

a3fr_status a3fr_fp64_probe(a3fr_ctx *c, const double *x, const double *y, double *sq, double *dv, int64_t n) {
    if (!c) return A3FR_EINVAL;
    if (n < 0 || (n > 0 && (!x || !y || !sq || !dv))) return fail(c, A3FR_EINVAL, "fp64_probe: bad arguments");
    launch_fp64_probe(x, y, sq, dv, n, c->stream);
    return check_launch(c, "fp64_probe");
}

}  // extern "C"
