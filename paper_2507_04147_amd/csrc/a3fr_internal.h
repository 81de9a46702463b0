// Internal declarations of the gfx950 library (kernels + host glue).
// Not part of the public ABI; shared only between the library's own sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/a3fr.h"

namespace a3fr {

constexpr int kTile = A3FR_TILE;          // 16 x 16 pixel tiles
constexpr int kWave = 64;                 // CDNA wavefront
constexpr double kZNear = 0.2;
constexpr double kDilate = 0.3;           // low-pass dilation of the 2D covariance, px^2
constexpr double kExtentQ = 11.1;         // footprint box of {d' S^-1 d <= Q}; Q >= 2 ln 255
// The footprint of a Gaussian of opacity o is the box of {d' S^-1 d <= Q(o)}:
// Q(o) = the smallest k/8, k = 1..kExtentSteps, with exp(k/16) >= (1.001 x 255) o,
// else kExtentQ.  The projection takes exp(k/16), k = 0..kExtentSteps, as a table.
constexpr int kExtentSteps = 88;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;
constexpr int kMaxViews = 384;
constexpr int kMaxEyes = 128;  // eye slots per frame batch (64 stereo frames)

// Blend record of one entry (a (view, Gaussian) pair that is drawn): centre in
// float64 (so that the tile-relative offset keeps full precision at any image
// size) and the inverse 2D covariance in LDL^T form scaled for exp2:
//   log2 G(d) = a2 (dx + k dy)^2 + c2 dy^2,
//   a2 = -log2(e)/2 * c/det, k = -b/c, c2 = -log2(e)/2 / c,
// where (a, b, c) is the dilated 2D covariance and det = a c - b^2; opacity,
// view-dependent colour and the float32 depth bits.  Records are stored per
// entry, contiguously; a key's value is its entry's record index.
struct alignas(16) Record {
    double u, v;
    float a2, k, c2, o;
    float r, g, b;
    uint32_t dbits;
};
static_assert(sizeof(Record) == 48, "record layout");

// One Gaussian's geometry packed for the record pass's gathers (written by the
// projection, which reads the structure-of-arrays scene coalesced):
// a = (mean x, y, z, opacity), b = (scale x, y, z, quat w), c = (quat x, y, z, 0).
struct alignas(16) GeomPack {
    float4 a, b, c;
};
static_assert(sizeof(GeomPack) == 48, "packed geometry layout");

// Device copy of the per-frame view table, plus derived tile-grid data.
struct DevView {
    a3fr_view v;
    int32_t tiles_x, tiles_y;
    int64_t tile_off;     // first global tile id
    int64_t img_off;      // first pixel of this view in the concatenated images
    int64_t mask_off;     // offset of this view's row tables (rows x (tiles_x + 1)) in the mask arrays
    int64_t cum_off;      // offset of this view's 2D active-tile prefix ((rows + 1) x (tiles_x + 1))
    double limx, limy;    // guard band of the projection Jacobian: (1.3 (W/2)) / fx, (1.3 (H/2)) / fy
    int32_t sel_slot;     // index among selecting views, -1 if none
    int32_t remask;       // 1: the tile mask may change after projection (full-resolution fallback,
                          //    incremental rounds); invisible (view, Gaussian) slots then get an
                          //    empty rectangle
    int32_t round_flags;  // incremental rounds: kRoundExclDone, kRoundFrozen
    int32_t rect_slot;    // >= 0: the projection keeps every slot's rectangle at rect[rect_slot * n + i]
                          //    (views whose mask may grow, and the fallback's periphery views)
    int32_t keep_visible; // 1: every visible slot of the view becomes an entry with a record, with keys or
                          //    not (the first round of an incremental frame, for the later rounds)
    // tile columns [ax0, ax1] x rows [ay0, ay1] hold every tile the view's mask
    // can activate (a margin of one tile; the whole grid for MASK_ALL; empty
    // when ax0 > ax1)
    int32_t ax0, ax1, ay0, ay1;
};
// tiles already rendered by an earlier round (the done flags) are left out, and the new ones marked done
constexpr int32_t kRoundExclDone = 1;
// no tile of the view is rendered in this round
constexpr int32_t kRoundFrozen = 2;

// rectangle of a (view, Gaussian) slot that is not visible (x0 > x1): x0 = 1, x1 = 0, y0 = 1, y1 = 0
constexpr uint64_t kEmptyRect = 0x0000000100000001ull;


// ---- upsampler ----
// flat float32 parameter vector: W1 [32][3][3][3], b1 [32], W2 [32][32][3][3],
// b2 [32], W3 [48][32][3][3], b3 [48] (weights [out][in][ky][kx])
constexpr int kNetW1 = 0, kNetB1 = 864, kNetW2 = 896, kNetB2 = 10112, kNetW3 = 10144, kNetB3 = 23968;
constexpr int kNetParams = 24016;
// bf16 packed weights: forward [9][co][cin padded to 8], input gradient [9][ci][co]
struct NetPacked {
    uint16_t *f1, *f2, *d2, *f3, *d3;
};
constexpr int64_t kNetPackedElems = 9 * 32 * 8 + 9 * 32 * 32 * 2 + 9 * 48 * 32 * 2;
struct NetConvArgs {
    const uint16_t *in;       // NHWC bf16, KIN channels
    const uint16_t *wpk;      // [9][NOUT][KIN] bf16
    const float *bias;        // forward: [NOUT]
    const uint16_t *mask;     // input gradient: NHWC bf16 activation whose sign masks the result
    uint16_t *out;            // NHWC bf16 (nullable)
    uint16_t *out_chw;        // zero-bordered channel-major copy (nullable)
    const float *img_in;      // last layer: float32 planar input (bilinear residual), batch stride img_bstride
    float *img_out;           // last layer: float32 planar output [B][3][4h][4w], batch stride out_bstride
    int64_t img_bstride, out_bstride;  // floats between batch items (0: 3 h w and 3 (4h)(4w))
    int B, h, w;
    int rows;                 // image rows per block (forward launches)
    // frame mode (the periphery of a foveated frame, batch item b = eye b): the gaze
    // of item b is gv[b * gv_stride].v.gx / gy; waves whose pixels (with the
    // layer's halo) all lie within r_mid of the gaze are skipped, and the last
    // layer writes only output pixels outside r_mid (the composite's periphery)
    const DevView *gv;        // nullable: frame mode off
    int gv_stride;
    double rm;
};
// inference forward of all three layers in one launch (float32 parameters,
// input and output, optional frame mode as in NetConvArgs)
struct NetFusedArgs {
    const float *img_in;             // float32 planar [B][3][h][w], batch stride img_bstride (0: 3 h w)
    const float *theta;              // float32 parameters (rounded to bf16 in the kernel)
    float *img_out;                  // float32 planar [B][3][4h][4w], batch stride out_bstride (0: 3 (4h)(4w))
    int64_t img_bstride, out_bstride;
    int B, h, w;
    const DevView *gv;               // frame mode as in NetConvArgs (nullable)
    int gv_stride;
    double rm;
};
struct NetWgradArgs {
    const uint16_t *g;        // channel-major zero-bordered bf16 gradient, NOUT channels
    const uint16_t *in;       // channel-major zero-bordered bf16 layer input, KIN channels
    float *grad;              // flat float32 gradient (accumulated with atomics)
    int off_w, off_b;
    int B, h, w;
};
__host__ __device__ int net_chw_stride(int w);

// ---- kernels' host launchers (all enqueue on `s`) ----
// up to kFillSegs device ranges of 32-bit words to clear in one launch
constexpr int kFillSegs = 8;
struct FillSegs {
    uint32_t *p[kFillSegs];
    int64_t n[kFillSegs];  // words; only the first count are used
    int count;
};
// zero: ranges the same launch clears (count 0: none), so that a frame's
// accumulators need no launch of their own
void launch_tile_masks(const DevView *views, int nv, int64_t rows_total, const int32_t *row_view,
                       const int32_t *row_y, uint16_t *row_prefix, uint16_t *row_list, uint8_t *active,
                       uint8_t *done /* [tiles] nullable: incremental rounds */, const FillSegs &zero, hipStream_t s);
// counts [nv][n] every slot; depth [nv][n] of entries; rect [n_rect_views][n] (views with rect_slot >= 0);
// score [nsel][n] (selecting views, by sel_slot); cum: the masked views' summed-area tables (launch_mask_cum)
void launch_preprocess(const a3fr_scene &sc, const DevView *views, int ngroups, const int32_t *groups,
                       const uint32_t *cum, uint32_t *counts, uint32_t *depth, uint64_t *rect, double *score,
                       GeomPack *pack /* [n] */, const double *exp_tab /* [kExtentSteps + 1] */, hipStream_t s);
// records and rectangles of the entries ent[0 .. min(*n_ent, cap)), at the entry's index; map[slot] = index;
// a count above cap raises bit 2 of err
void launch_entry_record(const a3fr_scene &sc, const GeomPack *pack /* this frame's projection */,
                         const DevView *views, const uint32_t *ent, const uint32_t *n_ent, int64_t m, int64_t cap,
                         const double *exp_tab, Record *rec, uint64_t *rect_e, uint32_t *map, uint32_t *err,
                         hipStream_t s);
void launch_select(const DevView *views, int nv, const int32_t *sel_views, int nsel, int64_t n,
                   const uint32_t *counts, const double *score, int keep_num, int keep_den,
                   uint32_t *sel_ws /* select_workspace_words(nsel, n) words */, uint8_t *keep, hipStream_t s,
                   bool zeroed = false /* the first select_hist_words(nsel) words already zero */);
int64_t select_hist_words(int nsel);
int64_t select_workspace_words(int nsel, int64_t n);
// scan workspace (uint64 words) for m = nv * n entry slots; the compaction
// clears it, so the key offsets must follow that compaction
int64_t scan_workspace_words(int64_t m);
// entries (slots with keys, kept; every visible slot of a keep_visible view) in slot order:
// ent[j] = slot, dkey[j] = depth bits, dval[j] = j, ecnt[j] = the slot's key count (ecnt nullable)
// keep: a byte per slot, or NULL when no view selects; rect NULL: keep_visible views count as others
void launch_compact_entries(const uint32_t *counts, const uint8_t *keep, const uint64_t *rect, const DevView *views,
                            int nv, int64_t n, const uint32_t *depth, uint32_t *ent, uint32_t *dkey, uint32_t *dval,
                            uint32_t *ecnt, uint64_t *ws, uint64_t *total, uint32_t *n_ent, uint32_t *err,
                            hipStream_t s, bool zeroed = false /* ws already zero */);
// key offsets of the entries in depth order: order[k] = entry index, its count ecnt[order[k]];
// sig (nullable, host-coherent): E, K and then seq are written there for the host
void launch_key_offsets(const uint32_t *ecnt, const uint32_t *order, const uint32_t *n_ent, int64_t m,
                        uint32_t *offsets, uint64_t *ws, uint64_t *total, uint32_t *total32, uint32_t *err,
                        uint64_t *sig, uint64_t seq, hipStream_t s);
// number of key chunks (blocks) of the emission for K keys; chunk_start needs one word per chunk
int64_t emit_chunks(int64_t K);
// The entries of one emission, in depth order: entry order[k] of this pass has slot ent[order[k]]
// and record r = map ? map[slot] : order[k]; its rectangle is rect_e[r].  rect_s, esort, rsort
// (capacity cap) receive the rectangle, slot and record per depth-ordered entry.
struct EmitEntries {
    const uint32_t *order, *ent, *map;
    const uint64_t *rect_e;
    uint64_t *rect_s;
    uint32_t *esort, *rsort;
    int64_t cap;
};
void launch_emit(const DevView *views, int nv, int64_t n, int64_t m, const EmitEntries &ee, const uint32_t *n_ent,
                 const uint32_t *offsets, const uint16_t *row_prefix, const uint16_t *row_list, const uint32_t *cum,
                 uint32_t *chunk_start, uint32_t *keys, uint32_t *vals, int64_t K,
                 const uint32_t *K_dev /* nullable: device key count (clamped to K) */,
                 uint32_t *zero, int zero_words /* cleared by the first kernel (nullable when 0) */, hipStream_t s);
void launch_clamp_keys(const uint64_t *total, int64_t cap, const uint32_t *n_ent, const uint32_t *offsets,
                       int64_t ecap, uint32_t *n32, uint32_t *err, hipStream_t s);
void launch_mask_cum(const DevView *views, int nv, int max_tiles_x, const uint16_t *row_prefix, uint32_t *cum,
                     hipStream_t s, const uint32_t *skip_if_zero = nullptr /* device count: 0 skips */);
// inspection helpers: 64-bit keys (tile << 32 | record depth bits); key values as Gaussian indices;
// gathers and dense scatters of per-entry arrays
void launch_make_keys64(const uint32_t *tiles, const uint32_t *vals, int64_t K, const Record *rec, int64_t n_rec,
                        uint64_t *out, hipStream_t s);
void launch_vals_to_index(const uint32_t *vals, int64_t K, const uint32_t *rent, int64_t n_rec, int64_t n,
                          uint32_t *out, hipStream_t s);
void launch_gather_u32(const uint32_t *src, const uint32_t *idx, int64_t cnt, uint32_t *out, hipStream_t s);
void launch_scatter_dense_u64(const uint64_t *src, const uint32_t *ent, int64_t cnt, uint64_t *out, hipStream_t s);
void launch_scatter_dense_rec(const Record *src, const uint32_t *ent, int64_t cnt, Record *out, hipStream_t s);
// keys per thread of the radix passes: 16 (8192-key partitions) for the
// tile-id sort, 4 (2048-key partitions) for the entry depth sort
constexpr int kSortItemsLarge = 16;
constexpr int kSortItemsSmall = 4;
// entry depth sort (onesweep): workspace of a sort of at most n_max keys in
// npass passes (u32 words); its leading words must be zero before
// launch_onesweep_prepare (which clears them unless zeroed)
int64_t onesweep_workspace_words(int64_t n_max, int npass);
int64_t onesweep_zero_words(int npass);
void launch_onesweep_prepare(const uint32_t *keys, const uint32_t *n_dev, int64_t n_max, int npass, uint32_t *ws,
                             hipStream_t s, bool zeroed = false);
void launch_onesweep_pass(const uint32_t *ki, const uint32_t *vi, uint32_t *ko, uint32_t *vo, const uint32_t *n_dev,
                          int64_t n_max, int npass, int p, uint32_t *ws, uint32_t *err, hipStream_t s);
// tile-id sort (count, scan, scatter): workspace for at most n_max keys (u32
// words); its first sort_zero_words(n_max) words must be zero before the first
// pass (every pass leaves them zero).  Pass p sorts *n_dev keys by digit p.
int64_t sort_workspace_words(int64_t n_max);
int64_t sort_zero_words(int64_t n_max);
void launch_sort_count(const uint32_t *ki, const uint32_t *n_dev, int64_t n_max, int p, uint32_t *ws, hipStream_t s);
void launch_sort_scatter(const uint32_t *ki, const uint32_t *vi, uint32_t *ko, uint32_t *vo, const uint32_t *n_dev,
                         int64_t n_max, int p, const uint32_t *ws, hipStream_t s);
void launch_ranges(const uint32_t *tiles, int64_t K, const uint32_t *K_dev, int64_t ntiles, uint32_t *ranges,
                   hipStream_t s);
// forward blend: variants (LDS batch depth x lane pixel block x schedule), all bit-identical
// Tile ids of one blend launch: range y holds the global tiles
// [base[y], base[y] + len[y]); count 0 means every tile.
constexpr int kMaxTileRanges = 8;
struct TileRanges {
    int count;
    int64_t base[kMaxTileRanges], len[kMaxTileRanges];
};
struct BlendArgs {
    const DevView *views;
    int nv;
    int64_t ntiles;
    const uint8_t *active;
    const uint32_t *ranges, *vals;
    const Record *rec;
    int64_t n;
    float *rgb, *T;
    uint32_t *last;
    unsigned long long *pairs;   // nullable: count evaluated pairs
    uint32_t *ws;                // kBlendWsWords words (queue schedule)
    uint32_t *order;             // [ntiles] (queue schedule)
    int64_t queue_waves;         // persistent waves of the queue schedule
    TileRanges tr;               // grid schedules only (the queue schedule takes every tile)
};
struct BlendVariant { int batch, rows; bool queue, quad; };
// batch {32, 64, 128} x rows {1, 2} x {grid, queue}, then the quadrant blocks with batch {64, 128, 256}
constexpr int kBlendVariants = A3FR_BLEND_VARIANTS;
constexpr int kBlendDefault = 1;      // batch 64, 4 x 1 pixels per lane, grid
constexpr int kBlendWsWords = 68;
BlendVariant blend_variant(int k);
// AMR of full views (gaze in the views): tile levels (eccentricity radii r, count fractions f, mode 0
// eccentricity / 1 count / 2 the smaller), then the level-L blend of the first L positions of each 2 x 2 block,
// the others inherited or interpolated
struct AmrLevels {
    double r[3], f[3];
    int mode, interp;
};
void launch_blend_amr(const DevView *views, int nv, int64_t ntiles, const uint32_t *ranges, const uint32_t *vals,
                      const Record *rec, int64_t n, const AmrLevels &a, uint64_t *thr /* [nv][3] */,
                      uint8_t *lv /* [ntiles] */, float *rgb, int64_t max_pixels /* largest view */, hipStream_t s);
void launch_blend(const BlendArgs &a, int variant, hipStream_t s);
void launch_blend_order(const uint8_t *active, const uint32_t *ranges, int64_t ntiles, uint32_t *ws, uint32_t *order,
                        hipStream_t s);
void launch_blend_bwd(const DevView *views, int nv, int64_t ntiles, const uint8_t *active, const uint32_t *ranges,
                      const uint32_t *vals, const Record *rec, int64_t n, const float *dl_drgb, const float *T,
                      const uint32_t *last, float *acc /* [records][12] (n = 0: indexed by the key value) */,
                      hipStream_t s);
void launch_activate(const a3fr_params &p, float *scale, float *opacity, hipStream_t s);
// per Gaussian, over the views where its slot is an entry (count > 0, kept): record map[slot], sums acc[record]
void launch_preprocess_bwd(const a3fr_params &p, const DevView *views, int nv, const uint32_t *counts,
                           const uint8_t *keep, const uint32_t *map, const float *acc, const Record *rec,
                           const a3fr_grads &g, hipStream_t s);
// the packed weights of theta and the bf16 input (NHWC8, plus the
// channel-major copy when chw is not NULL; x_bstride 0: 3 h w), one launch
void launch_net_prep(const float *theta, const NetPacked &pk, const float *x, int64_t x_bstride, int B, int h, int w,
                     uint16_t *nhwc, uint16_t *chw, hipStream_t s);
void launch_net_conv(int layer, bool dgrad, const NetConvArgs &a, hipStream_t s);
void launch_net_fused(const NetFusedArgs &a, hipStream_t s);
void launch_net_wgrad(int layer, const NetWgradArgs &a, int slabs, hipStream_t s);
void launch_net_mse(const float *out, const float *target, int B, int h, int w, uint16_t *g_nhwc, uint16_t *g_chw,
                    double *sse, float *loss, hipStream_t s);
void launch_net_adam(float *theta, const float *grad, float *m, float *v, int n, float lr, float beta1, float beta2,
                     float eps, float bc1, float bc2, hipStream_t s);
// The fallback pairs of a frame (one per eye): periphery view pv, its eye's
// full-resolution view fv, the mid radius, and where the pair's difference
// planes [2][tiles_y+1][tiles_x+1] (float64) start in the shared buffer.
constexpr int kFbMax = 16;
constexpr int kFbLdsBytes = 48 * 1024;
struct FbBatch {
    int count;
    int max_cells;  // largest 2 (tiles_y+1)(tiles_x+1) over the pairs
    int pv[kFbMax], fv[kFbMax];
    double r_mid[kFbMax];
    int64_t doff[kFbMax];
};
int drop_energy_parts();
// Mass maps of every pair of the batch, then each pair's periphery tiles
// flagged (estimate coef (dT^2)^power >= threshold, outside r_mid) with the
// covered full-resolution tiles activated and n_flagged counted.
void launch_drop_energy(const DevView *views, const FbBatch &b, int64_t n, const uint32_t *counts,
                        const uint8_t *keep, const uint64_t *rect, const double *score,
                        double *diff /* zeroed planes of every pair, at b.doff */,
                        double *partials /* [b.count][drop_energy_parts()][b.max_cells] */, int64_t ntiles,
                        float *energy /* [2][ntiles]: dropped mass, kept mass */, double threshold, double coef,
                        double power, uint8_t *flags, uint8_t *active, uint32_t *n_flagged, hipStream_t s);
void launch_rows_from_active(const DevView *views, int64_t rows_total, const int32_t *row_view, const int32_t *row_y,
                             const uint8_t *active, uint16_t *row_prefix, uint16_t *row_list,
                             const uint32_t *n_flagged, hipStream_t s);
void launch_recount(const DevView *views, const FbBatch &b, int64_t n, const uint64_t *rect,
                    const uint16_t *row_prefix, uint32_t *counts, const uint32_t *n_flagged, hipStream_t s);
void launch_composite(int W, int H, double gx, double gy, double rf, double rm, const float *fovea,
                      const float *mid, int sm, const float *periph, int sp, const float *periph_full,
                      bool periph_done /* outside r_mid already written (unless fallback-flagged) */,
                      const uint8_t *fb_flags /* nullable: periphery tiles taken from fovea */, int fb_tiles_x,
                      const DevView *gaze_view /* nullable: read the gaze (v.gx, v.gy) from this device view */,
                      float *out, hipStream_t s);
// every eye of a frame, all W x H, in one launch: eye e's gaze, layers (at layers + 3 img_off) and
// fallback flags (fb_flags + tile_off of its periphery view; nullable) from views[3e .. 3e + 2];
// output at out + 3 W H e
void launch_composite_eyes(int n_eyes, int W, int H, double rf, double rm, int sm, int sp, const DevView *views,
                           const float *layers, bool periph_done, const uint8_t *fb_flags, float *out,
                           hipStream_t s);
void launch_region_sse(int W, int H, double gx, double gy, double rf, double rm, const float *a,
                       const float *b, double *partial /* [nblk][3] */, unsigned long long *cnt /* [nblk][3] */,
                       int nblk, hipStream_t s);
// the three region sums of the partials of launch_region_sse into device outputs
void launch_region_sse_sum(const double *partial, const unsigned long long *cnt, int nblk, double *sse3,
                           int64_t *count3, hipStream_t s);
void launch_fp64_probe(const double *x, const double *y, double *sq, double *dv, int64_t n, hipStream_t s);
void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
void launch_zero_segs(const FillSegs &f, hipStream_t s);

}  // namespace a3fr
