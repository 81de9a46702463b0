/*
 * a3fr.h -- C ABI of the MI355X (gfx950) foveated 3D Gaussian Splatting library.
 *
 * The library renders a 3D Gaussian Splatting scene the way the paper's
 * renderer does it (Sec. 2.3: project every 3D Gaussian to a screen ellipse and
 * find the tiles it touches; sort each tile's ellipses by depth, near to far;
 * composite each pixel front to back), for several layers of several eyes at
 * once, reusing the projection of one pass over the scene for every layer
 * (Sec. 3.5: the projected Gaussians, per-tile subsets and depth-sorted lists
 * of the first round are buffered and reused by later rounds).  A foveated
 * frame has a full-resolution foveal layer around the gaze point and coarser
 * surrounding layers (Sec. 2.2 and Eq. 1, the foveal radius).
 *
 * Conventions (every entry point):
 *  - Pointers named *_dev are device pointers (hipMalloc'd or torch CUDA
 *    tensors), owned by the caller, which must keep them alive until the work
 *    enqueued on the context's stream has finished.  Host pointers are read
 *    before the call returns.
 *  - All work is enqueued on the context's HIP stream and is asynchronous,
 *    except where a call is documented to synchronise.
 *  - Errors: arguments are checked on the host before anything is enqueued
 *    and give A3FR_EINVAL (nothing enqueued); a failed device allocation gives
 *    A3FR_ENOMEM; a HIP runtime error gives A3FR_EDEVICE.  No C++ exception
 *    crosses this interface.  a3fr_last_error() returns a message for the
 *    last failure on the context.
 *  - Images are planar float32, [channel][row][column], row = y (down),
 *    column = x (right); pixel (x, y) is sampled at its centre (x+0.5, y+0.5).
 *  - The tile grid is 16 x 16 pixels; a view of W x H pixels has
 *    ceil(W/16) x ceil(H/16) tiles, row-major.
 */
#ifndef A3FR_H
#define A3FR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    A3FR_OK = 0,
    A3FR_EINVAL = 1,     /* bad argument; nothing was enqueued */
    A3FR_ENOMEM = 2,     /* device allocation failed */
    A3FR_ECAPACITY = 3,  /* a size limit of the library was exceeded (see each call) */
    A3FR_EDEVICE = 4,    /* HIP runtime error */
    A3FR_ENOTREADY = 5   /* call order violated (e.g. blend before bin_sort) */
} a3fr_status;

#define A3FR_TILE 16
#define A3FR_MASK_ALL 0      /* every tile of the view is rendered */
#define A3FR_MASK_DISC 1     /* tiles whose pixel-centre rectangle is within r_out of the gaze */
#define A3FR_MASK_ANNULUS 2  /* as DISC with r_out, minus tiles lying wholly within r_in */
/* (DISC and ANNULUS: a negative r_out selects no tile) */

typedef struct a3fr_ctx a3fr_ctx;

/* Scene (Sec. 2.3: every point carries a position, an anisotropic scale, a
 * rotation, an opacity and spherical-harmonic colour).  float32 device
 * pointers, already activated (scale = exp(log-scale), opacity =
 * sigmoid(logit)).  Geometry is structure-of-arrays (coalesced per-Gaussian
 * loads in projection); quat is (w, x, y, z) and is normalised inside the
 * library.  sh is per Gaussian, [n][(sh_degree+1)^2][3] (coefficient, then
 * channel), so that the colour of the few Gaussians that are drawn is one
 * contiguous gather. */
typedef struct {
    int64_t n;
    int32_t sh_degree;        /* 0..3 */
    int32_t reserved;
    const float *mean_dev;    /* [3][n] */
    const float *scale_dev;   /* [3][n] */
    const float *quat_dev;    /* [4][n] */
    const float *opacity_dev; /* [n] */
    const float *sh_dev;      /* [n][(sh_degree+1)^2][3] */
} a3fr_scene;

/* One rendered layer of one eye: a pinhole camera at this layer's resolution
 * plus the layer's active-tile mask.  OpenCV axes (x right, y down, z
 * forward); world->camera p = R x + t.  Views with the same eye index share
 * their colour (view-dependent spherical harmonics seen from campos) and must
 * carry the same R, t and campos.  Gaze and radii are in this layer's pixels. */
typedef struct {
    double R[9];          /* row-major */
    double t[3];
    double campos[3];     /* eye centre, world space (view direction for colour) */
    double fx, fy, cx, cy;
    int32_t width, height;
    int32_t eye;          /* 0 .. 127 */
    int32_t mask;         /* A3FR_MASK_* */
    int32_t select;       /* 1: draw only the kept periphery subset (see a3fr_preprocess) */
    int32_t reserved;
    double gx, gy;        /* gaze point */
    double r_in, r_out;   /* mask radii */
    float bg[3];          /* background colour */
    int32_t reserved2;
} a3fr_view;

/* An eye camera at full resolution. */
typedef struct {
    double R[9];
    double t[3];
    double campos[3];
    double fx, fy, cx, cy;
    int32_t width, height;
    float bg[3];
    int32_t reserved;
} a3fr_camera;

typedef struct { double x, y; } a3fr_gaze; /* full-resolution pixel coordinates */

/* Layered foveation (Sec. 2.2: foveal region at full resolution, surrounding
 * regions at progressively lower resolution; Eq. 1 sizes the foveal radius).
 * Full-resolution pixels within r_fovea of the gaze come from the fovea layer,
 * those within r_mid from the mid layer (1/scale_mid per axis, bilinear), the
 * rest from the periphery layer (1/scale_periph per axis, bilinear), which
 * draws only the ceil(keep_num/keep_den x N_vis) visible Gaussians of largest
 * opacity x projected area (ties to the lower index). */
typedef struct {
    double r_fovea, r_mid;    /* full-resolution pixels, 0 <= r_fovea <= r_mid */
    int32_t scale_mid;        /* 2 */
    int32_t scale_periph;     /* 4 */
    int32_t keep_num, keep_den; /* 3, 10 */
    double margin;            /* mid-layer bilinear support in mid-layer pixels (2.0) */
} a3fr_fovea;

/* Counters of the last bin_sort / blend. */
typedef struct {
    int64_t n_keys;         /* (tile, depth) keys emitted */
    int64_t n_kept[16];     /* kept periphery points per selecting view (first 16 views) */
    int64_t n_tiles;        /* tiles of all views */
    int64_t n_active_tiles; /* tiles rendered */
    int64_t n_fallback_tiles; /* periphery tiles re-rendered at full resolution (a3fr_set_fallback) */
} a3fr_counts;

/* ---- context ------------------------------------------------------------ */

/* Create a context bound to a HIP stream (hipStream_t; NULL = default
 * stream).  The context owns a growable device workspace (allocated with
 * hipMalloc on first use, freed by a3fr_destroy). */
a3fr_status a3fr_create(a3fr_ctx **out, void *hip_stream);
void a3fr_destroy(a3fr_ctx *ctx);
a3fr_status a3fr_set_stream(a3fr_ctx *ctx, void *hip_stream);
/* Debug option: keep a copy of the keys in emission order for a3fr_inspect
 * (costs one extra device copy of the keys per a3fr_bin_sort). */
a3fr_status a3fr_set_debug(a3fr_ctx *ctx, int32_t keep_emission_order);
/* Blocks until the context's stream is idle; reports deferred device errors. */
a3fr_status a3fr_sync(a3fr_ctx *ctx);
/* How the host thread waits inside the library (a3fr_sync and the key-count
 * read of a3fr_bin_sort): blocking = 0 polls (the lowest wake-up latency, the
 * default; the counts are then written by the kernel that forms them straight
 * into host-coherent memory and polled there, with no copy or event in the
 * stream); 1 sleeps on blocking-sync events, leaving the CPU to other threads
 * (the gaze tracker of Algorithm 1, which runs on the CPU beside the renderer,
 * Sec. 3.1).  A3FR_EINVAL for other values. */
a3fr_status a3fr_set_host_wait(a3fr_ctx *ctx, int32_t blocking);
const char *a3fr_status_str(a3fr_status s);
const char *a3fr_last_error(const a3fr_ctx *ctx);

/* ---- the rendering path ---------------------------------------------------*/

/* Projection of every (view, Gaussian) pair (Sec. 2.3, projection stage: each
 * ellipsoid becomes a screen ellipse and the tiles it intersects are found):
 * near-plane cull (z <= 0.2), EWA projection of the 3D covariance to a 2D
 * covariance Sigma2D dilated by 0.3 px^2, and the tile rectangle of the
 * axis-aligned box around the part of the ellipse where the Gaussian can be
 * drawn: {d : d' Sigma2D^-1 d <= Q(o)}, where Q(o), for opacity o, is the
 * smallest k/8 (k = 1..88) with exp(k/16) >= 1.001 x 255 o, else 11.1.  A
 * pixel outside that box has alpha = o exp(-q/2) < 1/255 and is skipped by
 * the blend, so the tile lists, and the images, do not depend on the tile
 * shape.  Then: the number of active tiles the rectangle covers, the float32
 * depth key, and the view-dependent SH colour per eye.  The integer results
 * are computed in float64 in a fixed operation order (bit-exact against the
 * reference definition).  For views with select = 1 the periphery subset is
 * chosen here: over the Gaussians whose box meets the view, the
 * ceil(keep_num/keep_den x N_vis) of largest opacity x pi x sqrt(det Sigma2D),
 * ties to the lower index (radix select on the float64 score bits).  Then the
 * key counts are prefix-summed.
 * views: host array of n_views (1..384) views.  keep = keep_num/keep_den
 * (ignored without selecting views).  The results stay in the context and are
 * reused by a3fr_bin_sort and a3fr_blend until the next a3fr_preprocess
 * (Sec. 3.5).  Limits: n < 2^31; every view <= 65535 tiles per axis. */
a3fr_status a3fr_preprocess(a3fr_ctx *ctx, const a3fr_scene *scene, const a3fr_view *views, int32_t n_views,
                            int32_t keep_num, int32_t keep_den);

/* Tile-key duplication and depth sort (Sec. 2.3, sorting stage): the result
 * is, per tile, the list of Gaussians whose footprint box covers it, ordered by
 * (float32 depth bits, Gaussian index) -- the order of a stable sort of
 * (global tile id << 32 | depth bits) keys emitted in index order.  It is
 * built as: visible entries sorted by depth (in a3fr_preprocess), one 32-bit
 * tile-id key per (entry, active tile) emitted in that order (value =
 * Gaussian index), a stable LSD radix sort by tile id, then each tile's
 * [start, end) run.  Global tile id = the view's tile offset (views in order)
 * + row x tiles_x + column.
 * SYNCHRONISES once (reads the entry and key counts; the entries' blend
 * records are formed meanwhile).  *n_keys_out (host, may be NULL) receives the
 * key count.  A3FR_ECAPACITY if the count reaches 2^32 (keys are addressed by
 * 32-bit positions). */
a3fr_status a3fr_bin_sort(a3fr_ctx *ctx, int64_t *n_keys_out);

/* Front-to-back blend of every active tile (Sec. 2.3, rasterization stage):
 * alpha = min(0.99, o exp(-q/2)), q the Mahalanobis distance of the pixel
 * centre; alpha < 1/255 is skipped; a pixel stops before the Gaussian that
 * would bring its transmittance below 1e-4; output = colour + T x bg.
 * rgb_dev: all views' images concatenated in view order, each [3][H][W];
 * T_dev (may be NULL): final transmittance, [H][W] per view, concatenated;
 * last_dev (may be NULL): 1 + list position of the last blended Gaussian
 * (0: none).  Pixels of inactive tiles are not written. */
a3fr_status a3fr_blend(a3fr_ctx *ctx, float *rgb_dev, float *T_dev, uint32_t *last_dev);

/* Plain full-resolution render (FRR) of n_cams eye cameras: every tile, every
 * Gaussian.  out_dev: [n_cams][3][H][W].  Synchronises once (a3fr_bin_sort). */
a3fr_status a3fr_render_full(a3fr_ctx *ctx, const a3fr_scene *scene, const a3fr_camera *cams, int32_t n_cams,
                             float *out_dev);

/* Foveated stereo frame: the three layers of each of n_eyes eyes
 * (a3fr_make_foveated_views) rendered in one preprocess / sort / blend,
 * then composited to full resolution: out_dev [n_eyes][3][H][W].
 * Synchronises once (a3fr_bin_sort).  With the upsampler set (and at most 8
 * eyes, a grid blend variant, profiling off) the fovea and mid layers are
 * blended on a second, internal stream beside the periphery's blend and the
 * network; the context's stream waits for it before the composite, so the
 * output is ordered on the context's stream as for any other call. */
a3fr_status a3fr_render_foveated(a3fr_ctx *ctx, const a3fr_scene *scene, const a3fr_camera *cams,
                                 const a3fr_gaze *gaze, int32_t n_eyes, const a3fr_fovea *fovea, float *out_dev);

/* Batched gaze trace: n_frames consecutive stereo frames, each with its own
 * head pose and gaze, rendered as ONE batch -- every layer of every eye of every
 * frame in one projection pass over the scene, one key sort and one blend
 * launch (tiles of all views in one grid, uneven tile counts), then
 * composited (Sec. 3.5: the projection and per-tile lists of the scene are
 * shared by all the regions rendered from it).  This is a3fr_render_foveated
 * with n_eyes = 2 n_frames, eye 2f + k being eye k (0 left, 1 right) of frame
 * f, and gives the same images as the frames rendered one at a time.
 * cams, gaze: host arrays [n_frames][2], frame-major.  out_dev: device
 * [n_frames][2][3][H][W].  n_frames in [1, 64].  Synchronises once
 * (a3fr_bin_sort); for a batch without host read-back capture it with
 * a3fr_graph_capture (n_eyes = 2 n_frames) and replay it per window. */
a3fr_status a3fr_render_batch(a3fr_ctx *ctx, const a3fr_scene *scene, const a3fr_camera *cams,
                              const a3fr_gaze *gaze, int32_t n_frames, const a3fr_fovea *fovea, float *out_dev);

/* Host helper: the 3 layer views of each eye (eye-major, layer-minor:
 * fovea disc of radius r_fovea at full resolution; mid annulus at 1/scale_mid
 * with radii r_fovea/s - margin and r_mid/s + margin; periphery at
 * 1/scale_periph, every tile, select = 1).  out: host array of 3*n_eyes. */
a3fr_status a3fr_make_foveated_views(const a3fr_camera *cams, const a3fr_gaze *gaze, int32_t n_eyes,
                                     const a3fr_fovea *fovea, a3fr_view *out);

/* Composite of one eye's three layers (fovea [3][H][W], mid [3][H/sm][W/sm],
 * periphery [3][H/sp][W/sp]) into out_dev [3][H][W]: region by the distance
 * of the pixel centre to the gaze (float64 test), bilinear with
 * align_corners = false and clamp-to-edge for the coarser layers.  If
 * periph_full_dev is not NULL it replaces the bilinear periphery (an
 * already-upsampled [3][H][W] image). */
a3fr_status a3fr_composite(a3fr_ctx *ctx, int32_t W, int32_t H, a3fr_gaze gaze, const a3fr_fovea *fovea,
                           const float *fovea_dev, const float *mid_dev, const float *periph_dev,
                           const float *periph_full_dev, float *out_dev);

/* Quality judge: squared error of two [3][H][W] images, both clamped to
 * [0,1], summed over RGB per region (0 fovea, 1 mid, 2 periphery; by the same
 * distance test as the composite) in float64, and the pixel count per
 * region.  sse3 and count3 are host arrays of 3; synchronises.
 * PSNR = 10 log10(count x 3 / sse). */
a3fr_status a3fr_region_sse(a3fr_ctx *ctx, int32_t W, int32_t H, a3fr_gaze gaze, double r_fovea, double r_mid,
                            const float *a_dev, const float *b_dev, double *sse3, int64_t *count3);

/* For callers that cannot allocate -- code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc: a3fr_region_sse with no
 * device or host allocation and no synchronisation.  The same sums, bit for
 * bit, written to device memory on the context's stream:
 * sse3_dev: double[3] and count3_dev: int64_t[3], device pointers owned by the
 * caller.  The per-block partial sums live in a static device array of the
 * library (1024 blocks x 3 regions x (8 + 8) bytes = 48 KiB; every GPU the
 * library runs on holds its own copy until the process ends), which every call
 * overwrites in full (nothing is cleared).  Calls that overlap on one GPU (on
 * different streams or contexts) race on that array: serialise them.
 * Limits: 1 <= W, H and W x H <= A3FR_NOALLOC_MAX_PIXELS, else A3FR_EINVAL
 * with nothing enqueued. */
#define A3FR_NOALLOC_MAX_PIXELS 2147483647
a3fr_status a3fr_region_sse_noalloc(a3fr_ctx *ctx, int32_t W, int32_t H, a3fr_gaze gaze, double r_fovea,
                                    double r_mid, const float *a_dev, const float *b_dev, double *sse3_dev,
                                    int64_t *count3_dev);

/* Counters of the last preprocess / bin_sort (host struct). */
a3fr_status a3fr_get_counts(a3fr_ctx *ctx, a3fr_counts *out);

/* ---- AMR levels -------------------------------------------------------------- */

/* Adaptive resolution by 2 x 2 pixel blocks (Sec. 3.4 and Fig. 8; Sec. 3.5:
 * tiles labelled with levels 1 to 4): every tile of the full-resolution view
 * is split into 2 x 2 blocks; a tile of level L renders the first L positions
 * of each block (top-left, top-right, bottom-left, bottom-right) with all
 * Gaussians; a level-4 tile equals a3fr_render_full's pixels.
 *
 * Levels (level_mode):
 *   0  eccentricity: 4 if the tile's pixel-centre rectangle lies within
 *      r_level[0] of the gaze, 3 within r_level[1], 2 within r_level[2], else 1
 *      (0 <= r_level[0] <= r_level[1] <= r_level[2], full-resolution pixels;
 *      the distance test of A3FR_MASK_DISC);
 *   1  Gaussian count: the view's T tiles ranked by the number of keys that
 *      land in them (descending, ties to the lower tile index y * tiles_x + x);
 *      the first ceil(count_frac[0] T) have level 4, the first
 *      ceil(count_frac[1] T) at least 3, the first ceil(count_frac[2] T) at
 *      least 2 (0 <= count_frac[0] <= count_frac[1] <= count_frac[2] <= 1):
 *      tiles with few Gaussians are smooth and take fewer samples (Sec. 3.6);
 *   2  the smaller of the two.
 * Unrendered positions (fill):
 *   0  inherit the rendered pixel above them, else the top-left one;
 *   1  interpolate the blocks' top-left samples (rendered at every level)
 *      bilinearly at the pixel's position on that half-resolution grid, the
 *      last block clamped: 0.5f * (a + b) between two samples (odd x or odd
 *      y), 0.25f * ((a + b) + (c + d)) among four (a top-left, b top-right, c
 *      bottom-left, d bottom-right neighbour sample), in float.
 * Fields a mode does not use are ignored; other values are A3FR_EINVAL. */
typedef struct {
    double r_level[3];
    int32_t level_mode;
    int32_t fill;
    double count_frac[3];
} a3fr_amr;

/* One full-resolution view per eye (as a3fr_render_full) rendered with AMR
 * levels around gaze[e]; out_dev [n_eyes][3][H][W] (every pixel written). */
a3fr_status a3fr_render_amr(a3fr_ctx *ctx, const a3fr_scene *scene, const a3fr_camera *cams, const a3fr_gaze *gaze,
                            int32_t n_eyes, const a3fr_amr *amr, float *out_dev);

/* ---- incremental foveal rendering -------------------------------------------- */

/* Incremental rendering of the foveal region as ever more accurate gaze
 * predictions arrive (Sec. 3.3): the layered frame of a3fr_render_foveated
 * built over several calls on one context.
 *
 * a3fr_incremental_begin: round 0, before any gaze.  Projects every layer of
 * every eye once and keeps the results in the context (Sec. 3.5: later rounds
 * use the buffered projection and never read the scene again), selects the
 * periphery subset and renders the periphery layer, which needs no gaze.
 * The fovea and mid layers are projected with empty masks; every visible
 * entry keeps its rectangle and record, coloured now.  Arguments as in
 * a3fr_render_foveated (no fallback in this mode).
 *
 * a3fr_incremental_round: for each eye, renders the fovea-layer tiles within
 * radius (full-resolution pixels, the same tile test as A3FR_MASK_DISC) of
 * gaze[e], and the mid-layer tiles within radius + (r_mid - r_fovea) of it
 * (plus the mid layer's margin, in its pixels), that no earlier round of this
 * frame rendered; radius 0 renders no fovea tile.  The radius of a round
 * follows from the expected distance E between this prediction and the final
 * one (Eq. 4: r_f - E, at least 0; with no newer prediction, rendering may
 * continue around the same gaze up to r_f + E, Eq. 5; the mid layer's outer
 * radius is offset by the same E) -- the caller's schedule.
 *
 * a3fr_incremental_finish: the final gaze (one per eye).  Renders the fovea
 * tiles within r_fovea of it and the mid layer's annulus around it that are
 * not yet rendered, then composites into out_dev [eyes][3][H][W].  With the
 * upsampler set at a3fr_incremental_begin the whole periphery is upsampled
 * there, before any gaze.  The result equals a3fr_render_foveated with that
 * gaze.
 *
 * Tiles and keys of each round: a3fr_get_counts after the call.  Any other
 * a3fr_preprocess, render or graph call on the context ends the frame (the
 * rounds share its buffers): a later round or finish then returns
 * A3FR_ENOTREADY.  A3FR_EINVAL while a captured graph is held. */
a3fr_status a3fr_incremental_begin(a3fr_ctx *ctx, const a3fr_scene *scene, const a3fr_camera *cams, int32_t n_eyes,
                                   const a3fr_fovea *fovea);
a3fr_status a3fr_incremental_round(a3fr_ctx *ctx, const a3fr_gaze *gaze, double radius);
a3fr_status a3fr_incremental_finish(a3fr_ctx *ctx, const a3fr_gaze *gaze, float *out_dev);

/* ---- training: device activation and the backward pass ------------------ */

/* The optimised (raw) parameters of the scene.  Sec. 2.3: every point carries
 * trainable position, scale, rotation, opacity and SH colour; the scale is
 * optimised as its logarithm and the opacity as a logit, so that any real
 * value is valid.  float32 device pointers, layouts as in a3fr_scene. */
typedef struct {
    int64_t n;
    int32_t sh_degree;          /* 0..3 */
    int32_t reserved;
    const float *mean_dev;      /* [3][n] */
    const float *log_scale_dev; /* [3][n] */
    const float *quat_dev;      /* [4][n] (w, x, y, z), any non-zero norm */
    const float *logit_dev;     /* [n] */
    const float *sh_dev;        /* [n][(sh_degree+1)^2][3] */
} a3fr_params;

/* Gradients of a scalar loss with respect to a3fr_params, same layouts,
 * float32 device pointers owned by the caller; overwritten (not accumulated). */
typedef struct {
    float *mean_dev;      /* [3][n] */
    float *log_scale_dev; /* [3][n] */
    float *quat_dev;      /* [4][n] */
    float *logit_dev;     /* [n] */
    float *sh_dev;        /* [n][(sh_degree+1)^2][3] */
} a3fr_grads;

/* Activation on the device: scale_dev [3][n] = exp(log_scale) and
 * opacity_dev [n] = 1/(1 + exp(-logit)), each evaluated in float64 and
 * rounded once to float32.  Together with params->mean_dev, quat_dev and
 * sh_dev they form the a3fr_scene of the forward render. */
a3fr_status a3fr_activate(a3fr_ctx *ctx, const a3fr_params *params, float *scale_dev, float *opacity_dev);

/* Reverse mode of a3fr_blend for the frame of the last a3fr_preprocess /
 * a3fr_bin_sort / a3fr_blend: given dL/d(rgb) (dl_drgb_dev, the layout of
 * a3fr_blend's rgb_dev) and that blend's T_dev and last_dev outputs, each
 * active tile walks its list back to front from the last blended Gaussian,
 * recovering the transmittance in front of every Gaussian by dividing by
 * (1 - alpha) -- nothing is stored per (pixel, Gaussian) -- and accumulates,
 * per (view, Gaussian), dL/d(opacity), dL/d(rgb) and the sums that give
 * dL/d(2D centre) and dL/d(inverse 2D covariance).  Alpha and the skip and
 * stop decisions are evaluated exactly as in the forward blend; where alpha
 * is clamped at 0.99 it passes no gradient.  The accumulators stay in the
 * context for a3fr_preprocess_backward.  Pixels of inactive tiles are
 * ignored; last values beyond a tile's list are clamped to its length. */
a3fr_status a3fr_blend_backward(a3fr_ctx *ctx, const float *dl_drgb_dev, const float *T_dev,
                                const uint32_t *last_dev);

/* Reverse mode of the projection and colour of a3fr_preprocess and of
 * a3fr_activate, after a3fr_blend_backward: for every Gaussian, the chain
 * rule in float64 from the accumulated 2D gradients of each view through the
 * EWA projection (with the guard-band clamp of the Jacobian), the view
 * covariance, the 3D covariance R(q) S S' R(q)', the quaternion
 * normalisation, the exponential of the log-scale and the sigmoid of the
 * logit, and from the colour gradient through the clamp at zero and the SH
 * basis to the SH coefficients and, through the viewing direction, the
 * mean.  Gradients are summed over the views and written to *grads.
 * params must be the parameters whose activation was rendered (same n and
 * sh_degree as the scene of the last a3fr_preprocess). */
a3fr_status a3fr_preprocess_backward(a3fr_ctx *ctx, const a3fr_params *params, const a3fr_grads *grads);

/* ---- learned peripheral upsampler ------------------------------------------ */

/* The periphery is rendered at 1/4 resolution per axis (Sec. 2.2: detail
 * decreases away from the fovea; Sec. 3.5: coarse regions are interpolated
 * from the rendered samples).  This network brings it back to full
 * resolution:
 *   out = pixel_shuffle_x4(conv3(relu(conv2(relu(conv1(x)))))) + bilinear_x4(x),
 * 3x3 convolutions (zero padding 1, bias) of 3->32, 32->32 and 32->48
 * channels; channel c*16 + 4i + j of conv3 goes to output pixel
 * (c, 4y+i, 4x+j); bilinear with align_corners = false, clamp to edge,
 * interpolated vertically and then horizontally (as the composite's
 * bilinear, so that a zero network gives the bilinear frame bit for bit).
 * bfloat16 operands (input, weights, post-ReLU activations) on the matrix
 * cores with float32 accumulation; the last layer, the shuffle and the
 * residual are float32.
 * theta_dev: the flat float32 parameter vector of A3FR_NET_PARAMS values,
 *   W1 [32][3][3][3], b1 [32], W2 [32][32][3][3], b2 [32], W3 [48][32][3][3],
 *   b3 [48] (weights [out][in][ky][kx]). */
#define A3FR_NET_PARAMS 24016

/* in_dev: float32 [B][3][h][w]; out_dev: float32 [B][3][4h][4w].
 * for_training = 0: one fused launch (the activations stay on chip; the
 * weights are rounded to bf16 in the kernel).  for_training = 1: the three
 * layers one launch each, keeping the activations (and their channel-major
 * copies) in the context for a3fr_net_backward.  Both give the same bits. */
a3fr_status a3fr_net_forward(a3fr_ctx *ctx, const float *theta_dev, const float *in_dev, int32_t batch, int32_t h,
                             int32_t w, float *out_dev, int32_t for_training);

/* Mean squared error of the last training forward's out_dev against
 * target_dev (float32 [B][3][4h][4w], both 16-byte aligned, else
 * A3FR_EINVAL) and its gradient with respect to theta:
 * grad_dev (float32 [A3FR_NET_PARAMS], overwritten); loss_dev (float32 [1],
 * may be NULL) receives the loss.  The gradient entering each convolution's
 * weight and input gradients is rounded to bfloat16 (matrix-core operands);
 * weight gradients accumulate in float32. */
a3fr_status a3fr_net_backward(a3fr_ctx *ctx, const float *theta_dev, const float *out_dev, const float *target_dev,
                              float *grad_dev, float *loss_dev);

/* One Adam step on theta_dev with moment buffers m_dev, v_dev (float32
 * [A3FR_NET_PARAMS], zero before step 1): bias-corrected moments, step >= 1. */
a3fr_status a3fr_net_adam(a3fr_ctx *ctx, float *theta_dev, const float *grad_dev, float *m_dev, float *v_dev,
                          int32_t step, float lr, float beta1, float beta2, float eps);

/* ---- foveated-frame options -------------------------------------------------- */

/* Upsample the periphery of a3fr_render_foveated with the learned network
 * (theta_dev: A3FR_NET_PARAMS float32 on the device, used by reference until
 * changed) instead of bilinear x4; NULL restores bilinear.  The frame width
 * and height must then be divisible by fovea->scale_periph, which must be 4. */
a3fr_status a3fr_set_upsampler(a3fr_ctx *ctx, const float *theta_dev);

/* Per-tile error estimate of the periphery with full-resolution fallback in
 * a3fr_render_foveated.  For each periphery tile, D and K are the opacity
 * mass per periphery pixel (integral of o exp(-q/2): 2 pi o sqrt(det Sigma2D),
 * each Gaussian's spread evenly over the tiles of its rectangle) of the
 * visible Gaussians the periphery subset dropped and kept; with the
 * transmittance model T ~ exp(-mass), dropping raises the tile's
 * transmittance by dT = exp(-K) - exp(-(K + D)), and the squared-error
 * estimate is coef x (dT^2)^power.  Tiles whose estimate is >= mse_threshold
 * and that reach outside r_mid are rendered at full resolution with every
 * Gaussian (they join the fovea layer's tile mask in the same pass) and
 * taken from there by the composite.  mse_threshold = 0: every such tile, so
 * the periphery equals the plain full-resolution render; +infinity: none
 * (the default).  mse_threshold >= 0, coef >= 0, power > 0. */
a3fr_status a3fr_set_fallback(a3fr_ctx *ctx, double mse_threshold, double coef, double power);

/* ---- blend variants and autotuning ----------------------------------------- */

/* The forward blend has A3FR_BLEND_VARIANTS implementations, all giving
 * bit-identical images (every pixel evaluates the same float32 expressions
 * over the same list in the same order):
 *   variant = schedule * 6 + rows_per_lane_index * 3 + batch_index,
 *   batch (records staged in LDS per step) = {32, 64, 128}[batch_index],
 *   lane pixel block = 4 x 1 (rows_per_lane_index 0) or 2 x 2 (1),
 *   schedule 0: one wave per tile in tile order; 1: persistent waves pulling
 *   active tiles longest list first (the paper's ordering of tiles by their
 *   number of Gaussians, Sec. 3.5), from an O(tiles) bucket order by the bit
 *   length of the list length;
 * and, for variant = 12 + batch_index, a block of four waves per tile in tile
 * order, each wave one 8 x 8 quadrant with one pixel per lane (the
 * cooperative groups of the paper's AMR renderer, Sec. 3.4), batch
 * {64, 128, 256}[batch_index]: each wave walks only the entries that can
 * reach its quadrant.
 * The tile itself stays 16 x 16 (the binning unit of the keys). */
#define A3FR_BLEND_VARIANTS 15
a3fr_status a3fr_set_blend_variant(a3fr_ctx *ctx, int32_t variant);

/* Times every variant on the current frame (after a3fr_bin_sort; writes a
 * scratch image, not the caller's), reps timed blends each after one
 * warm-up, and selects the fastest for later a3fr_blend calls.  ms_out (host,
 * A3FR_BLEND_VARIANTS, may be NULL): mean ms per blend; best_out (host, may
 * be NULL): the chosen variant.  Synchronises. */
a3fr_status a3fr_autotune_blend(a3fr_ctx *ctx, int32_t reps, double *ms_out, int32_t *best_out);

/* ---- HIP graphs ---------------------------------------------------------------- */

/* Records the whole foveated frame of a3fr_render_foveated (preprocess,
 * selection, fallback, key emission and sort, blend, upsampler, composite,
 * with the context's options at this moment) into a HIP graph, for frames of
 * the same layout (image sizes, eyes, fovea parameters) and poses and gazes
 * given at launch (n_eyes = 2 x frames for a batch of stereo frames, as in
 * a3fr_render_batch).  No host read-back happens inside the graph: key buffers
 * hold max_keys keys (1 <= max_keys < 2^32) and the key count stays on the
 * device; a frame with more keys is cut at max_keys and reported by a3fr_sync
 * as A3FR_ECAPACITY.  An exact frame first counts this layout's keys K0 and
 * entries E0 (A3FR_ECAPACITY if K0 > max_keys); the entries and their blend
 * records get a capacity of E0 x max_keys / K0 (+1024), also reported as
 * A3FR_ECAPACITY when exceeded.  A warm-up frame with those capacities then
 * sizes the workspace (both frames are also written to out_dev).
 * scene and out_dev must stay valid at the same addresses while the graph is
 * replayed.  If the context is bound to the null stream it is rebound to an
 * internal non-blocking stream (stream capture needs one).  While a graph is
 * held, other calls on the context also run with the key capacity. */
a3fr_status a3fr_graph_capture(a3fr_ctx *ctx, const a3fr_scene *scene, const a3fr_camera *cams,
                               const a3fr_gaze *gaze, int32_t n_eyes, const a3fr_fovea *fovea, float *out_dev,
                               int64_t max_keys);
/* Uploads this frame's views (cameras and gazes; same sizes as captured) and
 * replays the graph on the context's stream.  Asynchronous. */
a3fr_status a3fr_graph_launch(a3fr_ctx *ctx, const a3fr_camera *cams, const a3fr_gaze *gaze);
/* Releases the graph and returns the context to exact key counts. */
a3fr_status a3fr_graph_destroy(a3fr_ctx *ctx);

/* ---- per-stage timing (HIP events on the context's stream) -------------- */
typedef enum {
    A3FR_STAGE_MASKS = 0,      /* active-tile masks */
    A3FR_STAGE_PREPROCESS = 1, /* projection, blend records, key counts */
    A3FR_STAGE_SELECT = 2,     /* periphery radix select */
    A3FR_STAGE_SCAN = 3,       /* compaction of visible entries; key offsets in depth order */
    A3FR_STAGE_EMIT = 4,       /* key emission */
    A3FR_STAGE_SORT_HIST = 5,  /* per-partition digit counts and their scan, one launch per pass of the
                                  tile-id sort */
    A3FR_STAGE_SORT_PASS = 6,  /* the scatter of one pass of the tile-id sort (one launch per 8-bit digit) */
    A3FR_STAGE_RANGES = 7,     /* tile ranges */
    A3FR_STAGE_BLEND = 8,      /* front-to-back blend */
    A3FR_STAGE_COMPOSITE = 9,  /* foveated composite */
    A3FR_STAGE_DEPTH_SORT = 10,/* radix sort of the visible entries by depth (histograms + 4 onesweep passes) */
    A3FR_STAGE_ACTIVATE = 11,  /* device activation */
    A3FR_STAGE_BLEND_BWD = 12, /* reverse blend (including the clear of its accumulators) */
    A3FR_STAGE_PREPROCESS_BWD = 13, /* reverse projection, colour and activation */
    A3FR_STAGE_FALLBACK = 14,  /* periphery error estimate, fallback masks and recount */
    A3FR_STAGE_NET = 15,       /* upsampler inference in a3fr_render_foveated */
    A3FR_STAGE_COLOUR = 16,    /* view-dependent colour of the entries that emit keys */
    A3FR_STAGE_COUNT = 17
} a3fr_stage;

typedef struct {
    int64_t launches[A3FR_STAGE_COUNT]; /* timed intervals per stage */
    double ms[A3FR_STAGE_COUNT];        /* summed event time per stage */
    int64_t sort_keys;                  /* keys sorted by tile id, summed over the timed bin_sorts */
    int64_t sort_passes;                /* scatter passes of the tile-id sorts, summed */
    int64_t blend_pairs;                /* evaluated (pixel, Gaussian) pairs of the timed blends */
} a3fr_profile;

/* Per-stage event timing: enable = 0 off (the default), 1 on and blends also
 * count their evaluated (pixel, Gaussian) pairs (every list entry a pixel
 * evaluates while it has not stopped, the stopping one included; this runs
 * the counting variant of the blend), 2 on without pair counting (the blend
 * variant timed is the one used for rendering).  Each timed interval adds
 * two event records to the stream. */
a3fr_status a3fr_set_profiling(a3fr_ctx *ctx, int32_t enable);
/* Synchronises, returns the per-stage totals accumulated since the last call
 * (or since profiling was enabled) and resets them. */
a3fr_status a3fr_get_profile(a3fr_ctx *ctx, a3fr_profile *out);

/* ---- inspection of buffered intermediates (tests and tools) -------------- */
typedef enum {
    A3FR_BUF_COUNTS = 0,      /* uint32 [n_views][n] active tiles covered (before selection) */
    A3FR_BUF_DEPTH = 1,       /* uint32 [n_views][n] float32 depth bits (valid where count > 0) */
    A3FR_BUF_RECT = 2,        /* uint16 [n_views][n][4] x0,x1,y0,y1 tile rectangle (valid where count > 0) */
    A3FR_BUF_OFFSETS = 3,     /* uint32 [E + 1] exclusive prefix of the key counts of the E visible
                                 (kept) entries, in depth order (A3FR_BUF_DEPTH_ORDER) */
    A3FR_BUF_KEYS = 4,        /* uint64 [K] (tile << 32 | depth bits) keys in emission order: entries in
                                 depth order, tiles row-major (needs a3fr_set_debug) */
    A3FR_BUF_VALS = 5,        /* uint32 [K] values in emission order (needs a3fr_set_debug) */
    A3FR_BUF_SORTED_KEYS = 6, /* uint64 [K] (tile << 32 | depth bits), sorted */
    A3FR_BUF_SORTED_VALS = 7, /* uint32 [K] Gaussian indices, sorted */
    A3FR_BUF_RANGES = 8,      /* uint32 [n_tiles][2] start, end */
    A3FR_BUF_ACTIVE = 9,      /* uint8 [n_tiles] active-tile flags */
    A3FR_BUF_KEEP = 10,       /* uint8 [n_views][n] kept by the periphery subset (selecting views) */
    A3FR_BUF_RECORDS = 11,    /* 48-byte blend records [n_views][n]: f64 u, v; f32 conic terms, opacity, rgb
                                 (valid where count > 0) */
    A3FR_BUF_DEPTH_ORDER = 12,/* uint32 [E] visible (kept) entries view*n + index, sorted by (depth, view, index) */
    /* upsampler, after a3fr_net_forward(for_training = 1) (gradients after a3fr_net_backward);
       bfloat16 bits, [B][h][w][C] unless stated */
    A3FR_BUF_NET_X0 = 13,     /* rounded input, C = 8 (channels 3..7 zero) */
    A3FR_BUF_NET_A1 = 14,     /* bf16(relu(conv1)), C = 32 */
    A3FR_BUF_NET_A2 = 15,     /* bf16(relu(conv2)), C = 32 */
    A3FR_BUF_NET_G3 = 16,     /* bf16(dL/d conv3 output), C = 48 */
    A3FR_BUF_NET_G2 = 17,     /* bf16(dL/d conv2 output), C = 32 */
    A3FR_BUF_NET_G1 = 18,     /* bf16(dL/d conv1 output), [B][32][h+2][roundup(w,32)+16], data at row 1 and column 8 */
    /* full-resolution fallback, after an a3fr_render_foveated with a3fr_set_fallback */
    A3FR_BUF_FB_ENERGY = 19,  /* float32 [2][n_tiles]: dropped, kept opacity mass per pixel (periphery views' tiles) */
    A3FR_BUF_FB_FLAGS = 20,   /* uint8 [n_tiles]: 1 = periphery tile taken from the full-resolution layer */
    A3FR_BUF_SEL_STATE = 21,  /* uint32 [n_selecting_views][8]: periphery select of each selecting view:
                                 visible count, kept count k, rank left in the chosen bucket, mode (0 select,
                                 1 keep all, 2 keep none), level-1 and level-2 buckets, candidates, 0 */
    A3FR_BUF_AMR_LEVELS = 22  /* uint8 [n_tiles]: level 1..4 of every tile, after a3fr_render_amr */
} a3fr_buffer;

/* Device-to-device copy of an intermediate into dst_dev (at most max_bytes);
 * *bytes_out (host) receives its size.  dst_dev may be NULL to query. */
a3fr_status a3fr_inspect(a3fr_ctx *ctx, a3fr_buffer which, void *dst_dev, int64_t max_bytes, int64_t *bytes_out);

/* Device self-check used by the tests: out_sqrt[i] = sqrt(x[i]) and
 * out_div[i] = x[i] / y[i] in float64 on the device (the operations the
 * key path relies on being correctly rounded).  Device pointers, n >= 0. */
a3fr_status a3fr_fp64_probe(a3fr_ctx *ctx, const double *x_dev, const double *y_dev, double *sqrt_dev,
                            double *div_dev, int64_t n);

#ifdef __cplusplus
}
#endif
#endif /* A3FR_H */
