/*
 * a3fr_oracle.c -- plain FP64 CPU oracle for gaze-tracked foveated 3D Gaussian
 * Splatting.  TEST INFRASTRUCTURE ONLY: it is loaded by the tests, by the smoke
 * check and by the CPU-baseline leg of the benchmark, never by the product path.
 * It shares no code, header or constant table with the HIP library.
 *
 * What it computes follows the three stages of the 3DGS pipeline that the paper
 * builds on (Sec. 2.3 and the caption of the 3DGS-process figure: projection of
 * every ellipsoid to a screen ellipse and the tiles it touches; per-tile sort of
 * the ellipses by depth, near to far; front-to-back volume-rendering blend per
 * pixel), the buffering of the projected data for reuse by later layers
 * (Sec. 3.5), and a layered foveation (Sec. 2.2: a full-detail foveal region
 * with progressively coarser surrounding regions).  The paper states none of
 * the 3DGS formulas; the conventions used here are the textbook ones (EWA
 * splatting, real spherical harmonics of degree 3, alpha compositing) and are
 * listed with every other reading in DESIGN.md's "Readings" section.
 *
 * Everything is float64.  The key path (projection -> tile rectangle -> depth
 * key -> periphery score) follows a written operation order of fused
 * multiply-adds, correctly rounded divisions and square roots, so that its
 * integer results (tile rectangles, depth keys, kept set) are defined
 * bit-for-bit.  Build with -ffp-contract=off -fno-fast-math.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_ZNEAR 0.2
#define OR_DILATE 0.3
#define OR_EXTENT_Q 11.1          /* >= 2 ln 255: box of {d' S^-1 d <= Q} holds every alpha >= 1/255 */
#define OR_ALPHA_MIN (1.0 / 255.0)
#define OR_ALPHA_MAX 0.99
#define OR_T_MIN 1e-4

typedef struct {
    double R[9];        /* world -> camera rotation, row-major */
    double t[3];        /* world -> camera translation */
    double campos[3];   /* camera centre, world space */
    double fx, fy, cx, cy;
    int32_t width, height;
    int32_t eye;        /* colour slot shared by the layers of one eye */
    int32_t mask;       /* 0: every tile, 1: disc, 2: annulus */
    int32_t select;     /* 1: only the kept subset emits keys */
    int32_t pad_;
    double gx, gy;      /* gaze point in this view's pixels */
    double r_in, r_out; /* mask radii in this view's pixels */
    double bg[3];
} or_view;

/* ------------------------------------------------------------------------- */
/* tiny parallel-for                                                          */
/* ------------------------------------------------------------------------- */
typedef void (*or_body)(void *ctx, int64_t item);
typedef struct { or_body fn; void *ctx; int64_t n; int64_t next; } or_pool;

static void *or_worker(void *arg) {
    or_pool *p = (or_pool *)arg;
    for (;;) {
        int64_t i = __atomic_fetch_add(&p->next, 1, __ATOMIC_RELAXED);
        if (i >= p->n) break;
        p->fn(p->ctx, i);
    }
    return NULL;
}

static void or_parallel(int64_t n, or_body fn, void *ctx, int nthreads) {
    or_pool p = {fn, ctx, n, 0};
    if (nthreads <= 1 || n < 2) { or_worker(&p); return; }
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    int started = 0;
    for (int k = 0; k < nthreads - 1; ++k)
        if (pthread_create(&th[k], NULL, or_worker, &p) == 0) ++started;
    or_worker(&p);
    for (int k = 0; k < started; ++k) pthread_join(th[k], NULL);
}

/* ------------------------------------------------------------------------- */
/* tile grid                                                                  */
/* ------------------------------------------------------------------------- */
static inline int32_t or_tiles_x(const or_view *v, int32_t tw) { return (v->width + tw - 1) / tw; }
static inline int32_t or_tiles_y(const or_view *v, int32_t th) { return (v->height + th - 1) / th; }

/* Active-tile test.  A tile's pixel-centre rectangle [x0,x1]x[y0,y1] (clipped to
 * the image) is tested against the gaze disc(s). disc: active iff the squared
 * distance from the gaze to the rectangle is <= r_out^2. annulus: the same outer
 * test, and inactive when all four corners lie within r_in of the gaze (the tile
 * is covered by the inner layer).  A negative r_out is an empty mask (a layer
 * with nothing to render, as in the incremental rounds of Sec. 3.3 before a
 * radius is known). */
static int or_tile_active(const or_view *v, int32_t tw, int32_t th, int32_t tx, int32_t ty) {
    if (v->mask == 0) return 1;
    if (v->r_out < 0.0) return 0;
    int32_t xe = (tx + 1) * tw; if (xe > v->width) xe = v->width;
    int32_t ye = (ty + 1) * th; if (ye > v->height) ye = v->height;
    double x0 = (double)(tx * tw) + 0.5, x1 = (double)xe - 0.5;
    double y0 = (double)(ty * th) + 0.5, y1 = (double)ye - 0.5;
    double ddx = fmax(fmax(x0 - v->gx, v->gx - x1), 0.0);
    double ddy = fmax(fmax(y0 - v->gy, v->gy - y1), 0.0);
    double d2 = ddx * ddx + ddy * ddy;
    if (!(d2 <= v->r_out * v->r_out)) return 0;
    if (v->mask == 2 && v->r_in > 0.0) {
        double ri2 = v->r_in * v->r_in;
        double ax = x0 - v->gx, bx = x1 - v->gx, ay = y0 - v->gy, by = y1 - v->gy;
        int inside = (ax * ax + ay * ay <= ri2) && (bx * bx + ay * ay <= ri2) &&
                     (ax * ax + by * by <= ri2) && (bx * bx + by * by <= ri2);
        if (inside) return 0;
    }
    return 1;
}

void or_tile_masks(int32_t nv, const or_view *views, int32_t tw, int32_t th,
                   const int64_t *aoff, uint8_t *active) {
    for (int32_t v = 0; v < nv; ++v) {
        int32_t TX = or_tiles_x(&views[v], tw), TY = or_tiles_y(&views[v], th);
        for (int32_t ty = 0; ty < TY; ++ty)
            for (int32_t tx = 0; tx < TX; ++tx)
                active[aoff[v] + (int64_t)ty * TX + tx] = (uint8_t)or_tile_active(&views[v], tw, th, tx, ty);
    }
}

/* ------------------------------------------------------------------------- */
/* key path (FP64, written operation order)                                   */
/* ------------------------------------------------------------------------- */
/* View-space position and covariance of Gaussian i in the camera of view v.
 * Returns 0 when the point is culled by the near plane or has a degenerate
 * rotation quaternion. Sv holds (00,01,02,11,12,22). */
static int or_view_space(const float *mean, const float *scale, const float *quat, int64_t n, int64_t i,
                         const or_view *v, double p[3], double Sv[6]) {
    const double *Rw = v->R;
    double mx = mean[i], my = mean[n + i], mz = mean[2 * n + i];
    for (int k = 0; k < 3; ++k)
        p[k] = fma(Rw[3 * k + 0], mx, fma(Rw[3 * k + 1], my, fma(Rw[3 * k + 2], mz, v->t[k])));
    if (!(p[2] > OR_ZNEAR)) return 0;

    double qw = quat[i], qx = quat[n + i], qy = quat[2 * n + i], qz = quat[3 * n + i];
    double nq = sqrt(fma(qw, qw, fma(qx, qx, fma(qy, qy, qz * qz))));
    if (!(nq > 0.0)) return 0;
    double w = qw / nq, x = qx / nq, y = qy / nq, z = qz / nq;
    double xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z;
    double wx = w * x, wy = w * y, wz = w * z;
    double Rq[9] = {1.0 - 2.0 * (yy + zz), 2.0 * (xy - wz), 2.0 * (xz + wy),
                    2.0 * (xy + wz), 1.0 - 2.0 * (xx + zz), 2.0 * (yz - wx),
                    2.0 * (xz - wy), 2.0 * (yz + wx), 1.0 - 2.0 * (xx + yy)};
    double s0 = scale[i], s1 = scale[n + i], s2 = scale[2 * n + i];
    double M[9];
    for (int r = 0; r < 3; ++r) {
        M[3 * r + 0] = Rq[3 * r + 0] * s0;
        M[3 * r + 1] = Rq[3 * r + 1] * s1;
        M[3 * r + 2] = Rq[3 * r + 2] * s2;
    }
    /* Sigma3D = M M^T (symmetric, full matrix kept for the next product) */
    double S[9];
    for (int r = 0; r < 3; ++r)
        for (int c = r; c < 3; ++c) {
            double e = fma(M[3 * r + 0], M[3 * c + 0], fma(M[3 * r + 1], M[3 * c + 1], M[3 * r + 2] * M[3 * c + 2]));
            S[3 * r + c] = e; S[3 * c + r] = e;
        }
    /* A = Rw Sigma3D, then Sigma_view = A Rw^T */
    double A[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            A[3 * r + c] = fma(Rw[3 * r + 0], S[0 * 3 + c], fma(Rw[3 * r + 1], S[1 * 3 + c], Rw[3 * r + 2] * S[2 * 3 + c]));
    static const int pr[6] = {0, 0, 0, 1, 1, 2}, pc[6] = {0, 1, 2, 1, 2, 2};
    for (int k = 0; k < 6; ++k) {
        int r = pr[k], c = pc[k];
        Sv[k] = fma(A[3 * r + 0], Rw[3 * c + 0], fma(A[3 * r + 1], Rw[3 * c + 1], A[3 * r + 2] * Rw[3 * c + 2]));
    }
    return 1;
}

/* Exported for the pins: view-space mean and covariance (00,01,02,11,12,22)
 * of Gaussian i in view v; returns 0 when culled. */
int or_view_cov(const float *mean, const float *scale, const float *quat, int64_t n, int64_t i,
                const or_view *v, double *p, double *Sv) {
    return or_view_space(mean, scale, quat, n, i, v, p, Sv);
}

typedef struct {
    int ok;            /* projectable: in front of the near plane, det > 0 */
    int vis;           /* ok and the footprint box meets the image */
    double u, v;       /* centre, this view's pixels */
    double a, b, c;    /* dilated 2D covariance */
    double det;
    int32_t rect[4];   /* x0, x1, y0, y1 (inclusive tile indices) */
    uint32_t depth_bits;
} or_proj;

/* Footprint bound of a Gaussian of opacity o (Sec. 2.3: the tiles its ellipse
 * covers; a pixel takes it only where alpha = o exp(-q/2) >= 1/255, i.e.
 * q <= 2 ln(255 o)): Q(o) = the smallest k/8, k = 1..88, with
 * exp(k/16) >= (1.001 x 255) o, else 11.1 (>= 2 ln 255).  So
 * Q(o) >= 2 ln(255 o) + 2 ln 1.001, a margin far above the float32 rounding
 * of the blend's alpha, and the box of {d' S^-1 d <= Q(o)} holds every pixel
 * the Gaussian can reach.  Steps of 1/8 make Q(o) comparisons against exp at
 * fixed points, so no last bit of a logarithm moves a tile boundary. */
static double or_exp_tab[89];
static pthread_once_t or_exp_once = PTHREAD_ONCE_INIT;
static void or_exp_init(void) {
    for (int k = 0; k <= 88; ++k) or_exp_tab[k] = exp((double)k / 16.0);
}
static double or_extent_q(double o) {
    pthread_once(&or_exp_once, or_exp_init);
    const double t = (1.001 * 255.0) * o;
    for (int k = 1; k <= 88; ++k)
        if (or_exp_tab[k] >= t) return (double)k / 8.0;
    return OR_EXTENT_Q;
}

/* Exported for the pins: the footprint bound Q(o). */
double or_footprint_q(double o) { return or_extent_q(o); }

static void or_project_one(const float *mean, const float *scale, const float *quat, const float *opac, int64_t n,
                           int64_t i, const or_view *v, int32_t tw, int32_t th, or_proj *o) {
    memset(o, 0, sizeof(*o));
    double p[3], Sv[6];
    if (!or_view_space(mean, scale, quat, n, i, v, p, Sv)) return;
    const double S00 = Sv[0], S01 = Sv[1], S02 = Sv[2], S11 = Sv[3], S12 = Sv[4], S22 = Sv[5];
    double xz = p[0] / p[2], yz = p[1] / p[2];
    double limx = (1.3 * (0.5 * (double)v->width)) / v->fx;
    double limy = (1.3 * (0.5 * (double)v->height)) / v->fy;
    double txc = fmin(fmax(xz, -limx), limx);
    double tyc = fmin(fmax(yz, -limy), limy);
    double j00 = v->fx / p[2], j02 = -(j00 * txc);
    double j11 = v->fy / p[2], j12 = -(j11 * tyc);
    /* B = J Sigma_view (rows 0 and 1; only the entries needed) */
    double B00 = fma(j00, S00, j02 * S02), B01 = fma(j00, S01, j02 * S12), B02 = fma(j00, S02, j02 * S22);
    double B11 = fma(j11, S11, j12 * S12), B12 = fma(j11, S12, j12 * S22);
    double a = fma(B00, j00, B02 * j02) + OR_DILATE;
    double b = fma(B01, j11, B02 * j12);
    double c = fma(B11, j11, B12 * j12) + OR_DILATE;
    double det = fma(a, c, -(b * b));
    if (!(det > 0.0)) return;
    o->ok = 1;
    o->a = a; o->b = b; o->c = c; o->det = det;
    o->u = fma(v->fx, xz, v->cx);
    o->v = fma(v->fy, yz, v->cy);
    o->depth_bits = 0;
    float dz = (float)p[2];
    memcpy(&o->depth_bits, &dz, 4);

    const double q = or_extent_q((double)opac[i]);
    double ex = sqrt(q * a), ey = sqrt(q * c);
    double lox = o->u - ex, hix = o->u + ex, loy = o->v - ey, hiy = o->v + ey;
    if (!(hix >= 0.5 && lox <= (double)v->width - 0.5 && hiy >= 0.5 && loy <= (double)v->height - 0.5)) return;
    int32_t TX = or_tiles_x(v, tw), TY = or_tiles_y(v, th);
    double fx0 = ceil((lox - ((double)tw - 0.5)) / (double)tw);
    double fx1 = floor((hix - 0.5) / (double)tw);
    double fy0 = ceil((loy - ((double)th - 0.5)) / (double)th);
    double fy1 = floor((hiy - 0.5) / (double)th);
    fx0 = fmax(fx0, 0.0); fx1 = fmin(fx1, (double)(TX - 1));
    fy0 = fmax(fy0, 0.0); fy1 = fmin(fy1, (double)(TY - 1));
    if (!(fx0 <= fx1 && fy0 <= fy1)) return;
    o->vis = 1;
    o->rect[0] = (int32_t)fx0; o->rect[1] = (int32_t)fx1;
    o->rect[2] = (int32_t)fy0; o->rect[3] = (int32_t)fy1;
}

typedef struct {
    const float *mean, *scale, *quat, *opac;
    int64_t n; int32_t nv; const or_view *views; int32_t tw, th;
    const uint8_t *active; const int64_t *aoff;
    uint8_t *proj, *vis; uint32_t *depth_bits; int32_t *rect, *count;
    double *mu, *cov, *det, *score;
} or_project_ctx;

static void or_project_body(void *vctx, int64_t item) {
    or_project_ctx *C = (or_project_ctx *)vctx;
    int64_t n = C->n;
    int32_t v = (int32_t)(item / n);
    int64_t i = item % n;
    const or_view *vw = &C->views[v];
    or_proj o;
    or_project_one(C->mean, C->scale, C->quat, C->opac, n, i, vw, C->tw, C->th, &o);
    int64_t k = (int64_t)v * n + i;
    C->proj[k] = (uint8_t)o.ok;
    C->vis[k] = (uint8_t)o.vis;
    C->depth_bits[k] = o.depth_bits;
    C->mu[2 * k] = o.u; C->mu[2 * k + 1] = o.v;
    C->cov[3 * k] = o.a; C->cov[3 * k + 1] = o.b; C->cov[3 * k + 2] = o.c;
    C->det[k] = o.det;
    C->score[k] = o.ok ? ((double)C->opac[i] * M_PI) * sqrt(o.det) : 0.0;
    int32_t cnt = 0;
    if (o.vis) {
        int32_t TX = or_tiles_x(vw, C->tw);
        for (int32_t ty = o.rect[2]; ty <= o.rect[3]; ++ty)
            for (int32_t tx = o.rect[0]; tx <= o.rect[1]; ++tx)
                cnt += C->active ? C->active[C->aoff[v] + (int64_t)ty * TX + tx] : 1;
    }
    memcpy(&C->rect[4 * k], o.rect, sizeof(o.rect));
    C->count[k] = cnt;
}

/* Projection of every (view, Gaussian).  Outputs are [nv][n] (rect [nv][n][4],
 * mu [nv][n][2], cov [nv][n][3] = dilated (a,b,c)).  count is the number of
 * active tiles in the rectangle (before any periphery selection). */
void or_project(int64_t n, const float *mean, const float *scale, const float *quat, const float *opac,
                int32_t nv, const or_view *views, int32_t tw, int32_t th,
                const uint8_t *active, const int64_t *aoff,
                uint8_t *proj, uint8_t *vis, uint32_t *depth_bits, int32_t *rect, int32_t *count,
                double *mu, double *cov, double *det, double *score, int nthreads) {
    or_project_ctx C = {mean, scale, quat, opac, n, nv, views, tw, th, active, aoff,
                        proj, vis, depth_bits, rect, count, mu, cov, det, score};
    or_parallel((int64_t)nv * n, or_project_body, &C, nthreads);
}

/* ------------------------------------------------------------------------- */
/* colour: real spherical harmonics up to degree 3                            */
/* ------------------------------------------------------------------------- */
/* Real SH with the Condon-Shortley phase, ordered (l, m = -l..l), evaluated on
 * a unit direction (x, y, z).  Each constant is the closed-form normalisation
 * sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) (times sqrt 2 for m != 0) folded into
 * the Cartesian polynomial. */
void or_sh_basis(double x, double y, double z, double *Y) {
    const double pi = M_PI;
    double xx = x * x, yy = y * y, zz = z * z;
    Y[0] = 0.5 * sqrt(1.0 / pi);
    Y[1] = -sqrt(3.0 / (4.0 * pi)) * y;
    Y[2] = sqrt(3.0 / (4.0 * pi)) * z;
    Y[3] = -sqrt(3.0 / (4.0 * pi)) * x;
    Y[4] = 0.5 * sqrt(15.0 / pi) * x * y;
    Y[5] = -0.5 * sqrt(15.0 / pi) * y * z;
    Y[6] = 0.25 * sqrt(5.0 / pi) * (2.0 * zz - xx - yy);
    Y[7] = -0.5 * sqrt(15.0 / pi) * x * z;
    Y[8] = 0.25 * sqrt(15.0 / pi) * (xx - yy);
    Y[9] = -0.25 * sqrt(35.0 / (2.0 * pi)) * y * (3.0 * xx - yy);
    Y[10] = 0.5 * sqrt(105.0 / pi) * x * y * z;
    Y[11] = -0.25 * sqrt(21.0 / (2.0 * pi)) * y * (4.0 * zz - xx - yy);
    Y[12] = 0.25 * sqrt(7.0 / pi) * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
    Y[13] = -0.25 * sqrt(21.0 / (2.0 * pi)) * x * (4.0 * zz - xx - yy);
    Y[14] = 0.25 * sqrt(105.0 / pi) * z * (xx - yy);
    Y[15] = -0.25 * sqrt(35.0 / (2.0 * pi)) * x * (xx - 3.0 * yy);
}

/* colour[e][i][ch] = max(0, 0.5 + sum_k Y_k(d) sh[k][ch][i]), d = unit vector from
 * the eye centre to the Gaussian mean.  Only the first (deg+1)^2 coefficients. */
void or_colour(int64_t n, const float *mean, const float *sh, int32_t deg, int32_t ne,
               const double *campos, double *colour) {
    int nk = (deg + 1) * (deg + 1);
    for (int32_t e = 0; e < ne; ++e)
        for (int64_t i = 0; i < n; ++i) {
            double dx = (double)mean[i] - campos[3 * e], dy = (double)mean[n + i] - campos[3 * e + 1],
                   dz = (double)mean[2 * n + i] - campos[3 * e + 2];
            double len = sqrt(dx * dx + dy * dy + dz * dz);
            double Y[16];
            or_sh_basis(dx / len, dy / len, dz / len, Y);
            for (int ch = 0; ch < 3; ++ch) {
                double s = 0.0;
                for (int k = 0; k < nk; ++k) s += Y[k] * (double)sh[((int64_t)k * 3 + ch) * n + i];
                double c = 0.5 + s;
                colour[((int64_t)e * n + i) * 3 + ch] = c > 0.0 ? c : 0.0;
            }
        }
}

/* ------------------------------------------------------------------------- */
/* periphery subset: top ceil(num/den * N_vis) by (score desc, index asc)     */
/* ------------------------------------------------------------------------- */
typedef struct { double s; int64_t i; } or_si;
static int or_si_cmp(const void *pa, const void *pb) {
    const or_si *a = (const or_si *)pa, *b = (const or_si *)pb;
    if (a->s > b->s) return -1;
    if (a->s < b->s) return 1;
    return (a->i > b->i) - (a->i < b->i);
}

int64_t or_select(int64_t n, const uint8_t *vis, const double *score, int32_t num, int32_t den, uint8_t *keep) {
    int64_t nvis = 0;
    for (int64_t i = 0; i < n; ++i) nvis += vis[i] ? 1 : 0;
    or_si *arr = (or_si *)malloc(sizeof(or_si) * (size_t)(nvis > 0 ? nvis : 1));
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i)
        if (vis[i]) { arr[m].s = score[i]; arr[m].i = i; ++m; }
    qsort(arr, (size_t)m, sizeof(or_si), or_si_cmp);
    int64_t k = ((int64_t)num * nvis + den - 1) / den;
    memset(keep, 0, (size_t)n);
    for (int64_t j = 0; j < k; ++j) keep[arr[j].i] = 1;
    free(arr);
    return k;
}

/* ------------------------------------------------------------------------- */
/* key emission, sort, ranges                                                 */
/* ------------------------------------------------------------------------- */
/* Keys are emitted view by view, Gaussian by Gaussian in index order, and for
 * each Gaussian row by row over its tile rectangle (active tiles only):
 * key = (global tile id << 32) | depth bits, value = Gaussian index.
 * Returns the number of keys; writes them only if keys != NULL and K <= cap. */
int64_t or_emit(int64_t n, int32_t nv, const or_view *views, int32_t tw, int32_t th,
                const uint8_t *active, const int64_t *aoff, const int64_t *tile_off,
                const uint8_t *vis, const uint8_t *keep, const int32_t *rect, const uint32_t *depth_bits,
                uint64_t *keys, uint32_t *vals, int64_t cap) {
    int64_t K = 0;
    for (int32_t v = 0; v < nv; ++v) {
        int32_t TX = or_tiles_x(&views[v], tw);
        for (int64_t i = 0; i < n; ++i) {
            int64_t k = (int64_t)v * n + i;
            if (!vis[k]) continue;
            if (views[v].select && !(keep && keep[k])) continue;
            const int32_t *r = &rect[4 * k];
            for (int32_t ty = r[2]; ty <= r[3]; ++ty)
                for (int32_t tx = r[0]; tx <= r[1]; ++tx) {
                    int64_t lt = (int64_t)ty * TX + tx;
                    if (active && !active[aoff[v] + lt]) continue;
                    if (keys && K < cap) {
                        keys[K] = ((uint64_t)(tile_off[v] + lt) << 32) | (uint64_t)depth_bits[k];
                        vals[K] = (uint32_t)i;
                    }
                    ++K;
                }
        }
    }
    return K;
}

typedef struct { uint64_t k; uint32_t v; } or_kv;
static int or_kv_cmp(const void *pa, const void *pb) {
    const or_kv *a = (const or_kv *)pa, *b = (const or_kv *)pb;
    if (a->k != b->k) return a->k < b->k ? -1 : 1;
    return (a->v > b->v) - (a->v < b->v);
}

/* Sort by (key, value): the same order a stable sort of the index-ordered
 * emission by key produces. In place. */
void or_sort(int64_t K, uint64_t *keys, uint32_t *vals) {
    or_kv *a = (or_kv *)malloc(sizeof(or_kv) * (size_t)(K > 0 ? K : 1));
    for (int64_t j = 0; j < K; ++j) { a[j].k = keys[j]; a[j].v = vals[j]; }
    qsort(a, (size_t)K, sizeof(or_kv), or_kv_cmp);
    for (int64_t j = 0; j < K; ++j) { keys[j] = a[j].k; vals[j] = a[j].v; }
    free(a);
}

/* range[t] = [start, end) of tile t's run in the sorted keys; empty runs 0,0. */
void or_ranges(int64_t K, const uint64_t *keys, int64_t ntiles, int64_t *range) {
    memset(range, 0, sizeof(int64_t) * 2 * (size_t)ntiles);
    for (int64_t j = 0; j < K; ++j) {
        int64_t t = (int64_t)(keys[j] >> 32);
        if (t < 0 || t >= ntiles) continue;
        if (j == 0 || (keys[j - 1] >> 32) != keys[j] >> 32) range[2 * t] = j;
        if (j == K - 1 || (keys[j + 1] >> 32) != keys[j] >> 32) range[2 * t + 1] = j + 1;
    }
}

/* ------------------------------------------------------------------------- */
/* blend                                                                      */
/* ------------------------------------------------------------------------- */
/* A pixel is flagged ambiguous when a skip or stop decision lies within the
 * error a float32 evaluation of the same blend can make: eps_alpha bounds the
 * relative error of a float32 alpha, eps_step the relative rounding of one
 * float32 transmittance update.  The bound on T's relative error grows along the
 * list by alpha eps_alpha / (1 - alpha) + eps_step per blended Gaussian.
 *
 * For such a pixel the float32 renderer may take the other branch of the
 * decision.  Its colour then is the one the definition gives with that single
 * decision reversed (every other decision taken as in float64), so the
 * tolerance of an ambiguous pixel is derived by rendering it that way: amb_tol
 * is the sum, over its near-threshold decisions, of the largest channel change
 * that reversing the decision alone causes (a first-order bound when several
 * decisions are near their thresholds at once). */
typedef struct {
    double eps_alpha, eps_step;
} or_blend_opts;

typedef struct {
    double rgb[3], T;
    int32_t last;   /* 1 + list position of the last blended Gaussian, 0 if none */
    int32_t amb;    /* a skip/stop decision fell within the margin of its threshold */
    int64_t pairs;  /* list entries evaluated before the pixel stopped */
    double amb_tol; /* largest colour change a reversed near-threshold decision causes */
} or_pix;

enum { OR_FLIP_NONE = 0, OR_FLIP_SKIP = 1, OR_FLIP_STOP = 2 };
#define OR_MAX_FLIPS 16

/* Front-to-back compositing of one pixel (centre px, py) over an ordered list:
 * alpha = min(0.99, o exp(p)) with p = min(0, -q/2), q = d' Sigma^-1 d; skip
 * alpha < 1/255; stop before blending when T (1 - alpha) < 1e-4.  With flip_j
 * >= 0 the decision of kind flip_kind at list position flip_j goes the other
 * way.  Near-threshold decisions are recorded in flips (when not NULL). */
static void or_blend_path(double px, double py, const uint32_t *list, int64_t len, int32_t v, int64_t n,
                          const double *mu, const double *cov, const double *det, const float *opac,
                          const double *colour_e, const double *bg, const or_blend_opts *op, int64_t flip_j,
                          int flip_kind, or_pix *out, int64_t *flip_pos, int *flip_kinds, int *nflips) {
    double T = 1.0, C[3] = {0.0, 0.0, 0.0}, relT = 0.0;
    int32_t last = 0, amb = 0;
    int64_t pairs = 0;
    for (int64_t j = 0; j < len; ++j) {
        int64_t i = list[j];
        int64_t k = (int64_t)v * n + i;
        ++pairs;
        double dx = px - mu[2 * k], dy = py - mu[2 * k + 1];
        double A = cov[3 * k + 2] / det[k], B = -cov[3 * k + 1] / det[k], Cc = cov[3 * k] / det[k];
        double p = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy;
        if (p > 0.0) p = 0.0;
        double araw = (double)opac[i] * exp(p);
        if (fabs(araw - OR_ALPHA_MIN) <= op->eps_alpha * OR_ALPHA_MIN) {
            amb = 1;
            if (flip_pos && *nflips < OR_MAX_FLIPS) { flip_pos[*nflips] = j; flip_kinds[*nflips] = OR_FLIP_SKIP; }
            if (nflips) ++*nflips;
        }
        int skip = araw < OR_ALPHA_MIN;
        if (j == flip_j && flip_kind == OR_FLIP_SKIP) skip = !skip;
        if (skip) continue;
        double alpha = araw < OR_ALPHA_MAX ? araw : OR_ALPHA_MAX;
        double Tn = T * (1.0 - alpha);
        double relTn = relT + (araw < OR_ALPHA_MAX ? alpha * op->eps_alpha / (1.0 - alpha) : 0.0) + op->eps_step;
        if (fabs(Tn - OR_T_MIN) <= relTn * OR_T_MIN) {
            amb = 1;
            if (flip_pos && *nflips < OR_MAX_FLIPS) { flip_pos[*nflips] = j; flip_kinds[*nflips] = OR_FLIP_STOP; }
            if (nflips) ++*nflips;
        }
        int stop = Tn < OR_T_MIN;
        if (j == flip_j && flip_kind == OR_FLIP_STOP) stop = !stop;
        if (stop) break;
        const double *c = &colour_e[3 * i];
        for (int ch = 0; ch < 3; ++ch) C[ch] += alpha * T * c[ch];
        T = Tn;
        relT = relTn;
        last = (int32_t)(j + 1);
    }
    for (int ch = 0; ch < 3; ++ch) out->rgb[ch] = C[ch] + T * bg[ch];
    out->T = T; out->last = last; out->amb = amb; out->pairs = pairs; out->amb_tol = 0.0;
}

static void or_blend_pixel(double px, double py, const uint32_t *list, int64_t len, int32_t v, int64_t n,
                           const double *mu, const double *cov, const double *det, const float *opac,
                           const double *colour_e, const double *bg, const or_blend_opts *op, or_pix *out) {
    int64_t fpos[OR_MAX_FLIPS];
    int fkind[OR_MAX_FLIPS];
    int nf = 0;
    or_blend_path(px, py, list, len, v, n, mu, cov, det, opac, colour_e, bg, op, -1, OR_FLIP_NONE, out, fpos, fkind,
                  &nf);
    if (nf > OR_MAX_FLIPS) {  /* not expected: no bound derived, the colour is not checked */
        out->amb_tol = INFINITY;
        return;
    }
    double tol = 0.0;
    for (int f = 0; f < nf; ++f) {
        or_pix alt;
        or_blend_path(px, py, list, len, v, n, mu, cov, det, opac, colour_e, bg, op, fpos[f], fkind[f], &alt, NULL,
                      NULL, NULL);
        double d = 0.0;
        for (int ch = 0; ch < 3; ++ch) d = fmax(d, fabs(alt.rgb[ch] - out->rgb[ch]));
        tol += d;
    }
    out->amb_tol = tol;
}

typedef struct {
    int32_t nv; const or_view *views; int32_t tw, th;
    const uint8_t *active; const int64_t *aoff; const int64_t *tile_off; const int64_t *img_off;
    const uint32_t *vals; const int64_t *range;
    int64_t n; const double *mu, *cov, *det; const float *opac; const double *colour;
    or_blend_opts op;
    double *rgb, *Tout; int32_t *last; uint8_t *amb; int64_t *pairs; double *amb_tol;
    int64_t total_tiles;
} or_blend_ctx;

static void or_blend_tile(void *vctx, int64_t gt) {
    or_blend_ctx *C = (or_blend_ctx *)vctx;
    int32_t v = 0;
    while (v + 1 < C->nv && C->tile_off[v + 1] <= gt) ++v;
    const or_view *vw = &C->views[v];
    int64_t lt = gt - C->tile_off[v];
    int32_t TX = or_tiles_x(vw, C->tw);
    int32_t tx = (int32_t)(lt % TX), ty = (int32_t)(lt / TX);
    if (C->active && !C->active[C->aoff[v] + lt]) return;
    int64_t s = C->range[2 * gt], e = C->range[2 * gt + 1];
    const uint32_t *list = C->vals + s;
    int64_t W = vw->width, H = vw->height, HW = W * H;
    const double *col = C->colour + (int64_t)vw->eye * C->n * 3;
    for (int32_t yy = ty * C->th; yy < (ty + 1) * C->th && yy < H; ++yy)
        for (int32_t xx = tx * C->tw; xx < (tx + 1) * C->tw && xx < W; ++xx) {
            or_pix P;
            or_blend_pixel(xx + 0.5, yy + 0.5, list, e - s, v, C->n, C->mu, C->cov, C->det, C->opac, col,
                           vw->bg, &C->op, &P);
            int64_t pix = (int64_t)yy * W + xx;
            for (int ch = 0; ch < 3; ++ch) C->rgb[3 * C->img_off[v] + ch * HW + pix] = P.rgb[ch];
            C->Tout[C->img_off[v] + pix] = P.T;
            C->last[C->img_off[v] + pix] = P.last;
            C->amb[C->img_off[v] + pix] = (uint8_t)P.amb;
            if (C->amb_tol) C->amb_tol[C->img_off[v] + pix] = P.amb_tol;
            C->pairs[C->img_off[v] + pix] = P.pairs;
        }
}

/* Tiled blend of every active tile.  Images are per view, concatenated:
 * rgb at 3*img_off[v] as planar [3][H][W]; T/last/amb/pairs at img_off[v]. */
void or_blend(int32_t nv, const or_view *views, int32_t tw, int32_t th,
              const uint8_t *active, const int64_t *aoff, const int64_t *tile_off, const int64_t *img_off,
              const uint32_t *sorted_vals, const int64_t *range,
              int64_t n, const double *mu, const double *cov, const double *det, const float *opac,
              const double *colour, double eps_alpha, double eps_step,
              double *rgb, double *Tout, int32_t *last, uint8_t *amb, int64_t *pairs, double *amb_tol,
              int nthreads) {
    int64_t total = tile_off[nv];
    or_blend_ctx C = {nv, views, tw, th, active, aoff, tile_off, img_off, sorted_vals, range,
                      n, mu, cov, det, opac, colour, {eps_alpha, eps_step},
                      rgb, Tout, last, amb, pairs, amb_tol, total};
    or_parallel(total, or_blend_tile, &C, nthreads);
}

static int or_u64_cmp(const void *pa, const void *pb) {
    uint64_t a = *(const uint64_t *)pa, b = *(const uint64_t *)pb;
    return (a > b) - (a < b);
}

/* The plain definition, no tiles: every pixel composites all projectable (and,
 * for a selecting view, kept) Gaussians of the view sorted by (depth bits,
 * index).  For small scenes. */
void or_blend_brute(int64_t n, int32_t nv, const or_view *views, const int64_t *img_off,
                    const uint8_t *proj, const uint8_t *keep, const uint32_t *depth_bits,
                    const double *mu, const double *cov, const double *det, const float *opac,
                    const double *colour, double *rgb, double *Tout) {
    uint64_t *ord = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    uint32_t *list = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    or_blend_opts op = {0.0, 0.0};
    for (int32_t v = 0; v < nv; ++v) {
        const or_view *vw = &views[v];
        int64_t m = 0;
        for (int64_t i = 0; i < n; ++i) {
            int64_t k = (int64_t)v * n + i;
            if (!proj[k]) continue;
            if (vw->select && !(keep && keep[k])) continue;
            ord[m++] = ((uint64_t)depth_bits[k] << 32) | (uint64_t)i;
        }
        /* ascending (depth bits, index): the packed word orders exactly so */
        qsort(ord, (size_t)m, sizeof(uint64_t), or_u64_cmp);
        for (int64_t a = 0; a < m; ++a) list[a] = (uint32_t)(ord[a] & 0xffffffffu);
        int64_t W = vw->width, H = vw->height, HW = W * H;
        const double *col = colour + (int64_t)vw->eye * n * 3;
        for (int64_t yy = 0; yy < H; ++yy)
            for (int64_t xx = 0; xx < W; ++xx) {
                or_pix P;
                or_blend_pixel(xx + 0.5, yy + 0.5, list, m, v, n, mu, cov, det, opac, col, vw->bg, &op, &P);
                for (int ch = 0; ch < 3; ++ch) rgb[3 * img_off[v] + ch * HW + yy * W + xx] = P.rgb[ch];
                Tout[img_off[v] + yy * W + xx] = P.T;
            }
    }
    free(ord);
    free(list);
}

typedef struct {
    const uint32_t *list; int64_t len; int32_t v; int64_t n;
    const double *mu, *cov, *det; const float *opac; const double *col; const double *bg;
    or_blend_opts op; const int32_t *xs, *ys; double *rgb, *T; int32_t *amb; double *amb_tol;
} or_pixels_ctx;

static void or_pixels_body(void *vctx, int64_t j) {
    or_pixels_ctx *C = (or_pixels_ctx *)vctx;
    or_pix P;
    or_blend_pixel(C->xs[j] + 0.5, C->ys[j] + 0.5, C->list, C->len, C->v, C->n, C->mu, C->cov, C->det, C->opac,
                   C->col, C->bg, &C->op, &P);
    for (int ch = 0; ch < 3; ++ch) C->rgb[3 * j + ch] = P.rgb[ch];
    C->T[j] = P.T;
    C->amb[j] = P.amb;
    if (C->amb_tol) C->amb_tol[j] = P.amb_tol;
}

/* The plain definition for a sample of pixels of view v of a large scene:
 * every projectable (and, for a selecting view, kept) Gaussian sorted by
 * (depth bits, index), composited at each requested pixel centre. */
void or_blend_pixels(int64_t n, int32_t v, const or_view *views, const uint8_t *proj, const uint8_t *keep,
                     const uint32_t *depth_bits, const double *mu, const double *cov, const double *det,
                     const float *opac, const double *colour, double eps_alpha, double eps_step, int64_t npx,
                     const int32_t *xs, const int32_t *ys, double *rgb, double *T, int32_t *amb, double *amb_tol,
                     int nthreads) {
    const or_view *vw = &views[v];
    uint64_t *ord = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    uint32_t *list = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t k = (int64_t)v * n + i;
        if (!proj[k]) continue;
        if (vw->select && !(keep && keep[k])) continue;
        ord[m++] = ((uint64_t)depth_bits[k] << 32) | (uint64_t)i;
    }
    qsort(ord, (size_t)m, sizeof(uint64_t), or_u64_cmp);
    for (int64_t a = 0; a < m; ++a) list[a] = (uint32_t)(ord[a] & 0xffffffffu);
    or_pixels_ctx C = {list, m, v, n, mu, cov, det, opac, colour + (int64_t)vw->eye * n * 3, vw->bg,
                       {eps_alpha, eps_step}, xs, ys, rgb, T, amb, amb_tol};
    or_parallel(npx, or_pixels_body, &C, nthreads);
    free(ord);
    free(list);
}

/* Per-step transmittance of one pixel along its tile list (for the
 * monotonicity invariant): trace[j] = T after entry j (unchanged when skipped),
 * stops where the blend stops. Returns the number of entries written. */
int64_t or_pixel_trace(int32_t v, double px, double py, const uint32_t *list, int64_t len, int64_t n,
                       const double *mu, const double *cov, const double *det, const float *opac,
                       double *trace) {
    double T = 1.0;
    int64_t w = 0;
    for (int64_t j = 0; j < len; ++j) {
        int64_t i = list[j], k = (int64_t)v * n + i;
        double dx = px - mu[2 * k], dy = py - mu[2 * k + 1];
        double A = cov[3 * k + 2] / det[k], B = -cov[3 * k + 1] / det[k], Cc = cov[3 * k] / det[k];
        double p = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy;
        if (p > 0.0) p = 0.0;
        double araw = (double)opac[i] * exp(p);
        if (araw >= OR_ALPHA_MIN) {
            double alpha = araw < OR_ALPHA_MAX ? araw : OR_ALPHA_MAX;
            double Tn = T * (1.0 - alpha);
            if (Tn < OR_T_MIN) break;
            T = Tn;
        }
        trace[w++] = T;
    }
    return w;
}

/* ------------------------------------------------------------------------- */
/* foveated composite and the quality judge                                   */
/* ------------------------------------------------------------------------- */
static double or_bilinear(const double *img, int64_t W, int64_t H, double sx, double sy) {
    if (sx < 0.0) sx = 0.0;
    if (sx > (double)(W - 1)) sx = (double)(W - 1);
    if (sy < 0.0) sy = 0.0;
    if (sy > (double)(H - 1)) sy = (double)(H - 1);
    int64_t x0 = (int64_t)floor(sx), y0 = (int64_t)floor(sy);
    int64_t x1 = x0 + 1 < W ? x0 + 1 : W - 1, y1 = y0 + 1 < H ? y0 + 1 : H - 1;
    double wx = sx - (double)x0, wy = sy - (double)y0;
    double top = (1.0 - wx) * img[y0 * W + x0] + wx * img[y0 * W + x1];
    double bot = (1.0 - wx) * img[y1 * W + x0] + wx * img[y1 * W + x1];
    return (1.0 - wy) * top + wy * bot;
}

/* Region of a full-resolution pixel centre: 0 fovea (rho <= r_f), 1 mid
 * (rho <= r_m), 2 periphery. */
static int or_region(double px, double py, double gx, double gy, double rf, double rm) {
    double dx = px - gx, dy = py - gy;
    double r2 = dx * dx + dy * dy;
    if (r2 <= rf * rf) return 0;
    if (r2 <= rm * rm) return 1;
    return 2;
}

/* out[3][H][W]: fovea pixel inside r_f; bilinear x2 of mid up to r_m; bilinear
 * x(periph_scale) of the periphery (or the given upsampled periphery) beyond. */
void or_composite(int32_t W, int32_t H, double gx, double gy, double rf, double rm,
                  const double *fovea, const double *mid, int32_t mid_scale,
                  const double *periph, int32_t periph_scale, const double *periph_full, double *out) {
    int64_t Wm = W / mid_scale, Hm = H / mid_scale, Wp = W / periph_scale, Hp = H / periph_scale;
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x) {
            double px = x + 0.5, py = y + 0.5;
            int reg = or_region(px, py, gx, gy, rf, rm);
            for (int ch = 0; ch < 3; ++ch) {
                double val;
                if (reg == 0) val = fovea[(int64_t)ch * W * H + y * W + x];
                else if (reg == 1) val = or_bilinear(mid + (int64_t)ch * Wm * Hm, Wm, Hm, px / mid_scale - 0.5, py / mid_scale - 0.5);
                else if (periph_full) val = periph_full[(int64_t)ch * W * H + y * W + x];
                else val = or_bilinear(periph + (int64_t)ch * Wp * Hp, Wp, Hp, px / periph_scale - 0.5, py / periph_scale - 0.5);
                out[(int64_t)ch * W * H + y * W + x] = val;
            }
        }
}

/* Squared-error sums of two [3][H][W] images clamped to [0,1], per region
 * (fovea, mid, periphery), and pixel counts per region. */
void or_region_sse(int32_t W, int32_t H, double gx, double gy, double rf, double rm,
                   const double *a, const double *b, double *sse3, int64_t *cnt3) {
    for (int r = 0; r < 3; ++r) { sse3[r] = 0.0; cnt3[r] = 0; }
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x) {
            int reg = or_region(x + 0.5, y + 0.5, gx, gy, rf, rm);
            double s = 0.0;
            for (int ch = 0; ch < 3; ++ch) {
                double u = a[(int64_t)ch * W * H + y * W + x], w = b[(int64_t)ch * W * H + y * W + x];
                u = u < 0.0 ? 0.0 : (u > 1.0 ? 1.0 : u);
                w = w < 0.0 ? 0.0 : (w > 1.0 ? 1.0 : w);
                s += (u - w) * (u - w);
            }
            sse3[reg] += s;
            cnt3[reg] += 1;
        }
}
