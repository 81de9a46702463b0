/*
 * a3fr_oracle_grad.c -- FP64 oracle of the differentiable render (TEST INFRASTRUCTURE ONLY).
 *
 * Forward: the plain definition of one view (no tiles): every projectable
 * Gaussian, sorted by (float32 depth bits, index), composited front to back at
 * every pixel centre, from the raw parameters (mean, log-scale, quaternion,
 * opacity logit, SH) with scale = exp(log-scale) and opacity = sigmoid(logit).
 * The rendering conventions are those of a3fr_oracle.c (Sec. 2.3 of the
 * paper: projection, depth order, front-to-back blend).
 *
 * Backward: the analytic chain rule of that forward for a loss L = sum over
 * pixels and channels of w[ch][y][x] * I[ch][y][x] (w = dL/dI is given):
 *   blend -> per-Gaussian (2D mean, inverse 2D covariance, opacity, colour)
 *   -> Jacobian and view covariance -> 3D covariance -> scale and rotation
 *   -> log-scale and quaternion; colour -> SH coefficients and mean (through
 *   the viewing direction); mean also through the projection; opacity -> logit.
 * "smooth" mode drops every discontinuity (no alpha skip, no stop, no 0.99
 * clamp, no colour clamp) so that central finite differences pin the chain.
 *
 * Build with -ffp-contract=off -fno-fast-math (float64 throughout).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double R[9], t[3], campos[3];
    double fx, fy, cx, cy;
    int32_t width, height;
    int32_t eye, mask, select, pad_;
    double gx, gy, r_in, r_out;
    double bg[3];
} og_view;

#define OG_ZNEAR 0.2
#define OG_DILATE 0.3
#define OG_AMIN (1.0 / 255.0)
#define OG_AMAX 0.99
#define OG_TMIN 1e-4

/* real SH basis (Condon-Shortley phase) and its gradient w.r.t. (x, y, z) as
 * polynomials; closed-form normalisations */
static void og_sh(double x, double y, double z, double *Y, double (*dY)[3]) {
    const double pi = M_PI;
    const double C0 = 0.5 * sqrt(1.0 / pi), C1 = sqrt(3.0 / (4.0 * pi));
    const double C2a = 0.5 * sqrt(15.0 / pi), C2b = 0.25 * sqrt(5.0 / pi), C2c = 0.25 * sqrt(15.0 / pi);
    const double C3a = 0.25 * sqrt(35.0 / (2.0 * pi)), C3b = 0.5 * sqrt(105.0 / pi);
    const double C3c = 0.25 * sqrt(21.0 / (2.0 * pi)), C3d = 0.25 * sqrt(7.0 / pi), C3e = 0.25 * sqrt(105.0 / pi);
    const double xx = x * x, yy = y * y, zz = z * z;
    Y[0] = C0;
    Y[1] = -C1 * y; Y[2] = C1 * z; Y[3] = -C1 * x;
    Y[4] = C2a * x * y; Y[5] = -C2a * y * z; Y[6] = C2b * (2 * zz - xx - yy); Y[7] = -C2a * x * z; Y[8] = C2c * (xx - yy);
    Y[9] = -C3a * y * (3 * xx - yy); Y[10] = C3b * x * y * z; Y[11] = -C3c * y * (4 * zz - xx - yy);
    Y[12] = C3d * z * (2 * zz - 3 * xx - 3 * yy); Y[13] = -C3c * x * (4 * zz - xx - yy);
    Y[14] = C3e * z * (xx - yy); Y[15] = -C3a * x * (xx - 3 * yy);
    if (!dY) return;
    double g[16][3] = {
        {0, 0, 0},
        {0, -C1, 0}, {0, 0, C1}, {-C1, 0, 0},
        {C2a * y, C2a * x, 0}, {0, -C2a * z, -C2a * y}, {-2 * C2b * x, -2 * C2b * y, 4 * C2b * z},
        {-C2a * z, 0, -C2a * x}, {2 * C2c * x, -2 * C2c * y, 0},
        {-6 * C3a * x * y, -C3a * (3 * xx - 3 * yy), 0},
        {C3b * y * z, C3b * x * z, C3b * x * y},
        {2 * C3c * x * y, -C3c * (4 * zz - xx - 3 * yy), -8 * C3c * y * z},
        {-6 * C3d * x * z, -6 * C3d * y * z, C3d * (6 * zz - 3 * xx - 3 * yy)},
        {-C3c * (4 * zz - 3 * xx - yy), 2 * C3c * x * y, -8 * C3c * x * z},
        {2 * C3e * x * z, -2 * C3e * y * z, C3e * (xx - yy)},
        {-C3a * (3 * xx - 3 * yy), 6 * C3a * x * y, 0},
    };
    memcpy(dY, g, sizeof(g));
}

/* per-Gaussian forward state */
typedef struct {
    int ok;                 /* projectable */
    double s[3], o, qn[4], qnorm, Rq[9], M[9], S3[9];
    double p[3], Sv[9];
    double txc, tyc;        /* clamped x/z, y/z */
    int clx, cly;           /* clamped? */
    double J[6];            /* rows: (J00 J01 J02), (J10 J11 J12) */
    double a, b, c, det;    /* dilated 2D covariance */
    double A, B, Cc;        /* inverse (conic) */
    double u, v;
    double dir[3], vlen, Y[16], dY[16][3];
    double craw[3], col[3];
    uint32_t depth_bits;
} og_g;

static void og_forward_one(int64_t n, int64_t i, const float *mean, const float *log_s, const float *quat,
                           const float *logit, const float *sh, int nk, const og_view *v, int smooth, og_g *g) {
    memset(g, 0, sizeof(*g));
    const double *Rw = v->R;
    double mu[3] = {mean[i], mean[n + i], mean[2 * n + i]};
    for (int k = 0; k < 3; ++k) g->p[k] = Rw[3 * k] * mu[0] + Rw[3 * k + 1] * mu[1] + Rw[3 * k + 2] * mu[2] + v->t[k];
    for (int k = 0; k < 3; ++k) g->s[k] = exp((double)log_s[(int64_t)k * n + i]);
    g->o = 1.0 / (1.0 + exp(-(double)logit[i]));
    double q[4] = {quat[i], quat[n + i], quat[2 * n + i], quat[3 * n + i]};
    g->qnorm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (!(g->p[2] > OG_ZNEAR) || !(g->qnorm > 0.0)) return;
    for (int k = 0; k < 4; ++k) g->qn[k] = q[k] / g->qnorm;
    double w = g->qn[0], x = g->qn[1], y = g->qn[2], z = g->qn[3];
    double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                   2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                   2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
    memcpy(g->Rq, R, sizeof(R));
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) g->M[3 * r + c] = R[3 * r + c] * g->s[c];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double e = 0;
            for (int k = 0; k < 3; ++k) e += g->M[3 * r + k] * g->M[3 * c + k];
            g->S3[3 * r + c] = e;
        }
    double A[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double e = 0;
            for (int k = 0; k < 3; ++k) e += Rw[3 * r + k] * g->S3[3 * k + c];
            A[3 * r + c] = e;
        }
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double e = 0;
            for (int k = 0; k < 3; ++k) e += A[3 * r + k] * Rw[3 * c + k];
            g->Sv[3 * r + c] = e;
        }
    const double pz = g->p[2];
    const double limx = 1.3 * 0.5 * v->width / v->fx, limy = 1.3 * 0.5 * v->height / v->fy;
    double tx = g->p[0] / pz, ty = g->p[1] / pz;
    g->clx = tx < -limx || tx > limx;
    g->cly = ty < -limy || ty > limy;
    g->txc = tx < -limx ? -limx : (tx > limx ? limx : tx);
    g->tyc = ty < -limy ? -limy : (ty > limy ? limy : ty);
    double J[6] = {v->fx / pz, 0.0, -v->fx * g->txc / pz, 0.0, v->fy / pz, -v->fy * g->tyc / pz};
    memcpy(g->J, J, sizeof(J));
    double T2[4] = {0, 0, 0, 0};  /* J Sv J^T */
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) {
            double e = 0;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) e += J[3 * r + k] * g->Sv[3 * k + l] * J[3 * c + l];
            T2[2 * r + c] = e;
        }
    g->a = T2[0] + OG_DILATE;
    g->b = T2[1];
    g->c = T2[3] + OG_DILATE;
    g->det = g->a * g->c - g->b * g->b;
    if (!(g->det > 0.0)) return;
    g->A = g->c / g->det;
    g->B = -g->b / g->det;
    g->Cc = g->a / g->det;
    g->u = v->fx * tx + v->cx;
    g->v = v->fy * ty + v->cy;
    float dz = (float)pz;
    memcpy(&g->depth_bits, &dz, 4);
    /* colour */
    double dv[3] = {mu[0] - v->campos[0], mu[1] - v->campos[1], mu[2] - v->campos[2]};
    g->vlen = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    for (int k = 0; k < 3; ++k) g->dir[k] = dv[k] / g->vlen;
    og_sh(g->dir[0], g->dir[1], g->dir[2], g->Y, g->dY);
    for (int ch = 0; ch < 3; ++ch) {
        double s = 0.5;
        for (int k = 0; k < nk; ++k) s += g->Y[k] * (double)sh[((int64_t)k * 3 + ch) * n + i];
        g->craw[ch] = s;
        g->col[ch] = smooth ? s : (s > 0.0 ? s : 0.0);
    }
    g->ok = 1;
}

typedef struct {
    int64_t n; int nk; const og_view *v; int smooth;
    int64_t wx0, wy0, ww, wh;   /* pixel window */
    const og_g *G; const uint32_t *list; int64_t m;
    const double *wgt; double eps_alpha, eps_step;
    double *img; uint8_t *amb;
    int nchunks;
    double *acc;  /* [nchunks][m][9] by list position: dA dB dC du dv do dc0 dc1 dc2 */
} og_ctx;

static void og_pixels(void *vctx, int64_t chunk) {
    og_ctx *C = (og_ctx *)vctx;
    const og_view *v = C->v;
    const int64_t W = v->width, H = v->height, HW = W * H;
    int64_t y0 = C->wy0 + C->wh * chunk / C->nchunks, y1 = C->wy0 + C->wh * (chunk + 1) / C->nchunks;
    double *acc = C->acc + chunk * C->m * 9;  /* indexed by list position */
    int64_t *bl = (int64_t *)malloc(sizeof(int64_t) * (size_t)(C->m > 0 ? C->m : 1));
    double *al = (double *)malloc(sizeof(double) * (size_t)(C->m > 0 ? C->m : 1) * 4);
    for (int64_t py = y0; py < y1; ++py)
        for (int64_t px = C->wx0; px < C->wx0 + C->ww; ++px) {
            const double X = px + 0.5, Yc = py + 0.5;
            double T = 1.0, Col[3] = {0, 0, 0}, relT = 0.0;
            int amb = 0;
            int64_t nb = 0;
            for (int64_t j = 0; j < C->m; ++j) {
                const og_g *g = &C->G[C->list[j]];
                const double dx = X - g->u, dy = Yc - g->v;
                double p = -0.5 * (g->A * dx * dx + g->Cc * dy * dy) - g->B * dx * dy;
                if (p > 0.0) p = 0.0;
                const double G = exp(p);
                const double araw = g->o * G;
                double alpha = araw;
                int clamped = 0;
                if (!C->smooth) {
                    if (fabs(araw - OG_AMIN) <= C->eps_alpha * OG_AMIN) amb = 1;
                    if (araw < OG_AMIN) continue;
                    if (araw >= OG_AMAX) { alpha = OG_AMAX; clamped = 1; }
                    const double Tn = T * (1.0 - alpha);
                    const double relTn = relT + (clamped ? 0.0 : alpha * C->eps_alpha / (1.0 - alpha)) + C->eps_step;
                    if (fabs(Tn - OG_TMIN) <= relTn * OG_TMIN) amb = 1;
                    if (Tn < OG_TMIN) break;
                    relT = relTn;
                }
                for (int ch = 0; ch < 3; ++ch) Col[ch] += alpha * T * g->col[ch];
                bl[nb] = j;
                al[4 * nb + 0] = alpha;
                al[4 * nb + 1] = T;
                al[4 * nb + 2] = G;
                al[4 * nb + 3] = clamped;
                ++nb;
                T *= (1.0 - alpha);
            }
            const int64_t pix = py * W + px;
            for (int ch = 0; ch < 3; ++ch) C->img[ch * HW + pix] = Col[ch] + T * v->bg[ch];
            if (C->amb) C->amb[pix] = (uint8_t)amb;
            /* backward along the blended list */
            const double dC[3] = {C->wgt[pix], C->wgt[HW + pix], C->wgt[2 * HW + pix]};
            double S = T * (v->bg[0] * dC[0] + v->bg[1] * dC[1] + v->bg[2] * dC[2]);
            for (int64_t q = nb - 1; q >= 0; --q) {
                const int64_t j = bl[q];
                const og_g *g = &C->G[C->list[j]];
                const double alpha = al[4 * q], Tb = al[4 * q + 1], G = al[4 * q + 2];
                const int clamped = al[4 * q + 3] != 0.0;
                double *a9 = acc + j * 9;
                const double cd = g->col[0] * dC[0] + g->col[1] * dC[1] + g->col[2] * dC[2];
                for (int ch = 0; ch < 3; ++ch) a9[6 + ch] += alpha * Tb * dC[ch];
                const double dalpha = Tb * cd - S / (1.0 - alpha);
                S += cd * alpha * Tb;
                if (clamped) continue;
                a9[5] += dalpha * G;
                const double dp = dalpha * alpha;
                const double dx = X - g->u, dy = Yc - g->v;
                a9[0] += dp * (-0.5 * dx * dx);
                a9[1] += dp * (-dx * dy);
                a9[2] += dp * (-0.5 * dy * dy);
                a9[3] += dp * (g->A * dx + g->B * dy);
                a9[4] += dp * (g->B * dx + g->Cc * dy);
            }
        }
    free(bl);
    free(al);
}

#define OG_MAX_THREADS 256
typedef struct {
    og_ctx *c;
    int64_t k;
} og_arg;

static void *og_thread(void *p) {
    og_arg *a = (og_arg *)p;
    og_pixels(a->c, a->k);
    return NULL;
}

static int og_u64cmp(const void *pa, const void *pb) {
    uint64_t a = *(const uint64_t *)pa, b = *(const uint64_t *)pb;
    return (a > b) - (a < b);
}

/* Per-Gaussian chain from the 2D gradients a9 = (dA, dB, dC, du, dv, do, dcol[3]). */
static void og_chain(const og_g *g, const double *a9, const og_view *v, int smooth, int nk, const float *sh, int64_t n,
                     int64_t i, double *gm, double *gls, double *gq, double *glogit, double *gsh) {
    /* conic -> Sigma2D: dSigma = -K G_K K with K the conic matrix, G_K = [[dA, dB/2],[dB/2, dC]] */
    const double K[4] = {g->A, g->B, g->B, g->Cc};
    const double GK[4] = {a9[0], 0.5 * a9[1], 0.5 * a9[1], a9[2]};
    double t1[4], GS[4];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) t1[2 * r + c] = GK[2 * r] * K[c] + GK[2 * r + 1] * K[2 + c];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) GS[2 * r + c] = -(K[2 * r] * t1[c] + K[2 * r + 1] * t1[2 + c]);
    /* GS is the symmetric matrix gradient of (J Sv J^T); dJ = 2 GS J Sv, dSv = J^T GS J */
    const double *J = g->J;
    double JS[6];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) {
            double e = 0;
            for (int k = 0; k < 3; ++k) e += J[3 * r + k] * g->Sv[3 * k + c];
            JS[3 * r + c] = e;
        }
    double dJ[6];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) dJ[3 * r + c] = 2.0 * (GS[2 * r] * JS[c] + GS[2 * r + 1] * JS[3 + c]);
    double dSv[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double e = 0;
            for (int k = 0; k < 2; ++k)
                for (int l = 0; l < 2; ++l) e += J[3 * k + r] * GS[2 * k + l] * J[3 * l + c];
            dSv[3 * r + c] = e;
        }
    /* J(p) and (u, v)(p) -> dp */
    const double x = g->p[0], y = g->p[1], z = g->p[2];
    double dp[3] = {0, 0, 0};
    const double fx = v->fx, fy = v->fy;
    dp[2] += dJ[0] * (-fx / (z * z));
    dp[2] += dJ[4] * (-fy / (z * z));
    if (g->clx) {
        dp[2] += dJ[2] * (fx * g->txc / (z * z));
    } else {
        dp[0] += dJ[2] * (-fx / (z * z));
        dp[2] += dJ[2] * (2.0 * fx * x / (z * z * z));
    }
    if (g->cly) {
        dp[2] += dJ[5] * (fy * g->tyc / (z * z));
    } else {
        dp[1] += dJ[5] * (-fy / (z * z));
        dp[2] += dJ[5] * (2.0 * fy * y / (z * z * z));
    }
    dp[0] += a9[3] * (fx / z);
    dp[2] += a9[3] * (-fx * x / (z * z));
    dp[1] += a9[4] * (fy / z);
    dp[2] += a9[4] * (-fy * y / (z * z));
    const double *Rw = v->R;
    for (int k = 0; k < 3; ++k) gm[k] += Rw[k] * dp[0] + Rw[3 + k] * dp[1] + Rw[6 + k] * dp[2];
    /* Sv = Rw S3 Rw^T -> dS3 = Rw^T dSv Rw */
    double dS3[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double e = 0;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) e += Rw[3 * k + r] * dSv[3 * k + l] * Rw[3 * l + c];
            dS3[3 * r + c] = e;
        }
    /* S3 = M M^T -> dM = (dS3 + dS3^T) M */
    double dM[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double e = 0;
            for (int k = 0; k < 3; ++k) e += (dS3[3 * r + k] + dS3[3 * k + r]) * g->M[3 * k + c];
            dM[3 * r + c] = e;
        }
    /* M = Rq diag(s) */
    double dR[9], ds[3] = {0, 0, 0};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            dR[3 * r + c] = dM[3 * r + c] * g->s[c];
            ds[c] += dM[3 * r + c] * g->Rq[3 * r + c];
        }
    for (int c = 0; c < 3; ++c) gls[c] += ds[c] * g->s[c];
    /* rotation of the unit quaternion -> dq_hat -> dq */
    const double w = g->qn[0], qx = g->qn[1], qy = g->qn[2], qz = g->qn[3];
    double dqh[4];
    dqh[0] = 2 * qz * (dR[3] - dR[1]) + 2 * qy * (dR[2] - dR[6]) + 2 * qx * (dR[7] - dR[5]);
    dqh[1] = 2 * qy * (dR[1] + dR[3]) + 2 * qz * (dR[2] + dR[6]) + 2 * w * (dR[7] - dR[5]) - 4 * qx * (dR[4] + dR[8]);
    dqh[2] = -4 * qy * (dR[0] + dR[8]) + 2 * qx * (dR[1] + dR[3]) + 2 * w * (dR[2] - dR[6]) + 2 * qz * (dR[5] + dR[7]);
    dqh[3] = -4 * qz * (dR[0] + dR[4]) + 2 * w * (dR[3] - dR[1]) + 2 * qx * (dR[2] + dR[6]) + 2 * qy * (dR[5] + dR[7]);
    const double dotq = dqh[0] * g->qn[0] + dqh[1] * g->qn[1] + dqh[2] * g->qn[2] + dqh[3] * g->qn[3];
    for (int k = 0; k < 4; ++k) gq[k] += (dqh[k] - g->qn[k] * dotq) / g->qnorm;
    /* opacity -> logit */
    glogit[0] += a9[5] * g->o * (1.0 - g->o);
    /* colour -> SH and the viewing direction */
    double dcr[3];
    for (int ch = 0; ch < 3; ++ch) dcr[ch] = (smooth || g->craw[ch] > 0.0) ? a9[6 + ch] : 0.0;
    double dd[3] = {0, 0, 0};
    for (int k = 0; k < nk; ++k) {
        double dYk = 0;
        for (int ch = 0; ch < 3; ++ch) {
            gsh[((int64_t)k * 3 + ch) * n] += g->Y[k] * dcr[ch];
            dYk += (double)sh[((int64_t)k * 3 + ch) * n + i] * dcr[ch];
        }
        for (int a = 0; a < 3; ++a) dd[a] += dYk * g->dY[k][a];
    }
    const double dot = dd[0] * g->dir[0] + dd[1] * g->dir[1] + dd[2] * g->dir[2];
    for (int a = 0; a < 3; ++a) gm[a] += (dd[a] - g->dir[a] * dot) / g->vlen;
}

/* Render the pixels of the window [wx0, wx0+ww) x [wy0, wy0+wh) of one view
 * from raw parameters and back-propagate w = dL/dI (pixels outside the window
 * are neither rendered nor differentiated: their image entries stay as given).
 * Inputs are [k][n] structure-of-arrays (sh [16][3][n]); outputs image
 * [3][H][W], ambiguity flags [H][W] (non-smooth mode; may be NULL), and the
 * gradients (same layouts as the inputs, float64).  Returns the number of
 * Gaussians drawn (projectable and, in thresholded mode, with a footprint box
 * {d' Sigma2D^-1 d <= 11.1} meeting the window: outside it alpha < 1/255
 * for any opacity <= 1, as 2 ln 255 < 11.1, so the cull is exact). */
int64_t or_render_grad(int64_t n, const float *mean, const float *log_s, const float *quat, const float *logit,
                       const float *sh, int32_t deg, const og_view *v, int32_t smooth, const double *wgt,
                       double eps_alpha, double eps_step, int64_t wx0, int64_t wy0, int64_t ww, int64_t wh,
                       double *img, uint8_t *amb, double *g_mean, double *g_logs,
                       double *g_quat, double *g_logit, double *g_sh, int nthreads) {
    const int nk = (deg + 1) * (deg + 1);
    og_g *G = (og_g *)calloc((size_t)(n > 0 ? n : 1), sizeof(og_g));
    uint64_t *ord = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    uint32_t *list = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        og_forward_one(n, i, mean, log_s, quat, logit, sh, nk, v, smooth, &G[i]);
        if (G[i].ok && !smooth) {
            const double ex = sqrt(11.1 * G[i].a), ey = sqrt(11.1 * G[i].c);
            if (G[i].u + ex < (double)wx0 + 0.5 || G[i].u - ex > (double)(wx0 + ww) - 0.5 ||
                G[i].v + ey < (double)wy0 + 0.5 || G[i].v - ey > (double)(wy0 + wh) - 0.5)
                G[i].ok = 0;
        }
        if (G[i].ok) ord[m++] = ((uint64_t)G[i].depth_bits << 32) | (uint64_t)i;
    }
    qsort(ord, (size_t)m, sizeof(uint64_t), og_u64cmp);
    for (int64_t a = 0; a < m; ++a) list[a] = (uint32_t)(ord[a] & 0xffffffffu);
    int nchunks = nthreads > 0 ? nthreads : 1;
    if (nchunks > wh) nchunks = (int)wh;
    if (nchunks < 1) nchunks = 1;
    og_ctx C = {n, nk, v, smooth, wx0, wy0, ww, wh, G, list, m, wgt, eps_alpha, eps_step, img, amb, nchunks,
                (double *)calloc((size_t)nchunks * (size_t)(m > 0 ? m : 1) * 9, sizeof(double))};
    /* one chunk of image rows per thread, each with its own accumulator */
    if (nchunks > OG_MAX_THREADS) nchunks = OG_MAX_THREADS;
    C.nchunks = nchunks;
    pthread_t th[OG_MAX_THREADS];
    og_arg args[OG_MAX_THREADS];
    int created[OG_MAX_THREADS] = {0};
    for (int k = 0; k < nchunks; ++k) {
        args[k].c = &C;
        args[k].k = k;
    }
    for (int k = 1; k < nchunks; ++k) created[k] = pthread_create(&th[k], NULL, og_thread, &args[k]) == 0;
    og_pixels(&C, 0);
    for (int k = 1; k < nchunks; ++k) {
        if (created[k])
            pthread_join(th[k], NULL);
        else
            og_pixels(&C, k);
    }
    /* reduce the chunk accumulators */
    for (int k = 1; k < nchunks; ++k)
        for (int64_t j = 0; j < m * 9; ++j) C.acc[j] += C.acc[(int64_t)k * m * 9 + j];
    memset(g_mean, 0, sizeof(double) * 3 * (size_t)n);
    memset(g_logs, 0, sizeof(double) * 3 * (size_t)n);
    memset(g_quat, 0, sizeof(double) * 4 * (size_t)n);
    memset(g_logit, 0, sizeof(double) * (size_t)n);
    memset(g_sh, 0, sizeof(double) * (size_t)nk * 3 * (size_t)n);
    for (int64_t j = 0; j < m; ++j) {
        const int64_t i = list[j];
        double gm[3] = {0, 0, 0}, gls[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, glg = 0;
        og_chain(&G[i], C.acc + j * 9, v, smooth, nk, sh, n, i, gm, gls, gq, &glg, g_sh + i);
        for (int k = 0; k < 3; ++k) { g_mean[(int64_t)k * n + i] = gm[k]; g_logs[(int64_t)k * n + i] = gls[k]; }
        for (int k = 0; k < 4; ++k) g_quat[(int64_t)k * n + i] = gq[k];
        g_logit[i] = glg;
    }
    free(C.acc);
    free(G);
    free(ord);
    free(list);
    return m;
}
