// Training side of the library: device activation of the optimised
// parameters, and the reverse of the projection, colour and activation
// (paper Sec. 2.3: every point carries trainable position, scale, rotation,
// opacity and SH colour; the render is projection -> depth sort -> blend).
//
// The reverse projection runs one thread per Gaussian in float64: it
// recomputes the forward key path of each view it was drawn in (view-space
// position, 3D and view covariance, guard-band-clamped Jacobian, dilated 2D
// covariance), takes the per-(view, Gaussian) sums accumulated by the reverse
// blend, and applies the chain rule down to the raw parameters.  Memory
// traffic per Gaussian is the parameters once (236 B at degree 3), the 48-byte
// accumulator and record of each view it was drawn in, and the gradients once.
#include "a3fr_internal.h"

namespace a3fr {

// ------------------------------------------------------------------------
// activation
// ------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_activate(a3fr_params p, float *__restrict__ scale,
                                                  float *__restrict__ opacity) {
    const int64_t n = p.n;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) scale[k * n + i] = (float)exp((double)p.log_scale_dev[k * n + i]);
    opacity[i] = (float)(1.0 / (1.0 + exp(-(double)p.logit_dev[i])));
}

void launch_activate(const a3fr_params &p, float *scale, float *opacity, hipStream_t s) {
    if (p.n == 0) return;
    hipLaunchKernelGGL(k_activate, dim3((unsigned)((p.n + 255) / 256)), dim3(256), 0, s, p, scale, opacity);
}

// ------------------------------------------------------------------------
// reverse projection
// ------------------------------------------------------------------------
// Real SH up to degree 3 (Condon-Shortley phase) at the unit direction
// (x, y, z) and the gradient of each basis polynomial with respect to
// (x, y, z); normalisations sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!), x sqrt 2
// for m != 0.
__device__ __forceinline__ void sh_basis_grad64(double x, double y, double z, double *Y, double (*G)[3]) {
    const double c0 = 0.28209479177387814, c1 = 0.4886025119029199;
    const double c2a = 1.0925484305920792, c2b = 0.31539156525252005, c2c = 0.5462742152960396;
    const double c3a = 0.5900435899266435, c3b = 2.890611442640554, c3c = 0.4570457994644658;
    const double c3d = 0.3731763325901154, c3e = 1.445305721320277;
    const double xx = x * x, yy = y * y, zz = z * z;
    Y[0] = c0;                          G[0][0] = 0.0;            G[0][1] = 0.0;            G[0][2] = 0.0;
    Y[1] = -c1 * y;                     G[1][0] = 0.0;            G[1][1] = -c1;            G[1][2] = 0.0;
    Y[2] = c1 * z;                      G[2][0] = 0.0;            G[2][1] = 0.0;            G[2][2] = c1;
    Y[3] = -c1 * x;                     G[3][0] = -c1;            G[3][1] = 0.0;            G[3][2] = 0.0;
    Y[4] = c2a * x * y;                 G[4][0] = c2a * y;        G[4][1] = c2a * x;        G[4][2] = 0.0;
    Y[5] = -c2a * y * z;                G[5][0] = 0.0;            G[5][1] = -c2a * z;       G[5][2] = -c2a * y;
    Y[6] = c2b * (2.0 * zz - xx - yy);  G[6][0] = -2.0 * c2b * x; G[6][1] = -2.0 * c2b * y; G[6][2] = 4.0 * c2b * z;
    Y[7] = -c2a * x * z;                G[7][0] = -c2a * z;       G[7][1] = 0.0;            G[7][2] = -c2a * x;
    Y[8] = c2c * (xx - yy);             G[8][0] = 2.0 * c2c * x;  G[8][1] = -2.0 * c2c * y; G[8][2] = 0.0;
    // degree 3, each polynomial expanded, then differentiated term by term
    Y[9] = -c3a * y * (3.0 * xx - yy);
    G[9][0] = -6.0 * c3a * x * y; G[9][1] = -3.0 * c3a * (xx - yy); G[9][2] = 0.0;
    Y[10] = c3b * x * y * z;
    G[10][0] = c3b * y * z; G[10][1] = c3b * x * z; G[10][2] = c3b * x * y;
    Y[11] = -c3c * y * (4.0 * zz - xx - yy);
    G[11][0] = 2.0 * c3c * x * y; G[11][1] = -c3c * (4.0 * zz - xx - 3.0 * yy); G[11][2] = -8.0 * c3c * y * z;
    Y[12] = c3d * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
    G[12][0] = -6.0 * c3d * x * z; G[12][1] = -6.0 * c3d * y * z; G[12][2] = c3d * (6.0 * zz - 3.0 * xx - 3.0 * yy);
    Y[13] = -c3c * x * (4.0 * zz - xx - yy);
    G[13][0] = -c3c * (4.0 * zz - 3.0 * xx - yy); G[13][1] = 2.0 * c3c * x * y; G[13][2] = -8.0 * c3c * x * z;
    Y[14] = c3e * z * (xx - yy);
    G[14][0] = 2.0 * c3e * x * z; G[14][1] = -2.0 * c3e * y * z; G[14][2] = c3e * (xx - yy);
    Y[15] = -c3a * x * (xx - 3.0 * yy);
    G[15][0] = -3.0 * c3a * (xx - yy); G[15][1] = 6.0 * c3a * x * y; G[15][2] = 0.0;
}

__global__ void __launch_bounds__(256) k_preprocess_bwd(a3fr_params p, const DevView *__restrict__ views, int nv,
                                                        const uint32_t *__restrict__ counts,
                                                        const uint8_t *__restrict__ keep,
                                                        const uint32_t *__restrict__ map,
                                                        const float *__restrict__ acc,
                                                        const Record *__restrict__ rec, a3fr_grads g) {
    const int64_t n = p.n;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int nk = (p.sh_degree + 1) * (p.sh_degree + 1);
    const double mx = p.mean_dev[i], my = p.mean_dev[n + i], mz = p.mean_dev[2 * n + i];
    const double ls0 = p.log_scale_dev[i], ls1 = p.log_scale_dev[n + i], ls2 = p.log_scale_dev[2 * n + i];
    const double s0 = exp(ls0), s1 = exp(ls1), s2 = exp(ls2);
    const double qw = p.quat_dev[i], qx = p.quat_dev[n + i], qy = p.quat_dev[2 * n + i], qz = p.quat_dev[3 * n + i];
    const double lg = p.logit_dev[i];
    const double op = 1.0 / (1.0 + exp(-lg));
    const double nq = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);

    double gmean[3] = {0.0, 0.0, 0.0};
    double dS3[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // 00 01 02 11 12 22 of dL/dSigma3D (symmetric)
    double gop = 0.0;
    float gsh[48];
#pragma unroll
    for (int k = 0; k < 48; ++k) gsh[k] = 0.0f;
    bool any = false;

    // forward 3D covariance pieces (shared by every view)
    double w = 0.0, x = 0.0, y = 0.0, z = 0.0;
    double Rq[9], M[9], S[9];
    const bool valid = nq > 0.0;
    if (valid) {
        w = qw / nq; x = qx / nq; y = qy / nq; z = qz / nq;
        Rq[0] = 1.0 - 2.0 * (y * y + z * z); Rq[1] = 2.0 * (x * y - w * z); Rq[2] = 2.0 * (x * z + w * y);
        Rq[3] = 2.0 * (x * y + w * z); Rq[4] = 1.0 - 2.0 * (x * x + z * z); Rq[5] = 2.0 * (y * z - w * x);
        Rq[6] = 2.0 * (x * z - w * y); Rq[7] = 2.0 * (y * z + w * x); Rq[8] = 1.0 - 2.0 * (x * x + y * y);
        const double sc[3] = {s0, s1, s2};
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) M[3 * r + c] = Rq[3 * r + c] * sc[c];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                S[3 * r + c] = M[3 * r] * M[3 * c] + M[3 * r + 1] * M[3 * c + 1] + M[3 * r + 2] * M[3 * c + 2];
    }

    for (int vi = 0; vi < nv && valid; ++vi) {
        // the slot's entry (drawn: it has keys and, in a selecting view, is kept) and its record
        const int64_t slot = (int64_t)vi * n + i;
        if (counts[slot] == 0 || (views[vi].v.select && !keep[slot])) continue;
        const int64_t r = map[slot];
        const float4 *a4 = reinterpret_cast<const float4 *>(acc + r * 12);
        const float4 A0 = a4[0], A1 = a4[1], A2 = a4[2];
        const float sums[9] = {A0.x, A0.y, A0.z, A0.w, A1.x, A1.y, A1.z, A1.w, A2.x};
        bool nz = false;
#pragma unroll
        for (int k = 0; k < 9; ++k) nz |= sums[k] != 0.0f;
        if (!nz) continue;
        any = true;
        const DevView &dv = views[vi];
        const a3fr_view &v = dv.v;
        const double *Rw = v.R;
        double pv[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) pv[k] = Rw[3 * k] * mx + Rw[3 * k + 1] * my + Rw[3 * k + 2] * mz + v.t[k];
        // view covariance Sv = Rw S Rw'
        double Aw[9], Sv[9];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                Aw[3 * r + c] = Rw[3 * r] * S[c] + Rw[3 * r + 1] * S[3 + c] + Rw[3 * r + 2] * S[6 + c];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                Sv[3 * r + c] = Aw[3 * r] * Rw[3 * c] + Aw[3 * r + 1] * Rw[3 * c + 1] + Aw[3 * r + 2] * Rw[3 * c + 2];
        const double pz = pv[2];
        const double xz = pv[0] / pz, yz = pv[1] / pz;
        const bool clx = xz < -dv.limx || xz > dv.limx, cly = yz < -dv.limy || yz > dv.limy;
        const double txc = fmin(fmax(xz, -dv.limx), dv.limx), tyc = fmin(fmax(yz, -dv.limy), dv.limy);
        const double J[6] = {v.fx / pz, 0.0, -(v.fx / pz) * txc, 0.0, v.fy / pz, -(v.fy / pz) * tyc};
        double JS[6];
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                JS[3 * r + c] = J[3 * r] * Sv[c] + J[3 * r + 1] * Sv[3 + c] + J[3 * r + 2] * Sv[6 + c];
        const double a = JS[0] * J[0] + JS[1] * J[1] + JS[2] * J[2] + kDilate;
        const double b = JS[0] * J[3] + JS[1] * J[4] + JS[2] * J[5];
        const double c = JS[3] * J[3] + JS[4] * J[4] + JS[5] * J[5] + kDilate;
        const double det = a * c - b * b;
        const double L = 1.4426950408889634;  // log2(e)
        const double a2 = -0.5 * L * c / det, kk = -b / c, c2 = -0.5 * L / c;
        // pixel sums -> record terms -> 2D covariance
        const double d_a2 = sums[0];
        const double d_k = 2.0 * a2 * (double)sums[2];
        const double d_c2 = sums[3];
        const double d_u = -2.0 * a2 * (double)sums[1];
        const double d_v = -2.0 * a2 * kk * (double)sums[1] - 2.0 * c2 * (double)sums[4];
        const double det2 = det * det;
        const double da = d_a2 * (0.5 * L * c * c / det2);
        const double db = d_a2 * (-L * b * c / det2) - d_k / c;
        const double dc = d_a2 * (0.5 * L * b * b / det2) + d_k * b / (c * c) + d_c2 * (0.5 * L / (c * c));
        // symmetric gradient of J Sv J'
        const double G00 = da, G01 = 0.5 * db, G11 = dc;
        double dJ[6];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            dJ[cc] = 2.0 * (G00 * JS[cc] + G01 * JS[3 + cc]);
            dJ[3 + cc] = 2.0 * (G01 * JS[cc] + G11 * JS[3 + cc]);
        }
        double dSv[9];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
                dSv[3 * r + cc] = J[r] * (G00 * J[cc] + G01 * J[3 + cc]) + J[3 + r] * (G01 * J[cc] + G11 * J[3 + cc]);
        // Jacobian and centre as functions of the view-space position
        const double fx = v.fx, fy = v.fy, iz2 = 1.0 / (pz * pz);
        double dp0 = 0.0, dp1 = 0.0, dp2 = 0.0;
        dp2 += dJ[0] * (-fx * iz2) + dJ[4] * (-fy * iz2);
        if (clx) {
            dp2 += dJ[2] * (fx * txc * iz2);
        } else {
            dp0 += dJ[2] * (-fx * iz2);
            dp2 += dJ[2] * (2.0 * fx * pv[0] * iz2 / pz);
        }
        if (cly) {
            dp2 += dJ[5] * (fy * tyc * iz2);
        } else {
            dp1 += dJ[5] * (-fy * iz2);
            dp2 += dJ[5] * (2.0 * fy * pv[1] * iz2 / pz);
        }
        dp0 += d_u * (fx / pz);
        dp2 += d_u * (-fx * pv[0] * iz2);
        dp1 += d_v * (fy / pz);
        dp2 += d_v * (-fy * pv[1] * iz2);
#pragma unroll
        for (int k = 0; k < 3; ++k) gmean[k] += Rw[k] * dp0 + Rw[3 + k] * dp1 + Rw[6 + k] * dp2;
        // Sv = Rw S Rw'  ->  dS += Rw' dSv Rw
        double B[9];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
                B[3 * r + cc] = dSv[3 * r] * Rw[cc] + dSv[3 * r + 1] * Rw[3 + cc] + dSv[3 * r + 2] * Rw[6 + cc];
        const int ur[6] = {0, 0, 0, 1, 1, 2}, uc[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
        for (int e = 0; e < 6; ++e)
            dS3[e] += Rw[ur[e]] * B[uc[e]] + Rw[3 + ur[e]] * B[3 + uc[e]] + Rw[6 + ur[e]] * B[6 + uc[e]];
        gop += (double)sums[5];
        // colour: clamp at zero (the record holds the clamped forward colour), SH basis, direction
        const Record &rr = rec[r];
        const double dcol[3] = {rr.r > 0.0f ? (double)sums[6] : 0.0, rr.g > 0.0f ? (double)sums[7] : 0.0,
                                rr.b > 0.0f ? (double)sums[8] : 0.0};
        if (dcol[0] != 0.0 || dcol[1] != 0.0 || dcol[2] != 0.0) {
            const double ex = mx - v.campos[0], ey = my - v.campos[1], ez = mz - v.campos[2];
            const double len = sqrt(ex * ex + ey * ey + ez * ez);
            const double d0 = ex / len, d1 = ey / len, d2 = ez / len;
            double Y[16], GY[16][3];
            sh_basis_grad64(d0, d1, d2, Y, GY);
            const float *f = p.sh_dev + i * (int64_t)nk * 3;
            double gd0 = 0.0, gd1 = 0.0, gd2 = 0.0;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                if (k < nk) {
                    const double fc = (double)f[3 * k] * dcol[0] + (double)f[3 * k + 1] * dcol[1] +
                                      (double)f[3 * k + 2] * dcol[2];
                    gsh[3 * k] += (float)(Y[k] * dcol[0]);
                    gsh[3 * k + 1] += (float)(Y[k] * dcol[1]);
                    gsh[3 * k + 2] += (float)(Y[k] * dcol[2]);
                    gd0 += fc * GY[k][0];
                    gd1 += fc * GY[k][1];
                    gd2 += fc * GY[k][2];
                }
            }
            const double dot = gd0 * d0 + gd1 * d1 + gd2 * d2;
            gmean[0] += (gd0 - d0 * dot) / len;
            gmean[1] += (gd1 - d1 * dot) / len;
            gmean[2] += (gd2 - d2 * dot) / len;
        }
    }

    double gls[3] = {0.0, 0.0, 0.0}, gq[4] = {0.0, 0.0, 0.0, 0.0};
    if (any) {
        // S = M M'  ->  dM = 2 dS M;  M = Rq diag(s)
        const double D[9] = {dS3[0], dS3[1], dS3[2], dS3[1], dS3[3], dS3[4], dS3[2], dS3[4], dS3[5]};
        double dM[9];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                dM[3 * r + c] = 2.0 * (D[3 * r] * M[c] + D[3 * r + 1] * M[3 + c] + D[3 * r + 2] * M[6 + c]);
        const double sc[3] = {s0, s1, s2};
        double dR[9], ds[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                dR[3 * r + c] = dM[3 * r + c] * sc[c];
                ds[c] += dM[3 * r + c] * Rq[3 * r + c];
            }
#pragma unroll
        for (int c = 0; c < 3; ++c) gls[c] = ds[c] * sc[c];
        // rotation of the unit quaternion (w, x, y, z), then its normalisation
        const double gw = 2.0 * (z * (dR[3] - dR[1]) + y * (dR[2] - dR[6]) + x * (dR[7] - dR[5]));
        const double gx = 2.0 * (y * (dR[1] + dR[3]) + z * (dR[2] + dR[6]) + w * (dR[7] - dR[5])) -
                          4.0 * x * (dR[4] + dR[8]);
        const double gy = 2.0 * (x * (dR[1] + dR[3]) + w * (dR[2] - dR[6]) + z * (dR[5] + dR[7])) -
                          4.0 * y * (dR[0] + dR[8]);
        const double gz = 2.0 * (w * (dR[3] - dR[1]) + x * (dR[2] + dR[6]) + y * (dR[5] + dR[7])) -
                          4.0 * z * (dR[0] + dR[4]);
        const double dot = gw * w + gx * x + gy * y + gz * z;
        gq[0] = (gw - w * dot) / nq;
        gq[1] = (gx - x * dot) / nq;
        gq[2] = (gy - y * dot) / nq;
        gq[3] = (gz - z * dot) / nq;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        g.mean_dev[k * n + i] = (float)gmean[k];
        g.log_scale_dev[k * n + i] = (float)gls[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) g.quat_dev[k * n + i] = (float)gq[k];
    g.logit_dev[i] = (float)(gop * op * (1.0 - op));
    float *gs = g.sh_dev + i * (int64_t)nk * 3;
#pragma unroll
    for (int k = 0; k < 48; ++k)
        if (k < 3 * nk) gs[k] = gsh[k];
}

void launch_preprocess_bwd(const a3fr_params &p, const DevView *views, int nv, const uint32_t *counts,
                           const uint8_t *keep, const uint32_t *map, const float *acc, const Record *rec,
                           const a3fr_grads &g, hipStream_t s) {
    if (p.n == 0) return;
    hipLaunchKernelGGL(k_preprocess_bwd, dim3((unsigned)((p.n + 255) / 256)), dim3(256), 0, s, p, views, nv, counts,
                       keep, map, acc, rec, g);
}

}  // namespace a3fr
