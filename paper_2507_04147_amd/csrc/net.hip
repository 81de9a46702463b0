// Learned peripheral upsampler on the CDNA4 matrix cores (bfloat16 MFMA,
// float32 accumulation):
//   out = pixel_shuffle_x4(conv3(relu(conv2(relu(conv1(x)))))) + bilinear_x4(x),
// 3x3 convolutions 3->32->32->48 with zero padding, trained with the mean
// squared error against the full-resolution render.  (The periphery of the
// paper's foveated frame is rendered at reduced resolution, Sec. 2.2; this
// network replaces the interpolation that brings it back to full resolution.)
//
// Layouts (device):
//   NHWC bf16   [b][y][x][C]      input of a convolution (A operand: 8 channels
//                                 of one pixel = one 16-byte load per lane);
//   CHW* bf16   [b][C][h+2][WS]   zero-bordered channel-major copy (one zero row
//                                 above and below, data from column 8, WS =
//                                 roundup(w,32)+16) read by the weight gradient:
//                                 8 consecutive pixels of one channel = one
//                                 aligned 16-byte load;
//   packed weights [9][NOUT][KIN] bf16 (tap-major; KIN padded to 8).
//
// Implicit GEMM: M = 16 consecutive pixels of a row, N = 16 output channels,
// K = (tap, input channel) flattened, 32 per v_mfma_f32_16x16x32_bf16.  Lane l
// of the 16x16x32 instruction holds A row l%16 (a pixel) with K entries
// 8(l/16)..+7, B column l%16 (a channel) with the same K entries, and returns
// D rows 4(l/16)..+3 (four pixels) of column l%16.
#include "a3fr_internal.h"

namespace a3fr {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace {

__device__ __forceinline__ uint16_t bf16_bits(float x) {
    const __bf16 h = (__bf16)x;  // round to nearest, ties to even
    return __builtin_bit_cast(uint16_t, h);
}

__device__ __forceinline__ float bf16_val(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ __forceinline__ floatx4 mfma16(bf16x8 a, bf16x8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

constexpr int kRowsPerBlock = 8;

}  // namespace

__host__ __device__ int net_chw_stride(int w) { return ((w + 31) / 32) * 32 + 16; }

// ---------------------------------------------------------------------------
// weight packing: float32 master -> bf16 forward [9][co][cinpad] and
// input-gradient [9][ci][co] (taps rotated by 180 degrees) layouts
// ---------------------------------------------------------------------------
__device__ __forceinline__ void net_pack_item(const float *__restrict__ theta, const NetPacked &pk, int t) {
    // layer 1: W1 [32][3][3][3] -> f1 [9][32][8]
    if (t < 9 * 32 * 8) {
        const int c = t % 8, co = (t / 8) % 32, tap = t / 256;
        const float v = c < 3 ? theta[kNetW1 + (co * 3 + c) * 9 + tap] : 0.0f;
        pk.f1[t] = bf16_bits(v);
    }
    // layer 2: W2 [32][32][3][3] -> f2 [9][32][32] and d2 [9][32(ci)][32(co)]
    if (t < 9 * 32 * 32) {
        const int a = t % 32, b = (t / 32) % 32, tap = t / 1024;
        pk.f2[t] = bf16_bits(theta[kNetW2 + (b * 32 + a) * 9 + tap]);                 // co = b, ci = a
        pk.d2[t] = bf16_bits(theta[kNetW2 + (a * 32 + b) * 9 + (8 - tap)]);           // ci = b, co = a
    }
    // layer 3: W3 [48][32][3][3] -> f3 [9][48][32] and d3 [9][32(ci)][48(co)]
    if (t < 9 * 48 * 32) {
        {
            const int ci = t % 32, co = (t / 32) % 48, tap = t / (48 * 32);
            pk.f3[t] = bf16_bits(theta[kNetW3 + (co * 32 + ci) * 9 + tap]);
        }
        {
            const int co = t % 48, ci = (t / 48) % 32, tap = t / (48 * 32);
            pk.d3[t] = bf16_bits(theta[kNetW3 + (co * 32 + ci) * 9 + (8 - tap)]);
        }
    }
}

// FP32 planar [B][3][h][w] -> bf16 NHWC8 (channels 3..7 zero) and, if chw is
// not NULL, the zero-bordered channel-major copy [B][8][h+2][WS].
__device__ __forceinline__ void net_input_item(const float *__restrict__ x, int64_t x_bstride, int B, int h, int w,
                                               uint16_t *__restrict__ nhwc, uint16_t *__restrict__ chw, int64_t p) {
    const int64_t HW = (int64_t)h * w;
    if (p >= (int64_t)B * HW) return;
    const int64_t b = p / HW, q = p - b * HW;
    const int y = (int)(q / w), xx = (int)(q - (int64_t)y * w);
    uint16_t v[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) v[c] = c < 3 ? bf16_bits(x[b * x_bstride + c * HW + q]) : (uint16_t)0;
    uint4 pk;
    pk.x = v[0] | ((uint32_t)v[1] << 16);
    pk.y = v[2] | ((uint32_t)v[3] << 16);
    pk.z = v[4] | ((uint32_t)v[5] << 16);
    pk.w = v[6] | ((uint32_t)v[7] << 16);
    reinterpret_cast<uint4 *>(nhwc)[p] = pk;
    if (chw) {
        const int WS = net_chw_stride(w);
#pragma unroll
        for (int c = 0; c < 3; ++c) chw[((b * 8 + c) * (int64_t)(h + 2) + y + 1) * WS + 8 + xx] = v[c];
    }
}

// Both preparations of a forward in one launch (they are independent): the
// first pack_blocks blocks pack the weights, the others convert the input.
constexpr int kNetPackBlocks = (9 * 48 * 32 + 255) / 256;
__global__ void __launch_bounds__(256) k_net_prep(const float *__restrict__ theta, NetPacked pk,
                                                  const float *__restrict__ x, int64_t x_bstride, int B, int h, int w,
                                                  uint16_t *__restrict__ nhwc, uint16_t *__restrict__ chw) {
    if ((int)blockIdx.x < kNetPackBlocks)
        net_pack_item(theta, pk, blockIdx.x * 256 + threadIdx.x);
    else
        net_input_item(x, x_bstride, B, h, w, nhwc, chw, (int64_t)(blockIdx.x - kNetPackBlocks) * 256 + threadIdx.x);
}

// ---------------------------------------------------------------------------
// convolution (forward and input gradient)
// ---------------------------------------------------------------------------
enum { kEpiRelu = 0, kEpiShuffle = 1, kEpiMask = 2 };

// Frame mode: true when every full-resolution pixel centre of the x4 blocks of
// input pixels [xa, xb] x [ya, yb] (this layer's pixels widened by its halo)
// lies within r_mid of the gaze, i.e. the composite takes none of them from the
// periphery.  The region test is convex, so the four extreme centres decide;
// a relative margin keeps rounding on the safe side (such waves are computed).
__device__ __forceinline__ bool inside_mid(int xa, int xb, int ya, int yb, double gx, double gy, double rm) {
    const double x0 = 4.0 * xa + 0.5 - gx, x1 = 4.0 * xb + 3.5 - gx;
    const double y0 = 4.0 * ya + 0.5 - gy, y1 = 4.0 * yb + 3.5 - gy;
    const double mx = fmax(x0 * x0, x1 * x1), my = fmax(y0 * y0, y1 * y1);
    return mx + my <= rm * rm * (1.0 - 1e-12);
}

// Epilogue of one image row of a hidden layer (ReLU forward, or the
// activation mask of the input gradient): lane holds pixels xs + 4g + r
// (r = 0..3) of channel nb*16 + li of every 16-channel block nb.  The
// bfloat16 row of the wave (16 pixels x NOUT channels) is staged in LDS (st:
// 16 rows of kStageStride<NOUT> halves) and stored NHWC with 16-byte stores,
// NOUT/8 lanes per pixel; the channel-major copy (training) is written from
// the registers.
template <int NOUT>
constexpr int kStageStride = NOUT + 8;  // halves per staged pixel (16-byte aligned rows)

template <int KIN, int NOUT, int EPI>
__device__ __forceinline__ void conv_epilogue(const NetConvArgs &a, const floatx4 *acc, uint16_t *st, int b, int y,
                                              int xs, int li, int g, int lane, int WS) {
    constexpr int NB = NOUT / 16;
    constexpr int SS = kStageStride<NOUT>;
    const int h = a.h, w = a.w;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int ch = nb * 16 + li;
        uint16_t q[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int x = xs + 4 * g + r;
            float v = acc[nb][r];
            if (EPI == kEpiRelu) {
                v = fmaxf(v + a.bias[ch], 0.0f);
            } else {
                // active where the forward activation is positive (bf16 bits as int16 > 0)
                const bool on = x < w && (int16_t)a.mask[(((int64_t)b * h + y) * w + x) * NOUT + ch] > 0;
                v = on ? v : 0.0f;
            }
            q[r] = bf16_bits(v);
            st[(4 * g + r) * SS + ch] = q[r];
        }
        if (a.out_chw) {
            uint16_t *o = a.out_chw + (((int64_t)b * NOUT + ch) * (h + 2) + y + 1) * WS + 8 + xs + 4 * g;
            if (xs + 4 * g + 3 < w) {
                uint2 pk;
                pk.x = q[0] | ((uint32_t)q[1] << 16);
                pk.y = q[2] | ((uint32_t)q[3] << 16);
                *reinterpret_cast<uint2 *>(o) = pk;
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (xs + 4 * g + r < w) o[r] = q[r];
            }
        }
    }
    if (a.out) {
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        constexpr int kParts = NOUT / 8;  // 16-byte pieces per pixel
        for (int k = lane; k < 16 * kParts; k += 64) {
            const int px = k / kParts, part = k % kParts;
            if (xs + px < w)
                *reinterpret_cast<uint4 *>(a.out + (((int64_t)b * h + y) * w + xs + px) * NOUT + part * 8) =
                    *reinterpret_cast<const uint4 *>(st + px * SS + part * 8);
        }
    }
    __builtin_amdgcn_wave_barrier();  // the staging area is reused by the next row
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Epilogue of the last layer for one image row, through LDS: the wave's 16
// pixels x 48 channels are staged, then lane l produces output column
// X = 4 xs + l (pixel x = xs + l/4, j = l%4) of the four output rows and three
// colour channels: out(c, 4y+i, X) = y3[x][c*16 + 4i + j] + b3 + bilinear,
// so every store writes 64 consecutive floats.
constexpr int kShufStride = 49;  // floats per staged pixel (48 channels + 1: bank spread)

__device__ __forceinline__ void shuffle_epilogue(const NetConvArgs &a, const floatx4 *acc, float *st, int b, int y,
                                                 int xs, int li, int g, int lane, double gx, double gy) {
    const int h = a.h, w = a.w;
#pragma unroll
    for (int nb = 0; nb < 3; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) st[(4 * g + r) * kShufStride + nb * 16 + li] = acc[nb][r];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int x = xs + (lane >> 2), j = lane & 3;
    if (x < w) {
        const int H4 = 4 * h, W4 = 4 * w;
        const int X = 4 * x + j;
        float sx = ((float)X + 0.5f) * 0.25f - 0.5f;
        sx = fminf(fmaxf(sx, 0.0f), (float)(w - 1));
        const float fx0 = floorf(sx);
        const int xa = (int)fx0, xb = xa + 1 < w ? xa + 1 : w - 1;
        const float wx = sx - fx0;
        const float *px = st + (lane >> 2) * kShufStride;
        // the four output rows 4y + i sample input rows y - 1, y, y + 1 (clamped):
        // their horizontal interpolations, once per row and channel
        const int rows[3] = {y > 0 ? y - 1 : 0, y, y + 1 < h ? y + 1 : h - 1};
        float hz[3][3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float *src = a.img_in + (int64_t)b * a.img_bstride + (int64_t)c * h * w;
#pragma unroll
            for (int k = 0; k < 3; ++k)
                hz[c][k] = (1.0f - wx) * src[(int64_t)rows[k] * w + xa] + wx * src[(int64_t)rows[k] * w + xb];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int Y = 4 * y + i;
            if (a.gv) {  // frame mode: only the composite's periphery (outside r_mid)
                const double dx = ((double)X + 0.5) - gx, dy = ((double)Y + 0.5) - gy;
                if (!(dx * dx + dy * dy > a.rm * a.rm)) continue;
            }
            float sy = ((float)Y + 0.5f) * 0.25f - 0.5f;
            sy = fminf(fmaxf(sy, 0.0f), (float)(h - 1));
            const float fy0 = floorf(sy);
            const int ya = (int)fy0, yb = ya + 1 < h ? ya + 1 : h - 1;
            const float wy = sy - fy0;
            // ya and yb are among the three rows (equal rows hold equal values)
            const int ka = ya == rows[0] ? 0 : (ya == rows[1] ? 1 : 2);
            const int kb = yb == rows[0] ? 0 : (yb == rows[1] ? 1 : 2);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float *dst = a.img_out + (int64_t)b * a.out_bstride + (int64_t)c * H4 * W4;
                const float top = ka == 0 ? hz[c][0] : (ka == 1 ? hz[c][1] : hz[c][2]);
                const float bot = kb == 0 ? hz[c][0] : (kb == 1 ? hz[c][1] : hz[c][2]);
                const int ch = c * 16 + 4 * i + j;
                dst[(int64_t)Y * W4 + X] = (px[ch] + a.bias[ch]) + ((1.0f - wy) * top + wy * bot);
            }
        }
    }
    __builtin_amdgcn_wave_barrier();  // the staging area is reused by the next row
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int KIN, int NOUT, int EPI, bool PERSIST>
__global__ void __launch_bounds__(256) k_net_conv(NetConvArgs a) {
    constexpr int KS = KIN + 8;                       // padded LDS row (bank spread, 16-byte aligned)
    constexpr int KTOT = 9 * KIN;
    constexpr int NKS = (KTOT + 31) / 32;
    constexpr int NB = NOUT / 16;
    __shared__ __attribute__((aligned(16))) uint16_t wl[9 * NOUT * KS];
    __shared__ float shuf[EPI == kEpiShuffle ? 4 * 16 * kShufStride : 1];
    __shared__ __attribute__((aligned(16))) uint16_t stage[EPI == kEpiShuffle ? 8 : 4 * 16 * kStageStride<NOUT>];
    const int tid = threadIdx.x;
    // weights [9][NOUT][KIN] -> LDS, 16 bytes per thread per step
    for (int c = tid; c < 9 * NOUT * KIN / 8; c += 256) {
        const int row = c / (KIN / 8), part = c % (KIN / 8);
        *reinterpret_cast<uint4 *>(&wl[row * KS + part * 8]) = reinterpret_cast<const uint4 *>(a.wpk)[c];
    }
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, g = lane >> 4;
    const int h = a.h, w = a.w;
    const int WS = net_chw_stride(w);
    // frame mode: halo of this layer's outputs in the last layer's pixels
    constexpr int HALO = NOUT == 48 ? 0 : (KIN == 8 ? 2 : 1);
    // tiles of 64 pixels x a.rows rows: one per block (grid x, y, batch), or,
    // PERSIST, resident blocks taking them in a grid-stride loop, so that the
    // weights are staged once per block for several tiles
    const int nbx = (w + 63) / 64, nby = (h + a.rows - 1) / a.rows;
    const int64_t ntile = PERSIST ? (int64_t)nbx * nby * a.B : 1;
    for (int64_t tile = PERSIST ? (int64_t)blockIdx.x : 0; tile < ntile; tile += PERSIST ? gridDim.x : 1) {
        int bx = blockIdx.x, y0 = blockIdx.y * a.rows, b = blockIdx.z;
        if (PERSIST) {
            bx = (int)(tile % nbx);
            const int64_t rest = tile / nbx;
            y0 = (int)(rest % nby) * a.rows;
            b = (int)(rest / nby);
        }
        const int xs = bx * 64 + wave * 16;  // this wave's 16 pixels
        if (xs >= w) continue;
        const uint16_t *in = a.in + (int64_t)b * h * w * KIN;
        double gx = 0.0, gy = 0.0;
        if (a.gv) {
            gx = a.gv[(int64_t)b * a.gv_stride].v.gx;
            gy = a.gv[(int64_t)b * a.gv_stride].v.gy;
        }
        // two image rows per pass: each weight fragment read from LDS feeds two
        // matrix-core instructions (one per row)
        for (int y = y0; y < y0 + a.rows && y < h; y += 2) {
            const bool has1 = y + 1 < y0 + a.rows && y + 1 < h;
            const bool skip0 = a.gv && inside_mid(max(xs - HALO, 0), min(xs + 15 + HALO, w - 1), max(y - HALO, 0),
                                                  min(y + HALO, h - 1), gx, gy, a.rm);
            const bool skip1 = !has1 || (a.gv && inside_mid(max(xs - HALO, 0), min(xs + 15 + HALO, w - 1),
                                                            max(y + 1 - HALO, 0), min(y + 1 + HALO, h - 1), gx, gy, a.rm));
            if (skip0 && skip1) continue;  // wave-uniform
            floatx4 acc[2][NB];
    #pragma unroll
            for (int r = 0; r < 2; ++r)
    #pragma unroll
                for (int nb = 0; nb < NB; ++nb) acc[r][nb] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    #pragma unroll
            for (int s = 0; s < NKS; ++s) {
                const int k0 = 32 * s + 8 * g;
                uint4 av0 = {0u, 0u, 0u, 0u}, av1 = {0u, 0u, 0u, 0u};
                int tap = 0, c0 = 0;
                const bool kval = k0 < KTOT;
                if (kval) {
                    tap = k0 / KIN;
                    c0 = k0 - tap * KIN;
                    const int py = y + tap / 3 - 1, px = xs + li + tap % 3 - 1;
                    if (px >= 0 && px < w) {
                        if (py >= 0 && py < h)
                            av0 = *reinterpret_cast<const uint4 *>(in + ((int64_t)py * w + px) * KIN + c0);
                        if (has1 && py + 1 >= 0 && py + 1 < h)
                            av1 = *reinterpret_cast<const uint4 *>(in + ((int64_t)(py + 1) * w + px) * KIN + c0);
                    }
                }
                const bf16x8 A0 = as_bf16x8(av0), A1 = as_bf16x8(av1);
    #pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    uint4 bv = {0u, 0u, 0u, 0u};
                    if (kval) bv = *reinterpret_cast<const uint4 *>(&wl[(tap * NOUT + nb * 16 + li) * KS + c0]);
                    acc[0][nb] = mfma16(A0, as_bf16x8(bv), acc[0][nb]);
                    if (has1) acc[1][nb] = mfma16(A1, as_bf16x8(bv), acc[1][nb]);  // wave-uniform
                }
            }
    #pragma unroll
            for (int rr = 0; rr < 2; ++rr) {
                if (rr == 1 && !has1) break;
                if (EPI == kEpiShuffle)
                    shuffle_epilogue(a, acc[rr], shuf + wave * 16 * kShufStride, b, y + rr, xs, li, g, lane, gx, gy);
                else
                    conv_epilogue<KIN, NOUT, EPI>(a, acc[rr], stage + wave * 16 * kStageStride<NOUT>, b, y + rr, xs, li, g,
                                                  lane, WS);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// weight gradient: dW[co][ci][tap] = sum_p g[p][co] in[p + tap][ci]
// one wave per (m-block of 16 output channels, n-block of 16 input channels,
// row offset dy); the three taps dx = -1, 0, +1 share the aligned 16-byte
// load of 8 pixels and two single-pixel loads (funnel-shifted with
// alignbyte).  A = g^T (M = co, K = pixels), B = in (K = pixels, N = ci).
// ---------------------------------------------------------------------------
constexpr int kWgradUnroll = 4;

template <int CIN, int KIN, int NOUT>
__global__ void __launch_bounds__(64) k_net_wgrad(NetWgradArgs a) {
    constexpr int NBK = (KIN + 15) / 16;
    const int unit = blockIdx.x;
    const int dy = unit % 3 - 1, nb = (unit / 3) % NBK, mb = unit / (3 * NBK);
    const int lane = threadIdx.x, li = lane & 15, g = lane >> 4;
    const int h = a.h, w = a.w, WS = net_chw_stride(w);
    const int xchunks = (w + 31) / 32;
    const int64_t chunks = (int64_t)a.B * h * xchunks;
    const int co = mb * 16 + li, ci = nb * 16 + li;
    const bool cival = ci < KIN;
    floatx4 acc[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) acc[d] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    float dbias = 0.0f;
    const bool do_bias = nb == 0 && dy == 0;
    // kWgradUnroll chunks per step, their loads issued before any product so
    // that several round trips to memory overlap
    for (int64_t c0 = blockIdx.y; c0 < chunks; c0 += (int64_t)kWgradUnroll * gridDim.y) {
        uint4 av[kWgradUnroll], bc[kWgradUnroll];
        uint32_t left[kWgradUnroll], right[kWgradUnroll];
#pragma unroll
        for (int u = 0; u < kWgradUnroll; ++u) {
            const int64_t c = c0 + (int64_t)u * gridDim.y;
            av[u] = uint4{0u, 0u, 0u, 0u};
            bc[u] = uint4{0u, 0u, 0u, 0u};
            left[u] = right[u] = 0u;
            if (c < chunks) {
                const int xc = (int)(c % xchunks) * 32;
                const int64_t by = c / xchunks;
                const int y = (int)(by % h);
                const int b = (int)(by / h);
                const int p = xc + 8 * g;
                av[u] = *reinterpret_cast<const uint4 *>(a.g + (((int64_t)b * NOUT + co) * (h + 2) + y + 1) * WS + 8 + p);
                if (cival) {
                    const uint16_t *row = a.in + (((int64_t)b * KIN + ci) * (h + 2) + y + 1 + dy) * WS + 8 + p;
                    bc[u] = *reinterpret_cast<const uint4 *>(row);
                    left[u] = row[-1];
                    right[u] = row[8];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kWgradUnroll; ++u) {
            if (do_bias) {
                const uint32_t wd[4] = {av[u].x, av[u].y, av[u].z, av[u].w};
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    dbias += bf16_val((uint16_t)(wd[k] & 0xffffu)) + bf16_val((uint16_t)(wd[k] >> 16));
            }
            // pixels p-1 .. p+6 and p+1 .. p+8
            uint4 bm, bp;
            bm.x = __builtin_amdgcn_alignbyte(bc[u].x, left[u] << 16, 2);
            bm.y = __builtin_amdgcn_alignbyte(bc[u].y, bc[u].x, 2);
            bm.z = __builtin_amdgcn_alignbyte(bc[u].z, bc[u].y, 2);
            bm.w = __builtin_amdgcn_alignbyte(bc[u].w, bc[u].z, 2);
            bp.x = __builtin_amdgcn_alignbyte(bc[u].y, bc[u].x, 2);
            bp.y = __builtin_amdgcn_alignbyte(bc[u].z, bc[u].y, 2);
            bp.z = __builtin_amdgcn_alignbyte(bc[u].w, bc[u].z, 2);
            bp.w = __builtin_amdgcn_alignbyte(right[u], bc[u].w, 2);
            const bf16x8 A = as_bf16x8(av[u]);
            acc[0] = mfma16(A, as_bf16x8(bm), acc[0]);
            acc[1] = mfma16(A, as_bf16x8(bc[u]), acc[1]);
            acc[2] = mfma16(A, as_bf16x8(bp), acc[2]);
        }
    }
    // D lane: rows co = 16 mb + 4g + r, column ci = 16 nb + li
    if (ci < CIN) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int tap = (dy + 1) * 3 + d;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int o = mb * 16 + 4 * g + r;
                atomicAdd(&a.grad[a.off_w + (o * CIN + ci) * 9 + tap], acc[d][r]);
            }
        }
    }
    if (do_bias) {
        dbias += __shfl_xor(dbias, 16, 64);
        dbias += __shfl_xor(dbias, 32, 64);
        if (g == 0) atomicAdd(&a.grad[a.off_b + co], dbias);
    }
}

// ---------------------------------------------------------------------------
// loss: mean squared error; dL/dy3 = unshuffle(2 (out - target) / N) in bf16
// (NHWC48 and the channel-major copy); sum of squares accumulated in float64
// ---------------------------------------------------------------------------
// One thread per low-resolution pixel (x fastest): its 48 gradient channels
// come from 3 colours x 4 rows x 4 contiguous output pixels (16-byte loads,
// coalesced across the wave), its NHWC48 row is written as six 16-byte
// stores and each channel-major plane gets one coalesced 2-byte store per
// lane.  The sum of squares is reduced in the block, one atomic per block.
__global__ void __launch_bounds__(256) k_net_mse(const float *__restrict__ out, const float *__restrict__ target,
                                                 int B, int h, int w, uint16_t *__restrict__ g_nhwc,
                                                 uint16_t *__restrict__ g_chw, double *__restrict__ sse) {
    __shared__ double red[4];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t npix = (int64_t)B * h * w;
    double e2 = 0.0;
    if (t < npix) {
        const int x = (int)(t % w);
        const int64_t by = t / w;
        const int y = (int)(by % h), b = (int)(by / h);
        const int64_t H4 = 4 * (int64_t)h, W4 = 4 * (int64_t)w;
        const float inv_n = 1.0f / (float)((int64_t)B * 3 * H4 * W4);
        const int WS = net_chw_stride(w);
        uint32_t q[24];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t o = (((int64_t)b * 3 + c) * H4 + 4 * y + i) * W4 + 4 * x;
                const float4 ov = *reinterpret_cast<const float4 *>(out + o);
                const float4 tv = *reinterpret_cast<const float4 *>(target + o);
                const float d[4] = {ov.x - tv.x, ov.y - tv.y, ov.z - tv.z, ov.w - tv.w};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int ch = c * 16 + i * 4 + j;
                    const uint16_t v = bf16_bits(2.0f * d[j] * inv_n);
                    g_chw[(((int64_t)b * 48 + ch) * (h + 2) + y + 1) * WS + 8 + x] = v;
                    if (j & 1) q[ch >> 1] |= (uint32_t)v << 16;
                    else q[ch >> 1] = v;
                    e2 += (double)d[j] * (double)d[j];
                }
            }
        }
        uint4 *dst = reinterpret_cast<uint4 *>(g_nhwc + t * 48);
#pragma unroll
        for (int k = 0; k < 6; ++k) dst[k] = uint4{q[4 * k], q[4 * k + 1], q[4 * k + 2], q[4 * k + 3]};
    }
    for (int off = 32; off > 0; off >>= 1) e2 += __shfl_xor(e2, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e2;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double s4 = red[0] + red[1] + red[2] + red[3];
        if (s4 != 0.0) atomicAdd(sse, s4);
    }
}

__global__ void k_net_loss_final(const double *sse, int64_t n, float *loss) { *loss = (float)(*sse / (double)n); }

// ---------------------------------------------------------------------------
// Adam (bias-corrected moments), float32
// ---------------------------------------------------------------------------
__global__ void k_net_adam(float *__restrict__ theta, const float *__restrict__ grad, float *__restrict__ m,
                           float *__restrict__ v, int n, float lr, float beta1, float beta2, float eps, float bc1,
                           float bc2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = grad[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_net_prep(const float *theta, const NetPacked &pk, const float *x, int64_t x_bstride, int B, int h, int w,
                     uint16_t *nhwc, uint16_t *chw, hipStream_t s) {
    const int64_t n = (int64_t)B * h * w;
    if (x_bstride == 0) x_bstride = 3 * (int64_t)h * w;
    hipLaunchKernelGGL(k_net_prep, dim3((unsigned)(kNetPackBlocks + (n + 255) / 256)), dim3(256), 0, s, theta, pk, x,
                       x_bstride, B, h, w, nhwc, chw);
}

// persistent blocks of the last layer's forward: three per compute unit of the MI355X
constexpr int64_t kNetConvBlocks = 3 * 256;

void launch_net_conv(int layer, bool dgrad, const NetConvArgs &a_in, hipStream_t s) {
    NetConvArgs a = a_in;
    if (a.rows <= 0) a.rows = kRowsPerBlock;
    if (a.img_bstride == 0) a.img_bstride = 3 * (int64_t)a.h * a.w;
    if (a.out_bstride == 0) a.out_bstride = 3 * (int64_t)(4 * a.h) * (4 * a.w);
    const dim3 grid((unsigned)((a.w + 63) / 64), (unsigned)((a.h + a.rows - 1) / a.rows), (unsigned)a.B);
    if (!dgrad) {
        if (layer == 1) hipLaunchKernelGGL((k_net_conv<8, 32, kEpiRelu, false>), grid, dim3(256), 0, s, a);
        else if (layer == 2) hipLaunchKernelGGL((k_net_conv<32, 32, kEpiRelu, false>), grid, dim3(256), 0, s, a);
        else {
            // the last layer (the largest weights) keeps its blocks resident
            const int64_t ntile = (int64_t)grid.x * grid.y * grid.z;
            hipLaunchKernelGGL((k_net_conv<32, 48, kEpiShuffle, true>),
                               dim3((unsigned)std::min<int64_t>(ntile, kNetConvBlocks)), dim3(256), 0, s, a);
        }
    } else {
        // input gradient of layer 3 (g3: 48 channels -> 32) and of layer 2 (32 -> 32)
        if (layer == 3) hipLaunchKernelGGL((k_net_conv<48, 32, kEpiMask, false>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_net_conv<32, 32, kEpiMask, false>), grid, dim3(256), 0, s, a);
    }
}

void launch_net_wgrad(int layer, const NetWgradArgs &a, int slabs, hipStream_t s) {
    if (layer == 1) hipLaunchKernelGGL((k_net_wgrad<3, 8, 32>), dim3(2 * 1 * 3, slabs), dim3(64), 0, s, a);
    else if (layer == 2) hipLaunchKernelGGL((k_net_wgrad<32, 32, 32>), dim3(2 * 2 * 3, slabs), dim3(64), 0, s, a);
    else hipLaunchKernelGGL((k_net_wgrad<32, 32, 48>), dim3(3 * 2 * 3, slabs), dim3(64), 0, s, a);
}

void launch_net_mse(const float *out, const float *target, int B, int h, int w, uint16_t *g_nhwc, uint16_t *g_chw,
                    double *sse, float *loss, hipStream_t s) {
    const int64_t n = (int64_t)B * h * w;
    if (n > 0)
        hipLaunchKernelGGL(k_net_mse, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, target, B, h, w, g_nhwc,
                           g_chw, sse);
    if (loss) hipLaunchKernelGGL(k_net_loss_final, dim3(1), dim3(1), 0, s, sse, (int64_t)B * 3 * 16 * h * w, loss);
}

void launch_net_adam(float *theta, const float *grad, float *m, float *v, int n, float lr, float beta1, float beta2,
                     float eps, float bc1, float bc2, hipStream_t s) {
    hipLaunchKernelGGL(k_net_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, theta, grad, m, v, n, lr, beta1,
                       beta2, eps, bc1, bc2);
}

}  // namespace a3fr
