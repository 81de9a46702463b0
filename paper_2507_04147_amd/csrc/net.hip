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
// so every store writes 64 consecutive floats.  Pixels x >= xend are not
// written (xend <= w).
constexpr int kShufStride = 49;  // floats per staged pixel (48 channels + 1: bank spread)

__device__ __forceinline__ void shuffle_epilogue(const NetConvArgs &a, const floatx4 *acc, float *st, int b, int y,
                                                 int xs, int li, int g, int lane, double gx, double gy, int xend) {
    const int h = a.h, w = a.w;
#pragma unroll
    for (int nb = 0; nb < 3; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) st[(4 * g + r) * kShufStride + nb * 16 + li] = acc[nb][r];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int x = xs + (lane >> 2), j = lane & 3;
    if (x < xend) {
        const int H4 = 4 * h, W4 = 4 * w;
        const int X = 4 * x + j;
        float sx = ((float)X + 0.5f) * 0.25f - 0.5f;
        sx = fminf(fmaxf(sx, 0.0f), (float)(w - 1));
        const float fx0 = floorf(sx);
        const int xa = (int)fx0, xb = xa + 1 < w ? xa + 1 : w - 1;
        const float wx = sx - fx0;
        const float *px = st + (lane >> 2) * kShufStride;
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
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                // bilinear residual: vertical interpolation in columns xa and xb, then horizontal
                const float *src = a.img_in + (int64_t)b * a.img_bstride + (int64_t)c * h * w;
                const float va = (1.0f - wy) * src[(int64_t)ya * w + xa] + wy * src[(int64_t)yb * w + xa];
                const float vb = (1.0f - wy) * src[(int64_t)ya * w + xb] + wy * src[(int64_t)yb * w + xb];
                float *dst = a.img_out + (int64_t)b * a.out_bstride + (int64_t)c * H4 * W4;
                const int ch = c * 16 + 4 * i + j;
                dst[(int64_t)Y * W4 + X] = (px[ch] + a.bias[ch]) + ((1.0f - wx) * va + wx * vb);
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
                    shuffle_epilogue(a, acc[rr], shuf + wave * 16 * kShufStride, b, y + rr, xs, li, g, lane, gx, gy,
                                     w);
                else
                    conv_epilogue<KIN, NOUT, EPI>(a, acc[rr], stage + wave * 16 * kStageStride<NOUT>, b, y + rr, xs, li, g,
                                                  lane, WS);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// fused inference forward: conv1 -> conv2 -> conv3 (+ shuffle and bilinear
// residual) in one launch.  Resident blocks (one per compute unit) stage the
// three layers' weights once and then take output tiles of kFxTX x kFxTY
// pixels in turn, keeping everything a tile needs in LDS: its input with a
// 3-pixel halo (bf16 for the products, float32 for the residual), conv1's
// activations with a 2-pixel halo (L1) and conv2's with a 1-pixel halo (L2).
// Only the float32 input is read from memory (each tile's, prefetched into
// registers while the previous tile computes) and only the final image is
// written.
//
// The products are the transposes of the layer-by-layer kernels' (A = the
// weights, M = 16 output channels; B = the pixels, N = 16 pixels of a row),
// with the same K entries in the same lanes and the same order of steps, so
// every sum is the same and both paths give the same bits.  Lane (li, g) of
// D then holds channels nb * 16 + 4g .. + 3 of pixel li: a hidden layer
// stores them as one 8-byte word, and in the last layer they are the four
// output pixels X = 4x .. 4x + 3 of output row 4y + g for colour nb (the
// pixel shuffle), stored as one float4.
// ---------------------------------------------------------------------------
constexpr int kFxTX = 60;                  // output pixels per tile row (4 chunks of 16 cover the 64 of L1)
constexpr int kFxTY = 8;                   // output rows per tile
constexpr int kFxCols = 66;                // stored columns of every layer region
constexpr int kFxThreads = 512;
constexpr int kFxWaves = kFxThreads / 64;  // wave w computes chunk w % 4 of rows (w / 4) * (rows / 2) ...
constexpr int kFxL0Rows = kFxTY + 6, kFxL1Rows = kFxTY + 4, kFxL2Rows = kFxTY + 2;
constexpr int kFxR1 = kFxL1Rows / 2, kFxR2 = kFxL2Rows / 2, kFxR3 = kFxTY / 2;  // rows per wave and layer
constexpr int kFxIn = kFxL0Rows * kFxCols;                                     // input pixels per tile
constexpr int kFxInPer = (kFxIn + kFxThreads - 1) / kFxThreads;                // ... per thread
constexpr int kFxMaskWords = 64;           // frame mode: tiles the block-wide list can rank (x 64)
constexpr int kFxRow = kFxCols * 64;       // bytes per row of a 32-channel region
// LDS byte offsets.  32-channel regions (L1, L2) hold 64 bytes per pixel, the
// 16-byte piece j of column c at slot j ^ ((c >> 2) & 3), and the conv2 and
// conv3 weights 64 bytes per row [tap][co], piece j of row r at slot
// j ^ ((r >> 2) & 3): the 16 consecutive pixels (rows) that 16 lanes read
// with ds_read_b128 cover the 64 banks once.  L0 (8 channels, 16 B per
// pixel) shares its space with L2, which conv2 writes once conv1 is done.
// W1 holds 12 taps (9 .. 11 zero: the unused K entries of conv1's last step).
// F: the tile's float32 input, 16 bytes per pixel (3 channels and a zero).
constexpr int kFxL1 = 0;
constexpr int kFxL2 = kFxL1 + kFxL1Rows * kFxRow;
constexpr int kFxL0 = kFxL2;
constexpr int kFxW1 = kFxL2 + kFxL2Rows * kFxRow;
constexpr int kFxW2 = kFxW1 + 12 * 32 * 16;
constexpr int kFxW3 = kFxW2 + 9 * 32 * 64;
constexpr int kFxBias = kFxW3 + 9 * 48 * 64;
constexpr int kFxF32 = kFxBias + (32 + 32 + 48) * 4;
constexpr int kFxMask = kFxF32 + kFxIn * 16;
constexpr int kFxRank = kFxMask + kFxMaskWords * 8;
constexpr int kFxBytes = kFxRank + (kFxMaskWords + 1) * 4;
static_assert(kFxIn * 16 <= kFxL2Rows * kFxRow, "L0 must fit in L2's space");
static_assert(kFxWaves == 8 && kFxL1Rows % 2 == 0 && kFxL2Rows % 2 == 0 && kFxTY % 2 == 0, "two row groups of 4 chunks");
static_assert(kFxBytes <= 160 * 1024, "LDS of one compute unit");
static_assert((kFxR1 + 2) * kFxRow < 65536 && 12 * 32 * 16 < 65536 && 9 * 48 * 64 < 65536, "immediate LDS offsets");

// byte offset of piece j of pixel (row, col) in a 32-channel region
__device__ __forceinline__ int fx_px(int row, int col, int j) {
    return row * kFxRow + col * 64 + ((j ^ ((col >> 2) & 3)) << 4);
}
// byte offset of piece j of weight row r
__device__ __forceinline__ int fx_wr(int r, int j) { return r * 64 + ((j ^ ((r >> 2) & 3)) << 4); }

__device__ __forceinline__ uint4 lds16(const uint8_t *p) { return *reinterpret_cast<const uint4 *>(p); }

#ifndef FX_STEP_FENCE
#define FX_STEP_FENCE
#endif
// One wave's products of a hidden or last layer: NR rows x 16 pixels x NB x
// 16 channels.  Row i reads the source from row r0 + i + dy, column
// c0 + li + dx.  abase[dx]: the lane's byte address of (r0, c0 + li + dx, g)
// in the source region; wbase: of its piece g of weight row li.  FIRST: the
// source is L0 (16 B per pixel; step s holds tap 4 s + g, so abase[s] is the
// lane's address for step s and wbase its row of tap g) and there are three
// steps; else nine steps of one tap (32 channels, 8 per lane group).  The
// fragments of the next step are loaded before the products of this one.
template <int NR, int NB, bool FIRST>
__device__ __forceinline__ void fx_conv(const uint8_t *const (&abase)[3], const uint8_t *wbase, bool last_ok,
                                        floatx4 (&acc)[NR][NB]) {
    constexpr int NS = FIRST ? 3 : 9;
    constexpr int NOUT = NB * 16;
#pragma unroll
    for (int i = 0; i < NR; ++i)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[i][nb] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        uint4 a[NR], wv[NB];
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            if (FIRST) {
                a[i] = lds16(abase[s] + i * kFxCols * 16);
                if (s == 2 && !last_ok) a[i] = uint4{0u, 0u, 0u, 0u};  // K >= 72 (the weights are zero too)
            } else {
                a[i] = lds16(abase[s % 3] + (i + s / 3) * kFxRow);
            }
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
            wv[nb] = FIRST ? lds16(wbase + (4 * s * 32 + nb * 16) * 16) : lds16(wbase + (s * NOUT + nb * 16) * 64);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int i = 0; i < NR; ++i) acc[i][nb] = mfma16(as_bf16x8(wv[nb]), as_bf16x8(a[i]), acc[i][nb]);
        FX_STEP_FENCE
    }
}

// Epilogue of a hidden layer: ReLU(acc + bias) rounded to bf16, channels
// nb * 16 + 4g .. + 3 of the lane's pixel as one 8-byte store; zero for a
// pixel outside the image (the next layer's zero padding).  dst[nb]: the
// lane's address of its pixel in row r0, channels nb * 16 + 4g; rowin: bit i
// set when row r0 + i lies in the image; in: the lane's column does.
template <int NR>
__device__ __forceinline__ void fx_hidden_store(uint8_t *const (&dst)[2], const floatx4 (&acc)[NR][2],
                                                const float (&bias)[2][4], uint32_t rowin, bool in) {
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const bool on = in && ((rowin >> i) & 1u);
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            uint2 v;
            v.x = bf16_bits(fmaxf(acc[i][nb][0] + bias[nb][0], 0.0f)) |
                  ((uint32_t)bf16_bits(fmaxf(acc[i][nb][1] + bias[nb][1], 0.0f)) << 16);
            v.y = bf16_bits(fmaxf(acc[i][nb][2] + bias[nb][2], 0.0f)) |
                  ((uint32_t)bf16_bits(fmaxf(acc[i][nb][3] + bias[nb][3], 0.0f)) << 16);
            if (!on) v = uint2{0u, 0u};
            *reinterpret_cast<uint2 *>(dst[nb] + i * kFxRow) = v;
        }
    }
}

struct FxTile {
    int b, x0, y0;
};

__device__ __forceinline__ FxTile fx_tile(int64_t t, int tiles_x, int tiles_y) {
    FxTile r;
    r.x0 = (int)(t % tiles_x) * kFxTX;
    const int64_t rest = t / tiles_x;
    r.y0 = (int)(rest % tiles_y) * kFxTY;
    r.b = (int)(rest / tiles_y);
    return r;
}

// frame mode: true when the composite takes none of the tile's pixels from the periphery
__device__ __forceinline__ bool fx_tile_inside(const NetFusedArgs &a, const FxTile &t) {
    if (!a.gv) return false;
    const DevView &v = a.gv[(int64_t)t.b * a.gv_stride];
    return inside_mid(t.x0, min(t.x0 + kFxTX, a.w) - 1, t.y0, min(t.y0 + kFxTY, a.h) - 1, v.v.gx, v.v.gy, a.rm);
}

// Global loads of a tile's float32 input (3 channels of the thread's pixels;
// zero outside the image) into registers.
__device__ __forceinline__ void fx_fetch(const NetFusedArgs &a, const FxTile &t, int tid, float (&v)[kFxInPer][3]) {
    const float *src = a.img_in + (int64_t)t.b * a.img_bstride;
    const int64_t plane = (int64_t)a.h * a.w;
#pragma unroll
    for (int k = 0; k < kFxInPer; ++k) {
        const int q = tid + k * kFxThreads;
        const int r = q / kFxCols, c = q - r * kFxCols;
        const int y = t.y0 - 3 + r, x = t.x0 - 3 + c;
        v[k][0] = v[k][1] = v[k][2] = 0.0f;
        if (q < kFxIn && y >= 0 && y < a.h && x >= 0 && x < a.w) {
            const int64_t o = (int64_t)y * a.w + x;
            v[k][0] = src[o];
            v[k][1] = src[plane + o];
            v[k][2] = src[2 * plane + o];
        }
    }
}

// The last layer's epilogue for the wave's kFxR3 output rows: lane (li, g)
// holds channels c * 16 + 4g + r of pixel x = xs + li, i.e. output pixels
// (4x + r, 4y + g) of colour c (the pixel shuffle); it adds the bias and the
// bilinear residual (as shuffle_epilogue: vertical interpolation in columns
// xa_r and xb_r, then horizontal; those columns are among xl = max(x - 1, 0),
// x, xr = min(x + 1, w - 1): r >= 2 and x = 0 take (x, xr), else (xl, x)) and
// stores the four as one float4.  FAST: every row lies in the image and every
// output pixel outside r_mid (no checks but the tile's right edge).
template <bool FAST, int NR>
__device__ __forceinline__ void fx_last_epilogue(const NetFusedArgs &fa, const floatx4 (&acc)[NR][3],
                                                 const float4 *F, const float *b3, int b, int x0, int y0, int yb0,
                                                 int xs, int xend, int li, int g, int64_t oplane, bool vec_out,
                                                 double gx, double gy) {
    const int h = fa.h, w = fa.w;
    const int x = xs + li;
    if (!FAST && x >= xend) return;
    const int fx0 = x0 - 3, fy0 = y0 - 3;
    float wx[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        float sx = ((float)(4 * x + r) + 0.5f) * 0.25f - 0.5f;
        sx = fminf(fmaxf(sx, 0.0f), (float)(w - 1));
        wx[r] = sx - floorf(sx);
    }
    const int cl = max(x - 1, 0) - fx0, cm = x - fx0, cr = min(x + 1, w - 1) - fx0;
    const bool left = x >= 1;
    double dx2[4] = {0.0, 0.0, 0.0, 0.0};
    if (!FAST && fa.gv)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double dx = ((double)(4 * x + r) + 0.5) - gx;
            dx2[r] = dx * dx;
        }
    float *ob = fa.img_out + (int64_t)b * fa.out_bstride + (int64_t)4 * x;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const int y = yb0 + i;
        if (!FAST && y >= h) break;  // wave-uniform
        const int Y = 4 * y + g;
        float sy = ((float)Y + 0.5f) * 0.25f - 0.5f;
        sy = fminf(fmaxf(sy, 0.0f), (float)(h - 1));
        const float f0 = floorf(sy);
        const int ya_ = (int)f0, yb_ = ya_ + 1 < h ? ya_ + 1 : h - 1;
        const float wy = sy - f0;
        bool keep[4] = {true, true, true, true};
        if (!FAST && fa.gv) {
            const double dy = ((double)Y + 0.5) - gy, dy2 = dy * dy, rm2 = fa.rm * fa.rm;
#pragma unroll
            for (int r = 0; r < 4; ++r) keep[r] = dx2[r] + dy2 > rm2;
        }
        const bool all = keep[0] && keep[1] && keep[2] && keep[3];
        // vertical interpolation in the three columns
        const float4 *fa_ = F + (ya_ - fy0) * kFxCols, *fb_ = F + (yb_ - fy0) * kFxCols;
        const float4 ta[3] = {fa_[cl], fa_[cm], fa_[cr]}, tb[3] = {fb_[cl], fb_[cm], fb_[cr]};
        float v[3][3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            v[k][0] = (1.0f - wy) * ta[k].x + wy * tb[k].x;
            v[k][1] = (1.0f - wy) * ta[k].y + wy * tb[k].y;
            v[k][2] = (1.0f - wy) * ta[k].z + wy * tb[k].z;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float vlo_a = left ? v[0][c] : v[1][c], vlo_b = left ? v[1][c] : v[2][c];
            float o[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float va = r < 2 ? vlo_a : v[1][c], vb = r < 2 ? vlo_b : v[2][c];
                const int ch = c * 16 + 4 * g + r;
                o[r] = (acc[i][c][r] + b3[ch]) + ((1.0f - wx[r]) * va + wx[r] * vb);
            }
            float *dst = ob + c * oplane + (int64_t)Y * (4 * w);
            if (FAST) {
                *reinterpret_cast<float4 *>(dst) = float4{o[0], o[1], o[2], o[3]};
            } else if (vec_out && all) {
                *reinterpret_cast<float4 *>(dst) = float4{o[0], o[1], o[2], o[3]};
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (keep[r]) dst[r] = o[r];
            }
        }
    }
}

// frame mode: true when every output pixel of the whole tile at (x0, y0) lies
// outside r_mid (its rectangle's nearest point to the gaze does, with a
// relative margin that keeps rounding on the safe side); always true otherwise
__device__ __forceinline__ bool fx_tile_outside(const NetFusedArgs &a, int x0, int y0, double gx, double gy) {
    if (!a.gv) return true;
    const double xa = 4.0 * x0, xb = 4.0 * (x0 + kFxTX), ya = 4.0 * y0, yb = 4.0 * (y0 + kFxTY);
    const double dx = gx < xa ? xa - gx : (gx > xb ? gx - xb : 0.0);
    const double dy = gy < ya ? ya - gy : (gy > yb ? gy - yb : 0.0);
    return dx * dx + dy * dy > a.rm * a.rm * (1.0 + 1e-12);
}

// Block barrier that orders LDS only: the output stores and the next tile's
// input loads stay in flight across it (a plain __syncthreads would wait for
// them, serialising each tile's stores with the next tile's products).
__device__ __forceinline__ void fx_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__global__ void __launch_bounds__(kFxThreads) k_net_fused(NetFusedArgs fa) {
    __shared__ __attribute__((aligned(16))) uint8_t sm[kFxBytes];
    const int h = fa.h, w = fa.w;
    const int tiles_x = (w + kFxTX - 1) / kFxTX, tiles_y = (h + kFxTY - 1) / kFxTY;
    const int64_t ntiles = (int64_t)fa.B * tiles_x * tiles_y;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, g = lane >> 4;
    const int cb = 16 * (wave & 3), grp = wave >> 2;  // this wave's chunk and row group
    // the last layer's chunks end at the tile's edge: 0, 16, 32, 44 (pixels 44 .. 47 are
    // computed by two waves, with the same operands, and stored twice with the same bits)
    const int cb3 = min(cb, kFxTX - 16);
    uint64_t *mask = reinterpret_cast<uint64_t *>(sm + kFxMask);
    uint32_t *rank = reinterpret_cast<uint32_t *>(sm + kFxRank);

    // ---- the tiles this block takes: every G-th of the list, G = gridDim.x.  In
    // frame mode with at most 64 x kFxMaskWords tiles the list holds only the
    // tiles with periphery pixels (ranked once per block), so that blocks get
    // equal shares; otherwise it is every tile (inside ones are then skipped).
    const bool ranked = fa.gv && ntiles <= 64 * kFxMaskWords;
    int64_t nlist = ntiles;
    if (ranked) {
        for (int t0 = 0; t0 < ntiles; t0 += kFxThreads) {
            const int t = t0 + tid;
            const bool real = t < ntiles && !fx_tile_inside(fa, fx_tile(t, tiles_x, tiles_y));
            const uint64_t bal = __ballot(real);
            if (lane == 0) mask[(t0 >> 6) + wave] = bal;
        }
        fx_sync();
        if (tid == 0) {
            uint32_t acc = 0;
            const int nw = (int)((ntiles + 63) >> 6);
            for (int k = 0; k < nw; ++k) {
                rank[k] = acc;
                acc += (uint32_t)__popcll(mask[k]);
            }
            rank[nw] = acc;
        }
        fx_sync();
        nlist = rank[(ntiles + 63) >> 6];
    }
    // list entry -> tile index
    auto tile_of = [&](int64_t e) -> int64_t {
        if (!ranked) return e;
        int k = 0;
        while (rank[k + 1] <= (uint32_t)e) ++k;
        uint64_t m = mask[k];
        for (uint32_t n = (uint32_t)e - rank[k]; n > 0; --n) m &= m - 1;  // drop the lower set bits
        return (int64_t)k * 64 + __builtin_ctzll(m);
    };
    if ((int64_t)blockIdx.x >= nlist) return;  // block-uniform

    // ---- weights (rounded to bf16 here, as net_pack_item does) and biases, once per block
    {
        const float *th = fa.theta;
        // conv1 [co][c][tap] -> W1 rows [tap][co] of 8 channels (3 real); taps 9 .. 11 zero
        for (int rw = tid; rw < 12 * 32; rw += kFxThreads) {
            const int tap = rw / 32, co = rw % 32;
            uint4 v = {0u, 0u, 0u, 0u};
            if (tap < 9) {
                v.x = bf16_bits(th[kNetW1 + (co * 3 + 0) * 9 + tap]) |
                      ((uint32_t)bf16_bits(th[kNetW1 + (co * 3 + 1) * 9 + tap]) << 16);
                v.y = bf16_bits(th[kNetW1 + (co * 3 + 2) * 9 + tap]);
            }
            *reinterpret_cast<uint4 *>(sm + kFxW1 + rw * 16) = v;
        }
        // conv2 [co][ci][tap], conv3 [co][ci][tap] -> rows [tap][co] of 32 channels: every
        // load issued first (read in order), then rounded and scattered
        constexpr int N2 = 32 * 32 * 9 / kFxThreads, N3 = 48 * 32 * 9 / kFxThreads;
        static_assert(N2 * kFxThreads == 32 * 32 * 9 && N3 * kFxThreads == 48 * 32 * 9, "whole rounds");
        float v2[N2], v3[N3];
#pragma unroll
        for (int m = 0; m < N2; ++m) v2[m] = th[kNetW2 + tid + m * kFxThreads];
#pragma unroll
        for (int m = 0; m < N3; ++m) v3[m] = th[kNetW3 + tid + m * kFxThreads];
#pragma unroll
        for (int m = 0; m < N2; ++m) {
            const int k = tid + m * kFxThreads, tap = k % 9, ci = (k / 9) % 32, co = k / 288;
            *reinterpret_cast<uint16_t *>(sm + kFxW2 + fx_wr(tap * 32 + co, ci >> 3) + (ci & 7) * 2) = bf16_bits(v2[m]);
        }
#pragma unroll
        for (int m = 0; m < N3; ++m) {
            const int k = tid + m * kFxThreads, tap = k % 9, ci = (k / 9) % 32, co = k / 288;
            *reinterpret_cast<uint16_t *>(sm + kFxW3 + fx_wr(tap * 48 + co, ci >> 3) + (ci & 7) * 2) = bf16_bits(v3[m]);
        }
    }
    float *sb = reinterpret_cast<float *>(sm + kFxBias);
    if (tid < 112) sb[tid] = fa.theta[tid < 32 ? kNetB1 + tid : (tid < 64 ? kNetB2 + tid - 32 : kNetB3 + tid - 64)];
    float4 *F = reinterpret_cast<float4 *>(sm + kFxF32);

    // ---- per-lane addresses, the same for every tile
    const int r1 = grp * kFxR1, r2 = grp * kFxR2, r3 = grp * kFxR3;
    const uint8_t *a1[3], *a2[3], *a3[3];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const int tap = min(4 * s + g, 8);  // taps 9 .. 11: any valid pixel (its products are zeroed)
        a1[s] = sm + kFxL0 + ((r1 + tap / 3) * kFxCols + cb + li + tap % 3) * 16;
        a2[s] = sm + kFxL1 + fx_px(r2, cb + li + s, g);
        a3[s] = sm + kFxL2 + fx_px(r3, cb3 + li + s, g);
    }
    const bool ok1 = g == 0;  // the lane's K entries of conv1's last step are real (tap 8)
    const uint8_t *w1 = sm + kFxW1 + (g * 32 + li) * 16;
    const uint8_t *w2 = sm + kFxW2 + fx_wr(li, g), *w3 = sm + kFxW3 + fx_wr(li, g);
    uint8_t *d1[2], *d2[2];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
        const int j = 2 * nb + (g >> 1), sub = (g & 1) * 8;
        d1[nb] = sm + kFxL1 + fx_px(r1, cb + li, j) + sub;
        d2[nb] = sm + kFxL2 + fx_px(r2, cb + li, j) + sub;
    }
    float bias1[2][4], bias2[2][4];
    fx_sync();
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            bias1[nb][r] = sb[nb * 16 + 4 * g + r];
            bias2[nb][r] = sb[32 + nb * 16 + 4 * g + r];
        }
    const int64_t oplane = (int64_t)(4 * h) * (4 * w);
    const bool vec_out = (reinterpret_cast<uintptr_t>(fa.img_out) & 15) == 0 && (fa.out_bstride & 3) == 0;

    float pre[kFxInPer][3];
    FxTile cur = fx_tile(tile_of(blockIdx.x), tiles_x, tiles_y);
    fx_fetch(fa, cur, tid, pre);
    for (int64_t e = blockIdx.x; e < nlist; e += gridDim.x) {
        const FxTile t = cur;
        const bool skip_tile = !ranked && fx_tile_inside(fa, t);  // block-uniform
        double gx = 0.0, gy = 0.0;
        if (fa.gv) {
            gx = fa.gv[(int64_t)t.b * fa.gv_stride].v.gx;
            gy = fa.gv[(int64_t)t.b * fa.gv_stride].v.gy;
        }
        const int x0 = t.x0, y0 = t.y0;
        const int xend = min(x0 + kFxTX, w);
        // ---- the tile's input: bf16 NHWC8 (L0) and float32 planar (F)
#pragma unroll
        for (int k = 0; k < kFxInPer; ++k) {
            const int q = tid + k * kFxThreads;
            if (q < kFxIn) {
                uint4 pk;
                pk.x = bf16_bits(pre[k][0]) | ((uint32_t)bf16_bits(pre[k][1]) << 16);
                pk.y = bf16_bits(pre[k][2]);
                pk.z = pk.w = 0u;
                *reinterpret_cast<uint4 *>(sm + kFxL0 + q * 16) = pk;
                F[q] = float4{pre[k][0], pre[k][1], pre[k][2], 0.0f};
            }
        }
        fx_sync();
        // the next tile's input is fetched while this one computes
        if (e + gridDim.x < nlist) {
            cur = fx_tile(tile_of(e + gridDim.x), tiles_x, tiles_y);
            fx_fetch(fa, cur, tid, pre);
        }
        // ---- conv1: L1 rows r1 .. r1 + kFxR1 - 1 (image (y0 - 2, x0 - 2) at L1 (0, 0)); L0 row R + 1 + dy
        if (!skip_tile) {
            const int ya = y0 - 2 + r1, xa = x0 - 2 + cb;
            if (!(fa.gv && inside_mid(max(xa - 2, 0), min(xa + 17, w - 1), max(ya - 2, 0), min(ya + kFxR1 + 1, h - 1),
                                      gx, gy, fa.rm))) {  // wave-uniform
                floatx4 acc[kFxR1][2];
                fx_conv<kFxR1, 2, true>(a1, w1, ok1, acc);
                uint32_t rowin = 0;
#pragma unroll
                for (int i = 0; i < kFxR1; ++i) rowin |= (ya + i >= 0 && ya + i < h) ? 1u << i : 0u;
                const int x = xa + li;
                fx_hidden_store<kFxR1>(d1, acc, bias1, rowin, x >= 0 && x < w);
            }
        }
        fx_sync();
        // ---- conv2: L2 rows r2 .. (image (y0 - 1, x0 - 1) at L2 (0, 0)); L1 row R + 1 + dy
        if (!skip_tile) {
            const int ya = y0 - 1 + r2, xa = x0 - 1 + cb;
            if (!(fa.gv && inside_mid(max(xa - 1, 0), min(xa + 16, w - 1), max(ya - 1, 0), min(ya + kFxR2, h - 1), gx,
                                      gy, fa.rm))) {
                floatx4 acc[kFxR2][2];
                fx_conv<kFxR2, 2, false>(a2, w2, true, acc);
                uint32_t rowin = 0;
#pragma unroll
                for (int i = 0; i < kFxR2; ++i) rowin |= (ya + i >= 0 && ya + i < h) ? 1u << i : 0u;
                const int x = xa + li;
                fx_hidden_store<kFxR2>(d2, acc, bias2, rowin, x >= 0 && x < w);
            }
        }
        fx_sync();
        // ---- conv3 + pixel shuffle + bilinear residual: output rows y0 + r3 ..; L2 row R + 1 + dy
        if (!skip_tile) {
            const int yb0 = y0 + r3, xs = x0 + cb3;
            if (yb0 < h && xs < xend &&
                !(fa.gv && inside_mid(xs, min(xs + 15, w - 1), yb0, min(yb0 + kFxR3 - 1, h - 1), gx, gy, fa.rm))) {
                floatx4 acc[kFxR3][3];
                fx_conv<kFxR3, 3, false>(a3, w3, true, acc);
                // whole tiles whose every output pixel the composite takes: no checks per row or pixel
                if (vec_out && x0 + kFxTX <= w && y0 + kFxTY <= h && fx_tile_outside(fa, x0, y0, gx, gy))
                    fx_last_epilogue<true, kFxR3>(fa, acc, F, sb + 64, t.b, x0, y0, yb0, xs, xend, li, g, oplane, true,
                                                  gx, gy);
                else
                    fx_last_epilogue<false, kFxR3>(fa, acc, F, sb + 64, t.b, x0, y0, yb0, xs, xend, li, g, oplane,
                                                   vec_out, gx, gy);
            }
        }
        fx_sync();  // L0 / F are rewritten by the next tile
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

constexpr int64_t kNetFusedBlocks = 256;

void launch_net_fused(const NetFusedArgs &a_in, hipStream_t s) {
    NetFusedArgs a = a_in;
    if (a.img_bstride == 0) a.img_bstride = 3 * (int64_t)a.h * a.w;
    if (a.out_bstride == 0) a.out_bstride = 3 * (int64_t)(4 * a.h) * (4 * a.w);
    const int64_t tiles = (int64_t)a.B * ((a.h + kFxTY - 1) / kFxTY) * ((a.w + kFxTX - 1) / kFxTX);
    // resident blocks, one per compute unit (the tile's LDS fills most of one)
    hipLaunchKernelGGL(k_net_fused, dim3((unsigned)std::min<int64_t>(tiles, kNetFusedBlocks)), dim3(kFxThreads), 0, s,
                       a);
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
