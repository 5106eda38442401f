// Learned coarse-grid corrector: a 4-layer 3x3 convolutional network with circular
// padding, trained and evaluated by hand-written BF16 MFMA kernels with FP32
// accumulation, plus the kernels that connect it to the solver (block-mean
// coarsening of a fine state, input features, training residuals, and adding the
// predicted correction to a coarse state).
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16, in persistent
// workgroups that walk tiles of a few rows x 32 (or 64) pixels staged in LDS:
//   forward        M = 16 output channels, N = 16 pixels of one row, K = 9 taps x C_in;
//                  the weights stay in LDS for all tiles of a workgroup (read from the
//                  float32 master parameters and rounded to bf16 as they are staged)
//   fused pair     (inference) layers 1 and 2 in one pass, layer 1's output on the tile
//                  and its one-pixel ring kept in LDS; layer 1 reads the float32 features
//   backward-data  the forward kernel on dY with the weights flipped in the taps and
//                  transposed in the channels, times the ReLU mask of the layer input
//   backward-weight M = output channels, N = 9 taps x C_in, K = pixels: dY^T and three
//                  x-shifted copies of X^T per tile in LDS; each workgroup accumulates
//                  over its tiles and writes one set of partial sums, summed in a
//                  fixed order.
// Activations are NHWC bf16 with channels padded to a multiple of 8 (input) or 16
// (output); weights are [c_out][K] with k = tap * C_in + c_in, tap = (dy+1)*3 + (dx+1),
// K padded with zeros to a multiple of 32.
#include <math.h>
#include <string.h>

#include <new>

#include "runtime.h"

namespace phx {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

constexpr int NLAYERS = 4;

__device__ __forceinline__ u16 bf16_bits(float f)
{
    __bf16 b = (__bf16)f;  // round to nearest even
    return __builtin_bit_cast(u16, b);
}
__device__ __forceinline__ float bf16_value(u16 u) { return __builtin_bit_cast(float, (unsigned int)u << 16); }

struct LayerDims {
    int cin, cout;    // real channels
    int cinp, coutp;  // padded: multiple of 8 / 16
    int kp;           // padded K = ceil(9 cinp / 32) * 32
};

static LayerDims layer_dims(int cin, int cout)
{
    LayerDims d;
    d.cin = cin;
    d.cout = cout;
    d.cinp = (cin + 7) / 8 * 8;
    d.coutp = (cout + 15) / 16 * 16;
    d.kp = (9 * d.cinp + 31) / 32 * 32;
    return d;
}

// ------------------------------------------------------------------ conv forward

enum ConvMode { CONV_RELU_BF16 = 0, CONV_LINEAR_F32 = 1, CONV_MASK_BF16 = 2 };

// Tiled forward convolution, persistent over tiles.  A workgroup of 4 waves keeps the
// bf16 weights in LDS for all its tiles; a tile is TR rows x TW = 16*MT pixels of one
// image, staged in LDS with a one-pixel circular halo.  Wave w computes rows w, w + 4,
// ... of the tile as MT x NT MFMA blocks with the weights as operand A (16 output
// channels x 32 k) and the input as operand B (32 k x 16 pixels), so each lane's
// accumulator holds 4 consecutive output channels of one pixel and stores them with
// one write.  Taller tiles stage fewer halo rows per output row.
// in: [P][CINP] bf16, w: [COUTP][KP] bf16 or (WT = float) the
// float32 master weights, rounded to bf16 in LDS (zero beyond 9*CINP), bias: [COUTP] f32.
// MODE: CONV_RELU_BF16 -> out_bf16[P][COUTP] = relu(acc + bias)
//       CONV_LINEAR_F32 -> out_f32[P][out_stride], channels < out_stride, acc + bias
//       CONV_MASK_BF16 -> out_bf16[P][COUTP] = acc if mask[P][COUTP] > 0 else 0
// Requires W % TW == 0.
// The 16-byte chunks of one staged input tile (TR + 2 rows of TW + 2 pixels with the
// circular halo, CINP channels) that this thread moves: chunk threadIdx.x + 256 k.
// XCD-aware tile order (tile t = xcd_tile(v)): each XCD walks a contiguous band of
// tiles, so the halo rows shared by vertically adjacent tiles are read through one L2.
typedef unsigned int chunk16 __attribute__((ext_vector_type(4)));  // 16 bytes of a staged tile

__device__ __forceinline__ unsigned int bf16_pair(float lo, float hi)
{
    return bf16_bits(lo) | ((unsigned int)bf16_bits(hi) << 16);
}

template <int CINP, int TR, int TW, int NPER>
__device__ __forceinline__ void conv_fetch_tile(chunk16 (&stage)[NPER], const u16* __restrict__ in, int t, int H,
                                                int W, int tx_n, int ty_n)
{
    constexpr int C8 = CINP / 8, NE = (TR + 2) * (TW + 2) * C8;
    const int img = t / (ty_n * tx_n);
    const int rt = t - img * (ty_n * tx_n);
    const int y0 = (rt / tx_n) * TR, x0 = (rt - (rt / tx_n) * tx_n) * TW;
#pragma unroll
    for (int k = 0; k < NPER; ++k) {
        const int e = threadIdx.x + 256 * k;
        if (e < NE) {
            const int c8 = e % C8, pix = e / C8;
            const int r = pix / (TW + 2), c = pix - (pix / (TW + 2)) * (TW + 2);
            int yy = y0 - 1 + r, xx = x0 - 1 + c;
            if (yy < 0) yy += H;
            if (yy >= H) yy %= H;
            xx += (xx < 0) ? W : (xx >= W ? -W : 0);
            stage[k] = *(const chunk16*)&in[((size_t)(img * H + yy) * W + xx) * CINP + 8 * c8];
        }
    }
}

template <int CINP, int COUTP, int MODE, int MT, int TR, typename WT>
__global__ __launch_bounds__(256) void conv_fwd_kernel(const u16* __restrict__ in, const WT* __restrict__ w,
                                                       const float* __restrict__ bias, int H, int W, int images,
                                                       u16* __restrict__ out_bf16, float* __restrict__ out_f32,
                                                       int out_stride, const u16* __restrict__ mask)
{
    static_assert(TR % 4 == 0, "4 waves share the tile's rows");
    constexpr int KP = (9 * CINP + 31) / 32 * 32;
    constexpr int NT = COUTP / 16;
    constexpr int TW = 16 * MT, RW = TR / 4;  // rows per wave
    // LDS elements per staged pixel and per weight row: padding by 16 keeps the 16-byte
    // operand reads of a 16-pixel run almost free of bank conflicts (0.7 conflict cycles
    // per LDS instruction against 4.3 with 8); the 16-channel output layer keeps 8, so
    // that 4 workgroups still fit per CU.
    constexpr int PAD = COUTP >= 32 ? 16 : 8;
    constexpr int CS = CINP + PAD;
    constexpr int WS = KP + PAD;
    constexpr int C8 = CINP / 8;  // 16-byte chunks per pixel
    __shared__ __attribute__((aligned(16))) u16 sw[COUTP * WS];
    __shared__ __attribute__((aligned(16))) u16 sx[(TR + 2) * (TW + 2) * CS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, g = lane >> 4;
    for (int e = threadIdx.x; e < COUTP * (KP / 8); e += 256) {
        const int o = e / (KP / 8), k8 = e - o * (KP / 8);
        if constexpr (sizeof(WT) == 4) {
            const float4 lo = *(const float4*)&w[(size_t)o * KP + 8 * k8];
            const float4 hi = *(const float4*)&w[(size_t)o * KP + 8 * k8 + 4];
            *(uint4*)&sw[o * WS + 8 * k8] =
                uint4{bf16_pair(lo.x, lo.y), bf16_pair(lo.z, lo.w), bf16_pair(hi.x, hi.y), bf16_pair(hi.z, hi.w)};
        } else {
            *(uint4*)&sw[o * WS + 8 * k8] = *(const uint4*)&w[(size_t)o * KP + 8 * k8];
        }
    }
    const int tx_n = W / TW, ty_n = (H + TR - 1) / TR;
    const int tiles = images * ty_n * tx_n;
    // The next tile's input is loaded into registers while the current one is
    // computed, then written to LDS after the barrier that ends the current tile's
    // reads.
    constexpr int NE = (TR + 2) * (TW + 2) * C8;  // 16-byte chunks of a staged tile
    constexpr int NPER = (NE + 255) / 256;
    chunk16 stage[NPER];
    // (the last tile of a workgroup fetches its own tile again: no branch around the loads)
    if ((int)blockIdx.x < tiles)
        conv_fetch_tile<CINP, TR, TW, NPER>(stage, in, xcd_tile(blockIdx.x, tiles), H, W, tx_n, ty_n);
    for (int v = blockIdx.x; v < tiles; v += gridDim.x) {
        const int t = xcd_tile(v, tiles);
        const int img = t / (ty_n * tx_n);
        const int rt = t - img * (ty_n * tx_n);
        const int y0 = (rt / tx_n) * TR, x0 = (rt - (rt / tx_n) * tx_n) * TW;
        __syncthreads();  // the previous tile's reads of sx are done
#pragma unroll
        for (int k = 0; k < NPER; ++k) {
            const int e = threadIdx.x + 256 * k;
            if (e < NE) *(chunk16*)&sx[(e / C8) * CS + 8 * (e % C8)] = stage[k];
        }
        __syncthreads();
        const int vn = v + (int)gridDim.x < tiles ? v + (int)gridDim.x : v;
        conv_fetch_tile<CINP, TR, TW, NPER>(stage, in, xcd_tile(vn, tiles), H, W, tx_n, ty_n);
        f32x4 acc[RW][MT][NT];
#pragma unroll
        for (int rr = 0; rr < RW; ++rr)
#pragma unroll
            for (int i = 0; i < MT; ++i)
#pragma unroll
                for (int j = 0; j < NT; ++j) acc[rr][i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < KP / 32; ++c) {
            const int k0 = 32 * c + 8 * g;
            const int tap = k0 / CINP, ci = k0 - (k0 / CINP) * CINP;
            bf16x8 a[NT];
#pragma unroll
            for (int j = 0; j < NT; ++j) a[j] = *(const bf16x8*)&sw[(j * 16 + m) * WS + k0];
            const int dy = tap / 3, dx = tap - (tap / 3) * 3;  // offsets into the halo tile
#pragma unroll
            for (int rr = 0; rr < RW; ++rr)
#pragma unroll
                for (int i = 0; i < MT; ++i) {
                    bf16x8 b = bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
                    if (tap < 9) b = *(const bf16x8*)&sx[((wave + 4 * rr + dy) * (TW + 2) + i * 16 + m + dx) * CS + ci];
#pragma unroll
                    for (int j = 0; j < NT; ++j)
                        acc[rr][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[j], b, acc[rr][i][j], 0, 0, 0);
                }
        }
        // lane holds C[4g + r][m]: channel j*16 + 4g + r of pixel (y0 + wave + 4 rr, x0 + i*16 + m)
#pragma unroll
        for (int rr = 0; rr < RW; ++rr) {
            const int yrow = y0 + wave + 4 * rr;
            if (yrow >= H) continue;
#pragma unroll
            for (int i = 0; i < MT; ++i) {
                const size_t q = (size_t)(img * H + yrow) * W + x0 + i * 16 + m;
#pragma unroll
                for (int j = 0; j < NT; ++j) {
                    const int c0 = j * 16 + 4 * g;
                    if (MODE == CONV_RELU_BF16) {
                        u16 o[4];
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const float v = acc[rr][i][j][r] + bias[c0 + r];
                            o[r] = bf16_bits(v > 0.f ? v : 0.f);
                        }
                        *(uint2*)&out_bf16[q * COUTP + c0] =
                            uint2{o[0] | ((unsigned int)o[1] << 16), o[2] | ((unsigned int)o[3] << 16)};
                    } else if (MODE == CONV_LINEAR_F32) {
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            if (c0 + r < out_stride) out_f32[q * out_stride + c0 + r] = acc[rr][i][j][r] + bias[c0 + r];
                    } else {
                        const uint2 mk = *(const uint2*)&mask[q * COUTP + c0];
                        const u16 mv[4] = {(u16)(mk.x & 0xffffu), (u16)(mk.x >> 16), (u16)(mk.y & 0xffffu),
                                           (u16)(mk.y >> 16)};
                        u16 o[4];
#pragma unroll
                        for (int r = 0; r < 4; ++r) o[r] = bf16_bits(bf16_value(mv[r]) > 0.f ? acc[rr][i][j][r] : 0.f);
                        *(uint2*)&out_bf16[q * COUTP + c0] =
                            uint2{o[0] | ((unsigned int)o[1] << 16), o[2] | ((unsigned int)o[3] << 16)};
                    }
                }
            }
        }
    }
}

// ------------------------------------------------------ fused layer pairs

// Two consecutive layers in one pass, for inference: layer A (CINP -> 32, ReLU, bf16)
// is evaluated on the tile and a one-pixel ring around it into LDS, and layer B
// (32 -> COUTP, MODE as in conv_fwd_kernel) reads it there, so the 32-channel
// activation between the two never goes through HBM.  A tile is 8 rows x 32 pixels of
// one image and a workgroup has 8 waves, one output row of layer B each.  The input is
// staged with a two-pixel circular ring (12 x 36 pixels); layer A's 10 x 34 pixels are
// taken as 22 runs of 16 consecutive pixels of that region in row-major order (the
// last run 12 pixels short), runs w, w + 8, w + 16 on wave w.  Every output element
// is accumulated over the same K order as in the one-layer kernel, so the results are
// the same bits.  Weights: the float32 master copies, rounded to bf16 in LDS.
// XF32: the input is float32 with 4 channels per pixel (CINP = 8).
constexpr int PAIR_R = 8, PAIR_W = 32, PAIR_THREADS = 512;

template <int CINP, int NPER, bool XF32>
__device__ __forceinline__ void pair_fetch_tile(chunk16 (&stage)[NPER], const void* __restrict__ in, int t, int H,
                                                int W, int tx_n, int ty_n)
{
    static_assert(!XF32 || CINP == 8, "float32 input: 4 channels padded to 8");
    constexpr int XR = PAIR_R + 4, XW = PAIR_W + 4, C8 = CINP / 8, NE = XR * XW * C8;
    const int img = t / (ty_n * tx_n);
    const int rt = t - img * (ty_n * tx_n);
    const int y0 = (rt / tx_n) * PAIR_R, x0 = (rt - (rt / tx_n) * tx_n) * PAIR_W;
#pragma unroll
    for (int k = 0; k < NPER; ++k) {
        const int e = threadIdx.x + PAIR_THREADS * k;
        if (e < NE) {
            const int c8 = e % C8, pix = e / C8;
            const int r = pix / XW, c = pix - (pix / XW) * XW;
            int yy = (y0 - 2 + r) % H;  // the grid may have fewer rows than the ring
            if (yy < 0) yy += H;
            int xx = x0 - 2 + c;  // W >= 32: one wrap at most
            xx += (xx < 0) ? W : (xx >= W ? -W : 0);
            const size_t p = (size_t)(img * H + yy) * W + xx;
            if (XF32) {
                const float4 v = ((const float4*)in)[p];
                stage[k] = chunk16{bf16_pair(v.x, v.y), bf16_pair(v.z, v.w), 0u, 0u};
            } else {
                stage[k] = *(const chunk16*)&((const u16*)in)[p * CINP + 8 * c8];
            }
        }
    }
}

template <int COUTP, int KP, int WS>
__device__ __forceinline__ void stage_weights(u16* sw, const float* __restrict__ w)
{
    for (int e = threadIdx.x; e < COUTP * (KP / 8); e += PAIR_THREADS) {
        const int o = e / (KP / 8), k8 = e - o * (KP / 8);
        const float4 lo = *(const float4*)&w[(size_t)o * KP + 8 * k8];
        const float4 hi = *(const float4*)&w[(size_t)o * KP + 8 * k8 + 4];
        *(uint4*)&sw[o * WS + 8 * k8] =
            uint4{bf16_pair(lo.x, lo.y), bf16_pair(lo.z, lo.w), bf16_pair(hi.x, hi.y), bf16_pair(hi.z, hi.w)};
    }
}

template <int CINP, int COUTP, int MODE, bool XF32>
__global__ __launch_bounds__(PAIR_THREADS) void conv_pair_kernel(const void* __restrict__ in,
                                                                 const float* __restrict__ wa,
                                                                 const float* __restrict__ ba,
                                                                 const float* __restrict__ wb,
                                                                 const float* __restrict__ bb, int H, int W, int images,
                                                                 u16* __restrict__ out_bf16, float* __restrict__ out_f32,
                                                                 int out_stride)
{
    static_assert(MODE == CONV_RELU_BF16 || MODE == CONV_LINEAR_F32, "forward modes only");
    constexpr int XR = PAIR_R + 4, XW = PAIR_W + 4;  // staged input
    constexpr int EW = PAIR_W + 2;                   // layer A's region: (PAIR_R + 2) x EW
    constexpr int EP = (PAIR_R + 2) * EW;            // 340 pixels
    constexpr int ENT = (EP + 15) / 16;              // 22 runs
    constexpr int KPA = (9 * CINP + 31) / 32 * 32, KPB = 9 * 32;
    constexpr int NTB = COUTP / 16, MT = PAIR_W / 16;
    // LDS elements per pixel and per weight row, padded by 16 against bank conflicts
    // (1.4 conflict cycles per LDS instruction against 4.2 with 8: 10 % faster)
    constexpr int CS0 = CINP + 16, CS1 = 32 + 16;
    constexpr int WSA = KPA + 16, WSB = KPB + 16;
    constexpr int C8 = CINP / 8;
    constexpr int NE = XR * XW * C8, NPER = (NE + PAIR_THREADS - 1) / PAIR_THREADS;
    constexpr int RUNS = (ENT + 7) / 8;  // runs of layer A per wave
    __shared__ __attribute__((aligned(16))) u16 swa[32 * WSA];
    __shared__ __attribute__((aligned(16))) u16 swb[COUTP * WSB];
    __shared__ __attribute__((aligned(16))) u16 sx0[XR * XW * CS0];
    __shared__ __attribute__((aligned(16))) u16 sx1[EP * CS1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, g = lane >> 4;
    stage_weights<32, KPA, WSA>(swa, wa);
    stage_weights<COUTP, KPB, WSB>(swb, wb);
    const int tx_n = W / PAIR_W, ty_n = (H + PAIR_R - 1) / PAIR_R;
    const int tiles = images * ty_n * tx_n;
    chunk16 stage[NPER];
    if ((int)blockIdx.x < tiles)
        pair_fetch_tile<CINP, NPER, XF32>(stage, in, xcd_tile(blockIdx.x, tiles), H, W, tx_n, ty_n);
    for (int v = blockIdx.x; v < tiles; v += gridDim.x) {
        const int t = xcd_tile(v, tiles);
        const int img = t / (ty_n * tx_n);
        const int rt = t - img * (ty_n * tx_n);
        const int y0 = (rt / tx_n) * PAIR_R, x0 = (rt - (rt / tx_n) * tx_n) * PAIR_W;
        __syncthreads();  // the previous tile's reads of sx0 and sx1 are done
#pragma unroll
        for (int k = 0; k < NPER; ++k) {
            const int e = threadIdx.x + PAIR_THREADS * k;
            if (e < NE) *(chunk16*)&sx0[(e / C8) * CS0 + 8 * (e % C8)] = stage[k];
        }
        __syncthreads();
        const int vn = v + (int)gridDim.x < tiles ? v + (int)gridDim.x : v;
        pair_fetch_tile<CINP, NPER, XF32>(stage, in, xcd_tile(vn, tiles), H, W, tx_n, ty_n);

        // layer A on the 10 x 34 region: run q covers region pixels 16 q .. 16 q + 15
        {
            f32x4 acc[RUNS][2];
            int base[RUNS];  // the lane's pixel, as an offset of its top-left tap in sx0
#pragma unroll
            for (int u = 0; u < RUNS; ++u) {
                const int q = wave + 8 * u;
                const int p = q < ENT ? (16 * q + m < EP ? 16 * q + m : EP - 1) : 0;
                const int er = p / EW, ec = p - (p / EW) * EW;
                base[u] = er * XW + ec;
                acc[u][0] = acc[u][1] = f32x4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
            for (int c = 0; c < KPA / 32; ++c) {
                const int k0 = 32 * c + 8 * g;
                const int tap = k0 / CINP, ci = k0 - (k0 / CINP) * CINP;
                const int dy = tap / 3, dx = tap - (tap / 3) * 3;
                bf16x8 a[2];
#pragma unroll
                for (int j = 0; j < 2; ++j) a[j] = *(const bf16x8*)&swa[(j * 16 + m) * WSA + k0];
#pragma unroll
                for (int u = 0; u < RUNS; ++u) {
                    if (wave + 8 * u < ENT) {  // uniform over the wave
                        bf16x8 b = bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
                        if (tap < 9) b = *(const bf16x8*)&sx0[(base[u] + dy * XW + dx) * CS0 + ci];
#pragma unroll
                        for (int j = 0; j < 2; ++j)
                            acc[u][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[j], b, acc[u][j], 0, 0, 0);
                    }
                }
            }
            // lane holds C[4g + r][m]: channel j*16 + 4g + r of region pixel 16 q + m
#pragma unroll
            for (int u = 0; u < RUNS; ++u) {
                const int p = 16 * (wave + 8 * u) + m;
                if (wave + 8 * u < ENT && p < EP) {
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        const int c0 = j * 16 + 4 * g;
                        u16 o[4];
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const float x = acc[u][j][r] + ba[c0 + r];
                            o[r] = bf16_bits(x > 0.f ? x : 0.f);
                        }
                        *(uint2*)&sx1[p * CS1 + c0] =
                            uint2{o[0] | ((unsigned int)o[1] << 16), o[2] | ((unsigned int)o[3] << 16)};
                    }
                }
            }
        }
        __syncthreads();  // layer A's region is complete

        // layer B: wave w computes output row w from region rows w .. w + 2
        f32x4 acc[MT][NTB];
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
            for (int j = 0; j < NTB; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < KPB / 32; ++c) {
            const int k0 = 32 * c + 8 * g;
            const int tap = k0 / 32, ci = k0 - (k0 / 32) * 32;
            const int dy = tap / 3, dx = tap - (tap / 3) * 3;
            bf16x8 a[NTB];
#pragma unroll
            for (int j = 0; j < NTB; ++j) a[j] = *(const bf16x8*)&swb[(j * 16 + m) * WSB + k0];
#pragma unroll
            for (int i = 0; i < MT; ++i) {
                const bf16x8 b = *(const bf16x8*)&sx1[((wave + dy) * EW + i * 16 + m + dx) * CS1 + ci];
#pragma unroll
                for (int j = 0; j < NTB; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[j], b, acc[i][j], 0, 0, 0);
            }
        }
        const int yrow = y0 + wave;
        if (yrow < H) {
#pragma unroll
            for (int i = 0; i < MT; ++i) {
                const size_t q = (size_t)(img * H + yrow) * W + x0 + i * 16 + m;
#pragma unroll
                for (int j = 0; j < NTB; ++j) {
                    const int c0 = j * 16 + 4 * g;
                    if (MODE == CONV_RELU_BF16) {
                        u16 o[4];
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const float x = acc[i][j][r] + bb[c0 + r];
                            o[r] = bf16_bits(x > 0.f ? x : 0.f);
                        }
                        *(uint2*)&out_bf16[q * COUTP + c0] =
                            uint2{o[0] | ((unsigned int)o[1] << 16), o[2] | ((unsigned int)o[3] << 16)};
                    } else {
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            if (c0 + r < out_stride) out_f32[q * out_stride + c0 + r] = acc[i][j][r] + bb[c0 + r];
                    }
                }
            }
        }
    }
}

// ----------------------------------------------------------- backward weights

// dW[o][k] = sum_p dY[p][o] X[p + off(tap(k))][cin(k)] and db[o] = sum_p dY[p][o],
// persistent over tiles of TR = 2 rows x TW = 16*MT pixels of one image.  Per tile the
// workgroup stages dY^T [COUTP][TR*TW] and, for each x shift s = dx in {0, 1, 2}, X^T
// [s][TR+2 rows][CINP][TW] with X at column x0 + c + s - 1, both written as pixel
// pairs, so that both MFMA operands are 8 consecutive pixels per lane (K = pixels).
// Wave w owns the N-tiles nt = w, w+4, ... of dW (16 columns of K each) for all
// output channels and accumulates them over all tiles of the workgroup; at the end
// the workgroup writes one set of COUTP*KP + COUTP partial sums.  Requires W % TW == 0.
template <int CINP, int COUTP, int MT>
__global__ __launch_bounds__(256) void conv_bwd_weight_kernel(const u16* __restrict__ x, const u16* __restrict__ dy,
                                                              int H, int W, int images, float* __restrict__ partials)
{
    constexpr int KP = (9 * CINP + 31) / 32 * 32;
    constexpr int MTN = COUTP / 16, NTILES = KP / 16, NPW = (NTILES + 3) / 4;
    constexpr int TW = 16 * MT, TR = 2, NPX = TR * TW;
    constexpr int XS = TW + 8, DS = NPX + 8;  // padded LDS row strides (16-byte multiples)
    __shared__ __attribute__((aligned(16))) u16 sxt[3][TR + 2][CINP][XS];
    __shared__ __attribute__((aligned(16))) u16 sdt[COUTP][DS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, g = lane >> 4;
    f32x4 acc[MTN][NPW];
#pragma unroll
    for (int i = 0; i < MTN; ++i)
#pragma unroll
        for (int j = 0; j < NPW; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    float dbias = 0.f;  // thread t < COUTP accumulates channel t
    const int tx_n = W / TW, ty_n = (H + TR - 1) / TR;
    const int tiles = images * ty_n * tx_n;
    for (int v = blockIdx.x; v < tiles; v += gridDim.x) {
        const int t = xcd_tile(v, tiles);  // XCD-aware order, as in the forward kernel
        const int img = t / (ty_n * tx_n);
        const int rt = t - img * (ty_n * tx_n);
        const int y0 = (rt / tx_n) * TR, x0 = (rt - (rt / tx_n) * tx_n) * TW;
        __syncthreads();  // the previous tile's reads of the staging areas are done
        for (int e = threadIdx.x; e < 3 * (TR + 2) * (TW / 2) * (CINP / 8); e += 256) {
            const int c8 = e % (CINP / 8);
            int rest = e / (CINP / 8);
            const int c2 = rest % (TW / 2);
            rest /= TW / 2;
            const int r = rest % (TR + 2), sh = rest / (TR + 2);
            int yy = y0 - 1 + r;
            if (yy < 0) yy += H;
            if (yy >= H) yy %= H;
            int xa = x0 + 2 * c2 + sh - 1;
            xa += (xa < 0) ? W : (xa >= W ? -W : 0);
            const int xb = (xa + 1 == W) ? 0 : xa + 1;
            const size_t row = (size_t)(img * H + yy) * W;
            const uint4 va = *(const uint4*)&x[(row + xa) * CINP + 8 * c8];
            const uint4 vb = *(const uint4*)&x[(row + xb) * CINP + 8 * c8];
            const unsigned int aw[4] = {va.x, va.y, va.z, va.w}, bw[4] = {vb.x, vb.y, vb.z, vb.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                *(unsigned int*)&sxt[sh][r][8 * c8 + 2 * j][2 * c2] = (aw[j] & 0xffffu) | (bw[j] << 16);
                *(unsigned int*)&sxt[sh][r][8 * c8 + 2 * j + 1][2 * c2] = (aw[j] >> 16) | (bw[j] & 0xffff0000u);
            }
        }
        for (int e = threadIdx.x; e < (NPX / 2) * (COUTP / 8); e += 256) {
            const int c8 = e % (COUTP / 8), q = 2 * (e / (COUTP / 8));
            const int rr = q / TW, cc = q - (q / TW) * TW;
            uint4 va = uint4{0u, 0u, 0u, 0u}, vb = uint4{0u, 0u, 0u, 0u};
            if (y0 + rr < H) {  // rows past the image bottom contribute nothing
                const size_t base = ((size_t)(img * H + y0 + rr) * W + x0 + cc) * COUTP + 8 * c8;
                va = *(const uint4*)&dy[base];
                vb = *(const uint4*)&dy[base + COUTP];
            }
            const unsigned int aw[4] = {va.x, va.y, va.z, va.w}, bw[4] = {vb.x, vb.y, vb.z, vb.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                *(unsigned int*)&sdt[8 * c8 + 2 * j][q] = (aw[j] & 0xffffu) | (bw[j] << 16);
                *(unsigned int*)&sdt[8 * c8 + 2 * j + 1][q] = (aw[j] >> 16) | (bw[j] & 0xffff0000u);
            }
        }
        __syncthreads();
        if (threadIdx.x < COUTP) {
            float sacc = 0.f;
            for (int q = 0; q < NPX; q += 8) {
                const uint4 v = *(const uint4*)&sdt[threadIdx.x][q];
                const unsigned int vw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int j = 0; j < 4; ++j) sacc += bf16_value((u16)(vw[j] & 0xffffu)) + bf16_value((u16)(vw[j] >> 16));
            }
            dbias += sacc;
        }
#pragma unroll
        for (int kc = 0; kc < NPX / 32; ++kc) {
            const int rr = (kc * 32) / TW, cb = (kc * 32) % TW;
            bf16x8 a[MTN];
#pragma unroll
            for (int i = 0; i < MTN; ++i) a[i] = *(const bf16x8*)&sdt[i * 16 + m][kc * 32 + 8 * g];
#pragma unroll
            for (int j = 0; j < NPW; ++j) {
                const int nt = wave + 4 * j;
                if (nt < NTILES) {
                    const int k = nt * 16 + m;
                    const int tap = k / CINP, ci = k - (k / CINP) * CINP;
                    bf16x8 b = bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
                    if (tap < 9) b = *(const bf16x8*)&sxt[tap % 3][rr + tap / 3][ci][cb + 8 * g];
#pragma unroll
                    for (int i = 0; i < MTN; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b, acc[i][j], 0, 0, 0);
                }
            }
        }
    }
    // lane holds C[4g + r][m]: dW[i*16 + 4g + r][nt*16 + m]
    float* part = partials + (size_t)blockIdx.x * (COUTP * KP + COUTP);
#pragma unroll
    for (int j = 0; j < NPW; ++j) {
        const int nt = wave + 4 * j;
        if (nt < NTILES) {
#pragma unroll
            for (int i = 0; i < MTN; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) part[(size_t)(i * 16 + 4 * g + r) * KP + nt * 16 + m] = acc[i][j][r];
        }
    }
    if (threadIdx.x < COUTP) part[COUTP * KP + threadIdx.x] = dbias;
}

// grads[e] = sum over workgroups of partials[wg][e].  A workgroup takes 64 entries;
// its wave q sums the q-th quarter of the groups in eight interleaved running sums
// (group g of the quarter goes to sum g mod 8), each wave keeping 8 loads per lane
// in flight; the sums are combined in a fixed order, the quarters as (0 + 1) + (2 + 3).
__global__ __launch_bounds__(256) void sum_partials_kernel(const float* __restrict__ partials, int n, int groups,
                                                          float* __restrict__ out)
{
    __shared__ float part[4][64];
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + lane;
    const int per = (groups + 3) / 4;
    const int g0 = q * per, g1 = g0 + per < groups ? g0 + per : groups;
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (e < n) {
        int gi = g0;
        for (; gi + 8 <= g1; gi += 8)
#pragma unroll
            for (int r = 0; r < 8; ++r) s[r] += partials[(size_t)(gi + r) * n + e];
        for (int r = 0; gi + r < g1; ++r) s[r] += partials[(size_t)(gi + r) * n + e];
    }
    part[q][lane] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
    __syncthreads();
    if (q == 0 && e < n) out[e] = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
}

// ------------------------------------------------------------ small kernels

// tap-flipped, channel-transposed bf16 copy for backward-data:
// wt[ci][k'] = w[o][tap * cinp + ci] with k' = (8 - tap) * coutp + o; every entry of
// wt (cinp x kpt) is written, the K padding with zeros.
__global__ __launch_bounds__(256) void pack_flipped_kernel(const float* __restrict__ w, int coutp, int cinp, int kp,
                                                           int kpt, u16* __restrict__ wt)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= cinp * kpt) return;
    const int ci = e / kpt, kk = e - (e / kpt) * kpt;
    const int tp = kk / coutp, o = kk - (kk / coutp) * coutp;
    wt[e] = tp < 9 ? bf16_bits(w[(size_t)o * kp + (8 - tp) * cinp + ci]) : (u16)0;
}

// x_bf16[p][cinp] from x_f32[p][cin] (padded channels 0)
__global__ __launch_bounds__(256) void pack_input_kernel(const float* __restrict__ x, int cin, int cinp, int P,
                                                         u16* __restrict__ out)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= P * cinp) return;
    const int p = e / cinp, c = e - (e / cinp) * cinp;
    out[e] = c < cin ? bf16_bits(x[(size_t)p * cin + c]) : (u16)0;
}

// loss partial sums (one per workgroup; each thread takes pixels p, p + G, ... with G
// the grid's thread count, a fixed order for a given P) and dL/dy = scale (y - t) in
// bf16 [P][coutp], padded channels 0 (coutp is a multiple of 8)
__global__ __launch_bounds__(256) void mse_grad_kernel(const float* __restrict__ y, const float* __restrict__ t,
                                                       int cout, int coutp, int P, float scale,
                                                       u16* __restrict__ dy, double* __restrict__ loss_part)
{
    __shared__ double red[4];
    double l = 0.0;
    for (int p = blockIdx.x * 256 + threadIdx.x; p < P; p += gridDim.x * 256) {
        for (int c8 = 0; c8 < coutp; c8 += 8) {
            unsigned int wv[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                u16 h[2];
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const int c = c8 + 2 * j + b;
                    float gval = 0.f;
                    if (c < cout) {
                        const float d = y[(size_t)p * cout + c] - t[(size_t)p * cout + c];
                        l += (double)d * d;
                        gval = scale * d;
                    }
                    h[b] = bf16_bits(gval);
                }
                wv[j] = h[0] | ((unsigned int)h[1] << 16);
            }
            *(uint4*)&dy[(size_t)p * coutp + c8] = uint4{wv[0], wv[1], wv[2], wv[3]};
        }
    }
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) l += __shfl_xor(l, s, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = l;
    __syncthreads();
    if (threadIdx.x == 0) loss_part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ __launch_bounds__(256) void sum_loss_kernel(const double* __restrict__ part, int n, double scale,
                                                       double* __restrict__ out)
{
    __shared__ double red[4];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
#pragma unroll
    for (int k = 32; k >= 1; k >>= 1) s += __shfl_xor(s, k, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = scale * (((red[0] + red[1]) + red[2]) + red[3]);
}

// Adam (Kingma & Ba, Algorithm 1) on the FP32 master parameters.
__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ theta, float* __restrict__ m_,
                                                   float* __restrict__ v_, const float* __restrict__ g, int n,
                                                   float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const float gv = g[e];
    const float m = b1 * m_[e] + (1.f - b1) * gv;
    const float v = b2 * v_[e] + (1.f - b2) * gv * gv;
    m_[e] = m;
    v_[e] = v;
    theta[e] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// --------------------------------------------------------- solver coupling

// fine (nx_f x ny_f) -> coarse block means over factor x factor cells
template <typename R>
__global__ __launch_bounds__(256) void coarsen_kernel(const typename cvec<R>::type* __restrict__ psi,
                                                      const R* __restrict__ n, const R* __restrict__ P, int nxf,
                                                      int nxc, int nyc, int f, typename cvec<R>::type* __restrict__ psic,
                                                      R* __restrict__ nc, R* __restrict__ Pc)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= nxc * nyc) return;
    const int jc = e / nxc, ic = e - (e / nxc) * nxc;
    double sr = 0, si = 0, sn = 0, sp = 0;
    for (int a = 0; a < f; ++a)
        for (int b = 0; b < f; ++b) {
            const size_t k = (size_t)(jc * f + a) * nxf + ic * f + b;
            sr += psi[k].x;
            si += psi[k].y;
            if (n) sn += n[k];
            if (P) sp += P[k];
        }
    const double inv = 1.0 / (f * f);
    psic[e] = typename cvec<R>::type{(R)(sr * inv), (R)(si * inv)};
    if (nc) nc[e] = (R)(sn * inv);
    if (Pc) Pc[e] = (R)(sp * inv);
}

// features x[p] = (Re psi / s_psi, Im psi / s_psi, n / s_n, P / s_p)
template <typename R>
__global__ __launch_bounds__(256) void features_kernel(const typename cvec<R>::type* __restrict__ psi,
                                                       const R* __restrict__ n, const R* __restrict__ P, int cells,
                                                       float s_psi, float s_n, float s_p, float* __restrict__ x)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= cells) return;
    x[4 * (size_t)e + 0] = (float)psi[e].x / s_psi;
    x[4 * (size_t)e + 1] = (float)psi[e].y / s_psi;
    x[4 * (size_t)e + 2] = n ? (float)n[e] / s_n : 0.f;
    x[4 * (size_t)e + 3] = P ? (float)P[e] / s_p : 0.f;
}

// residual r[p] = ((psi_ref - psi) / s_psi, (n_ref - n) / s_n) as 3 channels
template <typename R>
__global__ __launch_bounds__(256) void residual_kernel(const typename cvec<R>::type* __restrict__ psi_ref,
                                                       const R* __restrict__ n_ref,
                                                       const typename cvec<R>::type* __restrict__ psi,
                                                       const R* __restrict__ n, int cells, float s_psi, float s_n,
                                                       float* __restrict__ r)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= cells) return;
    r[3 * (size_t)e + 0] = (float)(psi_ref[e].x - psi[e].x) / s_psi;
    r[3 * (size_t)e + 1] = (float)(psi_ref[e].y - psi[e].y) / s_psi;
    r[3 * (size_t)e + 2] = n ? (float)(n_ref[e] - n[e]) / s_n : 0.f;
}

// psi += s_psi (y0 + i y1), n += s_n y2
template <typename R>
__global__ __launch_bounds__(256) void apply_kernel(typename cvec<R>::type* __restrict__ psi, R* __restrict__ n,
                                                    const float* __restrict__ y, int cells, float s_psi, float s_n)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= cells) return;
    psi[e].x += (R)(s_psi * y[3 * (size_t)e + 0]);
    psi[e].y += (R)(s_psi * y[3 * (size_t)e + 1]);
    if (n) n[e] += (R)(s_n * y[3 * (size_t)e + 2]);
}

}  // namespace phx

// ================================================================= host side

using namespace phx;

struct phx_cnn {
    phx_cnn_config cfg;
    phx_cnn_buffers buf;
    hipStream_t stream;
    LayerDims dims[NLAYERS];
    size_t w_off[NLAYERS], b_off[NLAYERS];  // element offsets into params
    int64_t n_params;
    // workspace regions (byte offsets)
    size_t wt[NLAYERS], act[NLAYERS + 1], grad_act, grad_act2, out_f32, dy_last, partials,
        loss_part, loss, grads_tmp;
    int bw_groups;
    size_t total;
};

#define CNN_HIP(call)                                                                            \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) return fail(PHX_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

static phx_status cnn_plan(const phx_cnn_config* c, phx_cnn* h)
{
    if (!c) return fail(PHX_EINVAL, "config is NULL");
    if (c->in_channels != 4 || c->out_channels != 3 || c->hidden != 32)
        return fail(PHX_EUNSUPPORTED, "the corrector is built for 4 input, 32 hidden and 3 output channels");
    if (c->height < 1 || c->width < 32 || c->width % 32 != 0 || c->max_batch < 1)
        return fail(PHX_EINVAL, "height >= 1, width a multiple of 32, max_batch >= 1 required");
    const int64_t P = (int64_t)c->max_batch * c->height * c->width;
    if (P >= ((int64_t)1 << 31) / 64) return fail(PHX_EINVAL, "max_batch * height * width too large");
    const int ch[NLAYERS + 1] = {c->in_channels, c->hidden, c->hidden, c->hidden, c->out_channels};
    int64_t off = 0;
    for (int l = 0; l < NLAYERS; ++l) {
        h->dims[l] = layer_dims(ch[l], ch[l + 1]);
        h->w_off[l] = off;
        off += (int64_t)h->dims[l].coutp * h->dims[l].kp;
        h->b_off[l] = off;
        off += h->dims[l].coutp;
    }
    h->n_params = off;
    size_t o = 0;
    auto take = [&](size_t b) { size_t r = o; o += align_up(b); return r; };
    for (int l = 0; l < NLAYERS; ++l) {
        const LayerDims& d = h->dims[l];
        const int kpt = (9 * d.coutp + 31) / 32 * 32;
        h->wt[l] = take((size_t)d.cinp * kpt * 2);
    }
    h->act[0] = take((size_t)P * h->dims[0].cinp * 2);
    for (int l = 1; l < NLAYERS; ++l) h->act[l] = take((size_t)P * h->dims[l].cinp * 2);
    h->act[NLAYERS] = 0;
    h->grad_act = take((size_t)P * 32 * 2);
    h->grad_act2 = take((size_t)P * 32 * 2);
    h->out_f32 = take((size_t)P * c->out_channels * 4);
    h->dy_last = take((size_t)P * h->dims[NLAYERS - 1].coutp * 2);
    h->bw_groups = 512;
    h->partials = take((size_t)h->bw_groups * (32 * 288 + 32) * 4);
    h->loss_part = take((size_t)((P * 16 + 255) / 256) * 8);
    h->loss = take(8);
    h->grads_tmp = take((size_t)h->n_params * 4);
    h->total = o;
    return PHX_OK;
}

phx_status phx_cnn_sizes(const phx_cnn_config* cfg, int64_t* n_params, size_t* workspace_bytes)
{
    clear_error();
    phx_cnn tmp{};
    phx_status s = cnn_plan(cfg, &tmp);
    if (s != PHX_OK) return s;
    if (n_params) *n_params = tmp.n_params;
    if (workspace_bytes) *workspace_bytes = tmp.total;
    return PHX_OK;
}

phx_status phx_cnn_param_offsets(const phx_cnn_config* cfg, int64_t* w_off, int64_t* b_off, int32_t* kp,
                                 int32_t* cinp, int32_t* coutp)
{
    clear_error();
    phx_cnn tmp{};
    phx_status s = cnn_plan(cfg, &tmp);
    if (s != PHX_OK) return s;
    for (int l = 0; l < NLAYERS; ++l) {
        if (w_off) w_off[l] = (int64_t)tmp.w_off[l];
        if (b_off) b_off[l] = (int64_t)tmp.b_off[l];
        if (kp) kp[l] = tmp.dims[l].kp;
        if (cinp) cinp[l] = tmp.dims[l].cinp;
        if (coutp) coutp[l] = tmp.dims[l].coutp;
    }
    return PHX_OK;
}

phx_status phx_cnn_create(const phx_cnn_config* cfg, const phx_cnn_buffers* buf, void* stream, phx_cnn** out)
{
    clear_error();
    if (!out || !buf) return fail(PHX_EINVAL, "out or buffers is NULL");
    *out = nullptr;
    phx_cnn* h = new (std::nothrow) phx_cnn();
    if (!h) return fail(PHX_EINVAL, "out of host memory");
    phx_status s = cnn_plan(cfg, h);
    if (s != PHX_OK) {
        delete h;
        return s;
    }
    if (!buf->params || !buf->workspace || buf->workspace_bytes < h->total) {
        delete h;
        return fail(PHX_EWORKSPACE, "params and a workspace of %zu bytes are required", h->total);
    }
    const void* ptrs[] = {buf->params, buf->adam_m, buf->adam_v, buf->workspace};
    for (const void* p : ptrs)
        if (p && ((uintptr_t)p & 255u)) {
            delete h;
            return fail(PHX_EINVAL, "device pointers must be 256-byte aligned");
        }
    h->cfg = *cfg;
    h->buf = *buf;
    h->stream = (hipStream_t)stream;
    *out = h;
    return PHX_OK;
}

void phx_cnn_destroy(phx_cnn* h) { delete h; }

// Workgroups of `kernel` resident on the current device (occupancy per CU, cached in
// `per_cu` by the caller, times the CU count); 0 if the runtime cannot tell.
template <typename K>
static int resident_groups(K kernel, int threads, int& per_cu)
{
    int dev = 0, cus = 0;
    if (per_cu <= 0 && hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess)
        per_cu = 0;
    if (per_cu <= 0 || hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return per_cu * cus;
}

// Forward tiles of 8 rows x 32 pixels (the width is a multiple of 32): 1.33x the
// output pixels staged with the halo, against 1.55x for 4 x 64 tiles, at the same
// accumulator and LDS footprint (3 workgroups per CU for 32 channels); measured
// 2-3 % faster than 4 x 64 and than 8 x 64 (2 workgroups per CU) tiles.
constexpr int kConvRows = 8, kConvMT = 2;

template <int CINP, int COUTP, int MODE, typename WT>
static hipError_t launch_conv(const void* in, const WT* w, const float* bias, int H, int W, int P, u16* ob,
                              float* of, int ostride, const u16* mask, hipStream_t s)
{
    static int per_cu = 0;
    const int images = P / (H * W);
    const int tiles = images * ((H + kConvRows - 1) / kConvRows) * (W / (16 * kConvMT));
    auto k = conv_fwd_kernel<CINP, COUTP, MODE, kConvMT, kConvRows, WT>;
    const int res = resident_groups(k, 256, per_cu);
    const int grid = (res > 0 && res < tiles) ? res : tiles;
    k<<<grid, 256, 0, s>>>((const u16*)in, w, bias, H, W, images, ob, of, ostride, mask);
    return hipGetLastError();
}

// two fused layers (inference): persistent over 8 x 32 tiles
template <int CINP, int COUTP, int MODE, bool XF32 = false>
static hipError_t launch_pair(const void* in, const float* wa, const float* ba, const float* wb, const float* bb, int H,
                              int W, int P, u16* ob, float* of, int ostride, hipStream_t s)
{
    static int per_cu = 0;
    const int images = P / (H * W);
    const int tiles = images * ((H + PAIR_R - 1) / PAIR_R) * (W / PAIR_W);
    auto k = conv_pair_kernel<CINP, COUTP, MODE, XF32>;
    const int res = resident_groups(k, PAIR_THREADS, per_cu);
    const int grid = (res > 0 && res < tiles) ? res : tiles;
    k<<<grid, PAIR_THREADS, 0, s>>>(in, wa, ba, wb, bb, H, W, images, ob, of, ostride);
    return hipGetLastError();
}

// tap-flipped, channel-transposed bf16 weights of every layer (backward-data)
static hipError_t cnn_pack_flipped(phx_cnn* h)
{
    char* ws = (char*)h->buf.workspace;
    for (int l = 0; l < NLAYERS; ++l) {
        const LayerDims& d = h->dims[l];
        const int kpt = (9 * d.coutp + 31) / 32 * 32;
        const int nt = d.cinp * kpt;
        pack_flipped_kernel<<<(nt + 255) / 256, 256, 0, h->stream>>>(h->buf.params + h->w_off[l], d.coutp, d.cinp,
                                                                     d.kp, kpt, (u16*)(ws + h->wt[l]));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Forward pass.  Training (keep_input) keeps every layer's input in the workspace for
// the backward passes: x packed into bf16 [P][8], then one launch per layer.  Inference
// runs layers 1 and 2 as one fused pair, the first layer reading x itself when it is
// 16-byte aligned (else from its bf16 copy), then layers 3 and 4 one launch each (the
// fused pair of those two was slower: 25 % more matrix products for a 32-channel
// layer A, and one 8-wave workgroup per CU with its LDS).  All paths give the same
// bits.  Every layer reads the float32 master weights.
static phx_status cnn_forward_impl(phx_cnn* h, const float* x, int batch, float* y, bool keep_input)
{
    const int H = h->cfg.height, W = h->cfg.width, P = batch * H * W;
    char* ws = (char*)h->buf.workspace;
    hipStream_t s = h->stream;
    const float* bias[NLAYERS];
    const float* wf[NLAYERS];
    for (int l = 0; l < NLAYERS; ++l) {
        bias[l] = h->buf.params + h->b_off[l];
        wf[l] = h->buf.params + h->w_off[l];
    }
    const bool aligned = ((uintptr_t)x & 15u) == 0;
    if (keep_input || !aligned) {
        const int n0 = P * h->dims[0].cinp;
        pack_input_kernel<<<(n0 + 255) / 256, 256, 0, s>>>(x, h->dims[0].cin, h->dims[0].cinp, P,
                                                           (u16*)(ws + h->act[0]));
        CNN_HIP(hipGetLastError());
    }
    if (!keep_input) {
        if (aligned)
            CNN_HIP((launch_pair<8, 32, CONV_RELU_BF16, true>(x, wf[0], bias[0], wf[1], bias[1], H, W, P,
                                                              (u16*)(ws + h->act[2]), nullptr, 0, s)));
        else
            CNN_HIP((launch_pair<8, 32, CONV_RELU_BF16>(ws + h->act[0], wf[0], bias[0], wf[1], bias[1], H, W, P,
                                                        (u16*)(ws + h->act[2]), nullptr, 0, s)));
    } else {
        CNN_HIP((launch_conv<8, 32, CONV_RELU_BF16>(ws + h->act[0], wf[0], bias[0], H, W, P, (u16*)(ws + h->act[1]),
                                                    nullptr, 0, nullptr, s)));
        CNN_HIP((launch_conv<32, 32, CONV_RELU_BF16>(ws + h->act[1], wf[1], bias[1], H, W, P, (u16*)(ws + h->act[2]),
                                                     nullptr, 0, nullptr, s)));
    }
    CNN_HIP((launch_conv<32, 32, CONV_RELU_BF16>(ws + h->act[2], wf[2], bias[2], H, W, P, (u16*)(ws + h->act[3]),
                                                 nullptr, 0, nullptr, s)));
    CNN_HIP((launch_conv<32, 16, CONV_LINEAR_F32>(ws + h->act[3], wf[3], bias[3], H, W, P, nullptr, y,
                                                  h->cfg.out_channels, nullptr, s)));
    return PHX_OK;
}

static phx_status check_batch(phx_cnn* h, int batch)
{
    if (!h) return fail(PHX_EINVAL, "handle is NULL");
    if (batch < 1 || batch > h->cfg.max_batch) return fail(PHX_EINVAL, "batch must be in 1..max_batch");
    return PHX_OK;
}

phx_status phx_cnn_forward(phx_cnn* h, const float* x, int32_t batch, float* y)
{
    clear_error();
    phx_status st = check_batch(h, batch);
    if (st != PHX_OK) return st;
    if (!x || !y) return fail(PHX_EINVAL, "x and y required");
    return cnn_forward_impl(h, x, batch, y, false);
}

// At most `groups` workgroups (the size of the partials buffer), no more than fit.
template <int CINP, int COUTP>
static hipError_t launch_bwd_weight(const u16* x, const u16* dy, int H, int W, int P, float* partials, int groups,
                                    float* grads, hipStream_t s)
{
    static int per_cu[2] = {0, 0};
    const int images = P / (H * W);
    const int mt4 = (W % 64 == 0) ? 1 : 0;
    const int tiles = images * ((H + 1) / 2) * (W / (mt4 ? 64 : 32));
    auto k = mt4 ? conv_bwd_weight_kernel<CINP, COUTP, 4> : conv_bwd_weight_kernel<CINP, COUTP, 2>;
    int g = resident_groups(k, 256, per_cu[mt4]);
    if (g <= 0 || g > groups) g = groups;
    if (g > tiles) g = tiles;
    k<<<g, 256, 0, s>>>(x, dy, H, W, images, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    constexpr int KP = (9 * CINP + 31) / 32 * 32;
    const int n = COUTP * KP + COUTP;
    sum_partials_kernel<<<(n + 63) / 64, 256, 0, s>>>(partials, n, g, grads);
    return hipGetLastError();
}

phx_status phx_cnn_gradients(phx_cnn* h, const float* x, const float* target, int32_t batch, float* grads,
                             double* loss)
{
    clear_error();
    phx_status st = check_batch(h, batch);
    if (st != PHX_OK) return st;
    if (!x || !target || !grads) return fail(PHX_EINVAL, "x, target and grads required");
    const int H = h->cfg.height, W = h->cfg.width, P = batch * H * W;
    if (P % 32) return fail(PHX_EINVAL, "batch * height * width must be a multiple of 32");
    char* ws = (char*)h->buf.workspace;
    hipStream_t s = h->stream;
    st = cnn_forward_impl(h, x, batch, (float*)(ws + h->out_f32), true);
    if (st != PHX_OK) return st;
    CNN_HIP(cnn_pack_flipped(h));
    // loss and dL/dy
    const int cout = h->cfg.out_channels, coutp = h->dims[NLAYERS - 1].coutp;
    const int lblocks = (P + 255) / 256 < 1024 ? (P + 255) / 256 : 1024;
    mse_grad_kernel<<<lblocks, 256, 0, s>>>((const float*)(ws + h->out_f32), target, cout, coutp, P,
                                            2.0f / ((float)P * cout), (u16*)(ws + h->dy_last),
                                            (double*)(ws + h->loss_part));
    CNN_HIP(hipGetLastError());
    sum_loss_kernel<<<1, 256, 0, s>>>((const double*)(ws + h->loss_part), lblocks, 1.0 / ((double)P * cout),
                                      loss ? loss : (double*)(ws + h->loss));
    CNN_HIP(hipGetLastError());
    float* pp = (float*)(ws + h->partials);
    const u16* act[NLAYERS];
    for (int l = 0; l < NLAYERS; ++l) act[l] = (const u16*)(ws + h->act[l]);
    u16* ga = (u16*)(ws + h->grad_act);
    u16* gb = (u16*)(ws + h->grad_act2);
    // layer 4 (32 -> 16 padded): weights, then gradient into act[3]'s space
    CNN_HIP((launch_bwd_weight<32, 16>(act[3], (const u16*)(ws + h->dy_last), H, W, P, pp, h->bw_groups,
                                        grads + h->w_off[3], s)));
    CNN_HIP((launch_conv<16, 32, CONV_MASK_BF16>((const u16*)(ws + h->dy_last), (const u16*)(ws + h->wt[3]), nullptr,
                                                 H, W, P, ga, nullptr, 0, act[3], s)));
    // layer 3
    CNN_HIP((launch_bwd_weight<32, 32>(act[2], ga, H, W, P, pp, h->bw_groups, grads + h->w_off[2], s)));
    CNN_HIP((launch_conv<32, 32, CONV_MASK_BF16>(ga, (const u16*)(ws + h->wt[2]), nullptr, H, W, P, gb, nullptr, 0,
                                                 act[2], s)));
    // layer 2
    CNN_HIP((launch_bwd_weight<32, 32>(act[1], gb, H, W, P, pp, h->bw_groups, grads + h->w_off[1], s)));
    CNN_HIP((launch_conv<32, 32, CONV_MASK_BF16>(gb, (const u16*)(ws + h->wt[1]), nullptr, H, W, P, ga, nullptr, 0,
                                                 act[1], s)));
    // layer 1 (8 padded -> 32): weights only
    CNN_HIP((launch_bwd_weight<8, 32>(act[0], ga, H, W, P, pp, h->bw_groups, grads + h->w_off[0], s)));
    return PHX_OK;
}

phx_status phx_cnn_adam(phx_cnn* h, const float* grads, int32_t t, float lr, float beta1, float beta2, float eps)
{
    clear_error();
    if (!h || !grads) return fail(PHX_EINVAL, "handle and grads required");
    if (!h->buf.adam_m || !h->buf.adam_v) return fail(PHX_EINVAL, "adam_m and adam_v buffers required");
    if (t < 1 || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return fail(PHX_EINVAL, "bad Adam hyper-parameters");
    const float c1 = (float)(1.0 - pow((double)beta1, t)), c2 = (float)(1.0 - pow((double)beta2, t));
    const int n = (int)h->n_params;
    adam_kernel<<<(n + 255) / 256, 256, 0, h->stream>>>(h->buf.params, h->buf.adam_m, h->buf.adam_v, grads, n, lr,
                                                        beta1, beta2, eps, c1, c2);
    CNN_HIP(hipGetLastError());
    return PHX_OK;
}

phx_status phx_cnn_train_step(phx_cnn* h, const float* x, const float* target, int32_t batch, int32_t t, float lr,
                              double* loss)
{
    clear_error();
    phx_status st = check_batch(h, batch);
    if (st != PHX_OK) return st;
    float* g = (float*)((char*)h->buf.workspace + h->grads_tmp);
    st = phx_cnn_gradients(h, x, target, batch, g, loss);
    if (st != PHX_OK) return st;
    return phx_cnn_adam(h, g, t, lr, 0.9f, 0.999f, 1e-8f);
}

// ---------------------------------------------------------------- coupling

template <typename R>
static phx_status coarsen_t(const void* psi, const void* n, const void* P, int nxf, int nyf, int f, void* psic,
                            void* nc, void* Pc, hipStream_t s)
{
    using C = typename cvec<R>::type;
    const int nxc = nxf / f, nyc = nyf / f;
    coarsen_kernel<R><<<(nxc * nyc + 255) / 256, 256, 0, s>>>((const C*)psi, (const R*)n, (const R*)P, nxf, nxc,
                                                              nyc, f, (C*)psic, (R*)nc, (R*)Pc);
    CNN_HIP(hipGetLastError());
    return PHX_OK;
}

phx_status phx_coarsen(int32_t precision, const void* psi_f, const void* n_f, const void* P_f, int32_t nx_f,
                       int32_t ny_f, int32_t factor, void* psi_c, void* n_c, void* P_c, void* stream)
{
    clear_error();
    if (precision != PHX_C64 && precision != PHX_C128) return fail(PHX_EINVAL, "bad precision");
    if (factor < 1 || nx_f < factor || ny_f < factor || nx_f % factor || ny_f % factor)
        return fail(PHX_EINVAL, "grid must be a positive multiple of the factor");
    if (!psi_f || !psi_c || (n_f && !n_c) || (P_f && !P_c)) return fail(PHX_EINVAL, "missing array");
    hipStream_t s = (hipStream_t)stream;
    return precision == PHX_C64 ? coarsen_t<float>(psi_f, n_f, P_f, nx_f, ny_f, factor, psi_c, n_c, P_c, s)
                                : coarsen_t<double>(psi_f, n_f, P_f, nx_f, ny_f, factor, psi_c, n_c, P_c, s);
}

phx_status phx_corrector_features(int32_t precision, const void* psi, const void* n, const void* P, int32_t nx,
                                  int32_t ny, double s_psi, double s_n, double s_p, float* x, void* stream)
{
    clear_error();
    if (precision != PHX_C64 && precision != PHX_C128) return fail(PHX_EINVAL, "bad precision");
    if (nx < 1 || ny < 1 || !psi || !x || !(s_psi > 0) || !(s_n > 0) || !(s_p > 0)) return fail(PHX_EINVAL, "bad arguments");
    const int cells = nx * ny;
    hipStream_t s = (hipStream_t)stream;
    if (precision == PHX_C64)
        features_kernel<float><<<(cells + 255) / 256, 256, 0, s>>>((const float2*)psi, (const float*)n,
                                                                   (const float*)P, cells, (float)s_psi, (float)s_n,
                                                                   (float)s_p, x);
    else
        features_kernel<double><<<(cells + 255) / 256, 256, 0, s>>>((const double2*)psi, (const double*)n,
                                                                    (const double*)P, cells, (float)s_psi, (float)s_n,
                                                                    (float)s_p, x);
    CNN_HIP(hipGetLastError());
    return PHX_OK;
}

phx_status phx_corrector_residual(int32_t precision, const void* psi_ref, const void* n_ref, const void* psi,
                                  const void* n, int32_t nx, int32_t ny, double s_psi, double s_n, float* r,
                                  void* stream)
{
    clear_error();
    if (precision != PHX_C64 && precision != PHX_C128) return fail(PHX_EINVAL, "bad precision");
    if (nx < 1 || ny < 1 || !psi_ref || !psi || !r || (n && !n_ref) || !(s_psi > 0) || !(s_n > 0))
        return fail(PHX_EINVAL, "bad arguments");
    const int cells = nx * ny;
    hipStream_t s = (hipStream_t)stream;
    if (precision == PHX_C64)
        residual_kernel<float><<<(cells + 255) / 256, 256, 0, s>>>((const float2*)psi_ref, (const float*)n_ref,
                                                                   (const float2*)psi, (const float*)n, cells,
                                                                   (float)s_psi, (float)s_n, r);
    else
        residual_kernel<double><<<(cells + 255) / 256, 256, 0, s>>>((const double2*)psi_ref, (const double*)n_ref,
                                                                    (const double2*)psi, (const double*)n, cells,
                                                                    (float)s_psi, (float)s_n, r);
    CNN_HIP(hipGetLastError());
    return PHX_OK;
}

phx_status phx_corrector_apply(int32_t precision, void* psi, void* n, const float* y, int32_t nx, int32_t ny,
                               double s_psi, double s_n, void* stream)
{
    clear_error();
    if (precision != PHX_C64 && precision != PHX_C128) return fail(PHX_EINVAL, "bad precision");
    if (nx < 1 || ny < 1 || !psi || !y || !(s_psi > 0) || !(s_n > 0)) return fail(PHX_EINVAL, "bad arguments");
    const int cells = nx * ny;
    hipStream_t s = (hipStream_t)stream;
    if (precision == PHX_C64)
        apply_kernel<float><<<(cells + 255) / 256, 256, 0, s>>>((float2*)psi, (float*)n, y, cells, (float)s_psi,
                                                                (float)s_n);
    else
        apply_kernel<double><<<(cells + 255) / 256, 256, 0, s>>>((double2*)psi, (double*)n, y, cells, (float)s_psi,
                                                                 (float)s_n);
    CNN_HIP(hipGetLastError());
    return PHX_OK;
}
