// Learned coarse-grid corrector: a 4-layer 3x3 convolutional network with circular
// padding, trained and evaluated by hand-written BF16 MFMA kernels with FP32
// accumulation, plus the kernels that connect it to the solver (block-mean
// coarsening of a fine state, input features, training residuals, and adding the
// predicted correction to a coarse state).
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16:
//   forward        M = 16 pixels of one row, N = output channels, K = 9 taps x C_in
//   backward-data  the forward kernel on dY with the weights flipped in the taps and
//                  transposed in the channels, times the ReLU mask of the layer input
//   backward-weight M = output channels, N = 9 taps x C_in, K = pixels: each
//                  workgroup stages 32-pixel chunks of dY and of the three shifted
//                  copies of X in LDS and accumulates; per-workgroup partials are
//                  summed in a fixed order.
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

// One wave computes 16 consecutive pixels of a row times all COUTP output
// channels.  in: [P][CINP] bf16, w: [COUTP][KP] bf16, bias: [COUTP] f32.
// MODE: CONV_RELU_BF16 -> out_bf16[P][COUTP] = relu(acc + bias)
//       CONV_LINEAR_F32 -> out_f32[P][out_stride], channels < out_stride, acc + bias
//       CONV_MASK_BF16 -> out_bf16[P][COUTP] = acc if mask[P][COUTP] > 0 else 0
template <int CINP, int COUTP, int MODE>
__global__ __launch_bounds__(256) void conv_fwd_kernel(const u16* __restrict__ in, const u16* __restrict__ w,
                                                       const float* __restrict__ bias, int H, int W, int P,
                                                       u16* __restrict__ out_bf16, float* __restrict__ out_f32,
                                                       int out_stride, const u16* __restrict__ mask)
{
    constexpr int KP = (9 * CINP + 31) / 32 * 32;
    constexpr int NT = COUTP / 16;
    const int lane = threadIdx.x & 63;
    const int wv = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int p0 = wv * 16;
    if (p0 >= P) return;  // whole wave leaves together (P is a multiple of 16)
    const int m = lane & 15, g = lane >> 4;
    const int p = p0 + m;  // pixel of this lane's A row
    const int img = p / (H * W);
    const int rem = p - img * H * W;
    const int y = rem / W, x = rem - (rem / W) * W;
    f32x4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < KP / 32; ++c) {
        const int k0 = 32 * c + 8 * g;
        const int tap = k0 / CINP, ci = k0 - (k0 / CINP) * CINP;
        bf16x8 a;
        if (tap < 9) {
            const int dy = tap / 3 - 1, dx = tap - (tap / 3) * 3 - 1;
            int yy = y + dy, xx = x + dx;
            yy += (yy < 0) ? H : (yy >= H ? -H : 0);
            xx += (xx < 0) ? W : (xx >= W ? -W : 0);
            a = *(const bf16x8*)(in + ((size_t)(img * H + yy) * W + xx) * CINP + ci);
        } else {
            a = bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const bf16x8 b = *(const bf16x8*)(w + (size_t)(t * 16 + m) * KP + k0);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
        }
    }
    // lane holds C[4g + i][m]: pixel p0 + 4g + i, channel t*16 + m
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int co = t * 16 + m;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int q = p0 + 4 * g + i;
            float v = acc[t][i];
            if (MODE == CONV_RELU_BF16) {
                v += bias[co];
                out_bf16[(size_t)q * COUTP + co] = bf16_bits(v > 0.f ? v : 0.f);
            } else if (MODE == CONV_LINEAR_F32) {
                if (co < out_stride) out_f32[(size_t)q * out_stride + co] = v + bias[co];
            } else {
                const float mk = bf16_value(mask[(size_t)q * COUTP + co]);
                out_bf16[(size_t)q * COUTP + co] = bf16_bits(mk > 0.f ? v : 0.f);
            }
        }
    }
}

// ----------------------------------------------------------- backward weights

// dW[o][k] += sum_p dY[p][o] X[p + off(tap(k))][cin(k)], db[o] += sum_p dY[p][o] over
// the pixel chunks of this workgroup (32 consecutive pixels of one row each);
// writes COUTP*KP + COUTP partial sums per workgroup.
template <int CINP, int COUTP>
__global__ __launch_bounds__(256) void conv_bwd_weight_kernel(const u16* __restrict__ x, const u16* __restrict__ dy,
                                                              int H, int W, int P, float* __restrict__ partials)
{
    constexpr int KP = (9 * CINP + 31) / 32 * 32;
    constexpr int MT = COUTP / 16, NTILES = KP / 16;
    constexpr int BLOCKS = MT * NTILES;                 // 16x16 output blocks
    constexpr int PER_WAVE = (BLOCKS + 3) / 4;
    // LDS: dY^T [COUTP][32] and X shifted by dx in {-1,0,1}: [3 dx][3 dy][CINP][32]
    __shared__ __attribute__((aligned(16))) u16 sdy[COUTP][32];
    __shared__ __attribute__((aligned(16))) u16 sx[3][3][CINP][32];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, g = lane >> 4;
    f32x4 acc[PER_WAVE];
#pragma unroll
    for (int b = 0; b < PER_WAVE; ++b) acc[b] = f32x4{0.f, 0.f, 0.f, 0.f};
    float dbias = 0.f;  // thread t < COUTP accumulates channel t
    const int chunks = P / 32;
    for (int ch = blockIdx.x; ch < chunks; ch += gridDim.x) {
        const int p0 = ch * 32;
        const int img = p0 / (H * W);
        const int rem = p0 - img * H * W;
        const int y = rem / W, x0 = rem - (rem / W) * W;
        // stage dY^T
        for (int e = threadIdx.x; e < 32 * COUTP; e += 256) {
            const int px = e / COUTP, o = e - (e / COUTP) * COUTP;
            sdy[o][px] = dy[(size_t)(p0 + px) * COUTP + o];
        }
        // stage X rows y-1..y+1, columns x0-1+dx .. for the three dx shifts
        for (int e = threadIdx.x; e < 3 * 3 * 32 * CINP; e += 256) {
            const int ci = e % CINP;
            const int px = (e / CINP) % 32;
            const int r = (e / (CINP * 32)) % 3;
            const int s = e / (CINP * 32 * 3);
            int yy = y + r - 1, xx = x0 + px + s - 1;
            yy += (yy < 0) ? H : (yy >= H ? -H : 0);
            xx += (xx < 0) ? W : (xx >= W ? -W : 0);
            sx[s][r][ci][px] = x[((size_t)(img * H + yy) * W + xx) * CINP + ci];
        }
        __syncthreads();
        if (threadIdx.x < COUTP) {
            float sacc = 0.f;
            for (int px = 0; px < 32; ++px) sacc += bf16_value(sdy[threadIdx.x][px]);
            dbias += sacc;
        }
#pragma unroll
        for (int b = 0; b < PER_WAVE; ++b) {
            const int blk = wave + 4 * b;
            if (blk < BLOCKS) {
                const int mt = blk / NTILES, nt = blk - (blk / NTILES) * NTILES;
                // A[m][kr] = dY[p0 + kr][mt*16 + m], kr = 8g + j
                const bf16x8 a = *(const bf16x8*)&sdy[mt * 16 + m][8 * g];
                // B[kr][n] = X[p0 + kr + off(tap)][cin], column n -> k = nt*16 + m
                const int k = nt * 16 + m;
                const int tap = k / CINP, ci = k - (k / CINP) * CINP;
                bf16x8 bv;
                if (tap < 9) {
                    const int r = tap / 3, s = tap - (tap / 3) * 3;
                    bv = *(const bf16x8*)&sx[s][r][ci][8 * g];
                } else {
                    bv = bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
                }
                acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bv, acc[b], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    float* part = partials + (size_t)blockIdx.x * (COUTP * KP + COUTP);
#pragma unroll
    for (int b = 0; b < PER_WAVE; ++b) {
        const int blk = wave + 4 * b;
        if (blk < BLOCKS) {
            const int mt = blk / NTILES, nt = blk - (blk / NTILES) * NTILES;
#pragma unroll
            for (int i = 0; i < 4; ++i) part[(size_t)(mt * 16 + 4 * g + i) * KP + nt * 16 + m] = acc[b][i];
        }
    }
    if (threadIdx.x < COUTP) part[COUTP * KP + threadIdx.x] = dbias;
}

// grads[e] = sum over workgroups of partials[wg][e] (fixed order)
__global__ __launch_bounds__(256) void sum_partials_kernel(const float* __restrict__ partials, int n, int groups,
                                                          float* __restrict__ out)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    float s = 0.f;
    for (int gidx = 0; gidx < groups; ++gidx) s += partials[(size_t)gidx * n + e];
    out[e] = s;
}

// ------------------------------------------------------------ small kernels

// bf16 copy of the weights, wb[o][k] (same [coutp][kp] layout as the master copy)
__global__ __launch_bounds__(256) void pack_weights_kernel(const float* __restrict__ w, int n, u16* __restrict__ wb)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e < n) wb[e] = bf16_bits(w[e]);
}

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

// loss partial sums and dL/dy = 2 (y - t) / (P cout) in bf16 [P][coutp]
__global__ __launch_bounds__(256) void mse_grad_kernel(const float* __restrict__ y, const float* __restrict__ t,
                                                       int cout, int coutp, int P, float scale,
                                                       u16* __restrict__ dy, double* __restrict__ loss_part)
{
    __shared__ double red[4];
    const int e = blockIdx.x * 256 + threadIdx.x;
    double l = 0.0;
    if (e < P * coutp) {
        const int p = e / coutp, c = e - (e / coutp) * coutp;
        float gval = 0.f;
        if (c < cout) {
            const float d = y[(size_t)p * cout + c] - t[(size_t)p * cout + c];
            l = (double)d * d;
            gval = scale * d;
        }
        dy[e] = bf16_bits(gval);
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
    size_t wb[NLAYERS], wt[NLAYERS], act[NLAYERS + 1], grad_act, grad_act2, out_f32, dy_last, partials,
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
        h->wb[l] = take((size_t)d.coutp * d.kp * 2);
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

template <int CINP, int COUTP, int MODE>
static hipError_t launch_conv(const u16* in, const u16* w, const float* bias, int H, int W, int P, u16* ob,
                              float* of, int ostride, const u16* mask, hipStream_t s)
{
    const int waves = P / 16;
    conv_fwd_kernel<CINP, COUTP, MODE><<<(waves + 3) / 4, 256, 0, s>>>(in, w, bias, H, W, P, ob, of, ostride, mask);
    return hipGetLastError();
}

static hipError_t cnn_pack(phx_cnn* h, bool transposed)
{
    char* ws = (char*)h->buf.workspace;
    for (int l = 0; l < NLAYERS; ++l) {
        const LayerDims& d = h->dims[l];
        const int n = d.coutp * d.kp;
        pack_weights_kernel<<<(n + 255) / 256, 256, 0, h->stream>>>(h->buf.params + h->w_off[l], n,
                                                                    (u16*)(ws + h->wb[l]));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (transposed) {
            const int kpt = (9 * d.coutp + 31) / 32 * 32;
            const int nt = d.cinp * kpt;
            pack_flipped_kernel<<<(nt + 255) / 256, 256, 0, h->stream>>>(h->buf.params + h->w_off[l], d.coutp, d.cinp,
                                                                         d.kp, kpt, (u16*)(ws + h->wt[l]));
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

// forward pass; activations of every layer input kept in the workspace
static phx_status cnn_forward_impl(phx_cnn* h, const float* x, int batch, float* y)
{
    const int H = h->cfg.height, W = h->cfg.width, P = batch * H * W;
    char* ws = (char*)h->buf.workspace;
    hipStream_t s = h->stream;
    CNN_HIP(cnn_pack(h, false));
    const int n0 = P * h->dims[0].cinp;
    pack_input_kernel<<<(n0 + 255) / 256, 256, 0, s>>>(x, h->dims[0].cin, h->dims[0].cinp, P, (u16*)(ws + h->act[0]));
    CNN_HIP(hipGetLastError());
    const float* bias[NLAYERS];
    const u16* wb[NLAYERS];
    for (int l = 0; l < NLAYERS; ++l) {
        bias[l] = h->buf.params + h->b_off[l];
        wb[l] = (const u16*)(ws + h->wb[l]);
    }
    CNN_HIP((launch_conv<8, 32, CONV_RELU_BF16>((const u16*)(ws + h->act[0]), wb[0], bias[0], H, W, P,
                                                (u16*)(ws + h->act[1]), nullptr, 0, nullptr, s)));
    CNN_HIP((launch_conv<32, 32, CONV_RELU_BF16>((const u16*)(ws + h->act[1]), wb[1], bias[1], H, W, P,
                                                 (u16*)(ws + h->act[2]), nullptr, 0, nullptr, s)));
    CNN_HIP((launch_conv<32, 32, CONV_RELU_BF16>((const u16*)(ws + h->act[2]), wb[2], bias[2], H, W, P,
                                                 (u16*)(ws + h->act[3]), nullptr, 0, nullptr, s)));
    CNN_HIP((launch_conv<32, 16, CONV_LINEAR_F32>((const u16*)(ws + h->act[3]), wb[3], bias[3], H, W, P, nullptr, y,
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
    return cnn_forward_impl(h, x, batch, y);
}

template <int CINP, int COUTP>
static hipError_t launch_bwd_weight(const u16* x, const u16* dy, int H, int W, int P, float* partials, int groups,
                                    float* grads, hipStream_t s)
{
    const int chunks = P / 32;
    const int g = chunks < groups ? chunks : groups;
    conv_bwd_weight_kernel<CINP, COUTP><<<g, 256, 0, s>>>(x, dy, H, W, P, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    constexpr int KP = (9 * CINP + 31) / 32 * 32;
    const int n = COUTP * KP + COUTP;
    sum_partials_kernel<<<(n + 255) / 256, 256, 0, s>>>(partials, n, g, grads);
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
    st = cnn_forward_impl(h, x, batch, (float*)(ws + h->out_f32));
    if (st != PHX_OK) return st;
    CNN_HIP(cnn_pack(h, true));
    // loss and dL/dy
    const int cout = h->cfg.out_channels, coutp = h->dims[NLAYERS - 1].coutp;
    const int nl = P * coutp, lblocks = (nl + 255) / 256;
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
