// Complex Wiener increment of the stochastic form of Eqs. (PULSE_psi)/(PULSE_res)
// (truncated Wigner, Sec. 5): after every RK4 step each cell of each component gets
//   dW = sqrt(nu (R n + gamma_c) dt / (4 dV)) (xi1 + i xi2),
// so that <dW dW> = 0 and <dW dW*> = nu (R n + gamma_c) dt / (2 dV), with n the
// cell's reservoir value after the step (0 without the reservoir) and dV = dx dy.
//
// xi1, xi2 come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): one call
// serves the cells 2p and 2p + 1 of a component (q = j nx + i counts cells), with
// the counter (p, component, step low word, step high word) and the key (seed low
// word, seed high word); cell 2p takes output words (x0, x1), cell 2p + 1 words
// (x2, x3).  The two words become uniforms u = (x + 1/2) 2^-32 and the Box-Muller
// transform gives r cos(2 pi u2), r sin(2 pi u2) with r = sqrt(-2 ln u1).  The step
// index lives in device memory (a base plus the launch's offset within its run of
// steps), so that replays of a captured graph draw fresh numbers.
//
// The pass is pointwise: one thread per cell pair, 16-byte loads and stores where
// the pair is aligned.  Its bytes (complex read + write, reservoir read) bound it
// from below; the generator's ten rounds of two 32x32->64 products and the
// transform are its arithmetic, kept short by serving two cells per generator call
// and, in single precision, by the hardware log2/sin/cos (sin and cos take their
// argument in revolutions, so sin(2 pi u) needs no range reduction).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "runtime.h"

namespace {

struct Philox4 {
    uint32_t x[4];
};

// Ten Philox rounds: the two 32x32->64 products of counter words 0 and 2 with the
// round multipliers, high halves mixed with words 1, 3 and the key, key bumped by
// the Weyl constants.
__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                 uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Philox4{{c0, c1, c2, c3}};
}

template <typename R> struct BoxMuller;

// Single precision.  24 bits of x0 would lose 1 - u1 when u1 is close to 1, so for
// x0 >= 2^31 the logarithm is taken of w = 1 - eps, eps = (~x0 + 1/2) 2^-32 formed
// exactly from the complement, and corrected by eps / (1 - w) (Goldberg's log1p:
// ln(1 - eps) = ln(w) * (-eps) / (w - 1), exact to a few ulp; w = 1 leaves -eps).
template <> struct BoxMuller<float> {
    __device__ static float2 pair(uint32_t x0, uint32_t x1)
    {
        const float two_m32 = 2.3283064365386963e-10f;  // 2^-32
        const float ln2 = 0.693147180559945309f;
        const bool upper = x0 >= 0x80000000u;
        const float eps = ((float)(~x0) + 0.5f) * two_m32;
        const float w = 1.0f - eps;
        const float u1 = upper ? w : ((float)x0 + 0.5f) * two_m32;
        float ln_u1 = __builtin_amdgcn_logf(u1) * ln2;
        if (upper) ln_u1 = (w == 1.0f) ? -eps : ln_u1 * (-eps * __builtin_amdgcn_rcpf(w - 1.0f));
        const float r = __builtin_amdgcn_sqrtf(-2.0f * ln_u1);
        const float u2 = ((float)x1 + 0.5f) * two_m32;
        return make_float2(r * __builtin_amdgcn_cosf(u2), r * __builtin_amdgcn_sinf(u2));
    }
    __device__ static float amp(float var) { return var > 0.0f ? __builtin_amdgcn_sqrtf(var) : 0.0f; }
};

template <> struct BoxMuller<double> {
    __device__ static double2 pair(uint32_t x0, uint32_t x1)
    {
        const double u1 = ((double)x0 + 0.5) * 2.3283064365386962890625e-10;
        const double u2 = ((double)x1 + 0.5) * 2.3283064365386962890625e-10;
        const double r = sqrt(-2.0 * log(u1));
        double s, c;
        sincospi(2.0 * u2, &s, &c);
        return make_double2(r * c, r * s);
    }
    __device__ static double amp(double var) { return var > 0.0 ? sqrt(var) : 0.0; }
};

template <typename R, bool RES>
__device__ __forceinline__ typename phx::cvec<R>::type add_noise(typename phx::cvec<R>::type v, R nn, R a, R b,
                                                               uint32_t x0, uint32_t x1)
{
    const auto xi = BoxMuller<R>::pair(x0, x1);
    const R amp = BoxMuller<R>::amp(RES ? a * nn + b : b);
    v.x += amp * xi.x;
    v.y += amp * xi.y;
    return v;
}

// One thread per cell pair (2p, 2p + 1) of one component (blockIdx.y).
// var = a n + b with a = nu R dt / (4 dV), b = nu gamma_c dt / (4 dV), formed in
// double on the host.
template <typename R, bool RES>
__global__ __launch_bounds__(256) void wiener_noise_kernel(typename phx::cvec<R>::type* __restrict__ psi,
                                                           const R* __restrict__ n, int64_t cells, R a, R b,
                                                           const uint64_t* __restrict__ step_base,
                                                           int64_t offset, uint32_t k0, uint32_t k1)
{
    using C = typename phx::cvec<R>::type;
    static_assert(sizeof(C) == 2 * sizeof(R), "complex is two reals");
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t q = 2 * p;
    if (q >= cells) return;
    const uint32_t s = blockIdx.y;
    const uint64_t step = *step_base + (uint64_t)offset;
    const Philox4 x = philox4x32_10((uint32_t)p, s, (uint32_t)step, (uint32_t)(step >> 32), k0, k1);
    const int64_t k = (int64_t)s * cells + q;
    C* ps = psi + k;
    const R* ns = RES ? n + k : nullptr;
    if (q + 1 < cells && (k & 1) == 0) {  // both cells, pair aligned to twice the element size
        if constexpr (sizeof(R) == 4) {
            const float4 v = *(const float4*)ps;
            const float2 nv = RES ? *(const float2*)ns : make_float2(0.0f, 0.0f);
            const float2 lo = add_noise<float, RES>(make_float2(v.x, v.y), nv.x, a, b, x.x[0], x.x[1]);
            const float2 hi = add_noise<float, RES>(make_float2(v.z, v.w), nv.y, a, b, x.x[2], x.x[3]);
            *(float4*)ps = make_float4(lo.x, lo.y, hi.x, hi.y);
        } else {
            const double2 nv = RES ? *(const double2*)ns : make_double2(0.0, 0.0);
            const double2 lo = add_noise<double, RES>(ps[0], nv.x, a, b, x.x[0], x.x[1]);
            const double2 hi = add_noise<double, RES>(ps[1], nv.y, a, b, x.x[2], x.x[3]);
            ps[0] = lo;
            ps[1] = hi;
        }
    } else {
        ps[0] = add_noise<R, RES>(ps[0], RES ? ns[0] : (R)0, a, b, x.x[0], x.x[1]);
        if (q + 1 < cells) ps[1] = add_noise<R, RES>(ps[1], RES ? ns[1] : (R)0, a, b, x.x[2], x.x[3]);
    }
}

// Adds `by` to the step base; one thread, a plain vector store.
__global__ void noise_step_advance_kernel(uint64_t* base, int64_t by)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) base[0] += (uint64_t)by;
}

// Sets the step base; graph-safe replacement for a memset/copy of one word.
__global__ void noise_step_set_kernel(uint64_t* base, int64_t value)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) base[0] = (uint64_t)value;
}

}  // namespace

namespace phx {

template <typename R>
hipError_t launch_noise(const phx_handle* h, void* psi, const void* n, int64_t offset, hipStream_t s)
{
    const phx_config& c = h->cfg;
    const int64_t cells = (int64_t)c.nx * c.ny;
    const double scale = c.noise * c.dt / (4.0 * c.dx * c.dy);
    const R a = (R)(scale * c.R), b = (R)(scale * c.gamma_c);
    const uint64_t* base = (const uint64_t*)(h->ws + h->L.noise);
    const uint32_t k0 = (uint32_t)c.seed, k1 = (uint32_t)(c.seed >> 32);
    using C = typename cvec<R>::type;
    const int64_t pairs = (cells + 1) / 2;
    const dim3 grid((unsigned)((pairs + 255) / 256), (unsigned)c.components);
    if (c.reservoir)
        hipLaunchKernelGGL((wiener_noise_kernel<R, true>), grid, dim3(256), 0, s, (C*)psi, (const R*)n, cells, a,
                           b, base, offset, k0, k1);
    else
        hipLaunchKernelGGL((wiener_noise_kernel<R, false>), grid, dim3(256), 0, s, (C*)psi, (const R*)nullptr,
                           cells, a, b, base, offset, k0, k1);
    return hipGetLastError();
}

hipError_t advance_noise_step(const phx_handle* h, int64_t by, hipStream_t s)
{
    hipLaunchKernelGGL(noise_step_advance_kernel, dim3(1), dim3(64), 0, s, (uint64_t*)(h->ws + h->L.noise), by);
    return hipGetLastError();
}

hipError_t set_noise_step(const phx_handle* h, int64_t value, hipStream_t s)
{
    hipLaunchKernelGGL(noise_step_set_kernel, dim3(1), dim3(64), 0, s, (uint64_t*)(h->ws + h->L.noise), value);
    return hipGetLastError();
}

template hipError_t launch_noise<float>(const phx_handle*, void*, const void*, int64_t, hipStream_t);
template hipError_t launch_noise<double>(const phx_handle*, void*, const void*, int64_t, hipStream_t);

}  // namespace phx
