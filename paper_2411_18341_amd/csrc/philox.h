// Device-side generator of the Wiener increments (truncated-Wigner noise, Sec. 5):
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and the Box-Muller transform,
// shared by the single-grid and the batched noise passes so that both draw the same
// numbers for the same (cell pair, component, step, seed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "phx_kernels.h"

namespace phx {
namespace noise {

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

// Adds the increments of cell q (words x0, x1) and, when `two`, of cell q + 1
// (words x2, x3) of one component; ps and ns point at cell q.  With `aligned` (q at
// an even element index) the pair moves as one 16-byte access.
template <typename R, bool RES>
__device__ __forceinline__ void noise_pair(typename cvec<R>::type* ps, const R* ns, bool two, bool aligned, R a,
                                           R b, const Philox4& x)
{
    if (two && aligned) {
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
        if (two) ps[1] = add_noise<R, RES>(ps[1], RES ? ns[1] : (R)0, a, b, x.x[2], x.x[3]);
    }
}

}  // namespace noise
}  // namespace phx
