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

#include "philox.h"
#include "runtime.h"

namespace {

using phx::noise::noise_pair;
using phx::noise::philox4x32_10;
using phx::noise::Philox4;

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
    noise_pair<R, RES>(ps, ns, q + 1 < cells, (k & 1) == 0, a, b, x);
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
    R a, b;
    uint32_t k0, k1;
    noise_coefs<R>(c, a, b, k0, k1);
    const uint64_t* base = (const uint64_t*)(h->ws + h->L.noise);
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
