// Norm restoration of imaginary-time propagation (t -> -i tau, named in Sec. 6).
//
// After each RK4 step of d psi/d tau = -(1/hbar) H psi (the stage kernels rotate
// their derivative by -i) the state is scaled by sqrt(N0 / N), N = dx dy sum |psi|^2
// over all components and cells, N0 the value when the phx_step call began.  Both
// norms come from the same deterministic two-pass FP64 reduction: fixed contiguous
// chunks per workgroup, a fixed lane and wave order inside it, then one workgroup
// over the partials in index order.  The scale lives in device memory, so the step
// sequence can be captured and replayed as a graph.  The streaming whole-step kernel
// instead writes one partial per wave and applies the scale to its next input; the
// finish kernel and the final scale pass are shared.  Passes: the partial sums read
// psi (8 B/pt complex64), the scale reads and writes it (16 B/pt); both are bound by
// HBM.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "runtime.h"

namespace {

constexpr int kNormBlocks = 1024;  // upper bound of the partials (workspace slot size)

__device__ __forceinline__ double block_sum_256(double v)
{
    __shared__ double lds[4];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) lds[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) s = ((lds[0] + lds[1]) + lds[2]) + lds[3];
    __syncthreads();
    return s;  // valid in thread 0
}

template <typename R>
__global__ __launch_bounds__(256) void norm_partials_kernel(const typename phx::cvec<R>::type* __restrict__ psi,
                                                            int64_t M, int64_t chunk, double* __restrict__ partials)
{
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = lo + chunk < M ? lo + chunk : M;
    // four independent loads and sums per iteration keep enough reads in flight;
    // the combination order is fixed, so the result does not depend on timing
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int64_t q = lo + threadIdx.x;
    for (; q + 768 < hi; q += 1024) {
        const auto a = psi[q], b = psi[q + 256], c = psi[q + 512], d = psi[q + 768];
        s0 += (double)a.x * a.x + (double)a.y * a.y;
        s1 += (double)b.x * b.x + (double)b.y * b.y;
        s2 += (double)c.x * c.x + (double)c.y * c.y;
        s3 += (double)d.x * d.x + (double)d.y * d.y;
    }
    for (; q < hi; q += 256) {
        const auto a = psi[q];
        s0 += (double)a.x * a.x + (double)a.y * a.y;
    }
    double s = block_sum_256((s0 + s1) + (s2 + s3));
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// mode 0: slots[0] = N (the target of the call) and slots[1] = 1; mode 1:
// slots[1] = sqrt(slots[0] / N).
__global__ __launch_bounds__(256) void norm_finish_kernel(const double* __restrict__ partials, int blocks,
                                                          double cell_area, int mode, double* __restrict__ slots)
{
    // eight independent accumulators per thread keep eight loads in flight (the
    // partials were just written by other XCDs: each load is a far miss); the order of
    // the additions depends on `blocks` alone
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int b = threadIdx.x;
    for (; b + 7 * 256 < blocks; b += 8 * 256) {
#pragma unroll
        for (int k = 0; k < 8; ++k) a[k] += partials[b + k * 256];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (b + k * 256 < blocks) a[k] += partials[b + k * 256];
    double s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    s = block_sum_256(s);
    if (threadIdx.x == 0) {
        const double N = cell_area * s;
        if (mode == 0) {
            slots[0] = N;
            slots[1] = 1.0;
        } else
            slots[1] = N > 0.0 ? sqrt(slots[0] / N) : 1.0;
    }
}

template <typename R>
__global__ __launch_bounds__(256) void norm_scale_kernel(typename phx::cvec<R>::type* __restrict__ psi, int64_t M,
                                                         const double* __restrict__ slots)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= M) return;
    const R s = (R)slots[1];
    auto v = psi[q];
    v.x *= s;
    v.y *= s;
    psi[q] = v;
}

}  // namespace

namespace phx {

int imag_norm_blocks(int64_t M)
{
    const int64_t b = (M + 4095) / 4096;
    return (int)(b < 1 ? 1 : (b > kNormBlocks ? kNormBlocks : b));
}

// Deterministic total norm of psi into slots[0] (mode 0) or the restoring scale into
// slots[1] (mode 1).
template <typename R>
hipError_t launch_imag_norm(const phx_handle* h, const void* psi, int mode, hipStream_t s)
{
    const phx_config& c = h->cfg;
    const int64_t M = (int64_t)c.nx * c.ny * c.components;
    const int blocks = imag_norm_blocks(M);
    const int64_t chunk = (M + blocks - 1) / blocks;
    double* partials = (double*)(h->ws + h->L.imag_partials);
    double* slots = (double*)(h->ws + h->L.imag);
    hipLaunchKernelGGL(norm_partials_kernel<R>, dim3(blocks), dim3(256), 0, s,
                       (const typename cvec<R>::type*)psi, M, chunk, partials);
    hipLaunchKernelGGL(norm_finish_kernel, dim3(1), dim3(256), 0, s, (const double*)partials, blocks, c.dx * c.dy,
                       mode, slots);
    return hipGetLastError();
}

hipError_t launch_imag_finish(const phx_handle* h, int count, hipStream_t s)
{
    hipLaunchKernelGGL(norm_finish_kernel, dim3(1), dim3(256), 0, s, (const double*)(h->ws + h->L.imag_partials),
                       count, h->cfg.dx * h->cfg.dy, 1, (double*)(h->ws + h->L.imag));
    return hipGetLastError();
}

template <typename R>
hipError_t launch_imag_scale(const phx_handle* h, void* psi, hipStream_t s)
{
    const phx_config& c = h->cfg;
    const int64_t M = (int64_t)c.nx * c.ny * c.components;
    hipLaunchKernelGGL(norm_scale_kernel<R>, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s,
                       (typename cvec<R>::type*)psi, M, (const double*)(h->ws + h->L.imag));
    return hipGetLastError();
}

template hipError_t launch_imag_norm<float>(const phx_handle*, const void*, int, hipStream_t);
template hipError_t launch_imag_norm<double>(const phx_handle*, const void*, int, hipStream_t);
template hipError_t launch_imag_scale<float>(const phx_handle*, void*, hipStream_t);
template hipError_t launch_imag_scale<double>(const phx_handle*, void*, hipStream_t);

}  // namespace phx
