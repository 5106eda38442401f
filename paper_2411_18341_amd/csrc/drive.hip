// Phasors of the coherent drive of Eq. (PULSE_psi) for the stage-fused RK4 kernels.
//
// The drive term -(i/hbar) E_s(r) exp(-i omega t) is evaluated at each stage's own
// time, t_k + {0, 1/2, 1/2, 1} dt for the step that starts at t_k.  The step index k
// lives in device memory (advanced after each run of steps, like the noise's), so one
// thread forms t_k = t_set + (k - k_set) dt in double from the time and index of the
// last phx_create / phx_set_info, and writes the four phasors exp(-i omega t_s),
// rounded once to the kernel precision, where the stage kernels read them.  Captured
// graphs thus replay with the right phase.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "runtime.h"

namespace {

template <typename R>
__global__ void drive_phasor_kernel(typename phx::cvec<R>::type* __restrict__ out,
                                    const uint64_t* __restrict__ step_base, int64_t offset, double t_set,
                                    int64_t k_set, double dt, double omega)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int64_t k = (int64_t)(*step_base + (uint64_t)offset);
    const double t = t_set + (double)(k - k_set) * dt;
    const double c[4] = {0.0, 0.5, 0.5, 1.0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const double th = omega * (t + c[s] * dt);
        out[s].x = (R)cos(th);
        out[s].y = (R)(-sin(th));
    }
}

}  // namespace

namespace phx {

template <typename R>
hipError_t launch_drive_phasors(const phx_handle* h, int64_t offset, hipStream_t s)
{
    using C = typename cvec<R>::type;
    hipLaunchKernelGGL(drive_phasor_kernel<R>, dim3(1), dim3(64), 0, s, (C*)(h->ws + h->L.drive_ph),
                       (const uint64_t*)(h->ws + h->L.noise), offset, h->drive_t0, h->drive_k0, h->cfg.dt,
                       h->cfg.drive_omega);
    return hipGetLastError();
}

template hipError_t launch_drive_phasors<float>(const phx_handle*, int64_t, hipStream_t);
template hipError_t launch_drive_phasors<double>(const phx_handle*, int64_t, hipStream_t);

}  // namespace phx
