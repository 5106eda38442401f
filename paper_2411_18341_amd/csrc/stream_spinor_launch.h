// Streaming whole-step RK4 kernel for the two-component (spinor) form
// (stream_spinor.h) and its launch for one reservoir setting and band height; the
// translation units that instantiate it are split so that the large reservoir
// variants compile in parallel.
#pragma once
#include "runtime.h"
#include "stream_spinor.h"

namespace phx {

template <typename R, bool RES, bool HASV, bool GHOSTS, bool YZERO, int B>
__global__ __launch_bounds__(256) void rk4_stream_spinor_kernel(const StepArgs<R> a)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int groups_x = (a.tiles_x + 3) / 4;
    const int band = t / groups_x, strip = (t - band * groups_x) * 4 + wave;
    if (strip >= a.tiles_x) return;
    if (stream_band_spinor<R, RES, HASV, GHOSTS, YZERO, B>(a, strip, band, (band & 1) ? -1 : 1))
        a.flag[0] = 1u;  // benign race
}

template <typename R, bool RES, bool HASV, int B>
static hipError_t launch_spinor_t(const StepArgs<R>& a, hipStream_t s)
{
    const bool ghosts = a.bcx == PHX_BC_ZERO || a.bcy == PHX_BC_ZERO;
    if (a.bcy == PHX_BC_ZERO)
        rk4_stream_spinor_kernel<R, RES, HASV, true, true, B><<<a.tiles, 256, 0, s>>>(a);
    else if (ghosts)
        rk4_stream_spinor_kernel<R, RES, HASV, true, false, B><<<a.tiles, 256, 0, s>>>(a);
    else
        rk4_stream_spinor_kernel<R, RES, HASV, false, false, B><<<a.tiles, 256, 0, s>>>(a);
    return hipGetLastError();
}

template <typename R, bool RES, int B>
hipError_t launch_spinor_part(bool has_v, const StepArgs<R>& a, hipStream_t s)
{
    return has_v ? launch_spinor_t<R, RES, true, B>(a, s) : launch_spinor_t<R, RES, false, B>(a, s);
}

}  // namespace phx
