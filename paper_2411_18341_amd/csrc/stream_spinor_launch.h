// Streaming whole-step RK4 kernel for the two-component (spinor) form
// (stream_spinor.h) and its launch for one reservoir setting and band height; the
// translation units that instantiate it are split so that the large reservoir
// variants compile in parallel.
#pragma once
#include "runtime.h"
#include "stream_spinor.h"

namespace phx {

// IMAG (imaginary time): wave w of tile t writes the FP64 norm partial of its cells
// (both components) to a.imag_partials[4 t + w] (0 for a wave past the last strip),
// reduced over the lanes in a fixed butterfly order.
template <typename R, bool RES, bool HASV, bool GHOSTS, bool YZERO, int B, bool IMAG = false, bool DRIVE = false>
__global__ __launch_bounds__(256) void rk4_stream_spinor_kernel(const StepArgs<R> a)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int groups_x = (a.tiles_x + 3) / 4;
    const int band = t / groups_x, strip = (t - band * groups_x) * 4 + wave;
    if (strip >= a.tiles_x) {
        if (IMAG && (threadIdx.x & 63) == 0) a.imag_partials[4 * t + wave] = 0.0;
        return;
    }
    double nrm = 0.0;
    if (stream_band_spinor<R, RES, HASV, GHOSTS, YZERO, B, IMAG, DRIVE>(a, strip, band, (band & 1) ? -1 : 1, &nrm))
        a.flag[0] = 1u;  // benign race
    if constexpr (IMAG) {
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) nrm += __shfl_xor(nrm, m, 64);
        if ((threadIdx.x & 63) == 0) a.imag_partials[4 * t + wave] = nrm;
    }
}

template <typename R, bool RES, bool HASV, int B, bool IMAG = false, bool DRIVE = false>
static hipError_t launch_spinor_t(const StepArgs<R>& a, hipStream_t s)
{
    const bool ghosts = a.bcx == PHX_BC_ZERO || a.bcy == PHX_BC_ZERO;
    if (a.bcy == PHX_BC_ZERO)
        rk4_stream_spinor_kernel<R, RES, HASV, true, true, B, IMAG, DRIVE><<<a.tiles, 256, 0, s>>>(a);
    else if (ghosts)
        rk4_stream_spinor_kernel<R, RES, HASV, true, false, B, IMAG, DRIVE><<<a.tiles, 256, 0, s>>>(a);
    else
        rk4_stream_spinor_kernel<R, RES, HASV, false, false, B, IMAG, DRIVE><<<a.tiles, 256, 0, s>>>(a);
    return hipGetLastError();
}

// imaginary time (no reservoirs): instantiated in units of its own
template <typename R, int B>
hipError_t launch_spinor_imag(bool has_v, const StepArgs<R>& a, hipStream_t s)
{
    return has_v ? launch_spinor_t<R, false, true, B, true>(a, s) : launch_spinor_t<R, false, false, B, true>(a, s);
}

// the coherent drive (no reservoirs): instantiated in units of its own
template <typename R, int B>
hipError_t launch_spinor_drive(bool has_v, const StepArgs<R>& a, hipStream_t s)
{
    return has_v ? launch_spinor_t<R, false, true, B, false, true>(a, s)
                 : launch_spinor_t<R, false, false, B, false, true>(a, s);
}

template <typename R, bool RES, int B>
hipError_t launch_spinor_part(bool has_v, const StepArgs<R>& a, hipStream_t s)
{
    return has_v ? launch_spinor_t<R, RES, true, B>(a, s) : launch_spinor_t<R, RES, false, B>(a, s);
}

}  // namespace phx
