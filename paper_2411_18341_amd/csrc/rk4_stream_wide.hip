// Wide streaming whole-step RK4 kernel (complex64): one wave per strip of 128
// columns (two per lane) walks a band of rows with the four stages of Eqs.
// rk4_K1-rk4_final pipelined one row apart (stream_wide.h).  Workgroups are single
// waves, so the launch can hold any number of strips and bands; tile t (consecutive
// tiles on one XCD) is band t / strips, strip t % strips.
//
// Two ring configurations: an 8-row input ring loaded 3 rows ahead (fewer registers,
// more waves per SIMD) and a 12-row ring loaded 6 rows ahead (more loads in flight
// per wave, for launches with fewer, taller bands).
#include "runtime.h"
#include "stream_wide.h"

namespace phx {

// IMAG (imaginary time): the wave of tile t writes the FP64 norm partial of its cells
// to a.imag_partials[t], reduced over the lanes in a fixed butterfly order.
template <bool RES, bool HASV, bool GHOSTS, bool YZERO, int K, int PF, int WPE, bool CHECK, bool NOISE,
          bool IMAG = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE)))
void rk4_stream_wide_kernel(const StepArgs<float> a)
{
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int band = t / a.tiles_x, strip = t - band * a.tiles_x;
    double nrm = 0.0;
    if (stream_band_wide<RES, HASV, GHOSTS, YZERO, K, PF, CHECK, NOISE, IMAG>(a, strip, band, a.band_rows,
                                                                             (band & 1) ? -1 : 1, &nrm))
        a.flag[0] = 1u;  // benign race: every writer stores 1
    if constexpr (IMAG) {
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) nrm += __shfl_xor(nrm, m, 64);
        if (threadIdx.x == 0) a.imag_partials[t] = nrm;
    }
}

// Waves per SIMD the register budget of the (non-checking) kernel is set for: 3 with
// the 8-row ring (2 when the reservoir comes with a potential, a zero boundary or the
// Wiener increment drawn in the step, whose extra registers would not fit in 168), 2
// with the 12-row ring.
int wide_waves_per_simd(int ring, bool reservoir, bool has_v, bool ghosts, bool noise)
{
    return ring == 8 && !(reservoir && (has_v || ghosts || noise)) ? 3 : 2;
}

template <bool RES, bool HASV, bool GHOSTS, bool YZERO, int K, int PF>
static void launch_wide_k(const StepArgs<float>& a, hipStream_t s)
{
    constexpr int WPE = (K == 8 && !(RES && (HASV || GHOSTS))) ? 3 : 2;
    // the checking variant (the last step of a run) needs a few more registers: with
    // the reservoir it is built for 2 waves per SIMD
    constexpr int WPE_CHECK = RES ? 2 : WPE;
    // with the increment drawn in the step the reservoir variants need more than 168
    // registers: built for 2 waves per SIMD
    constexpr int WPE_NOISE = RES ? 2 : WPE;
    if constexpr (!RES) {  // imaginary time (no reservoir)
        if (a.imag_partials) {
            if (a.check)
                rk4_stream_wide_kernel<RES, HASV, GHOSTS, YZERO, K, PF, WPE_CHECK, true, false, true>
                    <<<a.tiles, 64, 0, s>>>(a);
            else
                rk4_stream_wide_kernel<RES, HASV, GHOSTS, YZERO, K, PF, WPE, false, false, true><<<a.tiles, 64, 0, s>>>(a);
            return;
        }
    }
    if constexpr (!GHOSTS && !YZERO) {  // the increment in the step: periodic grids (noise_in_step)
        if (a.noise_step) {
            if (a.check)
                rk4_stream_wide_kernel<RES, HASV, GHOSTS, YZERO, K, PF, WPE_CHECK, true, true><<<a.tiles, 64, 0, s>>>(a);
            else
                rk4_stream_wide_kernel<RES, HASV, GHOSTS, YZERO, K, PF, WPE_NOISE, false, true><<<a.tiles, 64, 0, s>>>(a);
            return;
        }
    }
    if (a.check)
        rk4_stream_wide_kernel<RES, HASV, GHOSTS, YZERO, K, PF, WPE_CHECK, true, false><<<a.tiles, 64, 0, s>>>(a);
    else
        rk4_stream_wide_kernel<RES, HASV, GHOSTS, YZERO, K, PF, WPE, false, false><<<a.tiles, 64, 0, s>>>(a);
}

template <bool RES, bool HASV, int K, int PF>
static hipError_t launch_wide_t(const StepArgs<float>& a, hipStream_t s)
{
    const bool ghosts = a.bcx == PHX_BC_ZERO || a.bcy == PHX_BC_ZERO;
    if (a.bcy == PHX_BC_ZERO)
        launch_wide_k<RES, HASV, true, true, K, PF>(a, s);
    else if (ghosts)
        launch_wide_k<RES, HASV, true, false, K, PF>(a, s);
    else
        launch_wide_k<RES, HASV, false, false, K, PF>(a, s);
    return hipGetLastError();
}

// ring: 8 (8-row ring, 3 rows ahead) or 12 (12-row ring, 6 rows ahead)
hipError_t launch_stream_wide(bool reservoir, bool has_v, int ring, const StepArgs<float>& a, hipStream_t s)
{
    if (ring == 8) {
        if (reservoir) return has_v ? launch_wide_t<true, true, 8, 3>(a, s) : launch_wide_t<true, false, 8, 3>(a, s);
        return has_v ? launch_wide_t<false, true, 8, 3>(a, s) : launch_wide_t<false, false, 8, 3>(a, s);
    }
    if (ring == 12) {
        if (reservoir) return has_v ? launch_wide_t<true, true, 12, 6>(a, s) : launch_wide_t<true, false, 12, 6>(a, s);
        return has_v ? launch_wide_t<false, true, 12, 6>(a, s) : launch_wide_t<false, false, 12, 6>(a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace phx
