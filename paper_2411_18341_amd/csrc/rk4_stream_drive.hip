// Streaming whole-step RK4 kernel with the coherent drive of Eq. (PULSE_psi): the
// same band walk as the undriven kernel (stream_body.h), with the drive profile in
// the input ring and the phasors of the four stage times (written once per step from
// the device step index) added to every stage's derivative.  Bands of 40 and 64
// rows; kept in a translation unit of its own so that it compiles beside the others.
#include "runtime.h"
#include "stream_body.h"

namespace phx {

template <typename R, bool RES, bool HASV, bool GHOSTS, bool YZERO, int B>
__global__ __launch_bounds__(256) void rk4_stream_drive_kernel(const StepArgs<R> a)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int groups_x = (a.tiles_x + 3) / 4;
    const int band = t / groups_x, strip = (t - band * groups_x) * 4 + wave;
    if (strip >= a.tiles_x) return;
    if (stream_band<R, RES, HASV, GHOSTS, YZERO, B, false, true>(a, strip, band, (band & 1) ? -1 : 1))
        a.flag[0] = 1u;  // benign race
}

template <typename R, bool RES, bool HASV, int B>
static hipError_t launch_drive_t(const StepArgs<R>& a, hipStream_t s)
{
    const bool ghosts = a.bcx == PHX_BC_ZERO || a.bcy == PHX_BC_ZERO;
    if (a.bcy == PHX_BC_ZERO)
        rk4_stream_drive_kernel<R, RES, HASV, true, true, B><<<a.tiles, 256, 0, s>>>(a);
    else if (ghosts)
        rk4_stream_drive_kernel<R, RES, HASV, true, false, B><<<a.tiles, 256, 0, s>>>(a);
    else
        rk4_stream_drive_kernel<R, RES, HASV, false, false, B><<<a.tiles, 256, 0, s>>>(a);
    return hipGetLastError();
}

bool drive_stream_rows(int rows) { return rows == 40 || rows == 64; }

template <typename R>
hipError_t launch_stream_drive(bool reservoir, bool has_v, int rows, const StepArgs<R>& a, hipStream_t s)
{
#define PHX_D(RS, HV, B) \
    if (reservoir == RS && has_v == HV && rows == B) return launch_drive_t<R, RS, HV, B>(a, s)
    PHX_D(true, false, 40); PHX_D(true, true, 40); PHX_D(false, false, 40); PHX_D(false, true, 40);
    PHX_D(true, false, 64); PHX_D(true, true, 64); PHX_D(false, false, 64); PHX_D(false, true, 64);
#undef PHX_D
    return hipErrorInvalidValue;
}

template hipError_t launch_stream_drive<float>(bool, bool, int, const StepArgs<float>&, hipStream_t);
template hipError_t launch_stream_drive<double>(bool, bool, int, const StepArgs<double>&, hipStream_t);

}  // namespace phx
