// Streaming whole-step RK4 kernel for the two-component (spinor) form, with or
// without the reservoirs (stream_spinor.h): bands of 40 and 64 rows.  This unit
// holds the dispatch and the variants without reservoirs; each precision and band
// height with reservoirs has a unit of its own (rk4_stream_spinor_res_*.hip), and so
// does each precision in imaginary time (rk4_stream_spinor_imag_*.hip) and with the
// coherent drive (rk4_stream_spinor_drive_*.hip).
#include "stream_spinor_launch.h"

namespace phx {

template <typename R>
hipError_t launch_stream_spinor(bool reservoir, bool has_v, int rows, const StepArgs<R>& a, hipStream_t s)
{
    if (a.imag_partials) {  // imaginary time (no reservoirs)
        if (reservoir) return hipErrorInvalidValue;
        if (rows == 40) return launch_spinor_imag<R, 40>(has_v, a, s);
        if (rows == 64) return launch_spinor_imag<R, 64>(has_v, a, s);
        return hipErrorInvalidValue;
    }
    if (a.E) {  // the coherent drive (no reservoirs)
        if (reservoir) return hipErrorInvalidValue;
        if (rows == 40) return launch_spinor_drive<R, 40>(has_v, a, s);
        if (rows == 64) return launch_spinor_drive<R, 64>(has_v, a, s);
        return hipErrorInvalidValue;
    }
#define PHX_S(RS, B) \
    if (reservoir == RS && rows == B) return launch_spinor_part<R, RS, B>(has_v, a, s)
    PHX_S(false, 40); PHX_S(true, 40); PHX_S(false, 64); PHX_S(true, 64);
#undef PHX_S
    return hipErrorInvalidValue;
}

// the reservoir variants are instantiated in their own units
extern template hipError_t launch_spinor_part<float, true, 40>(bool, const StepArgs<float>&, hipStream_t);
extern template hipError_t launch_spinor_part<float, true, 64>(bool, const StepArgs<float>&, hipStream_t);
extern template hipError_t launch_spinor_part<double, true, 40>(bool, const StepArgs<double>&, hipStream_t);
extern template hipError_t launch_spinor_part<double, true, 64>(bool, const StepArgs<double>&, hipStream_t);
// and so are the imaginary-time variants
extern template hipError_t launch_spinor_imag<float, 40>(bool, const StepArgs<float>&, hipStream_t);
extern template hipError_t launch_spinor_imag<float, 64>(bool, const StepArgs<float>&, hipStream_t);
extern template hipError_t launch_spinor_imag<double, 40>(bool, const StepArgs<double>&, hipStream_t);
extern template hipError_t launch_spinor_imag<double, 64>(bool, const StepArgs<double>&, hipStream_t);
// and the driven ones
extern template hipError_t launch_spinor_drive<float, 40>(bool, const StepArgs<float>&, hipStream_t);
extern template hipError_t launch_spinor_drive<float, 64>(bool, const StepArgs<float>&, hipStream_t);
extern template hipError_t launch_spinor_drive<double, 40>(bool, const StepArgs<double>&, hipStream_t);
extern template hipError_t launch_spinor_drive<double, 64>(bool, const StepArgs<double>&, hipStream_t);

template hipError_t launch_stream_spinor<float>(bool, bool, int, const StepArgs<float>&, hipStream_t);
template hipError_t launch_stream_spinor<double>(bool, bool, int, const StepArgs<double>&, hipStream_t);

}  // namespace phx
