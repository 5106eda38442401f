// Spinor streaming whole-step kernel in imaginary time (no reservoirs), double, bands of
// 40 and 64 rows.
#include "stream_spinor_launch.h"

namespace phx {
template hipError_t launch_spinor_imag<double, 40>(bool, const StepArgs<double>&, hipStream_t);
template hipError_t launch_spinor_imag<double, 64>(bool, const StepArgs<double>&, hipStream_t);
}  // namespace phx
