// Spinor streaming whole-step kernel with the coherent drive (no reservoirs), double,
// bands of 40 and 64 rows.
#include "stream_spinor_launch.h"

namespace phx {
template hipError_t launch_spinor_drive<double, 40>(bool, const StepArgs<double>&, hipStream_t);
template hipError_t launch_spinor_drive<double, 64>(bool, const StepArgs<double>&, hipStream_t);
}  // namespace phx
