// Spinor streaming whole-step kernel with the coherent drive (no reservoirs), float,
// bands of 40 and 64 rows.
#include "stream_spinor_launch.h"

namespace phx {
template hipError_t launch_spinor_drive<float, 40>(bool, const StepArgs<float>&, hipStream_t);
template hipError_t launch_spinor_drive<float, 64>(bool, const StepArgs<float>&, hipStream_t);
}  // namespace phx
