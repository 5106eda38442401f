// Spinor streaming whole-step kernel with reservoirs, float, bands of 40 rows.
#include "stream_spinor_launch.h"

namespace phx {
template hipError_t launch_spinor_part<float, true, 40>(bool, const StepArgs<float>&, hipStream_t);
}  // namespace phx
