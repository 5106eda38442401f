// Spinor streaming whole-step kernel with reservoirs, double, bands of 40 rows.
#include "stream_spinor_launch.h"

namespace phx {
template hipError_t launch_spinor_part<double, true, 40>(bool, const StepArgs<double>&, hipStream_t);
}  // namespace phx
