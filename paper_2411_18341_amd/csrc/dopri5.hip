// Adaptive Dormand-Prince 5(4) stepping (named in Sec. 2 as the adaptive
// alternative to RK4).
#include "runtime.h"

namespace phx {

phx_status create_rk45(phx_handle*) { return fail(PHX_EUNSUPPORTED, "PHX_RK45 is not available in this build"); }
phx_status step_rk45(phx_handle*, int64_t, phx_info*) { return fail(PHX_EUNSUPPORTED, "PHX_RK45 is not available in this build"); }
phx_status set_info_rk45(phx_handle*, const phx_info*) { return fail(PHX_EUNSUPPORTED, "PHX_RK45 is not available in this build"); }

}  // namespace phx
