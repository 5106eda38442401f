// Batched RK4 over many independent driven-dissipative instances.
#include "runtime.h"

using namespace phx;

phx_status phx_batch_workspace_bytes(const phx_batch_desc*, size_t*)
{
    clear_error();
    return fail(PHX_EUNSUPPORTED, "batches are not available in this build");
}

phx_status phx_batch_step(const phx_batch_desc*, int64_t, void*)
{
    clear_error();
    return fail(PHX_EUNSUPPORTED, "batches are not available in this build");
}
