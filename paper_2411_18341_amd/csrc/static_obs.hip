// Observables of caller-given fields without a handle and without device memory
// from the caller or the allocator: the two-pass reduction of phx_observables
// (same kernels, same block partition, same summation order) with its per-block
// partials and reduced slots in a library-owned array of static device memory.
//
// Each device holds its own copy of `scratch` until the process ends.  Host code
// never passes the array's name to a kernel or a copy (in host code that name is a
// stand-in, not a device address): the device address is taken once per device with
// hipGetSymbolAddress, with that device current, and kept in scratch_ptr.
#include <cmath>
#include <mutex>

#include "runtime.h"

namespace phx {

// partials of at most 1024 workgroups (the observables plan never launches more)
// followed by the reduced slots
constexpr int kStaticObsBlocks = PHX_STATIC_OBS_BLOCKS;
constexpr size_t kStaticScratchDoubles = (size_t)(kStaticObsBlocks + 1) * OBS_SLOTS;

static __device__ __align__(256) double scratch[kStaticScratchDoubles];

constexpr int kMaxDevices = 64;
static double* scratch_ptr[kMaxDevices];
static std::mutex scratch_mutex;

// Device address of this device's scratch array (taken on first use), or NULL with
// the error recorded.
static double* device_scratch(int dev)
{
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            fail(PHX_EHIP, "static scratch address: %s", hipGetErrorString(e));
            return nullptr;
        }
        scratch_ptr[dev] = (double*)p;
    }
    return scratch_ptr[dev];
}

}  // namespace phx

extern "C" phx_status phx_observables_static(const phx_config* cfg, const phx_fields* f, double t,
                                             void* hip_stream, phx_obs* out)
{
    using namespace phx;
    clear_error();
    if (!cfg || !f || !out) return fail(PHX_EINVAL, "cfg, fields or out is NULL");
    const phx_status s = validate_config(cfg);
    if (s != PHX_OK) return s;
    if (!f->psi) return fail(PHX_EINVAL, "psi is NULL");
    if (cfg->reservoir && (!f->n || !f->P)) return fail(PHX_EINVAL, "reservoir needs n and P");
    if (cfg->drive && !f->E) return fail(PHX_EINVAL, "drive needs the profile E");
    if (!std::isfinite(t)) return fail(PHX_EINVAL, "t must be finite");
    const void* ptrs[] = {f->psi, f->n, f->V, f->P, f->E};
    for (const void* p : ptrs)
        if (p && ((uintptr_t)p & 255u) != 0) return fail(PHX_EINVAL, "device pointers must be 256-byte aligned");
    const Layout L = make_layout(*cfg);
    if (L.obs_blocks < 1 || L.obs_blocks > kStaticObsBlocks)
        return fail(PHX_EWORKSPACE, "observables need %d workgroup partials; the static scratch holds %d",
                    L.obs_blocks, kStaticObsBlocks);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return fail(PHX_EHIP, "no usable current device (device %d)", dev);
    double* ptr = device_scratch(dev);
    if (!ptr) return PHX_EHIP;
    double* partials = ptr;
    double* slots = ptr + (size_t)kStaticObsBlocks * OBS_SLOTS;
    const hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e;
    if (cfg->precision == PHX_C64)
        e = launch_observables<float>(obs_args<float>(*cfg, L.tiles, f->psi, f->n, f->V, f->P, f->E, t, partials, slots),
                                      L.obs_blocks, st);
    else
        e = launch_observables<double>(obs_args<double>(*cfg, L.tiles, f->psi, f->n, f->V, f->P, f->E, t, partials,
                                                        slots),
                                       L.obs_blocks, st);
    if (e != hipSuccess) return fail(PHX_EHIP, "observables launch: %s", hipGetErrorString(e));
    double q[OBS_SLOTS];
    e = hipMemcpyAsync(q, slots, sizeof(q), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(PHX_EHIP, "observables read-back: %s", hipGetErrorString(e));
    obs_from_slots(*cfg, q, out);
    return PHX_OK;
}
