// Tile-shape search for the RK4 kernel families (phx_autotune).
#include <math.h>

#include <vector>

#include "runtime.h"

using namespace phx;

namespace {

template <typename F>
static phx_status time_launches(phx_handle* h, int reps, F launch, double* us)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(PHX_EHIP, "hipEventCreate failed");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(PHX_EHIP, "hipEventCreate failed");
    }
    hipError_t e = launch(0);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, h->stream);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch(r + 1);
    if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(PHX_EHIP, "tuning launch failed: %s", hipGetErrorString(e));
    *us = 1e3 * ms / reps;
    return PHX_OK;
}

template <typename R>
static phx_status tune_step(phx_handle* h, int reps, phx_tune_result* out)
{
    const StepShapeId* shapes;
    const int n = step_shapes(h->cfg.precision, &shapes);
    const StepShapeId before = h->step_shape;
    StepShapeId best = before;
    double best_us = INFINITY, before_us = INFINITY;
    int timed = 0;
    for (int k = 0; k < n; ++k) {
        const StepShapeId sh = shapes[k];
        if (!step_shape_allowed(h->cfg, sh)) continue;
        ++timed;
        double us;
        phx_status s = time_launches(h, reps, [&](int k) { return rk4_step_trial<R>(h, sh, k); }, &us);
        if (s != PHX_OK) return s;
        if (sh.waves == before.waves && sh.rows == before.rows) before_us = us;
        if (us < best_us) {
            best_us = us;
            best = sh;
        }
    }
    h->step_shape = best;
    h->graph_dirty = true;
    *out = phx_tune_result{PHX_KERNEL_STEP, best.waves, best.rows, timed, best_us, before_us};
    return PHX_OK;
}

template <typename R>
static phx_status tune_stage(phx_handle* h, int reps, phx_tune_result* out)
{
    const TileShape before = h->stage_tiles.ts;
    TileShape best = before;
    double best_us = INFINITY, before_us = INFINITY;
    int count = 0;
    const int wxs[] = {1, 2, 4};
    const int rows[] = {1, 2, 4, 8, 16, 32};
    for (int wx : wxs) {
        for (int r : rows) {
            const TileShape ts{wx, r};
            double us;
            phx_status s = time_launches(h, reps, [&](int) { return rk4_stage_trial<R>(h, ts); }, &us);
            if (s != PHX_OK) return s;
            ++count;
            if (wx == before.wx && r == before.rows) before_us = us;
            if (us < best_us) {
                best_us = us;
                best = ts;
            }
        }
    }
    h->stage_tiles = plan_tiles(h->cfg.nx, h->cfg.ny, best.wx, best.rows);
    h->graph_dirty = true;
    *out = phx_tune_result{PHX_KERNEL_STAGE, best.wx, best.rows, count, best_us, before_us};
    return PHX_OK;
}

}  // namespace

phx_status phx_autotune(phx_handle* h, int32_t reps, phx_tune_result* out)
{
    clear_error();
    if (!h || !out) return fail(PHX_EINVAL, "handle or out is NULL");
    if (reps < 1 || reps > 10000) return fail(PHX_EINVAL, "reps must be in 1..10000");
    if (h->cfg.integrator != PHX_RK4) return fail(PHX_EUNSUPPORTED, "tuning covers the RK4 kernel families");
    const bool f32 = h->cfg.precision == PHX_C64;
    if (h->L.family == PHX_KERNEL_STEP) return f32 ? tune_step<float>(h, reps, out) : tune_step<double>(h, reps, out);
    return f32 ? tune_stage<float>(h, reps, out) : tune_stage<double>(h, reps, out);
}
