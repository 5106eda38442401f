// Host-side internals of libphx shared by the runtime translation units: error
// reporting, workspace layout, tile plans, coefficient formation and the handle.
#pragma once

#include <stddef.h>

#include <vector>

#include "phx_kernels.h"

namespace phx {

// Region shape of the whole-step RK4 kernel: waves per workgroup, rows per wave.
struct StepShapeId {
    int waves, rows;
};

struct TilePlan {
    TileShape ts;
    int tiles_x;
    int tiles;
};

// Byte offsets of the workspace regions of one handle (all 256-byte aligned).
struct Layout {
    size_t flag;        // non-finite flag word(s)
    size_t obs;         // OBS_SLOTS doubles: reduced observables
    size_t partials;    // obs_blocks * OBS_SLOTS doubles
    size_t y[2], yn[2]; // RK4 stage arguments (ping-pong)
    size_t acc, accn;   // RK4 running sum K1 + 2 K2 + 2 K3
    size_t k[7];        // Dormand-Prince stage derivatives
    size_t ys;          // Dormand-Prince stage argument
    size_t alt;         // second state buffer for psi (whole-step RK4, Dormand-Prince)
    size_t alt_n;       // second state buffer for n (whole-step RK4)
    size_t alt2, alt2_n;  // third state buffer (whole-step RK4: the tuner's trial launches)
    size_t noise;       // uint64 index of the next step, read by the noise and the drive
                        // (allocated when either is on)
    size_t drive_ph;    // RK4 with drive: the four stage phasors of the current step
    size_t imag;        // imaginary time: [0] target norm of the call, [1] restoring scale
    size_t imag_partials;  // imaginary time: per-workgroup norm partials
    int family;         // PHX_KERNEL_STAGE or PHX_KERNEL_STEP for RK4
    size_t err;         // Dormand-Prince error partials
    int obs_blocks;
    int err_blocks;
    TilePlan tiles;
    size_t total;
};

phx_status fail(phx_status s, const char* fmt, ...);
void clear_error();
const char* last_error();
size_t align_up(size_t x);
phx_status validate_config(const phx_config* c);
Layout make_layout(const phx_config& c);
TilePlan plan_tiles(int nx, int ny, int wx, int rows);
bool valid_step_shape(int precision, int waves, int rows);
template <typename R> Coef<R> make_coef(const phx_config& c);

}  // namespace phx

struct phx_handle {
    phx_config cfg;
    phx_fields f;
    hipStream_t stream;
    phx::Layout L;
    char* ws;
    phx_info info;
    double* host;           // pinned: [0, OBS_SLOTS) observables, [OBS_SLOTS] flag word,
                            // [OBS_SLOTS + 1] error norm
    hipEvent_t flag_ready;  // recorded after the flag read-back of the last phx_step
    bool flag_pending;
    // Dormand-Prince: where the current state lives (the caller's psi or the
    // workspace copy) and whether K1 = f(state) is valid in k[fsal].
    void* cur;
    void* other;
    void* cur_n;
    void* other_n;
    phx::StepShapeId step_shape;  // whole-step RK4 region shape in use
    int cus;                      // compute units of the handle's device
    phx::TilePlan stage_tiles;    // stage-fused RK4 tile plan in use
    int step_parity;              // whole-step family: buffer holding the state (0 = caller's)
    // coherent drive: time and step index of the last phx_create / phx_set_info
    double drive_t0;
    int64_t drive_k0;
    int fsal;               // index of the buffer that holds K1 of the current state
    bool k1_valid;
    // attempt log of the caller (phx_log_attempts): (dt, err, accepted) per attempt
    double* att_log;
    int64_t att_cap;
    int64_t* att_count;
    // hipGraph of graph_steps RK4 steps, captured on cap_stream, replayed on stream
    hipStream_t cap_stream;
    hipGraphExec_t graph;
    bool graph_dirty;
    // kernel timing (phx_set_timing / phx_kernel_times)
    struct TimedLaunch {
        hipEvent_t start, stop;
        int kind;
    };
    bool timing;
    std::vector<hipEvent_t> free_events;
    std::vector<TimedLaunch> pending;
    double kind_ms[PHX_MAX_KERNEL_KINDS];
    int64_t kind_launches[PHX_MAX_KERNEL_KINDS];
};

namespace phx {
// Kernel kinds for phx_kernel_times; names in kernel_kind_name().
enum KernelKind {
    K_RK4_S1 = 0, K_RK4_S2, K_RK4_S3, K_RK4_S4, K_OBS, K_DP_S1, K_DP_S2, K_DP_S3, K_DP_S4,
    K_DP_S5, K_DP_S6, K_DP_S7, K_DP_ERR, K_BATCH, K_RK4_STEP, K_NOISE, K_IMAG_NORM, K_IMAG_SCALE, K_KINDS_
};
const char* kernel_kind_name(int k);
// Timing brackets around one launch (no-ops unless timing is on).
hipError_t timing_begin(phx_handle* h, hipEvent_t* start);
hipError_t timing_end(phx_handle* h, hipEvent_t start, int kind);
const void* state_psi(const phx_handle* h);
// Observables: kernel arguments from a configuration, its tile plan and the fields
// (drive phase at time t), and phx_obs from the reduced slots.
template <typename R>
ObsArgs<R> obs_args(const phx_config& c, const TilePlan& tiles, const void* psi, const void* n, const void* V,
                    const void* P, const void* E, double t, double* partials, double* out);
void obs_from_slots(const phx_config& c, const double* q, phx_obs* out);
const void* state_n(const phx_handle* h);
phx_status create_rk45(phx_handle* h);
template <typename R> phx_status rk4_fused_steps(phx_handle* h, int64_t n);
template <typename R> phx_status rk4_fused_launches(phx_handle* h, int64_t n, hipStream_t s);
template <typename R> phx_status rk4_stage_launches(phx_handle* h, int64_t n, hipStream_t s);
int graph_chunk(const phx_config& c);
template <typename R> phx_status rk4_run_graph(phx_handle* h, int64_t n);
template <typename R> hipError_t rk4_step_trial(phx_handle* h, const StepShapeId& sh, int k);
template <typename R> hipError_t rk4_stage_trial(phx_handle* h, const TileShape& ts);
int step_shapes(int precision, const StepShapeId** out);
bool step_shape_fits(const phx_config& c, int waves);
// A whole-step shape this configuration can run (size limit of the streaming form;
// imaginary time, the drive and the spinor only on streaming shapes, the drive and
// the spinor on bands of 40 and 64 rows).
bool step_shape_allowed(const phx_config& c, const StepShapeId& sh);
bool drive_stream_rows(int rows);
// Wide streaming form (shapes {2, B}: 8-row input ring, {3, B}: 12-row ring; B = 0
// chooses the band height that fills the device): strips of 120 output columns and
// the band height in rows for this grid on a device with `cus` compute units.
template <typename R> struct StepArgs;
bool wide_shape(int waves);
int wide_strips(int nx);
int wide_band_rows(const phx_config& c, const StepShapeId& sh, bool has_v, int cus);
int wide_waves_per_simd(int ring, bool reservoir, bool has_v, bool ghosts, bool noise);
hipError_t launch_stream_wide(bool reservoir, bool has_v, int ring, const StepArgs<float>& a, hipStream_t s);
int rk4_family(const phx_config& c);
phx_status step_rk45(phx_handle* h, int64_t n, phx_info* out);
phx_status set_info_rk45(phx_handle* h, const phx_info* in);
// Wiener increment of one step on (psi, n) with step index base + offset; the base
// is advanced after each run of steps and set at creation and by phx_set_info.
template <typename R> hipError_t launch_noise(const phx_handle* h, void* psi, const void* n, int64_t offset,
                                              hipStream_t s);
hipError_t advance_noise_step(const phx_handle* h, int64_t by, hipStream_t s);
// The increment's variance a n + b (a = nu R dt / (4 dV), b = nu gamma_c dt / (4 dV),
// formed in double) and the generator key (the seed's two words).
template <typename R>
inline void noise_coefs(const phx_config& c, R& a, R& b, uint32_t& k0, uint32_t& k1)
{
    const double scale = c.noise * c.dt / (4.0 * c.dx * c.dy);
    a = (R)(scale * c.R);
    b = (R)(scale * c.gamma_c);
    k0 = (uint32_t)c.seed;
    k1 = (uint32_t)(c.seed >> 32);
}
// The wide streaming step adds the increment itself before its final store (one
// component, complex64, periodic in x and y); elsewhere a separate pass follows the step.
bool noise_in_step(const phx_config& c, const StepShapeId& sh);
hipError_t set_noise_step(const phx_handle* h, int64_t value, hipStream_t s);
// Drive phasors exp(-i omega t_s) of the four RK4 stage times of the step with index
// base + offset, written to the workspace (one thread; graph-replay safe).
template <typename R> hipError_t launch_drive_phasors(const phx_handle* h, int64_t offset, hipStream_t s);
bool uses_step_index(const phx_config& c);
// Imaginary time: deterministic total norm of psi into the target (mode 0) or the
// restoring scale (mode 1), and the pointwise scale pass.
int imag_norm_blocks(int64_t M);
template <typename R> hipError_t launch_imag_norm(const phx_handle* h, const void* psi, int mode, hipStream_t s);
template <typename R> hipError_t launch_imag_scale(const phx_handle* h, void* psi, hipStream_t s);
// Imaginary time, streaming form: the restoring scale from `count` per-wave partials.
hipError_t launch_imag_finish(const phx_handle* h, int count, hipStream_t s);
}  // namespace phx
