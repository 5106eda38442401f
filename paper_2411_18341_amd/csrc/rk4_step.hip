// Whole-step RK4 kernel: all four stages of Eqs. rk4_K1-rk4_final in one launch.
//
// A workgroup owns a region of 64 columns x H rows of the grid (H = WAVES*ROWS)
// and produces the interior 56 x (H-8) cells: every stage applies the five-point
// stencil once, so after four stages the values are exact up to 4 cells from the
// region edge (the 4-cell halo of the paper's subgrids, Sec. 3.2.4, recomputed
// redundantly instead of exchanged).  The state is read from HBM once (with the
// halo) and written once; the stage arguments, K sums and reservoir values stay in
// registers for the whole step.
//
// Stage s evaluates only the region rows [s, H-s) that the output depends on.
// Lane l of every wave owns region column l; wave w owns rows [w*ROWS, (w+1)*ROWS).
// x-neighbours come from the adjacent lanes by DPP wave shifts, y-neighbours from
// the lane's own registers except at the wave's first and last row, which are
// exchanged through LDS (double-buffered by stage parity: one barrier per stage).
// Region cells outside a zero boundary are ghost cells held at 0 in every stage;
// with a periodic boundary the region wraps.  The output goes to a second state
// buffer (neighbouring regions still read the input's halo).
#include "runtime.h"
#include "step_body.h"
#include "stream_body.h"

namespace phx {

template <typename R, bool RES, bool HASV, bool GHOSTS, int WAVES, int ROWS>
__global__ __launch_bounds__(WAVES * 64) void rk4_step_kernel(const StepArgs<R> a)
{
    __shared__ typename cvec<R>::type edge[2][WAVES][2][64];
    const bool bad = step_region<R, RES, HASV, GHOSTS, WAVES, ROWS>(a, xcd_tile(blockIdx.x, gridDim.x), edge);
    if (bad) a.flag[0] = 1u;  // benign race: every writer stores 1
}

// Streaming form: a workgroup is 4 adjacent strips of one band of B rows (their
// x-halo columns are read through one L1); a.tiles_x counts strips, a.tiles
// workgroups.  Waves past the last strip leave at once (the kernel has no barrier).
// IMAG (imaginary time): wave w of tile t writes the FP64 norm partial of its cells
// to a.imag_partials[4 t + w] (0 for a wave past the last strip), reduced over the
// lanes in a fixed butterfly order.
template <typename R, bool RES, bool HASV, bool GHOSTS, bool YZERO, int B, bool IMAG>
__global__ __launch_bounds__(256) void rk4_stream_kernel(const StepArgs<R> a)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int groups_x = (a.tiles_x + 3) / 4;
    const int band = t / groups_x, strip = (t - band * groups_x) * 4 + wave;
    if (strip >= a.tiles_x) {
        if (IMAG && (threadIdx.x & 63) == 0) a.imag_partials[4 * t + wave] = 0.0;
        return;
    }
    double nrm = 0.0;
    if (stream_band<R, RES, HASV, GHOSTS, YZERO, B, IMAG>(a, strip, band, (band & 1) ? -1 : 1, &nrm))
        a.flag[0] = 1u;  // benign race
    if constexpr (IMAG) {
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) nrm += __shfl_xor(nrm, m, 64);
        if ((threadIdx.x & 63) == 0) a.imag_partials[4 * t + wave] = nrm;
    }
}

// GHOSTS: some boundary is zero, so region cells outside the grid must be held at 0
// after every stage; with periodic boundaries in both directions there are none.
// WAVES == 1 selects the streaming kernel with bands of ROWS rows.
template <typename R, bool RES, bool HASV, int WAVES, int ROWS>
static hipError_t launch_step_t(const StepArgs<R>& a, hipStream_t s)
{
    const bool ghosts = a.bcx == PHX_BC_ZERO || a.bcy == PHX_BC_ZERO;
    if constexpr (WAVES == 1) {
        if constexpr (!RES) {
            if (a.imag_partials) {  // imaginary time
                if (a.bcy == PHX_BC_ZERO)
                    rk4_stream_kernel<R, RES, HASV, true, true, ROWS, true><<<a.tiles, 256, 0, s>>>(a);
                else if (ghosts)
                    rk4_stream_kernel<R, RES, HASV, true, false, ROWS, true><<<a.tiles, 256, 0, s>>>(a);
                else
                    rk4_stream_kernel<R, RES, HASV, false, false, ROWS, true><<<a.tiles, 256, 0, s>>>(a);
                return hipGetLastError();
            }
        }
        if (a.bcy == PHX_BC_ZERO)
            rk4_stream_kernel<R, RES, HASV, true, true, ROWS, false><<<a.tiles, 256, 0, s>>>(a);
        else if (ghosts)
            rk4_stream_kernel<R, RES, HASV, true, false, ROWS, false><<<a.tiles, 256, 0, s>>>(a);
        else
            rk4_stream_kernel<R, RES, HASV, false, false, ROWS, false><<<a.tiles, 256, 0, s>>>(a);
    } else {
        if (ghosts)
            rk4_step_kernel<R, RES, HASV, true, WAVES, ROWS><<<a.tiles, WAVES * 64, 0, s>>>(a);
        else
            rk4_step_kernel<R, RES, HASV, false, WAVES, ROWS><<<a.tiles, WAVES * 64, 0, s>>>(a);
    }
    return hipGetLastError();
}

// Region shapes (waves per workgroup, rows per wave) instantiated per precision.
// A region of WAVES*ROWS rows yields WAVES*ROWS - 8 output rows; taller regions
// recompute less halo, shorter ones need fewer registers per lane (more waves
// per SIMD).  The first entry is the default; phx_autotune measures them all.
// Shapes {1, B} are the streaming kernel with bands of B rows (B + 8 a multiple of 24).
// Shapes {2, B} and {3, B} are the wide streaming kernel (two columns per lane) with
// bands of B rows, B = 0 choosing the height that fills the device in one wave of
// workgroups (complex64 only).
static const StepShapeId kFloatShapes[] = {{8, 4}, {16, 4}, {8, 8}, {12, 4}, {12, 6}, {8, 6}, {4, 8}, {16, 6},
                                           {1, 40}, {1, 64}, {1, 88}, {1, 112},
                                           {2, 0}, {3, 0}, {2, 40}, {2, 64}, {3, 64}, {3, 96}};
static const StepShapeId kDoubleShapes[] = {{8, 4}, {16, 2}, {8, 2}, {12, 4}, {4, 4}, {1, 40}, {1, 64}};

int step_shapes(int precision, const StepShapeId** out)
{
    if (precision == PHX_C64) {
        *out = kFloatShapes;
        return (int)(sizeof(kFloatShapes) / sizeof(kFloatShapes[0]));
    }
    *out = kDoubleShapes;
    return (int)(sizeof(kDoubleShapes) / sizeof(kDoubleShapes[0]));
}

template <typename R, bool RES, bool HASV>
static hipError_t launch_step_shape(const StepShapeId& sh, const StepArgs<R>& a, hipStream_t s)
{
#define PHX_SHAPE(W, K) \
    if (sh.waves == W && sh.rows == K) return launch_step_t<R, RES, HASV, W, K>(a, s)
    if constexpr (sizeof(R) == 4) {
        PHX_SHAPE(8, 4); PHX_SHAPE(16, 4); PHX_SHAPE(8, 8); PHX_SHAPE(12, 4);
        PHX_SHAPE(12, 6); PHX_SHAPE(8, 6); PHX_SHAPE(4, 8); PHX_SHAPE(16, 6);
        PHX_SHAPE(1, 40); PHX_SHAPE(1, 64); PHX_SHAPE(1, 88); PHX_SHAPE(1, 112);
    } else {
        PHX_SHAPE(8, 4); PHX_SHAPE(16, 2); PHX_SHAPE(8, 2); PHX_SHAPE(12, 4); PHX_SHAPE(4, 4);
        PHX_SHAPE(1, 40); PHX_SHAPE(1, 64);
    }
#undef PHX_SHAPE
    return hipErrorInvalidValue;
}

template <typename R>
hipError_t launch_stream_drive(bool reservoir, bool has_v, int rows, const StepArgs<R>& a, hipStream_t s);
template <typename R>
hipError_t launch_stream_spinor(bool reservoir, bool has_v, int rows, const StepArgs<R>& a, hipStream_t s);

template <typename R>
hipError_t launch_rk4_step(bool reservoir, bool has_v, const StepShapeId& sh, const StepArgs<R>& a,
                           hipStream_t s)
{
    if (a.E && a.comps == 1)
        return sh.waves == 1 ? launch_stream_drive<R>(reservoir, has_v, sh.rows, a, s) : hipErrorInvalidValue;
    if (wide_shape(sh.waves)) {
        if constexpr (sizeof(R) == 4) {
            if (a.comps != 1) return hipErrorInvalidValue;
            return launch_stream_wide(reservoir, has_v, sh.waves == 2 ? 8 : 12, a, s);
        }
        return hipErrorInvalidValue;
    }
    if (a.comps == 2)
        return sh.waves == 1 ? launch_stream_spinor<R>(reservoir, has_v, sh.rows, a, s) : hipErrorInvalidValue;
    if (reservoir) return has_v ? launch_step_shape<R, true, true>(sh, a, s) : launch_step_shape<R, true, false>(sh, a, s);
    return has_v ? launch_step_shape<R, false, true>(sh, a, s) : launch_step_shape<R, false, false>(sh, a, s);
}

// Arguments of one whole step from `src` to `dst` (state buffers) with shape sh.
template <typename R>
static StepArgs<R> step_args(const phx_handle* h, const StepShapeId& sh, const void* src, const void* src_n,
                             void* dst, void* dst_n)
{
    using C = typename cvec<R>::type;
    const phx_config& c = h->cfg;
    StepArgs<R> a{};
    a.nx = c.nx;
    a.ny = c.ny;
    a.bcx = c.bc_x;
    a.bcy = c.bc_y;
    a.tiles_x = (c.nx + 55) / 56;
    if (wide_shape(sh.waves)) {  // wide streaming: strips of 120 columns, one wave per band of a strip
        a.tiles_x = wide_strips(c.nx);
        a.band_rows = wide_band_rows(c, sh, h->f.V != nullptr, h->cus);
        a.tiles = a.tiles_x * ((c.ny + a.band_rows - 1) / a.band_rows);
    } else if (sh.waves == 1) {  // streaming: strips of 56 columns, workgroups of 4 strips x one band
        a.tiles = ((a.tiles_x + 3) / 4) * ((c.ny + sh.rows - 1) / sh.rows);
    } else {
        const int oh = sh.waves * sh.rows - 8;
        a.tiles = a.tiles_x * ((c.ny + oh - 1) / oh);
    }
    a.c = make_coef<R>(c);
    a.half_dt = (R)(0.5 * c.dt);
    a.dt = (R)c.dt;
    a.dt6 = (R)(c.dt / 6.0);
    a.V = (const R*)h->f.V;
    a.P = (const R*)h->f.P;
    a.flag = (unsigned int*)(h->ws + h->L.flag);
    a.psi_in = (const C*)src;
    a.n_in = (const R*)src_n;
    a.psi_out = (C*)dst;
    a.n_out = (R*)dst_n;
    a.comps = c.components;
    if (c.imag_time) {
        a.imag_slots = (const double*)(h->ws + h->L.imag);
        a.imag_partials = (double*)(h->ws + h->L.imag_partials);
    }
    if (c.drive) {
        a.E = (const C*)h->f.E;
        a.drive_ph = (const C*)(h->ws + h->L.drive_ph);
    }
    return a;
}

// Trial launch k of the tuner.  k = 0 steps the caller's state into the workspace
// copy; later trials alternate between the two workspace copies, so that each one
// reads the state the previous one wrote, as real steps do (a launch that re-read one
// unchanged input would find part of it in the Infinity Cache).  The caller's state
// is never written.
template <typename R>
hipError_t rk4_step_trial(phx_handle* h, const StepShapeId& sh, int k)
{
    const bool res = h->cfg.reservoir != 0;
    char* A = h->ws + h->L.alt;
    char* An = res ? h->ws + h->L.alt_n : nullptr;
    char* B = h->ws + h->L.alt2;
    char* Bn = res ? h->ws + h->L.alt2_n : nullptr;
    StepArgs<R> a;
    if (k == 0)
        a = step_args<R>(h, sh, h->f.psi, h->f.n, A, An);
    else if (k & 1)
        a = step_args<R>(h, sh, A, An, B, Bn);
    else
        a = step_args<R>(h, sh, B, Bn, A, An);
    return launch_rk4_step<R>(res, h->f.V != nullptr, sh, a, h->stream);
}

template hipError_t rk4_step_trial<float>(phx_handle*, const StepShapeId&, int);
template hipError_t rk4_step_trial<double>(phx_handle*, const StepShapeId&, int);

// Enqueues n whole steps on stream s, alternating between the caller's arrays
// (buffer 0) and the workspace copy (buffer 1); h->step_parity is the buffer that
// holds the state before the first of them.
template <typename R>
phx_status rk4_fused_launches(phx_handle* h, int64_t n, hipStream_t s)
{
    const phx_config& c = h->cfg;
    void* S[2] = {h->f.psi, h->ws + h->L.alt};
    void* SN[2] = {h->f.n, c.reservoir ? h->ws + h->L.alt_n : nullptr};
    const bool res = c.reservoir != 0, hv = h->f.V != nullptr;
    const StepShapeId sh = h->step_shape;
    const bool fused_noise = c.noise > 0.0 && noise_in_step(c, sh);
    int cur = h->step_parity;
    for (int64_t k = 0; k < n; ++k) {
        StepArgs<R> a = step_args<R>(h, sh, S[cur], SN[cur], S[cur ^ 1], SN[cur ^ 1]);
        a.check = k == n - 1;  // the wide form tests the last step of the run (values stay non-finite)
        if (fused_noise) {
            a.noise_step = (const uint64_t*)(h->ws + h->L.noise);
            a.noise_offset = k;
            noise_coefs<R>(c, a.noise_a, a.noise_b, a.noise_k0, a.noise_k1);
        }
        if (c.drive && launch_drive_phasors<R>(h, k, s) != hipSuccess)
            return fail(PHX_EHIP, "drive phasor launch failed");
        hipEvent_t t0 = nullptr;
        hipError_t e = timing_begin(h, &t0);
        if (e == hipSuccess) e = launch_rk4_step<R>(res, hv, sh, a, s);
        if (e == hipSuccess) e = timing_end(h, t0, K_RK4_STEP);
        if (e != hipSuccess) return fail(PHX_EHIP, "RK4 step kernel launch: %s", hipGetErrorString(e));
        cur ^= 1;
        if (c.imag_time) {  // the scale that restores the norm, applied by the next step
            e = timing_begin(h, &t0);
            // one norm partial per wave: 4 per workgroup of the one-column walk, 1 for the wide
            if (e == hipSuccess) e = launch_imag_finish(h, wide_shape(sh.waves) ? a.tiles : 4 * a.tiles, s);
            if (e == hipSuccess) e = timing_end(h, t0, K_IMAG_NORM);
            if (e != hipSuccess) return fail(PHX_EHIP, "imaginary-time norm launch: %s", hipGetErrorString(e));
        }
        if (c.noise > 0.0 && !fused_noise) {
            e = timing_begin(h, &t0);
            if (e == hipSuccess) e = launch_noise<R>(h, S[cur], SN[cur], k, s);
            if (e == hipSuccess) e = timing_end(h, t0, K_NOISE);
            if (e != hipSuccess) return fail(PHX_EHIP, "noise launch: %s", hipGetErrorString(e));
        }
    }
    h->step_parity = cur;
    if (uses_step_index(c) && n > 0 && advance_noise_step(h, n, s) != hipSuccess)
        return fail(PHX_EHIP, "step index advance launch failed");
    return PHX_OK;
}

template phx_status rk4_fused_launches<float>(phx_handle*, int64_t, hipStream_t);
template phx_status rk4_fused_launches<double>(phx_handle*, int64_t, hipStream_t);

// n whole steps ending in the caller's arrays.  An odd count first copies the state
// into the workspace and takes one step back; the remaining even count alternates
// (graph replays of an even chunk start and end in the caller's arrays).
template <typename R>
phx_status rk4_fused_steps(phx_handle* h, int64_t n)
{
    const phx_config& c = h->cfg;
    const size_t rs = sizeof(R);
    const size_t cells = (size_t)c.nx * c.ny;
    h->step_parity = 0;
    if (n & 1) {
        void* alt = h->ws + h->L.alt;
        if (hipMemcpyAsync(alt, h->f.psi, cells * c.components * 2 * rs, hipMemcpyDeviceToDevice, h->stream) !=
                hipSuccess ||
            (c.reservoir && hipMemcpyAsync(h->ws + h->L.alt_n, h->f.n, cells * c.components * rs, hipMemcpyDeviceToDevice,
                                           h->stream) != hipSuccess))
            return fail(PHX_EHIP, "state copy failed");
        h->step_parity = 1;
        phx_status st = rk4_fused_launches<R>(h, 1, h->stream);
        if (st != PHX_OK) return st;
        --n;
    }
    return rk4_run_graph<R>(h, n);
}

template phx_status rk4_fused_steps<float>(phx_handle*, int64_t);
template phx_status rk4_fused_steps<double>(phx_handle*, int64_t);

}  // namespace phx
