// Adaptive Dormand-Prince 5(4) stepping, named in Sec. 2 as the adaptive
// alternative to RK4.  Tableau: Dormand & Prince, J. Comput. Appl. Math. 6 (1980),
// method RK5(4)7M; step-size control as in Hairer, Norsett & Wanner, Solving ODEs I,
// Sec. II.4.
//
// One launch per stage.  Stage s (1..6) evaluates K_s = f(y_s) with the stencil
// window over its stage argument y_s, stores K_s, and forms the next stage argument
// at its own cell, y_{s+1} = psi + sum_{j<=s} (dt a_{s+1,j}) K_j, reading K_1..K_{s-1}
// there.  y_7 is the fifth-order solution and goes to the second state buffer.
// Stage 7 evaluates K_7 = f(y_7) (first-same-as-last: it is K_1 of the next step
// when the step is accepted) and the embedded error e = sum_j dt (b_j - bhat_j) K_j,
// whose weighted squares are reduced in double precision per workgroup.  A second
// pass sums the partials in a fixed order; the host reads the norm, accepts or
// rejects, and adapts dt.  After an attempt the next attempt starts from a
// pointwise kernel that forms y_2 from the state and K_1.
#include <math.h>
#include <string.h>

#include "runtime.h"
#include "stencil.h"

namespace phx {

// Dormand-Prince RK5(4)7M coefficients (rows of A, fifth- and fourth-order weights).
static const double DP_A[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5.0, 0, 0, 0, 0, 0},
    {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0, 0},
    {44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0, 0, 0, 0},
    {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0, 0, 0},
    {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0, 0},
    {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0},
};
static const double DP_B[7] = {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0,
                               -2187.0 / 6784.0, 11.0 / 84.0, 0.0};
static const double DP_BHAT[7] = {5179.0 / 57600.0, 0.0, 7571.0 / 16695.0, 393.0 / 640.0,
                                  -92097.0 / 339200.0, 187.0 / 2100.0, 1.0 / 40.0};
// nodes: stage s is evaluated at t + c_s dt (the coherent drive's phase)
static const double DP_C[7] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 4.0 / 5.0, 8.0 / 9.0, 1.0, 1.0};

template <typename R>
struct DpArgs {
    using C = typename cvec<R>::type;
    int nx, ny, bcx, bcy, comps;
    int tiles_x, tiles;
    TileShape ts;
    int64_t cstride;
    Coef<R> c;
    const C* y;  const R* yn;     // stage argument y_s
    const C* psi; const R* n;     // state at the start of the attempt
    const R* V;  const R* P;
    C* k[7];  R* kn[7];           // K_1..K_7
    C* y_out; R* yn_out;          // y_{s+1}
    R ca[6];                      // dt a_{s+1,j}, j = 1..s
    R ce[7];                      // dt (b_j - bhat_j)
    double rtol, atol;
    double* partials;             // stage 7: one double per workgroup
    const C* E;                   // drive profile, or NULL
    C drive_ph;                   // exp(-i omega t_s) at this stage's time
};

__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

template <typename R, int COMPS, bool RES, bool HASV, int STAGE>
__global__ __launch_bounds__(256) void dp_stage_kernel(const DpArgs<R> a)
{
    using C = typename cvec<R>::type;
    __shared__ double lds[4];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = tile % a.tiles_x;
    const int ty = tile / a.tiles_x;
    const int wxi = wave % a.ts.wx;
    const int wyi = wave / a.ts.wx;
    const int i = (tx * a.ts.wx + wxi) * 64 + lane;
    const int j0 = (ty * (4 / a.ts.wx) + wyi) * a.ts.rows;
    const int cs = (int)a.cstride;
    double err = 0.0;
    if (i < a.nx && j0 < a.ny) {
        const int j1 = min(j0 + a.ts.rows, a.ny);
        const Cols q = make_cols(i, a.nx, a.bcx);
        Row3<C> U[COMPS], M[COMPS], D[COMPS];
#pragma unroll
        for (int s = 0; s < COMPS; ++s) {
            U[s] = load_row(a.y + s * cs, j0 - 1, a.nx, a.ny, a.bcy, q);
            M[s] = load_row(a.y + s * cs, j0, a.nx, a.ny, a.bcy, q);
        }
        for (int j = j0; j < j1; ++j) {
#pragma unroll
            for (int s = 0; s < COMPS; ++s) D[s] = load_row(a.y + s * cs, j + 1, a.nx, a.ny, a.bcy, q);
            const int idx = j * a.nx + i;
            R nn[COMPS];
#pragma unroll
            for (int s = 0; s < COMPS; ++s) nn[s] = RES ? a.yn[s * cs + idx] : R(0);
            const R v = HASV ? a.V[idx] : R(0);
            C f[COMPS];
            R rho[COMPS];
            rhs_cell<R, COMPS, HASV>(a.c, U, M, D, nn, v, f, rho);
            if (a.E) {
#pragma unroll
                for (int s = 0; s < COMPS; ++s) add_drive(f[s], a.E[s * cs + idx], a.drive_ph, a.c.inv_hbar);
            }
#pragma unroll
            for (int s = 0; s < COMPS; ++s) {
                const int o = s * cs + idx;
                R fn = R(0);
                if (RES) fn = a.P[o] - (a.c.gamma_r + a.c.R_ * rho[s]) * nn[s];
                a.k[STAGE - 1][o] = f[s];
                if (RES) a.kn[STAGE - 1][o] = fn;
                if (STAGE < 7) {
                    // y_{s+1} = psi + sum_{j<s} ca_j K_j + ca_s K_s
                    C acc = a.psi[o];
#pragma unroll
                    for (int jj = 0; jj < STAGE - 1; ++jj) {
                        const C kj = a.k[jj][o];
                        acc.x += a.ca[jj] * kj.x;
                        acc.y += a.ca[jj] * kj.y;
                    }
                    acc.x += a.ca[STAGE - 1] * f[s].x;
                    acc.y += a.ca[STAGE - 1] * f[s].y;
                    a.y_out[o] = acc;
                    if (RES) {
                        R an = a.n[o];
#pragma unroll
                        for (int jj = 0; jj < STAGE - 1; ++jj) an += a.ca[jj] * a.kn[jj][o];
                        a.yn_out[o] = an + a.ca[STAGE - 1] * fn;
                    }
                } else {
                    // embedded error e = sum_j dt (b_j - bhat_j) K_j  (b_2 = bhat_2 = 0)
                    C e = C{a.ce[6] * f[s].x, a.ce[6] * f[s].y};
#pragma unroll
                    for (int jj = 0; jj < 6; ++jj) {
                        if (jj == 1) continue;
                        const C kj = a.k[jj][o];
                        e.x += a.ce[jj] * kj.x;
                        e.y += a.ce[jj] * kj.y;
                    }
                    const C p0 = a.psi[o];
                    const C p1 = M[s].c;
                    const double m0 = sqrt((double)p0.x * p0.x + (double)p0.y * p0.y);
                    const double m1 = sqrt((double)p1.x * p1.x + (double)p1.y * p1.y);
                    const double sc = a.atol + a.rtol * fmax(m0, m1);
                    err += ((double)e.x * e.x + (double)e.y * e.y) / (sc * sc);
                    if (RES) {
                        R en = a.ce[6] * fn;
#pragma unroll
                        for (int jj = 0; jj < 6; ++jj) {
                            if (jj == 1) continue;
                            en += a.ce[jj] * a.kn[jj][o];
                        }
                        const double sn = a.atol + a.rtol * fmax(fabs((double)a.n[o]), fabs((double)nn[s]));
                        err += (double)en * en / (sn * sn);
                    }
                }
            }
#pragma unroll
            for (int s = 0; s < COMPS; ++s) {
                U[s] = M[s];
                M[s] = D[s];
            }
        }
    }
    if (STAGE == 7) {
        // every thread reaches this point (no early return), so the barrier is safe
        err = wave_sum_d(err);
        if (lane == 0) lds[wave] = err;
        __syncthreads();
        if (threadIdx.x == 0) a.partials[blockIdx.x] = ((lds[0] + lds[1]) + lds[2]) + lds[3];
    }
}

// y_2 = psi + dt a_21 K_1 at every cell (restart of an attempt from K_1).
template <typename R, bool RES>
__global__ __launch_bounds__(256) void dp_restart_kernel(const DpArgs<R> a, int cells)
{
    using C = typename cvec<R>::type;
    const int o = blockIdx.x * 256 + threadIdx.x;
    if (o >= cells) return;
    const C p = a.psi[o];
    const C k = a.k[0][o];
    a.y_out[o] = C{p.x + a.ca[0] * k.x, p.y + a.ca[0] * k.y};
    if (RES) a.yn_out[o] = a.n[o] + a.ca[0] * a.kn[0][o];
}

// Fixed-order sum of the per-workgroup error partials: one workgroup.
__global__ __launch_bounds__(256) void dp_err_sum_kernel(const double* __restrict__ partials, int blocks,
                                                         double* __restrict__ out)
{
    __shared__ double lds[4];
    double s = 0.0;
    for (int b = threadIdx.x; b < blocks; b += 256) s += partials[b];
    s = wave_sum_d(s);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = ((lds[0] + lds[1]) + lds[2]) + lds[3];
}

template <typename R, int COMPS, bool RES, bool HASV>
static hipError_t launch_dp_t(int stage, const DpArgs<R>& a, hipStream_t s)
{
    const dim3 grid(a.tiles), block(256);
    switch (stage) {
    case 1: dp_stage_kernel<R, COMPS, RES, HASV, 1><<<grid, block, 0, s>>>(a); break;
    case 2: dp_stage_kernel<R, COMPS, RES, HASV, 2><<<grid, block, 0, s>>>(a); break;
    case 3: dp_stage_kernel<R, COMPS, RES, HASV, 3><<<grid, block, 0, s>>>(a); break;
    case 4: dp_stage_kernel<R, COMPS, RES, HASV, 4><<<grid, block, 0, s>>>(a); break;
    case 5: dp_stage_kernel<R, COMPS, RES, HASV, 5><<<grid, block, 0, s>>>(a); break;
    case 6: dp_stage_kernel<R, COMPS, RES, HASV, 6><<<grid, block, 0, s>>>(a); break;
    default: dp_stage_kernel<R, COMPS, RES, HASV, 7><<<grid, block, 0, s>>>(a); break;
    }
    return hipGetLastError();
}

template <typename R>
static hipError_t launch_dp(int stage, bool res, bool hv, const DpArgs<R>& a, hipStream_t s)
{
    if (a.comps == 1) {
        if (res) return hv ? launch_dp_t<R, 1, true, true>(stage, a, s) : launch_dp_t<R, 1, true, false>(stage, a, s);
        return hv ? launch_dp_t<R, 1, false, true>(stage, a, s) : launch_dp_t<R, 1, false, false>(stage, a, s);
    }
    if (res) return hv ? launch_dp_t<R, 2, true, true>(stage, a, s) : launch_dp_t<R, 2, true, false>(stage, a, s);
    return hv ? launch_dp_t<R, 2, false, true>(stage, a, s) : launch_dp_t<R, 2, false, false>(stage, a, s);
}

// ------------------------------------------------------------------ host side

#define HIP_OR_FAIL(call)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) return fail(PHX_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

static size_t complex_bytes(const phx_handle* h)
{
    const size_t rs = h->cfg.precision == PHX_C64 ? 4 : 8;
    return (size_t)h->cfg.nx * h->cfg.ny * h->cfg.components * 2 * rs;
}

static size_t real_bytes(const phx_handle* h)
{
    const size_t rs = h->cfg.precision == PHX_C64 ? 4 : 8;
    return (size_t)h->cfg.nx * h->cfg.ny * h->cfg.components * rs;
}

// Per-handle Dormand-Prince buffers inside the workspace: 7 K arrays, two stage
// arguments and a second state, each for psi and (with the reservoir) n.
struct DpBuffers {
    char* k[7];
    char* kn[7];
    char* ys[2];
    char* yns[2];
    char* alt;
    char* alt_n;
    double* partials;
    double* err;
};

static DpBuffers dp_buffers(const phx_handle* h)
{
    DpBuffers b{};
    const Layout& L = h->L;
    const size_t cb = align_up(complex_bytes(h)), rb = align_up(real_bytes(h));
    char* base = h->ws + L.k[0];
    for (int s = 0; s < 7; ++s) b.k[s] = base + s * cb;
    b.ys[0] = base + 7 * cb;
    b.ys[1] = base + 8 * cb;
    b.alt = base + 9 * cb;
    char* nb = base + 10 * cb;
    if (h->cfg.reservoir) {
        for (int s = 0; s < 7; ++s) b.kn[s] = nb + s * rb;
        b.yns[0] = nb + 7 * rb;
        b.yns[1] = nb + 8 * rb;
        b.alt_n = nb + 9 * rb;
    }
    b.partials = (double*)(h->ws + L.err);
    b.err = (double*)(h->ws + L.obs);  // the observables slot doubles as the norm output
    return b;
}

// Buffer slot of K_s (s = 1..7) when K_1 sits in slot fsal: the other six slots
// follow in increasing order.
static void dp_slots(int fsal, int (&slot)[7])
{
    slot[0] = fsal;
    for (int s = 1, q = 0; s < 7; ++s, ++q) {
        if (q == fsal) ++q;
        slot[s] = q;
    }
}

template <typename R>
static phx_status dp_attempt(phx_handle* h, double dt, bool need_k1, double* err_out)
{
    using C = typename cvec<R>::type;
    const phx_config& c = h->cfg;
    const DpBuffers b = dp_buffers(h);
    const bool res = c.reservoir != 0, hv = h->f.V != nullptr;
    DpArgs<R> a{};
    a.nx = c.nx;
    a.ny = c.ny;
    a.bcx = c.bc_x;
    a.bcy = c.bc_y;
    a.comps = c.components;
    a.tiles_x = h->L.tiles.tiles_x;
    a.tiles = h->L.tiles.tiles;
    a.ts = h->L.tiles.ts;
    a.cstride = (int64_t)c.nx * c.ny;
    a.c = make_coef<R>(c);
    a.V = (const R*)h->f.V;
    a.P = (const R*)h->f.P;
    a.psi = (const C*)h->cur;
    a.n = (const R*)h->cur_n;
    int slot[7];
    dp_slots(h->fsal, slot);
    for (int s = 0; s < 7; ++s) {
        a.k[s] = (C*)b.k[slot[s]];
        a.kn[s] = res ? (R*)b.kn[slot[s]] : nullptr;
    }
    for (int j = 0; j < 7; ++j) a.ce[j] = (R)(dt * (DP_B[j] - DP_BHAT[j]));
    a.rtol = c.rtol;
    a.atol = c.atol;
    a.partials = b.partials;
    a.E = c.drive ? (const C*)h->f.E : nullptr;
    auto set_phasor = [&](int s) {  // exp(-i omega t_s) at the time of stage s (1..7)
        if (!c.drive) return;
        const double th = c.drive_omega * (h->info.t + DP_C[s - 1] * dt);
        a.drive_ph = C{(R)cos(th), (R)-sin(th)};
    };
    const int cells = c.nx * c.ny * c.components;
    hipEvent_t t0 = nullptr;
    hipError_t e = hipSuccess;
    auto set_ca = [&](int s) {  // coefficients of y_{s+1}
        for (int j = 0; j < 6; ++j) a.ca[j] = (R)(j < s ? dt * DP_A[s][j] : 0.0);
    };
    // stage 1 (only when K_1 of the current state is unknown) or the restart kernel
    set_ca(1);
    a.y_out = (C*)b.ys[0];
    a.yn_out = res ? (R*)b.yns[0] : nullptr;
    if (need_k1) {
        a.y = (const C*)h->cur;
        a.yn = (const R*)h->cur_n;
        set_phasor(1);
        e = timing_begin(h, &t0);
        if (e == hipSuccess) e = launch_dp<R>(1, res, hv, a, h->stream);
        if (e == hipSuccess) e = timing_end(h, t0, K_DP_S1);
    } else {
        e = timing_begin(h, &t0);
        if (e == hipSuccess) {
            const int blocks = (cells + 255) / 256;
            if (res) dp_restart_kernel<R, true><<<blocks, 256, 0, h->stream>>>(a, cells);
            else dp_restart_kernel<R, false><<<blocks, 256, 0, h->stream>>>(a, cells);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = timing_end(h, t0, K_DP_S1);
    }
    if (e != hipSuccess) return fail(PHX_EHIP, "Dormand-Prince stage 1: %s", hipGetErrorString(e));
    for (int s = 2; s <= 7; ++s) {
        a.y = (const C*)(s == 7 ? h->other : b.ys[(s - 2) & 1]);
        a.yn = res ? (const R*)(s == 7 ? h->other_n : b.yns[(s - 2) & 1]) : nullptr;
        if (s < 7) {
            set_ca(s);
            a.y_out = (C*)(s == 6 ? h->other : b.ys[(s - 1) & 1]);
            a.yn_out = res ? (R*)(s == 6 ? h->other_n : b.yns[(s - 1) & 1]) : nullptr;
        }
        set_phasor(s);
        e = timing_begin(h, &t0);
        if (e == hipSuccess) e = launch_dp<R>(s, res, hv, a, h->stream);
        if (e == hipSuccess) e = timing_end(h, t0, K_DP_S1 + s - 1);
        if (e != hipSuccess) return fail(PHX_EHIP, "Dormand-Prince stage %d: %s", s, hipGetErrorString(e));
    }
    e = timing_begin(h, &t0);
    if (e == hipSuccess) {
        dp_err_sum_kernel<<<1, 256, 0, h->stream>>>(b.partials, a.tiles, b.err);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = timing_end(h, t0, K_DP_ERR);
    if (e != hipSuccess) return fail(PHX_EHIP, "Dormand-Prince error sum: %s", hipGetErrorString(e));
    HIP_OR_FAIL(hipMemcpyAsync(&h->host[OBS_SLOTS + 1], b.err, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_OR_FAIL(hipStreamSynchronize(h->stream));
    const double real_unknowns = 2.0 * cells + (res ? (double)cells : 0.0);
    *err_out = sqrt(h->host[OBS_SLOTS + 1] / real_unknowns);
    return PHX_OK;
}

phx_status create_rk45(phx_handle* h)
{
    const DpBuffers b = dp_buffers(h);
    h->cur = h->f.psi;
    h->cur_n = h->f.n;
    h->other = b.alt;
    h->other_n = b.alt_n;
    h->fsal = 0;
    h->k1_valid = false;
    h->info.dt = h->cfg.dt;
    return PHX_OK;
}

// Copies the state back into the caller's arrays when it lives in the workspace.
static phx_status settle_state(phx_handle* h)
{
    if (h->cur == h->f.psi) return PHX_OK;
    HIP_OR_FAIL(hipMemcpyAsync(h->f.psi, h->cur, complex_bytes(h), hipMemcpyDeviceToDevice, h->stream));
    if (h->cfg.reservoir)
        HIP_OR_FAIL(hipMemcpyAsync(h->f.n, h->cur_n, real_bytes(h), hipMemcpyDeviceToDevice, h->stream));
    h->other = h->cur;
    h->other_n = h->cur_n;
    h->cur = h->f.psi;
    h->cur_n = h->f.n;
    return PHX_OK;
}

phx_status step_rk45(phx_handle* h, int64_t n, phx_info* out)
{
    const phx_config& c = h->cfg;
    int64_t done = 0;
    phx_status st = PHX_OK;
    while (done < n) {
        const double dt = h->info.dt;
        if (!(dt >= c.dt_min)) {
            st = fail(PHX_EDTMIN, "step size %g fell below dt_min %g after %lld accepted steps", dt, c.dt_min,
                      (long long)h->info.steps_accepted);
            break;
        }
        double err = 0.0;
        st = c.precision == PHX_C64 ? dp_attempt<float>(h, dt, !h->k1_valid, &err)
                                    : dp_attempt<double>(h, dt, !h->k1_valid, &err);
        if (st != PHX_OK) break;
        h->k1_valid = true;  // K_1 of the current state now sits in slot fsal
        if (h->att_log && *h->att_count >= 0 && *h->att_count < h->att_cap) {
            double* e = h->att_log + 3 * *h->att_count;
            e[0] = dt;
            e[1] = err;
            e[2] = err <= 1.0 ? 1.0 : 0.0;
            *h->att_count += 1;
        }
        const double fmax_ = h->info.last_rejected ? 1.0 : 5.0;
        double fac;
        if (!isfinite(err)) fac = 0.2;
        else if (err > 0.0) fac = 0.9 * pow(err, -0.2);
        else fac = fmax_;
        if (fac < 0.2) fac = 0.2;
        if (fac > fmax_) fac = fmax_;
        if (err <= 1.0) {
            // accept: the fifth-order solution becomes the state, K_7 becomes K_1
            void* t = h->cur;
            h->cur = h->other;
            h->other = t;
            t = h->cur_n;
            h->cur_n = h->other_n;
            h->other_n = t;
            int slot[7];
            dp_slots(h->fsal, slot);
            h->fsal = slot[6];
            h->info.t += dt;
            h->info.steps_accepted += 1;
            h->info.last_rejected = 0;
            ++done;
        } else {
            h->info.steps_rejected += 1;
            h->info.last_rejected = 1;
        }
        h->info.dt = fmin(dt * fac, c.dt_max);
    }
    phx_status s2 = settle_state(h);
    if (st == PHX_OK) st = s2;
    if (out) *out = h->info;
    return st;
}

phx_status set_info_rk45(phx_handle* h, const phx_info* in)
{
    // the caller may have replaced the state: K_1 must be recomputed
    phx_status s = settle_state(h);
    if (s != PHX_OK) return s;
    h->info = *in;
    h->k1_valid = false;
    return PHX_OK;
}

}  // namespace phx
