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
// Lane l of every wave owns region column l; wave w owns rows [w*ROWS, (w+1)*ROWS).
// x-neighbours come from the adjacent lanes by DPP wave shifts, y-neighbours from
// the lane's own registers except at the wave's first and last row, which are
// exchanged through LDS (double-buffered by stage parity: one barrier per stage).
// Region cells outside a zero boundary are ghost cells held at 0 in every stage;
// with a periodic boundary the region wraps.  The output goes to a second state
// buffer (neighbouring regions still read the input's halo).
#include "runtime.h"
#include "stencil.h"

namespace phx {

template <typename R>
struct StepArgs {
    using C = typename cvec<R>::type;
    int nx, ny, bcx, bcy;
    int tiles_x, tiles;
    Coef<R> c;
    R half_dt, dt, dt6;
    const C* psi_in; const R* n_in;
    C* psi_out; R* n_out;
    const R* V; const R* P;
    unsigned int* flag;
};

// value held by lane-1 (lane 0 receives 0) and by lane+1 (lane 63 receives 0)
__device__ __forceinline__ float lane_prev(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float lane_next(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ double lane_prev(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_next(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x130, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// index of grid coordinate g under the boundary rule; -1 for a ghost (zero boundary)
__device__ __forceinline__ int wrap_any(int g, int n, int bc)
{
    if (g >= 0 && g < n) return g;
    if (bc != PHX_BC_PERIODIC) return -1;
    const int m = g % n;
    return m < 0 ? m + n : m;
}

template <typename R, bool RES, bool HASV, int WAVES, int ROWS>
__global__ __launch_bounds__(WAVES * 64) void rk4_step_kernel(const StepArgs<R> a)
{
    using C = typename cvec<R>::type;
    constexpr int H = WAVES * ROWS;
    constexpr int OW = 56, OH = H - 8;
    __shared__ C edge[2][WAVES][2][64];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = tile % a.tiles_x;
    const int ty = tile / a.tiles_x;
    const int gi = tx * OW - 4 + lane;
    const int ci = wrap_any(gi, a.nx, a.bcx);
    const int row0 = ty * OH - 4 + wave * ROWS;

    C p0[ROWS], y[ROWS], acc[ROWS];
    R n0[ROWS], yn[ROWS], accn[ROWS], pp[ROWS], vv[ROWS];
    unsigned int ghost = 0;  // bit k: row k of this lane is a ghost cell
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
        const int rj = wrap_any(row0 + k, a.ny, a.bcy);
        const bool g = ci < 0 || rj < 0;
        ghost |= (g ? 1u : 0u) << k;
        const int idx = g ? 0 : rj * a.nx + ci;
        const C v = a.psi_in[idx];
        p0[k] = g ? czero<C>() : v;
        if (RES) {
            const R nv = a.n_in[idx];
            const R pv = a.P[idx];
            n0[k] = g ? R(0) : nv;
            pp[k] = g ? R(0) : pv;
        }
        if (HASV) {
            const R vv_ = a.V[idx];
            vv[k] = g ? R(0) : vv_;
        }
        y[k] = p0[k];
        if (RES) yn[k] = n0[k];
    }

#pragma unroll
    for (int s = 1; s <= 4; ++s) {
        const int par = s & 1;
        edge[par][wave][0][lane] = y[0];
        edge[par][wave][1][lane] = y[ROWS - 1];
        __syncthreads();
        C prev = wave > 0 ? edge[par][wave - 1][1][lane] : czero<C>();
        const C below = wave < WAVES - 1 ? edge[par][wave + 1][0][lane] : czero<C>();
        const R adt = (s == 3) ? a.dt : a.half_dt;
#pragma unroll
        for (int k = 0; k < ROWS; ++k) {
            const C cur = y[k];
            const C nxt = (k + 1 < ROWS) ? y[k + 1] : below;
            Row3<C> U[1], M[1], D[1];
            M[0].c = cur;
            M[0].l = C{lane_prev(cur.x), lane_prev(cur.y)};
            M[0].r = C{lane_next(cur.x), lane_next(cur.y)};
            U[0].c = prev;
            D[0].c = nxt;
            U[0].l = U[0].r = D[0].l = D[0].r = czero<C>();  // corners unused by the scalar stencil
            R nn[1] = {RES ? yn[k] : R(0)};
            C f[1];
            R rho[1];
            rhs_cell<R, 1>(a.c, U, M, D, nn, HASV ? vv[k] : R(0), f, rho);
            R fn = R(0);
            if (RES) fn = pp[k] - (a.c.gamma_r + a.c.R_ * rho[0]) * nn[0];
            const bool g = (ghost >> k) & 1u;
            if (s == 1) {
                acc[k] = f[0];
                if (RES) accn[k] = fn;
            } else if (s < 4) {
                acc[k] = C{acc[k].x + R(2) * f[0].x, acc[k].y + R(2) * f[0].y};
                if (RES) accn[k] = accn[k] + R(2) * fn;
            }
            C nv;
            R nnv = R(0);
            if (s < 4) {
                nv = C{p0[k].x + adt * f[0].x, p0[k].y + adt * f[0].y};
                if (RES) nnv = n0[k] + adt * fn;
            } else {
                nv = C{p0[k].x + a.dt6 * (acc[k].x + f[0].x), p0[k].y + a.dt6 * (acc[k].y + f[0].y)};
                if (RES) nnv = n0[k] + a.dt6 * (accn[k] + fn);
            }
            y[k] = g ? czero<C>() : nv;
            if (RES) yn[k] = g ? R(0) : nnv;
            prev = cur;
        }
    }

    // interior of the region: lanes 4..59, region rows 4..H-5, inside the grid
    bool bad = false;
    if (lane >= 4 && lane < 4 + OW && gi < a.nx) {
#pragma unroll
        for (int k = 0; k < ROWS; ++k) {
            const int r = wave * ROWS + k;
            const int gj = row0 + k;
            if (r >= 4 && r < 4 + OH && gj < a.ny) {
                const int idx = gj * a.nx + gi;
                a.psi_out[idx] = y[k];
                bad = bad || !(isfinite(y[k].x) && isfinite(y[k].y));
                if (RES) {
                    a.n_out[idx] = yn[k];
                    bad = bad || !isfinite(yn[k]);
                }
            }
        }
    }
    if (bad) a.flag[0] = 1u;  // benign race: every writer stores 1
}

template <typename R, bool RES, bool HASV, int WAVES, int ROWS>
static hipError_t launch_step_t(const StepArgs<R>& a, hipStream_t s)
{
    rk4_step_kernel<R, RES, HASV, WAVES, ROWS><<<a.tiles, WAVES * 64, 0, s>>>(a);
    return hipGetLastError();
}

// Region height per precision: 8 waves of 8 rows (64) for float, 8 waves of 4 rows
// (32) for double, which keeps the register footprint per lane without spills.
template <typename R> struct StepShape;
template <> struct StepShape<float> { static constexpr int WAVES = 8, ROWS = 8; };
template <> struct StepShape<double> { static constexpr int WAVES = 8, ROWS = 4; };

int step_tile_rows(int precision)
{
    return precision == PHX_C64 ? StepShape<float>::WAVES * StepShape<float>::ROWS - 8
                                : StepShape<double>::WAVES * StepShape<double>::ROWS - 8;
}

template <typename R>
hipError_t launch_rk4_step(bool reservoir, bool has_v, const StepArgs<R>& a, hipStream_t s)
{
    constexpr int W = StepShape<R>::WAVES, K = StepShape<R>::ROWS;
    if (reservoir) return has_v ? launch_step_t<R, true, true, W, K>(a, s) : launch_step_t<R, true, false, W, K>(a, s);
    return has_v ? launch_step_t<R, false, true, W, K>(a, s) : launch_step_t<R, false, false, W, K>(a, s);
}

template <typename R>
phx_status rk4_fused_steps(phx_handle* h, int64_t n)
{
    using C = typename cvec<R>::type;
    const phx_config& c = h->cfg;
    const size_t rs = sizeof(R);
    const size_t cells = (size_t)c.nx * c.ny;
    StepArgs<R> a{};
    a.nx = c.nx;
    a.ny = c.ny;
    a.bcx = c.bc_x;
    a.bcy = c.bc_y;
    const int oh = step_tile_rows(c.precision);
    a.tiles_x = (c.nx + 55) / 56;
    a.tiles = a.tiles_x * ((c.ny + oh - 1) / oh);
    a.c = make_coef<R>(c);
    a.half_dt = (R)(0.5 * c.dt);
    a.dt = (R)c.dt;
    a.dt6 = (R)(c.dt / 6.0);
    a.V = (const R*)h->f.V;
    a.P = (const R*)h->f.P;
    a.flag = (unsigned int*)(h->ws + h->L.flag);
    C* S[2] = {(C*)h->f.psi, (C*)(h->ws + h->L.alt)};
    R* SN[2] = {(R*)h->f.n, c.reservoir ? (R*)(h->ws + h->L.alt_n) : nullptr};
    int cur = 0;
    if (n & 1) {
        // odd count: start from the workspace copy so that the last step lands in
        // the caller's arrays
        if (hipMemcpyAsync(S[1], S[0], cells * 2 * rs, hipMemcpyDeviceToDevice, h->stream) != hipSuccess ||
            (c.reservoir && hipMemcpyAsync(SN[1], SN[0], cells * rs, hipMemcpyDeviceToDevice, h->stream) != hipSuccess))
            return fail(PHX_EHIP, "state copy failed");
        cur = 1;
    }
    const bool res = c.reservoir != 0, hv = h->f.V != nullptr;
    for (int64_t k = 0; k < n; ++k) {
        a.psi_in = S[cur];
        a.n_in = SN[cur];
        a.psi_out = S[cur ^ 1];
        a.n_out = SN[cur ^ 1];
        hipEvent_t t0 = nullptr;
        hipError_t e = timing_begin(h, &t0);
        if (e == hipSuccess) e = launch_rk4_step<R>(res, hv, a, h->stream);
        if (e == hipSuccess) e = timing_end(h, t0, K_RK4_STEP);
        if (e != hipSuccess) return fail(PHX_EHIP, "RK4 step kernel launch: %s", hipGetErrorString(e));
        cur ^= 1;
    }
    return PHX_OK;
}

template phx_status rk4_fused_steps<float>(phx_handle*, int64_t);
template phx_status rk4_fused_steps<double>(phx_handle*, int64_t);

}  // namespace phx
