// Device code of the whole-step RK4 kernel, shared by the single-grid launch and the
// batched persistent launch.
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
#pragma once

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

// value held by lane-1 (lane 0 receives 0) and by lane+1 (lane 63 receives 0):
// DPP wave shifts by one lane; out-of-range lanes read 0 (bound control).
__device__ __forceinline__ float lane_prev(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float lane_next(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double lane_prev(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x138, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_next(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x130, 0xf, 0xf, true);
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

// One whole RK4 step of the region `tile` of the grid described by `a`, computed
// by the WAVES waves of the calling workgroup; `edge` is the workgroup's LDS
// exchange buffer.  Returns true (in every lane that stored a cell) when a stored
// value is not finite.  Every thread of the workgroup must call it (barriers).
template <typename R, bool RES, bool HASV, bool GHOSTS, int WAVES, int ROWS>
__device__ __forceinline__ bool step_region(const StepArgs<R>& a, int tile,
                                            typename cvec<R>::type (&edge)[2][WAVES][2][64])
{
    using C = typename cvec<R>::type;
    constexpr int H = WAVES * ROWS;
    constexpr int OW = 56, OH = H - 8;

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
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
        const bool g = GHOSTS && (ci < 0 || rj < 0);
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
            // Stage s only feeds the rows [s, H-s) of the region that the output
            // rows depend on; the branch is uniform over the wave.
            const int r = wave * ROWS + k;
            if (r < s || r >= H - s) {
                prev = cur;
                continue;
            }
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
            const bool g = GHOSTS && ((ghost >> k) & 1u);
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
            y[k] = (GHOSTS && g) ? czero<C>() : nv;
            if (RES) yn[k] = (GHOSTS && g) ? R(0) : nnv;
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
    return bad;
}

}  // namespace phx
