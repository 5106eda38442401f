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
    // imaginary time (streaming form only): the input is scaled by imag_slots[1]
    // as it is read, and each wave writes the FP64 norm partial of the cells it stores
    const double* imag_slots;
    double* imag_partials;
    // coherent drive (streaming form only): profile [ny][nx] and the phasors
    // exp(-i omega t_s) of the four stage times of this step
    const C* E;
    const C* drive_ph;
    int comps;  // 2: the spinor streaming kernel (component stride nx*ny)
    int band_rows;        // wide streaming form: rows per band (a launch argument)
    int check;            // wide streaming form: test the stored values for non-finite ones
    // wide streaming form with the Wiener increment added before the final store
    // (null: no noise): step index *noise_step + noise_offset, variance a n + b, key
    const uint64_t* noise_step;
    int64_t noise_offset;
    R noise_a, noise_b;
    uint32_t noise_k0, noise_k1;
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

// native two-element vector of R (the store builtins take these, not the HIP structs)
template <typename R>
using rvec2 = R __attribute__((ext_vector_type(2)));

// index of grid coordinate g under the boundary rule; -1 for a ghost (zero boundary)
__device__ __forceinline__ int wrap_any(int g, int n, int bc)
{
    if (g >= 0 && g < n) return g;
    if (bc != PHX_BC_PERIODIC) return -1;
    const int m = g % n;
    return m < 0 ? m + n : m;
}

// The four stages of one region, run by one wave over its ROWS rows.  EDGE waves
// hold region rows that some stage skips (the first and last 4 rows of the region);
// the other waves run every row of every stage with no per-row test, so that the
// unrolled code has no branch joins (and no register copies at them).
//
// Per cell, with p = the stage argument, lr / ud the sums of its left+right and
// up+down neighbours, and kv = V/hbar + 2 (ax + ay) held for the whole step:
//   om = kv + g_r/hbar n + g/hbar |p|^2,   u = (R n - gamma_c)/2,
//   f.x = u p.x + om p.y - (ax lr.y + ay ud.y)
//   f.y = u p.y - om p.x + (ax lr.x + ay ud.x)
// which is i (hbar/2m) Lap p + (u - i w) p of Eq. (1) / Eq. (PULSE_psi) with the
// -2(ax+ay) p centre term of the five-point Laplacian folded into om.
template <typename R, bool RES, bool HASV, bool GHOSTS, int WAVES, int ROWS, bool EDGE>
__device__ __forceinline__ void step_stages(const StepArgs<R>& a, int lane, int wave,
                                            unsigned int ghost,
                                            const typename cvec<R>::type (&p0)[ROWS],
                                            typename cvec<R>::type (&y)[ROWS],
                                            const R (&n0)[ROWS], R (&yn)[ROWS],
                                            const R (&pp)[ROWS], const R (&kv)[ROWS],
                                            typename cvec<R>::type (&edge)[2][WAVES][2][64])
{
    using C = typename cvec<R>::type;
    constexpr int H = WAVES * ROWS;
    const Coef<R>& c = a.c;
    C acc[ROWS];
    R accn[ROWS];
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
            if (EDGE) {
                // stage s only feeds the region rows [s, H-s) that the output depends on
                const int r = wave * ROWS + k;
                if (r < s || r >= H - s) {
                    prev = cur;
                    continue;
                }
            }
            const R lrx = lane_prev(cur.x) + lane_next(cur.x);
            const R lry = lane_prev(cur.y) + lane_next(cur.y);
            const R udx = prev.x + nxt.x;
            const R udy = prev.y + nxt.y;
            const R rho = fma(cur.x, cur.x, cur.y * cur.y);
            R om = kv[k];
            if (RES) om = fma(c.grh, yn[k], om);
            om = fma(c.gh, rho, om);
            const R u = RES ? fma(c.half_R, yn[k], -c.half_gamma) : -c.half_gamma;
            const R tx = fma(c.ax, lrx, c.ay * udx);
            const R ty = fma(c.ax, lry, c.ay * udy);
            const R fx = fma(u, cur.x, fma(om, cur.y, -ty));
            const R fy = fma(u, cur.y, fma(-om, cur.x, tx));
            R fn = R(0);
            if (RES) fn = fma(-fma(c.R_, rho, c.gamma_r), yn[k], pp[k]);
            C nv;
            R nnv = R(0);
            if (s == 1) {
                acc[k] = C{fx, fy};
                if (RES) accn[k] = fn;
            } else if (s < 4) {
                acc[k] = C{fma(R(2), fx, acc[k].x), fma(R(2), fy, acc[k].y)};
                if (RES) accn[k] = fma(R(2), fn, accn[k]);
            }
            if (s < 4) {
                nv = C{fma(adt, fx, p0[k].x), fma(adt, fy, p0[k].y)};
                if (RES) nnv = fma(adt, fn, n0[k]);
            } else {
                nv = C{fma(a.dt6, acc[k].x + fx, p0[k].x), fma(a.dt6, acc[k].y + fy, p0[k].y)};
                if (RES) nnv = fma(a.dt6, accn[k] + fn, n0[k]);
            }
            const bool g = GHOSTS && ((ghost >> k) & 1u);
            y[k] = g ? czero<C>() : nv;
            if (RES) yn[k] = g ? R(0) : nnv;
            prev = cur;
        }
    }
}

// What a region's step reads from HBM, per lane and row of the calling wave: the
// state, the pump, the per-cell part of om (kv) and the ghost mask.  Loading it is
// separate from computing so that a persistent workgroup can fetch the next region
// while it computes the current one.
template <typename R, int ROWS>
struct RegionIn {
    typename cvec<R>::type p0[ROWS];
    R n0[ROWS], pp[ROWS], kv[ROWS];
    unsigned int ghost;  // bit k: row k of this lane is a ghost cell
};

// Issues the loads of region `tile` for the calling wave (no barrier, no LDS).
template <typename R, bool RES, bool HASV, bool GHOSTS, int WAVES, int ROWS>
__device__ __forceinline__ void load_region(const StepArgs<R>& a, int tile, RegionIn<R, ROWS>& in)
{
    using C = typename cvec<R>::type;
    constexpr int OW = 56, OH = WAVES * ROWS - 8;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tx = tile % a.tiles_x;
    const int ty = tile / a.tiles_x;
    const int ci = wrap_any(tx * OW - 4 + lane, a.nx, a.bcx);
    const int row0 = ty * OH - 4 + wave * ROWS;
    const R kdiag = R(2) * (a.c.ax + a.c.ay);
    in.ghost = 0;
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
        const int rj = wrap_any(row0 + k, a.ny, a.bcy);
        const bool g = GHOSTS && (ci < 0 || rj < 0);
        in.ghost |= (g ? 1u : 0u) << k;
        const int idx = g ? 0 : rj * a.nx + ci;
        const C v = a.psi_in[idx];
        in.p0[k] = g ? czero<C>() : v;
        if (RES) {
            const R nv = a.n_in[idx];
            const R pv = a.P[idx];
            in.n0[k] = g ? R(0) : nv;
            in.pp[k] = g ? R(0) : pv;
        }
        in.kv[k] = kdiag;
        if (HASV) {
            const R vv_ = a.V[idx];
            in.kv[k] = g ? kdiag : fma(a.c.inv_hbar, vv_, kdiag);
        }
    }
}

// The four stages of region `tile` from its loaded inputs, then the store of its
// interior.  Returns true (in every lane that stored a cell) when a stored value is
// not finite.  Every thread of the workgroup must call it (barriers).
template <typename R, bool RES, bool HASV, bool GHOSTS, int WAVES, int ROWS>
__device__ __forceinline__ bool run_region(const StepArgs<R>& a, int tile, const RegionIn<R, ROWS>& in,
                                           typename cvec<R>::type (&edge)[2][WAVES][2][64])
{
    using C = typename cvec<R>::type;
    constexpr int H = WAVES * ROWS;
    constexpr int OW = 56, OH = H - 8;
    const int lane = threadIdx.x & 63;
    // the wave index is the same in every lane: keep it in a scalar register so that
    // the branches on it below are scalar branches, not lane masks
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tx = tile % a.tiles_x;
    const int ty = tile / a.tiles_x;
    const int gi = tx * OW - 4 + lane;
    const int row0 = ty * OH - 4 + wave * ROWS;

    C y[ROWS];
    R yn[ROWS];
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
        y[k] = in.p0[k];
        yn[k] = RES ? in.n0[k] : R(0);
    }

    // waves whose rows all lie in [4, H-4) run every row of every stage
    if (wave * ROWS >= 4 && (wave + 1) * ROWS <= H - 4)
        step_stages<R, RES, HASV, GHOSTS, WAVES, ROWS, false>(a, lane, wave, in.ghost, in.p0, y, in.n0, yn,
                                                              in.pp, in.kv, edge);
    else
        step_stages<R, RES, HASV, GHOSTS, WAVES, ROWS, true>(a, lane, wave, in.ghost, in.p0, y, in.n0, yn,
                                                             in.pp, in.kv, edge);

    // interior of the region: lanes 4..59, region rows 4..H-5, inside the grid
    bool bad = false;
    if (lane >= 4 && lane < 4 + OW && gi < a.nx) {
#pragma unroll
        for (int k = 0; k < ROWS; ++k) {
            const int r = wave * ROWS + k;
            const int gj = row0 + k;
            if (r >= 4 && r < 4 + OH && gj < a.ny) {
                const int idx = gj * a.nx + gi;
                // non-temporal: the new state is not read again within this step
                __builtin_nontemporal_store(rvec2<R>{y[k].x, y[k].y}, (rvec2<R>*)&a.psi_out[idx]);
                bad = bad || !(isfinite(y[k].x) && isfinite(y[k].y));
                if (RES) {
                    __builtin_nontemporal_store(yn[k], &a.n_out[idx]);
                    bad = bad || !isfinite(yn[k]);
                }
            }
        }
    }
    return bad;
}

// One whole RK4 step of the region `tile` of the grid described by `a`, computed
// by the WAVES waves of the calling workgroup; `edge` is the workgroup's LDS
// exchange buffer.  Every thread of the workgroup must call it (barriers).
template <typename R, bool RES, bool HASV, bool GHOSTS, int WAVES, int ROWS>
__device__ __forceinline__ bool step_region(const StepArgs<R>& a, int tile,
                                            typename cvec<R>::type (&edge)[2][WAVES][2][64])
{
    RegionIn<R, ROWS> in;
    load_region<R, RES, HASV, GHOSTS, WAVES, ROWS>(a, tile, in);
    return run_region<R, RES, HASV, GHOSTS, WAVES, ROWS>(a, tile, in, edge);
}

}  // namespace phx
