// Stage-fused RK4 kernels (Eqs. rk4_K1-rk4_final, Sec. 2).
//
// One launch per stage.  Each launch evaluates K_s = f(y_s) (the derivative
// kernel of Sec. 3.2.8: five-point stencil plus the pointwise terms) and folds the
// paper's separate two-term and five-term sums into its epilogue, so that K_s never
// goes to memory:
//   stage 1: acc = K1,          y2 = psi + dt/2 K1
//   stage 2: acc = acc + 2 K2,  y3 = psi + dt/2 K2
//   stage 3: acc = acc + 2 K3,  y4 = psi + dt K3
//   stage 4: psi = psi + dt/6 (acc + K4)   (in place: psi is read only at the centre)
// and likewise for the reservoir n.  The sum order equals that of Eq. rk4_final.
//
// Memory layout and access: a wave owns 64 consecutive columns (one per lane, so
// every load and store of a row is one coalesced 512 B / 1 KiB access) and marches
// down `rows` rows, keeping a 3x3 window of the stage argument in registers: each
// row of the stage argument is fetched once by the wave that marches over it, and
// the column neighbours of a row come from the same or the adjacent cache line.
// No LDS and no barrier is needed; lanes past the grid edge simply exit.
#include "stencil.h"

namespace phx {

template <typename R, int COMPS, bool RES, bool HASV, int STAGE>
__global__ __launch_bounds__(256) void rk4_stage_kernel(const Rk4Args<R> a)
{
    using C = typename cvec<R>::type;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = tile % a.tiles_x;
    const int ty = tile / a.tiles_x;
    const int wxi = wave % a.ts.wx;
    const int wyi = wave / a.ts.wx;
    const int i = (tx * a.ts.wx + wxi) * 64 + lane;
    const int j0 = (ty * (4 / a.ts.wx) + wyi) * a.ts.rows;
    if (i >= a.nx || j0 >= a.ny) return;
    const int j1 = min(j0 + a.ts.rows, a.ny);
    const Cols q = make_cols(i, a.nx, a.bcx);
    const int cs = (int)a.cstride;

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
        if (a.E) {  // uniform over the launch
            const C ph = a.drive_ph[STAGE - 1];
#pragma unroll
            for (int s = 0; s < COMPS; ++s) add_drive(f[s], a.E[s * cs + idx], ph, a.c.inv_hbar);
        }
        if (a.imag) {  // t -> -i tau: d psi/d tau = -i (d psi/dt)
#pragma unroll
            for (int s = 0; s < COMPS; ++s) f[s] = C{f[s].y, -f[s].x};
        }
#pragma unroll
        for (int s = 0; s < COMPS; ++s) {
            const int o = s * cs + idx;
            R fn = R(0);
            if (RES) fn = a.P[o] - (a.c.gamma_r + a.c.R_ * rho[s]) * nn[s];
            if (STAGE == 1) {
                const C p0 = M[s].c;
                a.acc[o] = f[s];
                a.y_out[o] = C{p0.x + a.a_dt * f[s].x, p0.y + a.a_dt * f[s].y};
                if (RES) {
                    a.accn[o] = fn;
                    a.yn_out[o] = nn[s] + a.a_dt * fn;
                }
            } else if (STAGE == 2 || STAGE == 3) {
                const C p0 = a.psi[o];
                const C ac = a.acc[o];
                a.acc[o] = C{ac.x + R(2) * f[s].x, ac.y + R(2) * f[s].y};
                a.y_out[o] = C{p0.x + a.a_dt * f[s].x, p0.y + a.a_dt * f[s].y};
                if (RES) {
                    const R n0 = a.n[o];
                    a.accn[o] = a.accn[o] + R(2) * fn;
                    a.yn_out[o] = n0 + a.a_dt * fn;
                }
            } else {
                const C p0 = a.psi_io[o];
                const C ac = a.acc[o];
                const C p1 = C{p0.x + a.dt6 * (ac.x + f[s].x), p0.y + a.dt6 * (ac.y + f[s].y)};
                a.psi_io[o] = p1;
                bool bad = !(isfinite(p1.x) && isfinite(p1.y));
                if (RES) {
                    const R n1 = a.n_io[o] + a.dt6 * (a.accn[o] + fn);
                    a.n_io[o] = n1;
                    bad = bad || !isfinite(n1);
                }
                if (bad) a.flag[0] = 1u;  // benign race: every writer stores 1
            }
        }
#pragma unroll
        for (int s = 0; s < COMPS; ++s) {
            U[s] = M[s];
            M[s] = D[s];
        }
    }
}

template <typename R, int COMPS, bool RES, bool HASV>
static hipError_t launch_stage_t(int stage, const Rk4Args<R>& a, hipStream_t s)
{
    const dim3 grid(a.tiles), block(256);
    switch (stage) {
    case 1: rk4_stage_kernel<R, COMPS, RES, HASV, 1><<<grid, block, 0, s>>>(a); break;
    case 2: rk4_stage_kernel<R, COMPS, RES, HASV, 2><<<grid, block, 0, s>>>(a); break;
    case 3: rk4_stage_kernel<R, COMPS, RES, HASV, 3><<<grid, block, 0, s>>>(a); break;
    default: rk4_stage_kernel<R, COMPS, RES, HASV, 4><<<grid, block, 0, s>>>(a); break;
    }
    return hipGetLastError();
}

template <typename R>
hipError_t launch_rk4_stage(int stage, bool reservoir, bool has_v, const Rk4Args<R>& a,
                            hipStream_t s)
{
    if (a.comps == 1) {
        if (reservoir) return has_v ? launch_stage_t<R, 1, true, true>(stage, a, s)
                                    : launch_stage_t<R, 1, true, false>(stage, a, s);
        return has_v ? launch_stage_t<R, 1, false, true>(stage, a, s)
                     : launch_stage_t<R, 1, false, false>(stage, a, s);
    }
    if (reservoir) return has_v ? launch_stage_t<R, 2, true, true>(stage, a, s)
                                : launch_stage_t<R, 2, true, false>(stage, a, s);
    return has_v ? launch_stage_t<R, 2, false, true>(stage, a, s)
                 : launch_stage_t<R, 2, false, false>(stage, a, s);
}

template hipError_t launch_rk4_stage<float>(int, bool, bool, const Rk4Args<float>&, hipStream_t);
template hipError_t launch_rk4_stage<double>(int, bool, bool, const Rk4Args<double>&, hipStream_t);

}  // namespace phx
