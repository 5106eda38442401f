// Observables of the state as deterministic two-pass FP64 reductions.
//
// Pass 1: each workgroup walks a fixed set of tiles (grid-stride over the same
// tile geometry as the stencil kernels), each lane accumulating its cells' terms in
// double precision; the 64 lanes of a wave are combined by a butterfly of
// cross-lane exchanges and the 4 waves through LDS in a fixed order.  One row of
// OBS_SLOTS partials per workgroup goes to the workspace.
// Pass 2: one workgroup sums the partials in a fixed order.  Both passes are
// independent of timing, so repeated calls give bit-identical results.
#include "stencil.h"

namespace phx {

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m, 64));
    return v;
}

// Reduces q[] over the 256 threads of the workgroup; thread k < OBS_SLOTS returns
// the result of slot k in *out_k.
__device__ __forceinline__ void block_reduce(double (&q)[OBS_SLOTS], double* lds, int tid)
{
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int k = 0; k < OBS_SLOTS; ++k) {
        const double r = (k == O_MAXRHO) ? wave_max(q[k]) : wave_sum(q[k]);
        if (lane == 0) lds[wave * OBS_SLOTS + k] = r;
    }
    __syncthreads();
    if (tid < OBS_SLOTS) {
        double r = lds[tid];
        for (int w = 1; w < 4; ++w) {
            const double x = lds[w * OBS_SLOTS + tid];
            r = (tid == O_MAXRHO) ? fmax(r, x) : r + x;
        }
        q[0] = r;  // caller stores it
    }
}

template <typename R, int COMPS, bool RES, bool HASV>
__global__ __launch_bounds__(256) void obs_pass1(const ObsArgs<R> a, double delta_lt, double inv_4dxdy)
{
    using C = typename cvec<R>::type;
    __shared__ double lds[4 * OBS_SLOTS];
    double q[OBS_SLOTS];
#pragma unroll
    for (int k = 0; k < OBS_SLOTS; ++k) q[k] = 0.0;

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wxi = wave % a.ts.wx;
    const int wyi = wave / a.ts.wx;
    const int cs = (int)a.cstride;
    for (int tile = blockIdx.x; tile < a.tiles; tile += gridDim.x) {
        const int tx = tile % a.tiles_x;
        const int ty = tile / a.tiles_x;
        const int i = (tx * a.ts.wx + wxi) * 64 + lane;
        const int j0 = (ty * (4 / a.ts.wx) + wyi) * a.ts.rows;
        if (i >= a.nx || j0 >= a.ny) continue;
        const int j1 = min(j0 + a.ts.rows, a.ny);
        const Cols cq = make_cols(i, a.nx, a.bcx);
        Row3<C> U[COMPS], M[COMPS], D[COMPS];
#pragma unroll
        for (int s = 0; s < COMPS; ++s) {
            U[s] = load_row(a.psi + s * cs, j0 - 1, a.nx, a.ny, a.bcy, cq);
            M[s] = load_row(a.psi + s * cs, j0, a.nx, a.ny, a.bcy, cq);
        }
        for (int j = j0; j < j1; ++j) {
#pragma unroll
            for (int s = 0; s < COMPS; ++s) D[s] = load_row(a.psi + s * cs, j + 1, a.nx, a.ny, a.bcy, cq);
            const int idx = j * a.nx + i;
            R nn[COMPS];
#pragma unroll
            for (int s = 0; s < COMPS; ++s) nn[s] = RES ? a.n[s * cs + idx] : R(0);
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
                const C p = M[s].c;
                const double pr = p.x, pi = p.y;
                const double r = pr * pr + pi * pi;
                q[s == 0 ? O_NORM0 : O_NORM1] += r;
                // forward links x and y; ghost neighbours read as 0 in the window
                const double dxr = (double)M[s].r.x - pr, dxi = (double)M[s].r.y - pi;
                const double dyr = (double)D[s].c.x - pr, dyi = (double)D[s].c.y - pi;
                double kin = (dxr * dxr + dxi * dxi) * a.inv_dx2 + (dyr * dyr + dyi * dyi) * a.inv_dy2;
                if (a.bcx == PHX_BC_ZERO && i == 0) kin += r * a.inv_dx2;  // link from the left ghost
                if (a.bcy == PHX_BC_ZERO && j == 0) kin += r * a.inv_dy2;  // link from the lower ghost
                q[O_KIN] += kin;
                q[O_POT] += (double)v * r;
                q[O_RHO2] += r * r;
                q[O_MAXRHO] = fmax(q[O_MAXRHO], r);
                const double drho = 2.0 * (pr * (double)f[s].x + pi * (double)f[s].y);
                q[O_DRHO2] += drho * drho;
                q[O_NONFINITE] += (isfinite(p.x) && isfinite(p.y)) ? 0.0 : 1.0;
                if (RES) {
                    const double nd = nn[s];
                    const double pd = a.P[s * cs + idx];
                    const double fn = pd - (a.gamma_r_d + a.R_d * r) * nd;
                    q[O_NSUM] += nd;
                    q[O_RES] += nd * r;
                    q[O_FN2] += fn * fn;
                    q[O_P2] += pd * pd;
                    q[O_NONFINITE] += isfinite(nn[s]) ? 0.0 : 1.0;
                }
            }
            if (COMPS == 2) {
                const C pp = M[0].c;
                const double rp = (double)pp.x * pp.x + (double)pp.y * pp.y;
                const double rm = (double)M[1].c.x * M[1].c.x + (double)M[1].c.y * M[1].c.y;
                q[O_CROSS] += rp * rm;
                // J_+ psi_- = delta_lt (Dxx - Dyy - 2 i Dxy) psi_-
                const Row3<C>& u = U[COMPS - 1];
                const Row3<C>& m = M[COMPS - 1];
                const Row3<C>& d = D[COMPS - 1];
                const double xxr = ((double)m.l.x + m.r.x - 2.0 * m.c.x) * a.inv_dx2;
                const double xxi = ((double)m.l.y + m.r.y - 2.0 * m.c.y) * a.inv_dx2;
                const double yyr = ((double)u.c.x + d.c.x - 2.0 * m.c.x) * a.inv_dy2;
                const double yyi = ((double)u.c.y + d.c.y - 2.0 * m.c.y) * a.inv_dy2;
                const double xyr = (((double)d.r.x - u.r.x) - ((double)d.l.x - u.l.x)) * inv_4dxdy;
                const double xyi = (((double)d.r.y - u.r.y) - ((double)d.l.y - u.l.y)) * inv_4dxdy;
                // (a + i b) - 2 i (c + i e) = (a + 2 e) + i (b - 2 c)
                const double jr = delta_lt * ((xxr - yyr) + 2.0 * xyi);
                const double ji = delta_lt * ((xxi - yyi) - 2.0 * xyr);
                // 2 Re(conj(pp) * J)
                q[O_TETM] += 2.0 * ((double)pp.x * jr + (double)pp.y * ji);
            }
#pragma unroll
            for (int s = 0; s < COMPS; ++s) {
                U[s] = M[s];
                M[s] = D[s];
            }
        }
    }
    block_reduce(q, lds, threadIdx.x);
    if (threadIdx.x < OBS_SLOTS) a.partials[blockIdx.x * OBS_SLOTS + threadIdx.x] = q[0];
}

__global__ __launch_bounds__(256) void obs_pass2(const double* __restrict__ partials, int blocks,
                                                 double* __restrict__ out)
{
    __shared__ double lds[4 * OBS_SLOTS];
    double q[OBS_SLOTS];
#pragma unroll
    for (int k = 0; k < OBS_SLOTS; ++k) q[k] = 0.0;
    for (int b = threadIdx.x; b < blocks; b += 256) {
#pragma unroll
        for (int k = 0; k < OBS_SLOTS; ++k) {
            const double x = partials[b * OBS_SLOTS + k];
            q[k] = (k == O_MAXRHO) ? fmax(q[k], x) : q[k] + x;
        }
    }
    block_reduce(q, lds, threadIdx.x);
    if (threadIdx.x < OBS_SLOTS) out[threadIdx.x] = q[0];
}

template <typename R, int COMPS, bool RES, bool HASV>
static hipError_t obs_t(const ObsArgs<R>& a, int blocks, hipStream_t s, double delta_lt,
                        double inv_4dxdy)
{
    obs_pass1<R, COMPS, RES, HASV><<<blocks, 256, 0, s>>>(a, delta_lt, inv_4dxdy);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    obs_pass2<<<1, 256, 0, s>>>(a.partials, blocks, a.out);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_observables(const ObsArgs<R>& a, int blocks, hipStream_t s)
{
    const double d = a.delta_lt, x = a.inv_4dxdy;
    const bool v = a.V != nullptr;
    if (a.comps == 1) {
        if (a.reservoir) return v ? obs_t<R, 1, true, true>(a, blocks, s, 0, 0)
                                  : obs_t<R, 1, true, false>(a, blocks, s, 0, 0);
        return v ? obs_t<R, 1, false, true>(a, blocks, s, 0, 0)
                 : obs_t<R, 1, false, false>(a, blocks, s, 0, 0);
    }
    if (a.reservoir) return v ? obs_t<R, 2, true, true>(a, blocks, s, d, x)
                              : obs_t<R, 2, true, false>(a, blocks, s, d, x);
    return v ? obs_t<R, 2, false, true>(a, blocks, s, d, x)
             : obs_t<R, 2, false, false>(a, blocks, s, d, x);
}

template hipError_t launch_observables<float>(const ObsArgs<float>&, int, hipStream_t);
template hipError_t launch_observables<double>(const ObsArgs<double>&, int, hipStream_t);

}  // namespace phx
