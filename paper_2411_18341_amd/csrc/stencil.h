// Device-side building blocks of the stencil kernels: boundary-aware column and row
// indices, the 3x3 register window of one component, and the per-cell right-hand
// side of Eq. (1) and Eqs. (PULSE_psi), (PULSE_res).
#pragma once

#include "phx_kernels.h"

namespace phx {

template <typename C> __device__ __forceinline__ C czero();
template <> __device__ __forceinline__ float2 czero<float2>() { return make_float2(0.f, 0.f); }
template <> __device__ __forceinline__ double2 czero<double2>() { return make_double2(0.0, 0.0); }

// Column i and its two neighbours under the x boundary rule.  A ghost neighbour
// (zero boundary) keeps a valid in-row index so that the load stays in bounds and
// is then replaced by 0.
struct Cols {
    int i, il, ir;
    bool zl, zr;
};

__device__ __forceinline__ Cols make_cols(int i, int nx, int bcx)
{
    Cols c{i, i - 1, i + 1, false, false};
    if (c.il < 0) {
        if (bcx == PHX_BC_PERIODIC) c.il += nx; else { c.il = i; c.zl = true; }
    }
    if (c.ir >= nx) {
        if (bcx == PHX_BC_PERIODIC) c.ir -= nx; else { c.ir = i; c.zr = true; }
    }
    return c;
}

// Row j under the y boundary rule; returns -1 for a ghost row of a zero boundary.
__device__ __forceinline__ int wrap_row(int j, int ny, int bcy)
{
    if (j < 0) return bcy == PHX_BC_PERIODIC ? j + ny : -1;
    if (j >= ny) return bcy == PHX_BC_PERIODIC ? j - ny : -1;
    return j;
}

// Values of one component at columns i-1, i, i+1 of one row.
template <typename C>
struct Row3 {
    C l, c, r;
};

template <typename C>
__device__ __forceinline__ Row3<C> load_row(const C* __restrict__ f, int j, int nx, int ny,
                                            int bcy, const Cols& q)
{
    Row3<C> w;
    const int jj = wrap_row(j, ny, bcy);
    if (jj < 0) {
        w.l = w.c = w.r = czero<C>();
        return w;
    }
    const C* p = f + jj * nx;
    w.c = p[q.i];
    const C l = p[q.il];
    const C r = p[q.ir];
    w.l = q.zl ? czero<C>() : l;
    w.r = q.zr ? czero<C>() : r;
    return w;
}

// Right-hand side at the centre of the windows (U: row j-1, M: row j, D: row j+1)
// for every component.  nn are the reservoir values, v the potential (ignored
// without HASV).  Writes f_psi and rho = |psi|^2 per component.  See Coef for the
// formula; the one-component form skips the coupling terms altogether.
template <typename R, int COMPS, bool HASV = true>
__device__ __forceinline__ void rhs_cell(const Coef<R>& k,
                                         const Row3<typename cvec<R>::type> (&U)[COMPS],
                                         const Row3<typename cvec<R>::type> (&M)[COMPS],
                                         const Row3<typename cvec<R>::type> (&D)[COMPS],
                                         const R (&nn)[COMPS], R v,
                                         typename cvec<R>::type (&f)[COMPS], R (&rho)[COMPS])
{
    using C = typename cvec<R>::type;
#pragma unroll
    for (int s = 0; s < COMPS; ++s) {
        const C p = M[s].c;
        rho[s] = p.x * p.x + p.y * p.y;
    }
#pragma unroll
    for (int s = 0; s < COMPS; ++s) {
        const int o = COMPS - 1 - s;
        const C p = M[s].c;
        // undivided second differences of this component
        const R sxx_x = M[s].l.x + M[s].r.x - R(2) * p.x;
        const R sxx_y = M[s].l.y + M[s].r.y - R(2) * p.y;
        const R syy_x = U[s].c.x + D[s].c.x - R(2) * p.x;
        const R syy_y = U[s].c.y + D[s].c.y - R(2) * p.y;
        R tx = k.ax * sxx_x + k.ay * syy_x;
        R ty = k.ax * sxx_y + k.ay * syy_y;
        // w / hbar (the potential enters only when present)
        R om = k.gh * rho[s] + k.grh * nn[s];
        if (HASV) om += k.inv_hbar * v;
        const R u = k.half_R * nn[s] - k.half_gamma;
        if (COMPS == 2) {
            const C q = M[o].c;
            const R oxx_x = M[o].l.x + M[o].r.x - R(2) * q.x;
            const R oxx_y = M[o].l.y + M[o].r.y - R(2) * q.y;
            const R oyy_x = U[o].c.x + D[o].c.x - R(2) * q.x;
            const R oyy_y = U[o].c.y + D[o].c.y - R(2) * q.y;
            tx += -k.bx * oxx_x + k.by * oyy_x;
            ty += -k.bx * oxx_y + k.by * oyy_y;
            om += k.gxh * rho[o];
            // X = o[i+1,j+1] - o[i+1,j-1] - o[i-1,j+1] + o[i-1,j-1]
            const R xx = (D[o].r.x - U[o].r.x) - (D[o].l.x - U[o].l.x);
            const R xy = (D[o].r.y - U[o].r.y) - (D[o].l.y - U[o].l.y);
            const R sb = (s == 0) ? -k.bxy : k.bxy;  // -sgn * bxy
            // i T + (u - i om) p - sgn bxy X
            f[s].x = sb * xx - ty + u * p.x + om * p.y;
            f[s].y = sb * xy + tx + u * p.y - om * p.x;
        } else {
            // i T + (u - i om) p
            f[s].x = u * p.x + om * p.y - ty;
            f[s].y = u * p.y - om * p.x + tx;
        }
    }
}

}  // namespace phx
