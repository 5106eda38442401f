// Device code of the streaming whole-step RK4 kernel for the two-component (spinor)
// form of Eqs. (PULSE_psi), (PULSE_res): self and cross interaction, the potential,
// the TE-TM coupling J_+- = Delta_LT (d_x -+ i d_y)^2, whose mixed derivative needs
// the diagonal neighbours of the other component, and (RES) the reservoirs n_+-
// with gain, reservoir interaction and pumps P_+-.
//
// The band walk is the one-component kernel's (stream_body.h): one wave per strip of
// 56 columns plus a 4-column halo, rows walked once with the four stages pipelined
// one row apart, inputs in an 8-row ring, running sums in a 4-row ring, stage
// arguments in 3-row windows -- here for both components.  x-neighbours come from
// DPP lane shifts; the mixed difference
//   X = o[i+1,j+1] - o[i+1,j-1] - o[i-1,j+1] + o[i-1,j-1]
// is the lane shift of (row below - row above) of the other component, and changes
// sign with the walking direction (odd bands walk upwards).
#pragma once

#include "stream_body.h"

namespace phx {

// f_s for both components from the stage arguments (cur), the neighbour sums in x
// (lr) and y (ud), the y-differences of the rows below and above (dy = below - above,
// for the mixed term), the per-cell constant kv = V/hbar + 2 (ax + ay) and (RES) the
// reservoir values nn and pumps pv.
//   f_s = i T_s + (u_s - i om_s) p_s - sgn_s bxy X_o,   u_s = (R n_s - gamma)/2,
//   T_s = ax lr_s + ay ud_s - 2(ax + ay) p_s - bx (lr_o - 2 q) + by (ud_o - 2 q),
//   om_s = V/hbar + gh rho_s + gxh rho_o + grh n_s (the -2(ax + ay) p_s term folded into kv),
//   fn_s = P_s - (gamma_r + R rho_s) n_s,
// X_o = dir (next(dy_o) - prev(dy_o)), sgn = +1 for psi_+, -1 for psi_-; dir bxy is passed in as
// bxyd (dir is +-1: the same value bit for bit as multiplying X by dir).
template <typename R, bool RES, bool IMAG = false>
__device__ __forceinline__ void spinor_rhs(const Coef<R>& c, const typename cvec<R>::type (&cur)[2],
                                           const typename cvec<R>::type (&lr)[2],
                                           const typename cvec<R>::type (&ud)[2],
                                           const typename cvec<R>::type (&dy)[2], R kv, R bxyd,
                                           const R (&nn)[2], const R (&pv)[2], typename cvec<R>::type (&f)[2],
                                           R (&fn)[2])
{
    using C = typename cvec<R>::type;
    const R rho0 = fma(cur[0].x, cur[0].x, cur[0].y * cur[0].y);
    const R rho1 = fma(cur[1].x, cur[1].x, cur[1].y * cur[1].y);
    const R cb = R(2) * (c.bx - c.by);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int o = 1 - s;
        const C p = cur[s], q = cur[o];
        const R rs = s == 0 ? rho0 : rho1;
        R om = fma(c.gh, rs, fma(c.gxh, s == 0 ? rho1 : rho0, kv));
        if (RES) om = fma(c.grh, nn[s], om);
        const R u = RES ? fma(c.half_R, nn[s], -c.half_gamma) : -c.half_gamma;
        fn[s] = RES ? fma(-fma(c.R_, rs, c.gamma_r), nn[s], pv[s]) : R(0);
        // other component's second differences: -bx (lr_o - 2q) + by (ud_o - 2q)
        const R ox = fma(-c.bx, lr[o].x, fma(c.by, ud[o].x, cb * q.x));
        const R oy = fma(-c.bx, lr[o].y, fma(c.by, ud[o].y, cb * q.y));
        const R tx = fma(c.ax, lr[s].x, fma(c.ay, ud[s].x, ox));
        const R ty = fma(c.ax, lr[s].y, fma(c.ay, ud[s].y, oy));
        // the walking direction's sign rides on the coefficient (bxyd = dir bxy, chosen
        // once per band), not on each difference
        const R xx = lane_next(dy[o].x) - lane_prev(dy[o].x);
        const R xy = lane_next(dy[o].y) - lane_prev(dy[o].y);
        const R sb = s == 0 ? -bxyd : bxyd;
        f[s].x = fma(sb, xx, fma(u, p.x, fma(om, p.y, -ty)));
        f[s].y = fma(sb, xy, fma(u, p.y, fma(-om, p.x, tx)));
        if constexpr (IMAG) {  // imaginary time: -i f
            const R t = f[s].x;
            f[s].x = f[s].y;
            f[s].y = -t;
        }
    }
}

// IMAG: imaginary time (no reservoirs): each stage's derivative is rotated by -i, the
// input is multiplied by the scale a.imag_slots[1] that restores the previous step's
// norm, and *norm receives this lane's FP64 sum of |psi_out|^2 over both components of
// the cells it stores.
// DRIVE (no reservoirs, real time): the coherent drive -(i/hbar) E_s(r) exp(-i omega t_k)
// joins the derivative of component s at stage k; both components of E ride in the
// input ring beside psi, the four stage phasors come from a.drive_ph.
template <typename R, bool RES, bool HASV, bool GHOSTS, bool YZERO, int B, bool IMAG = false, bool DRIVE = false>
__device__ __forceinline__ bool stream_band_spinor(const StepArgs<R>& a, int strip, int band, int dir,
                                                   double* norm = nullptr)
{
    static_assert(!(IMAG && RES), "imaginary time has no reservoir");
    static_assert(!(DRIVE && (RES || IMAG)), "the drive runs without reservoirs, in real time");
    const R sc = IMAG ? (R)a.imag_slots[1] : R(1);  // uniform
    double nrm = 0.0;
    using C = typename cvec<R>::type;
    static_assert((B + 8) % 24 == 0, "band rows + 8 must be a multiple of the unroll length");
    constexpr int PF = 3;
    const int lane = threadIdx.x & 63;
    const Coef<R>& c = a.c;
    const int gi = strip * 56 - 4 + lane;
    const int ci = wrap_any(gi, a.nx, a.bcx);
    const bool gcol = GHOSTS && ci < 0;
    // Ghost columns and rows stay 0 in every stage: their inputs read as 0, so the stage
    // argument p0 + h f is 0 there when the step h is taken as 0 (the lane's h values,
    // and per row a uniform choice between them and 0).
    const R kh2 = gcol ? R(0) : a.half_dt;
    const R kh = gcol ? R(0) : a.dt;
    const int b0 = band * B;
    const R kdiag = R(2) * (c.ax + c.ay);
    const R bxyd = dir > 0 ? c.bxy : -c.bxy;  // uniform over the wave
    const size_t cells = (size_t)a.nx * a.ny;
    const __amdgpu_buffer_rsrc_t rpo = buffer_of(a.psi_out, 2 * cells * sizeof(C));
    const __amdgpu_buffer_rsrc_t rno = buffer_of(a.n_out, RES ? 2 * cells * sizeof(R) : 0);
    // inputs through buffer loads: the lane's column offset in a VGPR (past the buffer
    // for a ghost column, which then reads 0), the row and component offsets in
    // scalars; a ghost row (zero y boundary) reads through a descriptor of size 0
    const __amdgpu_buffer_rsrc_t rpi = buffer_of(a.psi_in, 2 * cells * sizeof(C));
    const __amdgpu_buffer_rsrc_t rni = buffer_of(a.n_in, RES ? 2 * cells * sizeof(R) : 0);
    const __amdgpu_buffer_rsrc_t rP = buffer_of(a.P, RES ? 2 * cells * sizeof(R) : 0);
    const __amdgpu_buffer_rsrc_t rV = buffer_of(a.V, HASV ? cells * sizeof(R) : 0);
    const __amdgpu_buffer_rsrc_t rnull = buffer_of(a.psi_in, 0);
    const __amdgpu_buffer_rsrc_t rE = buffer_of(a.E, DRIVE ? 2 * cells * sizeof(C) : 0);

    C sp[2][8];
    C sE[2][8];  // DRIVE: the profile of both components, in the input ring
    C ph[4];     // DRIVE: the phasors of the four stage times
    R sk[8];
    R sn[2][8], sP[2][8];
    C acc[2][4];
    R accn[2][4];
    C w2[2][3], w3[2][3], w4[2][3];
    R n2[2][2], n3[2][2], n4[2][2];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        sp[0][s] = sp[1][s] = czero<C>();
        sn[0][s] = sn[1][s] = sP[0][s] = sP[1][s] = R(0);
        sk[s] = kdiag;
        if constexpr (DRIVE) sE[0][s] = sE[1][s] = czero<C>();
    }
    if constexpr (DRIVE) {
#pragma unroll
        for (int s = 0; s < 4; ++s) ph[s] = a.drive_ph[s];
    }
    // DRIVE: adds -(i/hbar) E ph to f
    auto drive = [&](C& f, const C e, const C p) {
        const R zx = e.x * p.x - e.y * p.y;
        const R zy = e.x * p.y + e.y * p.x;
        f.x = fma(c.inv_hbar, zy, f.x);
        f.y = fma(-c.inv_hbar, zx, f.y);
    };
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        acc[0][s] = acc[1][s] = czero<C>();
        accn[0][s] = accn[1][s] = R(0);
    }
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int m = 0; m < 2; ++m) w2[m][s] = w3[m][s] = w4[m][s] = czero<C>();
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int m = 0; m < 2; ++m) n2[m][s] = n3[m][s] = n4[m][s] = R(0);

    const int start = dir > 0 ? b0 - 4 : b0 + B + 3;
    int g = start;
    int rw = wrap_any(g, a.ny, a.bcy);
    const int ci0 = ci < 0 ? 0 : ci;
    const int vc = gcol ? kOutOfRange : ci0 * (int)sizeof(C);
    const int vr = gcol ? kOutOfRange : ci0 * (int)sizeof(R);
    const int comp_c = (int)(cells * sizeof(C)), comp_r = (int)(cells * sizeof(R));
    const int row_c = a.nx * (int)sizeof(C), row_r = a.nx * (int)sizeof(R);
    auto fetch = [&](int s, bool use) {
        const bool grow = YZERO && rw < 0;  // uniform
        const int rr = grow ? 0 : rw;
        sp[0][s] = buf_load<C>(grow ? rnull : rpi, vc, rr * row_c);
        sp[1][s] = buf_load<C>(grow ? rnull : rpi, vc, comp_c + rr * row_c);
        if constexpr (DRIVE) {
            sE[0][s] = buf_load<C>(grow ? rnull : rE, vc, rr * row_c);
            sE[1][s] = buf_load<C>(grow ? rnull : rE, vc, comp_c + rr * row_c);
        }
        if constexpr (IMAG) {
#pragma unroll
            for (int m = 0; m < 2; ++m) sp[m][s] = C{sp[m][s].x * sc, sp[m][s].y * sc};
        }
        if (RES) {
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                sn[m][s] = buf_load<R>(grow ? rnull : rni, vr, m * comp_r + rr * row_r);
                sP[m][s] = buf_load<R>(grow ? rnull : rP, vr, m * comp_r + rr * row_r);
            }
        }
        if (HASV) {
            const R vv = buf_load<R>(grow ? rnull : rV, vr, rr * row_r);
            sk[s] = fma(c.inv_hbar, vv, kdiag);
        }
        const int gn = g + dir;
        int rn;
        if (YZERO) {
            rn = (gn >= 0 && gn < a.ny) ? gn : -1;
        } else {
            rn = rw + dir;
            rn = rn == a.ny ? 0 : (rn < 0 ? a.ny - 1 : rn);
        }
        g = use ? gn : g;
        rw = use ? rn : rw;
    };
#pragma unroll
    for (int t = 0; t < PF; ++t) fetch(t, true);

    // the lane's step h, or 0 on a ghost row (zero y boundary; uniform over the wave)
    auto row_h = [&](int r, R h) { return (YZERO && (unsigned)r >= (unsigned)a.ny) ? R(0) : h; };

    // neighbour sums and y-differences of one stage argument (rows above, at, below
    // in walking order) for both components
    auto sums = [&](const C (&up)[2], const C (&cur)[2], const C (&dn)[2], C (&lr)[2], C (&ud)[2], C (&dy)[2]) {
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            lr[m] = C{lane_prev(cur[m].x) + lane_next(cur[m].x), lane_prev(cur[m].y) + lane_next(cur[m].y)};
            ud[m] = C{up[m].x + dn[m].x, up[m].y + dn[m].y};
            dy[m] = C{dn[m].x - up[m].x, dn[m].y - up[m].y};
        }
    };

    bool bad = false;
    const bool out_col = lane >= 4 && lane < 60 && gi < a.nx;
    for (int base = 0; base < B + 8; base += 24) {
#pragma unroll
        for (int u = 0; u < 24; ++u) {
            const int j = start + dir * (base + u);
            fetch(slot<8>(u, -PF), base + u + PF < B + 8);
            C f[2], lr[2], ud[2], dy[2];
            R fn[2], nn[2], pv[2];
            // stage 1 at row j-1 from the input ring
            {
                const int s0 = slot<8>(u, 1);
                const C cur[2] = {sp[0][s0], sp[1][s0]};
                const C up[2] = {sp[0][slot<8>(u, 2)], sp[1][slot<8>(u, 2)]};
                const C dn[2] = {sp[0][slot<8>(u, 0)], sp[1][slot<8>(u, 0)]};
                sums(up, cur, dn, lr, ud, dy);
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    nn[m] = sn[m][s0];
                    pv[m] = sP[m][s0];
                }
                spinor_rhs<R, RES, IMAG>(c, cur, lr, ud, dy, sk[s0], bxyd, nn, pv, f, fn);
                if constexpr (DRIVE) {
                    drive(f[0], sE[0][s0], ph[0]);
                    drive(f[1], sE[1][s0], ph[0]);
                }
                const R hk = row_h(j - 1 * dir, kh2);
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    acc[m][slot<4>(u, 1)] = f[m];
                    w2[m][slot<3>(u, 1)] = C{fma(hk, f[m].x, cur[m].x), fma(hk, f[m].y, cur[m].y)};
                    if (RES) {
                        accn[m][slot<4>(u, 1)] = fn[m];
                        n2[m][slot<2>(u, 1)] = fma(hk, fn[m], sn[m][s0]);
                    }
                }
            }
            // stage 2 at row j-2 from w2
            {
                const int s0 = slot<8>(u, 2);
                const C cur[2] = {w2[0][slot<3>(u, 2)], w2[1][slot<3>(u, 2)]};
                const C up[2] = {w2[0][slot<3>(u, 3)], w2[1][slot<3>(u, 3)]};
                const C dn[2] = {w2[0][slot<3>(u, 1)], w2[1][slot<3>(u, 1)]};
                sums(up, cur, dn, lr, ud, dy);
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    nn[m] = n2[m][slot<2>(u, 2)];
                    pv[m] = sP[m][s0];
                }
                spinor_rhs<R, RES, IMAG>(c, cur, lr, ud, dy, sk[s0], bxyd, nn, pv, f, fn);
                if constexpr (DRIVE) {
                    drive(f[0], sE[0][s0], ph[1]);
                    drive(f[1], sE[1][s0], ph[1]);
                }
                const R hk = row_h(j - 2 * dir, kh2);
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    C& ac = acc[m][slot<4>(u, 2)];
                    ac = C{fma(R(2), f[m].x, ac.x), fma(R(2), f[m].y, ac.y)};
                    const C p0 = sp[m][s0];
                    w3[m][slot<3>(u, 2)] = C{fma(hk, f[m].x, p0.x), fma(hk, f[m].y, p0.y)};
                    if (RES) {
                        accn[m][slot<4>(u, 2)] = fma(R(2), fn[m], accn[m][slot<4>(u, 2)]);
                        n3[m][slot<2>(u, 2)] = fma(hk, fn[m], sn[m][s0]);
                    }
                }
            }
            // stage 3 at row j-3 from w3
            {
                const int s0 = slot<8>(u, 3);
                const C cur[2] = {w3[0][slot<3>(u, 3)], w3[1][slot<3>(u, 3)]};
                const C up[2] = {w3[0][slot<3>(u, 4)], w3[1][slot<3>(u, 4)]};
                const C dn[2] = {w3[0][slot<3>(u, 2)], w3[1][slot<3>(u, 2)]};
                sums(up, cur, dn, lr, ud, dy);
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    nn[m] = n3[m][slot<2>(u, 3)];
                    pv[m] = sP[m][s0];
                }
                spinor_rhs<R, RES, IMAG>(c, cur, lr, ud, dy, sk[s0], bxyd, nn, pv, f, fn);
                if constexpr (DRIVE) {
                    drive(f[0], sE[0][s0], ph[2]);
                    drive(f[1], sE[1][s0], ph[2]);
                }
                const R hk = row_h(j - 3 * dir, kh);
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    C& ac = acc[m][slot<4>(u, 3)];
                    ac = C{fma(R(2), f[m].x, ac.x), fma(R(2), f[m].y, ac.y)};
                    const C p0 = sp[m][s0];
                    w4[m][slot<3>(u, 3)] = C{fma(hk, f[m].x, p0.x), fma(hk, f[m].y, p0.y)};
                    if (RES) {
                        accn[m][slot<4>(u, 3)] = fma(R(2), fn[m], accn[m][slot<4>(u, 3)]);
                        n4[m][slot<2>(u, 3)] = fma(hk, fn[m], sn[m][s0]);
                    }
                }
            }
            // stage 4 at row j-4 from w4; the finished row is stored when it lies in the
            // band and in the grid
            {
                const int s0 = slot<8>(u, 4);
                const C cur[2] = {w4[0][slot<3>(u, 4)], w4[1][slot<3>(u, 4)]};
                const C up[2] = {w4[0][slot<3>(u, 5)], w4[1][slot<3>(u, 5)]};
                const C dn[2] = {w4[0][slot<3>(u, 3)], w4[1][slot<3>(u, 3)]};
                sums(up, cur, dn, lr, ud, dy);
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    nn[m] = n4[m][slot<2>(u, 4)];
                    pv[m] = sP[m][s0];
                }
                spinor_rhs<R, RES, IMAG>(c, cur, lr, ud, dy, sk[s0], bxyd, nn, pv, f, fn);
                if constexpr (DRIVE) {
                    drive(f[0], sE[0][s0], ph[3]);
                    drive(f[1], sE[1][s0], ph[3]);
                }
                const int r = j - 4 * dir;
                const bool st = out_col && r >= b0 && r < b0 + B && r < a.ny;
                const int cell = r * a.nx + gi;
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    const C ac = acc[m][slot<4>(u, 4)];
                    const C p0 = sp[m][s0];
                    const C y = C{fma(a.dt6, ac.x + f[m].x, p0.x), fma(a.dt6, ac.y + f[m].y, p0.y)};
                    buf_store_nt(y, rpo, st ? (int)((m * cells + cell) * sizeof(C)) : kOutOfRange);
                    if constexpr (IMAG) nrm += st ? (double)y.x * y.x + (double)y.y * y.y : 0.0;
                    bool b = !(isfinite(y.x) && isfinite(y.y));
                    if (RES) {
                        const R yn = fma(a.dt6, accn[m][slot<4>(u, 4)] + fn[m], sn[m][s0]);
                        buf_store_nt(yn, rno, st ? (int)((m * cells + cell) * sizeof(R)) : kOutOfRange);
                        b = b || !isfinite(yn);
                    }
                    bad = bad || (st && b);
                }
            }
        }
    }
    if constexpr (IMAG) *norm = nrm;
    return bad;
}

}  // namespace phx
