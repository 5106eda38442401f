// Device code of the streaming whole-step RK4 kernel: all four stages of Eqs.
// rk4_K1-rk4_final in one pass down a band of rows, one wave per strip of columns,
// with no LDS and no barrier.
//
// Lane l of a wave owns grid column strip*56 - 4 + l (the strip's 56 output columns
// plus a 4-column halo on each side, recomputed as in the region kernel; x-neighbours
// come from DPP wave shifts).  The wave walks the rows j = b0-4 .. b0+B+3 of its band
// [b0, b0+B) once; at row j it evaluates
//   stage 1 at row j-1, stage 2 at row j-2, stage 3 at row j-3, stage 4 at row j-4
// (each stage needs its argument at rows r-1..r+1, produced by the previous stage at
// this or an earlier row), and stores the finished row j-4 when it lies in the band;
// the walk ends with row b0+B+3, which finishes row b0+B-1.
// (Rows are named for a downward walk; an upward walk mirrors them.)
// Per-row inputs (psi, n, P, V) wait in an 8-row ring, loaded 3 rows ahead of their
// first use; the running sums K1 + 2K2 + 2K3 in a 4-row ring; the stage arguments
// of stages 2..4 in 3-row windows.  The row loop is unrolled by 24 (a multiple of
// every ring length; the B + 8 rows of the walk are a multiple of 24), so every ring slot is a fixed
// register and no value moves.  Ring slots before row b0-4 hold zeros and feed only
// rows that are never stored.
#pragma once

#include "step_body.h"

namespace phx {

// ring slot of the value that belongs to loop position t - back, ring length K
// (t and back are compile-time constants after unrolling)
template <int K>
__device__ __forceinline__ constexpr int slot(int t, int back)
{
    return ((t - back) % K + K) % K;
}

// Right-hand side of one cell from its stage argument p, the neighbour sums lr
// (x) and ud (y), the reservoir value nn and the per-cell constant kv (see
// step_stages for the formula).  Returns f and fn; IMAG (imaginary time, t -> -i tau)
// returns -i f.
template <typename R, bool RES, bool IMAG = false>
__device__ __forceinline__ void cell_rhs(const Coef<R>& c, typename cvec<R>::type p, R lrx, R lry, R udx, R udy,
                                         R nn, R pv, R kv, R& fx, R& fy, R& fn)
{
    const R rho = fma(p.x, p.x, p.y * p.y);
    R om = kv;
    if (RES) om = fma(c.grh, nn, om);
    om = fma(c.gh, rho, om);
    const R u = RES ? fma(c.half_R, nn, -c.half_gamma) : -c.half_gamma;
    const R tx = fma(c.ax, lrx, c.ay * udx);
    const R ty = fma(c.ax, lry, c.ay * udy);
    fx = fma(u, p.x, fma(om, p.y, -ty));
    fy = fma(u, p.y, fma(-om, p.x, tx));
    fn = RES ? fma(-fma(c.R_, rho, c.gamma_r), nn, pv) : R(0);
    if constexpr (IMAG) {
        const R t = fx;
        fx = fy;
        fy = -t;
    }
}

// Raw buffer stores (hardware range check: a store at an offset past the buffer's
// size is dropped), so lanes and rows that must not store take an out-of-range
// offset instead of a branch.  Offsets are in bytes; the output buffers are smaller
// than 2 GiB (enforced when the shape is chosen).
constexpr unsigned int kBufferWord3 = 0x00020000u;  // raw 32-bit data, gfx9 family
constexpr int kOutOfRange = 0x7fffffff;
constexpr int kNonTemporal = 2;  // cache-policy bit of the store

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void* p, size_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, (int)kBufferWord3);
}

__device__ __forceinline__ void buf_store_nt(float v, __amdgpu_buffer_rsrc_t r, int off)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, kNonTemporal);
}
__device__ __forceinline__ void buf_store_nt(double v, __amdgpu_buffer_rsrc_t r, int off)
{
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, off, 0, kNonTemporal);
}
__device__ __forceinline__ void buf_store_nt(float2 v, __amdgpu_buffer_rsrc_t r, int off)
{
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(u2{__builtin_bit_cast(unsigned int, v.x), __builtin_bit_cast(unsigned int, v.y)},
                                          r, off, 0, kNonTemporal);
}
__device__ __forceinline__ void buf_store_nt(double2 v, __amdgpu_buffer_rsrc_t r, int off)
{
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    const unsigned long long x = __builtin_bit_cast(unsigned long long, v.x);
    const unsigned long long y = __builtin_bit_cast(unsigned long long, v.y);
    __builtin_amdgcn_raw_buffer_store_b128(u4{(unsigned int)x, (unsigned int)(x >> 32), (unsigned int)y,
                                              (unsigned int)(y >> 32)},
                                           r, off, 0, kNonTemporal);
}

// Raw buffer loads of one element (an offset past the buffer's size reads 0).
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ float2 buf_load<float2>(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    // reinterpret the loaded bits as the whole vector (a bit cast of one element of an
    // extended vector has been compiled into a copy of its first element)
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ double2 buf_load<double2>(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

// YZERO: the y boundary is zero (ghost rows); else periodic in y.  dir = +1 walks the
// band downwards (rows b0-4 .. b0+B+3), dir = -1 upwards (rows b0+B+3 .. b0-4): odd
// bands walk up, so that neighbouring bands reach the 8 rows they both read at the same
// time (the second read is an L2 hit).  The stencil is symmetric in y, so the result
// does not depend on the direction.
// IMAG: imaginary time (no reservoir): the derivative is rotated by -i, the input is
// multiplied by the scale a.imag_slots[1] that restores the previous step's norm, and
// *norm receives this lane's sum of |psi_out|^2 over the cells it stores (FP64).
// DRIVE: the coherent drive -(i/hbar) E(r) exp(-i omega t_s) joins each stage's
// derivative; E rides in the input ring, the four stage phasors come from a.drive_ph.
template <typename R, bool RES, bool HASV, bool GHOSTS, bool YZERO, int B, bool IMAG = false, bool DRIVE = false>
__device__ __forceinline__ bool stream_band(const StepArgs<R>& a, int strip, int band, int dir,
                                            double* norm = nullptr)
{
    using C = typename cvec<R>::type;
    static_assert((B + 8) % 24 == 0, "band rows + 8 must be a multiple of the unroll length");
    constexpr int PF = 3;  // rows loaded ahead of their first use
    const int lane = threadIdx.x & 63;
    const Coef<R>& c = a.c;
    const int gi = strip * 56 - 4 + lane;
    const int ci = wrap_any(gi, a.nx, a.bcx);
    const bool gcol = GHOSTS && ci < 0;
    const R keep = gcol ? R(0) : R(1);  // ghost columns stay 0 in every stage
    const int b0 = band * B;
    const R kdiag = R(2) * (c.ax + c.ay);
    const size_t cells = (size_t)a.nx * a.ny;
    const __amdgpu_buffer_rsrc_t rpo = buffer_of(a.psi_out, cells * sizeof(C));
    const __amdgpu_buffer_rsrc_t rno = buffer_of(a.n_out, RES ? cells * sizeof(R) : 0);
    static_assert(!(IMAG && RES), "imaginary time has no reservoir");
    const R sc = IMAG ? (R)a.imag_slots[1] : R(1);
    double nrm = 0.0;
    C ph[4];
    C sE[8];
    if constexpr (DRIVE) {
#pragma unroll
        for (int s = 0; s < 4; ++s) ph[s] = a.drive_ph[s];
#pragma unroll
        for (int s = 0; s < 8; ++s) sE[s] = czero<C>();
    }
    // adds -(i/hbar) E ph to (fx, fy)
    auto drive = [&](R& fx, R& fy, const C e, const C p) {
        const R zx = e.x * p.x - e.y * p.y;
        const R zy = e.x * p.y + e.y * p.x;
        fx = fma(c.inv_hbar, zy, fx);
        fy = fma(-c.inv_hbar, zx, fy);
    };

    // 8-row ring of inputs, read through buffer loads: the lane's column offset in a
    // VGPR, the row offset in a scalar.  Zero boundaries: a ghost column's offset lies
    // past the buffer and a ghost row reads through a descriptor of size 0, so both
    // read 0; every stage argument is multiplied by keep (0 in ghost columns) and by
    // the factor of its row (0 in ghost rows), which leaves the other cells' values
    // unchanged.
    const __amdgpu_buffer_rsrc_t rpi = buffer_of(a.psi_in, cells * sizeof(C));
    const __amdgpu_buffer_rsrc_t rni = buffer_of(a.n_in, RES ? cells * sizeof(R) : 0);
    const __amdgpu_buffer_rsrc_t rP = buffer_of(a.P, RES ? cells * sizeof(R) : 0);
    const __amdgpu_buffer_rsrc_t rV = buffer_of(a.V, HASV ? cells * sizeof(R) : 0);
    const __amdgpu_buffer_rsrc_t rE = buffer_of(a.E, DRIVE ? cells * sizeof(C) : 0);
    const __amdgpu_buffer_rsrc_t rnull = buffer_of(a.psi_in, 0);
    C sp[8];
    R sn[8], sP[8], sk[8];
    C acc[4];
    R accn[4];
    C w2[3], w3[3], w4[3];
    R n2[2], n3[2], n4[2];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        sp[s] = czero<C>();
        sn[s] = R(0);
        sP[s] = R(0);
        sk[s] = kdiag;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        acc[s] = czero<C>();
        accn[s] = R(0);
    }
#pragma unroll
    for (int s = 0; s < 3; ++s) w2[s] = w3[s] = w4[s] = czero<C>();
#pragma unroll
    for (int s = 0; s < 2; ++s) n2[s] = n3[s] = n4[s] = R(0);

    // The row to fetch advances by one per position: g unwrapped, rw its index under
    // the boundary rule (-1 for a ghost row), advanced with selects so that the
    // unrolled body has no branch.  Past the band's last needed row (use == false) rw
    // stays put: the load repeats a row just read (a cache hit) and is never used.
    const int start = dir > 0 ? b0 - 4 : b0 + B + 3;
    int g = start;
    int rw = wrap_any(g, a.ny, a.bcy);
    const int ci0 = ci < 0 ? 0 : ci;
    const int vc = gcol ? kOutOfRange : ci0 * (int)sizeof(C);
    const int vr = gcol ? kOutOfRange : ci0 * (int)sizeof(R);
    const int row_c = a.nx * (int)sizeof(C), row_r = a.nx * (int)sizeof(R);
    auto fetch = [&](int s, bool use) {
        const bool grow = YZERO && rw < 0;  // uniform
        const int rr = grow ? 0 : rw;
        const C v = buf_load<C>(grow ? rnull : rpi, vc, rr * row_c);
        if constexpr (IMAG)
            sp[s] = C{v.x * sc, v.y * sc};
        else
            sp[s] = v;
        if (RES) {
            sn[s] = buf_load<R>(grow ? rnull : rni, vr, rr * row_r);
            sP[s] = buf_load<R>(grow ? rnull : rP, vr, rr * row_r);
        }
        if (HASV) {
            const R vv = buf_load<R>(grow ? rnull : rV, vr, rr * row_r);
            sk[s] = fma(c.inv_hbar, vv, kdiag);
        }
        if constexpr (DRIVE) sE[s] = buf_load<C>(grow ? rnull : rE, vc, rr * row_c);
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

    // 0 for a ghost row (zero y boundary), else 1: the row is uniform over the wave
    auto row_keep = [&](int r) { return (YZERO && (unsigned)r >= (unsigned)a.ny) ? R(0) : R(1); };

    bool bad = false;
    const bool out_col = lane >= 4 && lane < 60 && gi < a.nx;
    for (int base = 0; base < B + 8; base += 24) {
#pragma unroll
        for (int u = 0; u < 24; ++u) {
            const int j = start + dir * (base + u);  // newest row of this position
            fetch(slot<8>(u, -PF), base + u + PF < B + 8);  // row j + PF
            R fx, fy, fn;
            // stage 1 at row j-1: argument = the state, rows j-2..j from the input ring
            {
                const int s0 = slot<8>(u, 1);
                const C cur = sp[s0];
                const C up = sp[slot<8>(u, 2)], dn = sp[slot<8>(u, 0)];
                const R lrx = lane_prev(cur.x) + lane_next(cur.x);
                const R lry = lane_prev(cur.y) + lane_next(cur.y);
                cell_rhs<R, RES, IMAG>(c, cur, lrx, lry, up.x + dn.x, up.y + dn.y, sn[s0], sP[s0], sk[s0], fx, fy, fn);
                if constexpr (DRIVE) drive(fx, fy, sE[s0], ph[0]);
                const R kk = YZERO ? keep * row_keep(j - 1 * dir) : keep;
                acc[slot<4>(u, 1)] = C{fx, fy};
                accn[slot<4>(u, 1)] = fn;
                w2[slot<3>(u, 1)] = C{kk * fma(a.half_dt, fx, cur.x), kk * fma(a.half_dt, fy, cur.y)};
                n2[slot<2>(u, 1)] = kk * fma(a.half_dt, fn, sn[s0]);
            }
            // stage 2 at row j-2: argument in w2 (rows j-3..j-1)
            {
                const int s0 = slot<8>(u, 2);
                const C cur = w2[slot<3>(u, 2)];
                const C up = w2[slot<3>(u, 3)], dn = w2[slot<3>(u, 1)];
                const R nn = n2[slot<2>(u, 2)];
                const R lrx = lane_prev(cur.x) + lane_next(cur.x);
                const R lry = lane_prev(cur.y) + lane_next(cur.y);
                cell_rhs<R, RES, IMAG>(c, cur, lrx, lry, up.x + dn.x, up.y + dn.y, nn, sP[s0], sk[s0], fx, fy, fn);
                if constexpr (DRIVE) drive(fx, fy, sE[s0], ph[1]);
                const R kk = YZERO ? keep * row_keep(j - 2 * dir) : keep;
                C& ac = acc[slot<4>(u, 2)];
                ac = C{fma(R(2), fx, ac.x), fma(R(2), fy, ac.y)};
                accn[slot<4>(u, 2)] = fma(R(2), fn, accn[slot<4>(u, 2)]);
                const C p0 = sp[s0];
                w3[slot<3>(u, 2)] = C{kk * fma(a.half_dt, fx, p0.x), kk * fma(a.half_dt, fy, p0.y)};
                n3[slot<2>(u, 2)] = kk * fma(a.half_dt, fn, sn[s0]);
            }
            // stage 3 at row j-3: argument in w3 (rows j-4..j-2)
            {
                const int s0 = slot<8>(u, 3);
                const C cur = w3[slot<3>(u, 3)];
                const C up = w3[slot<3>(u, 4)], dn = w3[slot<3>(u, 2)];
                const R nn = n3[slot<2>(u, 3)];
                const R lrx = lane_prev(cur.x) + lane_next(cur.x);
                const R lry = lane_prev(cur.y) + lane_next(cur.y);
                cell_rhs<R, RES, IMAG>(c, cur, lrx, lry, up.x + dn.x, up.y + dn.y, nn, sP[s0], sk[s0], fx, fy, fn);
                if constexpr (DRIVE) drive(fx, fy, sE[s0], ph[2]);
                const R kk = YZERO ? keep * row_keep(j - 3 * dir) : keep;
                C& ac = acc[slot<4>(u, 3)];
                ac = C{fma(R(2), fx, ac.x), fma(R(2), fy, ac.y)};
                accn[slot<4>(u, 3)] = fma(R(2), fn, accn[slot<4>(u, 3)]);
                const C p0 = sp[s0];
                w4[slot<3>(u, 3)] = C{kk * fma(a.dt, fx, p0.x), kk * fma(a.dt, fy, p0.y)};
                n4[slot<2>(u, 3)] = kk * fma(a.dt, fn, sn[s0]);
            }
            // stage 4 at row j-4: argument in w4 (rows j-5..j-3); the row is finished and
            // stored when it lies in the band and in the grid (else the offset is out of
            // range and the store is dropped)
            {
                const int s0 = slot<8>(u, 4);
                const C cur = w4[slot<3>(u, 4)];
                const C up = w4[slot<3>(u, 5)], dn = w4[slot<3>(u, 3)];
                const R nn = n4[slot<2>(u, 4)];
                const R lrx = lane_prev(cur.x) + lane_next(cur.x);
                const R lry = lane_prev(cur.y) + lane_next(cur.y);
                cell_rhs<R, RES, IMAG>(c, cur, lrx, lry, up.x + dn.x, up.y + dn.y, nn, sP[s0], sk[s0], fx, fy, fn);
                if constexpr (DRIVE) drive(fx, fy, sE[s0], ph[3]);
                const C ac = acc[slot<4>(u, 4)];
                const C p0 = sp[s0];
                const C y = C{fma(a.dt6, ac.x + fx, p0.x), fma(a.dt6, ac.y + fy, p0.y)};
                const R yn = fma(a.dt6, accn[slot<4>(u, 4)] + fn, sn[s0]);
                const int r = j - 4 * dir;
                const bool st = out_col && r >= b0 && r < b0 + B && r < a.ny;
                const int cell = r * a.nx + gi;
                buf_store_nt(y, rpo, st ? cell * (int)sizeof(C) : kOutOfRange);
                if constexpr (IMAG) nrm += st ? (double)y.x * y.x + (double)y.y * y.y : 0.0;
                bool b = !(isfinite(y.x) && isfinite(y.y));
                if (RES) {
                    buf_store_nt(yn, rno, st ? cell * (int)sizeof(R) : kOutOfRange);
                    b = b || !isfinite(yn);
                }
                bad = bad || (st && b);
            }
        }
    }
    if constexpr (IMAG) *norm = nrm;
    return bad;
}

}  // namespace phx
