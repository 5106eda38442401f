// Device code of the wide streaming whole-step RK4 kernel (complex64 state): the
// band walk of stream_body.h with two grid columns per lane, so that one wave covers
// a strip of 128 columns and produces 120 of them.
//
// Lane l owns the column pair x0 + 2l, x0 + 2l + 1 with x0 = strip*120 - 4 (the
// strip's 120 output columns plus a 4-column halo on each side, recomputed as in the
// other whole-step forms).  Of the two x-neighbours of a column, one is the lane's
// other column and one comes from the adjacent lane by a DPP wave shift, so a pair
// needs two shifted operands per component instead of four.  Per output cell this
// halves the x-halo (128/120 instead of 64/56) and the shift work of the one-column
// walk; the arithmetic per cell is the same, in the same order, as in the other
// whole-step forms (their results agree bit for bit).
//
// The walk over the rows of the band, the ring buffers and the stage pipeline are
// those of stream_band: at position t (row j = start + dir t) stage s runs at row
// j - s and the finished row j - 4 is stored when it lies in the band.  The band
// height is a launch argument, not a template constant: the position loop is unrolled
// by 24 with a uniform exit test at every position, so the launch can choose any band
// height (and with it the number of waves) to fill the device evenly.
//
// Loads and stores are buffer instructions: the lane's column offset is a constant
// VGPR and the row offset a scalar, so no vector instruction computes an address.
// A ghost column (zero x boundary) has an out-of-range column offset and reads 0;
// a ghost row (zero y boundary) multiplies its state by 0.  The grid width must be
// even (a column pair never straddles the periodic seam or the right edge).
#pragma once

#include "philox.h"
#include "stream_body.h"

namespace phx {

typedef float wf4 __attribute__((ext_vector_type(4)));
typedef float wf2 __attribute__((ext_vector_type(2)));
typedef unsigned int wu4 __attribute__((ext_vector_type(4)));
typedef unsigned int wu2 __attribute__((ext_vector_type(2)));

constexpr int kWideCols = 120;  // output columns per strip (128 lanes-columns minus 2 x 4 halo)

__device__ __forceinline__ wf4 wload4(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    return __builtin_bit_cast(wf4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
__device__ __forceinline__ wf2 wload2(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    return __builtin_bit_cast(wf2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
// The pair of complex values a lane stores per row: one 128-bit store whose whole
// offset (column and row) is in the VGPR operand.  With the row offset in the scalar
// operand instead, the compiler puts no wait state between the store and a following
// VALU write to its data registers, and on gfx950 such a write can reach the data
// while the store still reads it (the stored row then holds wrong values in the last
// four lanes of some 16-lane rows); with a constant scalar offset it keeps the wait
// state.  The sum is formed unsigned: a masked lane's offset (kOutOfRange) plus a row
// offset below 2 GiB stays out of range and never wraps.
__device__ __forceinline__ void wstore4(wf4 v, __amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    const int off = (int)((unsigned)voff + (unsigned)soff);
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(wu4, v), r, off, 0, kNonTemporal);
}
__device__ __forceinline__ void wstore2(wf2 v, __amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(wu2, v), r, voff, soff, kNonTemporal);
}

// One band of `B` rows of strip `strip`; K is the length of the input ring (rows
// j-4 .. j+PF must fit: PF <= K - 5) and must divide 24.  CHECK: returns true when a
// stored value is not finite (else false without testing: a non-finite value never
// becomes finite again in later steps, so testing the last step of a run of steps
// detects it).  NOISE: each stored pair of cells (2p, 2p + 1) first gets its Wiener
// increment, drawn exactly as the separate noise pass draws it (one generator call
// per pair, the reservoir value after the step), so both give the same bits.  IMAG:
// imaginary time (no reservoir): the derivative is rotated by -i, the input is
// multiplied by the scale a.imag_slots[1] that restores the previous step's norm, and
// *norm receives this lane's FP64 sum of |psi_out|^2 over the cells it stores.
template <bool RES, bool HASV, bool GHOSTS, bool YZERO, int K, int PF, bool CHECK, bool NOISE = false,
          bool IMAG = false>
__device__ __forceinline__ bool stream_band_wide(const StepArgs<float>& a, int strip, int band, int B, int dir,
                                                 double* norm = nullptr)
{
    using C = float2;
    static_assert(24 % K == 0 && PF <= K - 5 && PF >= 1, "input ring");
    const int lane = threadIdx.x & 63;
    const Coef<float>& c = a.c;
    const int gi = strip * kWideCols - 4 + 2 * lane;  // first column of the lane's pair
    const int ci = wrap_any(gi, a.nx, a.bcx);           // -1: ghost pair (zero x boundary)
    const bool gcol = GHOSTS && ci < 0;
    const float keep = gcol ? 0.f : 1.f;
    const int b0 = band * B;
    const float kdiag = 2.f * (c.ax + c.ay);
    const int row8 = a.nx * 8, row4 = a.nx * 4;
    const size_t cells = (size_t)a.nx * a.ny;
    const __amdgpu_buffer_rsrc_t rpi = buffer_of(a.psi_in, cells * 8);
    const __amdgpu_buffer_rsrc_t rni = buffer_of(a.n_in, RES ? cells * 4 : 0);
    const __amdgpu_buffer_rsrc_t rP = buffer_of(a.P, RES ? cells * 4 : 0);
    const __amdgpu_buffer_rsrc_t rV = buffer_of(a.V, HASV ? cells * 4 : 0);
    const __amdgpu_buffer_rsrc_t rpo = buffer_of(a.psi_out, cells * 8);
    const __amdgpu_buffer_rsrc_t rno = buffer_of(a.n_out, RES ? cells * 4 : 0);
    const __amdgpu_buffer_rsrc_t rnull = buffer_of(a.psi_out, 0);  // every access out of range
    // column offsets within a row; a ghost pair reads past the buffer (0)
    const int v8 = gcol ? kOutOfRange : (ci < 0 ? 0 : ci) * 8;
    const int v4 = gcol ? kOutOfRange : (ci < 0 ? 0 : ci) * 4;
    // output lanes: the pair lies in the strip's 120 output columns and in the grid
    const bool out_col = lane >= 2 && lane < 62 && gi < a.nx;
    const int o8 = out_col ? gi * 8 : kOutOfRange;
    const int o4 = out_col ? gi * 4 : kOutOfRange;

    static_assert(!NOISE || (!GHOSTS && !YZERO), "the increment is drawn for periodic grids");
    static_assert(!(IMAG && (RES || NOISE)), "imaginary time has no reservoir and no noise");
    const float sc = IMAG ? (float)a.imag_slots[1] : 1.f;  // uniform
    double nrm = 0.0;
    const uint64_t nstep = NOISE ? *a.noise_step + (uint64_t)a.noise_offset : 0u;  // uniform

    // rings: [slot][cell of the pair]
    C sp[K][2];
    float sn[K][2], sP[K][2], sk[K][2];
    C acc[4][2];
    float accn[4][2];
    C w2[3][2], w3[3][2], w4[3][2];
    float n2[2][2], n3[2][2], n4[2][2];
#pragma unroll
    for (int s = 0; s < K; ++s) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            sp[s][e] = czero<C>();
            sn[s][e] = sP[s][e] = 0.f;
            sk[s][e] = kdiag;
        }
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            acc[s][e] = czero<C>();
            accn[s][e] = 0.f;
        }
#pragma unroll
        for (int s = 0; s < 3; ++s) w2[s][e] = w3[s][e] = w4[s][e] = czero<C>();
#pragma unroll
        for (int s = 0; s < 2; ++s) n2[s][e] = n3[s][e] = n4[s][e] = 0.f;
    }

    // Row to fetch: g unwrapped, rw its index under the boundary rule (-1 for a ghost
    // row).  Past the last row the walk needs (use == false) rw stays put: the load
    // repeats a row just read and is never used.
    const int npos = B + 8;
    const int start = dir > 0 ? b0 - 4 : b0 + B + 3;
    int g = start;
    int rw = wrap_any(g, a.ny, a.bcy);
    auto fetch = [&](int s, bool use) {
        const int rr = rw < 0 ? 0 : rw;
        const wf4 v = wload4(rpi, v8, rr * row8);
        const float rk = (YZERO && rw < 0) ? 0.f : 1.f;
        if (IMAG) {  // the input times the restoring scale (a ghost row reads 0 through rk)
            sp[s][0] = C{rk * (v.x * sc), rk * (v.y * sc)};
            sp[s][1] = C{rk * (v.z * sc), rk * (v.w * sc)};
        } else if (YZERO) {
            sp[s][0] = C{rk * v.x, rk * v.y};
            sp[s][1] = C{rk * v.z, rk * v.w};
        } else {
            sp[s][0] = C{v.x, v.y};
            sp[s][1] = C{v.z, v.w};
        }
        if (RES) {
            const wf2 nv = wload2(rni, v4, rr * row4);
            const wf2 pv = wload2(rP, v4, rr * row4);
            sn[s][0] = nv.x;
            sn[s][1] = nv.y;
            sP[s][0] = pv.x;
            sP[s][1] = pv.y;
        }
        if (HASV) {
            const wf2 vv = wload2(rV, v4, rr * row4);
            sk[s][0] = fmaf(c.inv_hbar, vv.x, kdiag);
            sk[s][1] = fmaf(c.inv_hbar, vv.y, kdiag);
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

    // 0 for a ghost row (zero y boundary), else 1: row r is uniform over the wave
    auto row_keep = [&](int r) { return (YZERO && (unsigned)r >= (unsigned)a.ny) ? 0.f : 1.f; };

    // stage right-hand side of the lane's pair from the argument rows (cur, up, dn):
    // the left neighbour of cell 0 and the right neighbour of cell 1 come from the
    // adjacent lanes; the other two are the pair's own cells
    auto rhs_pair = [&](const C (&cur)[2], const C (&up)[2], const C (&dn)[2], const float (&nn)[2],
                        const float (&pv)[2], const float (&kv)[2], float (&fx)[2], float (&fy)[2],
                        float (&fn)[2]) {
        const float lrx0 = lane_prev(cur[1].x) + cur[1].x;
        const float lry0 = lane_prev(cur[1].y) + cur[1].y;
        const float lrx1 = cur[0].x + lane_next(cur[0].x);
        const float lry1 = cur[0].y + lane_next(cur[0].y);
        cell_rhs<float, RES, IMAG>(c, cur[0], lrx0, lry0, up[0].x + dn[0].x, up[0].y + dn[0].y, nn[0], pv[0],
                                   kv[0], fx[0], fy[0], fn[0]);
        cell_rhs<float, RES, IMAG>(c, cur[1], lrx1, lry1, up[1].x + dn[1].x, up[1].y + dn[1].y, nn[1], pv[1],
                                   kv[1], fx[1], fy[1], fn[1]);
    };

    unsigned bad = 0u;
    for (int base = 0; base < npos; base += 24) {
#pragma unroll
        for (int u = 0; u < 24; ++u) {
            if (base + u >= npos) break;  // uniform
            const int j = start + dir * (base + u);  // newest row of this position
            fetch(slot<K>(u, -PF), base + u + PF < npos);  // row j + PF
            float fx[2], fy[2], fn[2];
            // stage 1 at row j-1: argument = the state (input ring)
            {
                const int s0 = slot<K>(u, 1);
                rhs_pair(sp[s0], sp[slot<K>(u, 2)], sp[slot<K>(u, 0)], sn[s0], sP[s0], sk[s0], fx, fy, fn);
                const float kk = YZERO ? keep * row_keep(j - 1 * dir) : keep;
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const C cur = sp[s0][e];
                    acc[slot<4>(u, 1)][e] = C{fx[e], fy[e]};
                    accn[slot<4>(u, 1)][e] = fn[e];
                    w2[slot<3>(u, 1)][e] = C{kk * fmaf(a.half_dt, fx[e], cur.x), kk * fmaf(a.half_dt, fy[e], cur.y)};
                    n2[slot<2>(u, 1)][e] = kk * fmaf(a.half_dt, fn[e], sn[s0][e]);
                }
            }
            // stage 2 at row j-2: argument in w2 (rows j-3..j-1)
            {
                const int s0 = slot<K>(u, 2);
                rhs_pair(w2[slot<3>(u, 2)], w2[slot<3>(u, 3)], w2[slot<3>(u, 1)], n2[slot<2>(u, 2)], sP[s0], sk[s0],
                         fx, fy, fn);
                const float kk = YZERO ? keep * row_keep(j - 2 * dir) : keep;
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    C& ac = acc[slot<4>(u, 2)][e];
                    ac = C{fmaf(2.f, fx[e], ac.x), fmaf(2.f, fy[e], ac.y)};
                    accn[slot<4>(u, 2)][e] = fmaf(2.f, fn[e], accn[slot<4>(u, 2)][e]);
                    const C p0 = sp[s0][e];
                    w3[slot<3>(u, 2)][e] = C{kk * fmaf(a.half_dt, fx[e], p0.x), kk * fmaf(a.half_dt, fy[e], p0.y)};
                    n3[slot<2>(u, 2)][e] = kk * fmaf(a.half_dt, fn[e], sn[s0][e]);
                }
            }
            // stage 3 at row j-3: argument in w3 (rows j-4..j-2)
            {
                const int s0 = slot<K>(u, 3);
                rhs_pair(w3[slot<3>(u, 3)], w3[slot<3>(u, 4)], w3[slot<3>(u, 2)], n3[slot<2>(u, 3)], sP[s0], sk[s0],
                         fx, fy, fn);
                const float kk = YZERO ? keep * row_keep(j - 3 * dir) : keep;
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    C& ac = acc[slot<4>(u, 3)][e];
                    ac = C{fmaf(2.f, fx[e], ac.x), fmaf(2.f, fy[e], ac.y)};
                    accn[slot<4>(u, 3)][e] = fmaf(2.f, fn[e], accn[slot<4>(u, 3)][e]);
                    const C p0 = sp[s0][e];
                    w4[slot<3>(u, 3)][e] = C{kk * fmaf(a.dt, fx[e], p0.x), kk * fmaf(a.dt, fy[e], p0.y)};
                    n4[slot<2>(u, 3)][e] = kk * fmaf(a.dt, fn[e], sn[s0][e]);
                }
            }
            // stage 4 at row j-4: argument in w4 (rows j-5..j-3); the finished row is
            // stored when it lies in the band and in the grid
            {
                const int s0 = slot<K>(u, 4);
                rhs_pair(w4[slot<3>(u, 4)], w4[slot<3>(u, 5)], w4[slot<3>(u, 3)], n4[slot<2>(u, 4)], sP[s0], sk[s0],
                         fx, fy, fn);
                float y[4], yn[2];
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const C ac = acc[slot<4>(u, 4)][e];
                    const C p0 = sp[s0][e];
                    y[2 * e] = fmaf(a.dt6, ac.x + fx[e], p0.x);
                    y[2 * e + 1] = fmaf(a.dt6, ac.y + fy[e], p0.y);
                    yn[e] = fmaf(a.dt6, accn[slot<4>(u, 4)][e] + fn[e], sn[s0][e]);
                }
                // Stores are issued at every position (no branch: the memory counters
                // then stay the same on every path through the loop); a row outside
                // the band goes to a descriptor of size 0, whose stores are dropped.
                const int r = j - 4 * dir;
                const bool st = r >= b0 && r < b0 + B && r < a.ny;  // uniform
                const int rr = st ? r : 0;
                if (NOISE && st) {
                    const uint32_t pair = (uint32_t)(r * a.nx + gi) >> 1;  // nx and gi even
                    const noise::Philox4 x = noise::philox4x32_10(pair, 0u, (uint32_t)nstep, (uint32_t)(nstep >> 32),
                                                                  a.noise_k0, a.noise_k1);
                    const C lo = noise::add_noise<float, RES>(C{y[0], y[1]}, yn[0], a.noise_a, a.noise_b, x.x[0],
                                                              x.x[1]);
                    const C hi = noise::add_noise<float, RES>(C{y[2], y[3]}, yn[1], a.noise_a, a.noise_b, x.x[2],
                                                              x.x[3]);
                    y[0] = lo.x;
                    y[1] = lo.y;
                    y[2] = hi.x;
                    y[3] = hi.y;
                }
                wstore4(wf4{y[0], y[1], y[2], y[3]}, st ? rpo : rnull, o8, rr * row8);
                if constexpr (IMAG) {
                    const bool stn = st && out_col;
                    nrm += stn ? (double)y[0] * y[0] + (double)y[1] * y[1] : 0.0;
                    nrm += stn ? (double)y[2] * y[2] + (double)y[3] * y[3] : 0.0;
                }
                if (RES) wstore2(wf2{yn[0], yn[1]}, st ? rno : rnull, o4, rr * row4);
                if (CHECK) {
                    unsigned nf = (unsigned)!isfinite(y[0]) | (unsigned)!isfinite(y[1]) |
                                  (unsigned)!isfinite(y[2]) | (unsigned)!isfinite(y[3]);
                    if (RES) nf |= (unsigned)!isfinite(yn[0]) | (unsigned)!isfinite(yn[1]);
                    bad |= (st && out_col) ? nf : 0u;
                }
            }
        }
    }
    if constexpr (IMAG) *norm = nrm;
    return bad != 0u;
}

}  // namespace phx
