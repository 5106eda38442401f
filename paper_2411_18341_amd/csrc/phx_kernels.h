// Internal declarations shared by the HIP translation units of libphx: complex
// vector types, the coefficient block every kernel receives, the 3x3 register
// window the stencil kernels march down the grid, the per-cell right-hand side of
// Eq. (1) / Eqs. (PULSE_psi), (PULSE_res), and the host-side launch entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "phx.h"

namespace phx {

template <typename R> struct cvec;
template <> struct cvec<float> { using type = float2; };
template <> struct cvec<double> { using type = double2; };

// Right-hand-side coefficients, formed in double on the host and rounded once.
//   d psi_s/dt = i T - sgn bxy X + (u - i w) psi_s,   u = (R n - gamma_c)/2,
//   w = (V + g rho_s + g_x rho_o + g_r n)/hbar (1/hbar folded into the coefficients),
//   T = ax Dxx' psi_s + ay Dyy' psi_s - bx Dxx' psi_o + by Dyy' psi_o,
//   X = psi_o[i+1,j+1] - psi_o[i+1,j-1] - psi_o[i-1,j+1] + psi_o[i-1,j-1],
// where Dxx' f = f[i+1] + f[i-1] - 2 f[i] (undivided second difference),
// ax = hbar/(2 m dx^2), ay = hbar/(2 m dy^2), bx = delta_lt/(hbar dx^2),
// by = delta_lt/(hbar dy^2), bxy = delta_lt/(2 hbar dx dy).  The spinor terms follow
// from -(i/hbar) delta_lt (Dxx - Dyy - 2 i sgn Dxy) psi_o with Dxy = X/(4 dx dy).
template <typename R>
struct Coef {
    R ax, ay;
    R inv_hbar;
    R gh, gxh, grh;           // g/hbar, g_x/hbar, g_r/hbar: w = V/hbar + gh rho_s + gxh rho_o + grh n
    R half_R, half_gamma;
    R R_, gamma_r;
    R bx, by, bxy;
};

// Boundary handling of one grid axis: neighbour index and whether it is a ghost.
struct Axis {
    int n;
    int bc;  // PHX_BC_PERIODIC or PHX_BC_ZERO
};

// Maps a linear workgroup id to a tile id so that consecutive tiles land on the
// same XCD: workgroups are dispatched round-robin over the 8 XCDs of the chip,
// so XCD x receives ids x, x+8, x+16, ...; giving each XCD a contiguous range of
// tiles keeps the halo rows shared by vertically adjacent tiles in one L2.
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7, l = b >> 3;
    return (x < r) ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

// Coherent drive of Eq. (PULSE_psi): adds -(i/hbar) E ph to f, with E the cell's
// drive profile value and ph = exp(-i omega t) the phasor of the stage's time.
template <typename C, typename R>
__device__ __forceinline__ void add_drive(C& f, const C e, const C ph, R inv_hbar)
{
    const R zx = e.x * ph.x - e.y * ph.y;
    const R zy = e.x * ph.y + e.y * ph.x;
    f.x += inv_hbar * zy;
    f.y -= inv_hbar * zx;
}

// ------------------------------------------------------------- launch API
// Tile geometry of the stencil kernels: a workgroup of 4 waves covers wx*64
// columns and (4/wx)*rows rows; each wave marches `rows` rows of its 64 columns.
struct TileShape {
    int wx;    // waves across x: 1, 2 or 4
    int rows;  // rows per wave
};

template <typename R>
struct Rk4Args {
    using C = typename cvec<R>::type;
    int nx, ny, bcx, bcy, comps;
    int tiles_x, tiles;
    TileShape ts;
    int64_t cstride;   // nx*ny: offset between components
    Coef<R> c;
    R a_dt;            // y_out = psi + a_dt k (stages 1-3)
    R dt6;             // psi += dt6 (acc + k) (stage 4)
    const C* y;  const R* yn;   // stage argument (stage 1: the state itself)
    const C* psi; const R* n;   // state at the start of the step (stages 2, 3)
    const R* V;  const R* P;
    C* y_out; R* yn_out;
    C* acc; R* accn;
    C* psi_io; R* n_io;         // stage 4: state, updated in place
    unsigned int* flag;         // set to 1 when stage 4 produces a non-finite value
    const C* E;                 // drive profile [comps][ny][nx], or NULL
    const C* drive_ph;          // phasors exp(-i omega t_s) of the four stage times
    int imag;                   // 1: imaginary time, the derivative is -i f
};

template <typename R>
hipError_t launch_rk4_stage(int stage, bool reservoir, bool has_v, const Rk4Args<R>& a,
                            hipStream_t s);

// Observables: first pass writes OBS_SLOTS doubles per workgroup, second pass
// reduces them in a fixed order into OBS_SLOTS doubles at `out`.
constexpr int OBS_SLOTS = 16;
enum ObsSlot {
    O_NORM0 = 0, O_NORM1, O_NSUM, O_KIN, O_POT, O_RHO2, O_CROSS, O_TETM, O_RES,
    O_DRHO2, O_FN2, O_P2, O_NONFINITE, O_MAXRHO, O_COUNT_
};

template <typename R>
struct ObsArgs {
    using C = typename cvec<R>::type;
    int nx, ny, bcx, bcy, comps, reservoir;
    int tiles_x, tiles;
    TileShape ts;
    int64_t cstride;
    Coef<R> c;
    double inv_dx2, inv_dy2;   // kinetic links
    double delta_lt, inv_4dxdy;  // TE-TM energy (spinor)
    double gamma_r_d, R_d;       // reservoir residual, in double precision
    const C* psi; const R* n; const R* V; const R* P;
    double* partials;          // [blocks][OBS_SLOTS]
    double* out;               // [OBS_SLOTS]
    const C* E;                // drive profile, or NULL
    C drive_ph;                // exp(-i omega t) at the handle's time
};

template <typename R>
hipError_t launch_observables(const ObsArgs<R>& a, int blocks, hipStream_t s);

}  // namespace phx
