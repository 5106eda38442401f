/*
 * CPU oracle for the PHOENIX solver (arXiv 2411.18341): plain complex128 RK4 and
 * Dormand-Prince 5(4) time stepping of the 2D dissipative nonlinear Schroedinger /
 * Gross-Pitaevskii equation with its reservoir and spinor extensions.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code, header,
 * table or constant with the GPU path; the two meet only through seeded input
 * arrays.  It is written for readability: one loop nest per definition, no
 * blocking, no fusion, double precision throughout, built with -ffp-contract=off.
 *
 * Equations followed (paper sections):
 *   - Eq. (1), Sec. 1: i hbar dpsi/dt = (-hbar^2/2m Lap + V + g|psi|^2 - i hbar gamma/2) psi.
 *   - Eqs. (PULSE_psi), (PULSE_res), Sec. 5: spinor psi_+-, cross interaction g_x,
 *     reservoir coupling g_r n, gain R n, TE-TM coupling J_+- = Delta_LT (d_x -+ i d_y)^2,
 *     reservoir rate equation dn/dt = P - (gamma_r + R|psi|^2) n.
 *   - Eqs. (rk4_K1)-(rk4_final), Sec. 2: the classical RK4 step.
 *   - Five-point Laplacian, Sec. 3.2.8.
 *   - Boundary conditions periodic or zero, independently in x and y, Sec. 5.
 *   - Adaptive Dormand-Prince 5(4), named in Sec. 2; tableau from Dormand & Prince,
 *     J. Comput. Appl. Math. 6 (1980) 19-26; step controller as in Hairer, Norsett &
 *     Wanner, Solving ODEs I, Sec. II.4.
 *   - Complex Wiener noise dW of Eq. (PULSE_psi) with the correlations of Sec. 5
 *     (truncated Wigner), drawn from Philox4x32-10 and the Box-Muller transform.
 *   - Coherent drive E_+- of Eq. (PULSE_psi), a term -(i/hbar) E_s(r, t) in d psi_s/dt,
 *     with E_s(r, t) = E_s(r) exp(-i omega t) evaluated at each stage's own time.
 *   - Imaginary-time propagation (named in Sec. 6): t -> -i tau, RK4 steps of
 *     d psi/d tau = -(1/hbar) H psi, each followed by restoring the norm.
 *
 * Readings where the paper is silent (each is also listed in the design notes):
 *   - f in Eqs. (rk4_K1)-(rk4_K4) is the time derivative d psi/dt = -(i/hbar) H psi.
 *   - "zero" boundary: ghost cells outside the grid hold 0 and every grid cell evolves.
 *   - TE-TM: d_xx, d_yy are 3-point second differences, d_xy the 4-corner cross stencil
 *     (psi[i+1,j+1] - psi[i+1,j-1] - psi[i-1,j+1] + psi[i-1,j-1]) / (4 dx dy).
 *   - (psi, n) form one coupled state advanced by the same Runge-Kutta stages.
 *   - The loss gamma of Eq. (1) and the gamma of Eq. (PULSE_psi) are the same
 *     parameter (gamma_c here).
 *   - The noise correlation carries the factor dt of a Wiener increment and the
 *     intensity factor nu; it is added after each deterministic RK4 step (Euler-
 *     Maruyama splitting) with the reservoir value after that step.
 *
 * Layout: psi is [components][ny][nx] complex, x fastest; n and P are
 * [components][ny][nx] real when the reservoir is on; V is [ny][nx] real (NULL = 0).
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

enum { ORC_BC_PERIODIC = 0, ORC_BC_ZERO = 1 };

typedef struct {
    int32_t nx, ny;
    double dx, dy;
    int32_t bc_x, bc_y;
    int32_t components; /* 1 scalar, 2 spinor */
    int32_t reservoir;  /* 0 or 1 */
    double hbar, mass;
    double g, g_x, g_r, R, gamma_c, gamma_r, delta_lt;
    /* coherent drive E_s(r, t) = E[s][q] exp(-i omega t) (Eq. PULSE_psi); E NULL = none */
    const cplx *E;
    double omega;
    double t0;          /* time at the start of the call (RK4 step k starts at t0 + k dt) */
} orc_params;

/* Observables, each a plain sum over the grid times the cell area dx*dy. */
typedef struct {
    double norm[2];       /* dxdy * sum |psi_c|^2 per component                     */
    double reservoir;     /* dxdy * sum n                                            */
    double energy;        /* e_kin + e_pot + e_int + e_cross + e_tetm + e_res        */
    double e_kin, e_pot, e_int, e_cross, e_tetm, e_res;
    double max_density;   /* max |psi_c|^2                                            */
    double steady_res_density;   /* ||2 Re(psi* f_psi)||_2 / ||rho||_2                */
    double steady_res_reservoir; /* ||f_n||_2 / ||P||_2 (0 without reservoir or pump)  */
    int64_t nonfinite;    /* number of non-finite values in psi and n                 */
} orc_obs;

/* ---------------------------------------------------------------- grid access */

static size_t cells(const orc_params *p) { return (size_t)p->nx * (size_t)p->ny; }

/* Value of one real-space component at integer position (i, j) under the boundary
 * rule: indices outside [0, N) wrap (periodic) or read a ghost cell holding 0. */
static cplx at(const orc_params *p, const cplx *f, int i, int j)
{
    if (i < 0 || i >= p->nx) {
        if (p->bc_x == ORC_BC_ZERO) return 0.0;
        i = ((i % p->nx) + p->nx) % p->nx;
    }
    if (j < 0 || j >= p->ny) {
        if (p->bc_y == ORC_BC_ZERO) return 0.0;
        j = ((j % p->ny) + p->ny) % p->ny;
    }
    return f[(size_t)j * p->nx + i];
}

/* Second differences and the mixed difference (Sec. 3.2.8 stencil; TE-TM reading). */
static cplx d_xx(const orc_params *p, const cplx *f, int i, int j)
{
    return (at(p, f, i + 1, j) + at(p, f, i - 1, j) - 2.0 * at(p, f, i, j)) / (p->dx * p->dx);
}
static cplx d_yy(const orc_params *p, const cplx *f, int i, int j)
{
    return (at(p, f, i, j + 1) + at(p, f, i, j - 1) - 2.0 * at(p, f, i, j)) / (p->dy * p->dy);
}
static cplx d_xy(const orc_params *p, const cplx *f, int i, int j)
{
    return (at(p, f, i + 1, j + 1) - at(p, f, i + 1, j - 1) - at(p, f, i - 1, j + 1) +
            at(p, f, i - 1, j - 1)) / (4.0 * p->dx * p->dy);
}
/* Five-point Laplacian, Sec. 3.2.8. */
static cplx laplacian(const orc_params *p, const cplx *f, int i, int j)
{
    return d_xx(p, f, i, j) + d_yy(p, f, i, j);
}

/* ------------------------------------------------------------- right-hand side */

/* Time derivative of the coupled state at every cell (Eq. 1 / Eqs. PULSE_psi, PULSE_res):
 *   f_psi_s = -(i/hbar) [ -(hbar^2/2m) Lap psi_s + (V + g rho_s + g_x rho_o + g_r n_s) psi_s
 *                         + Delta_LT (d_xx - d_yy - 2 i sgn_s d_xy) psi_o ]
 *             + (1/2)(R n_s - gamma_c) psi_s
 *   f_n_s   = P_s - (gamma_r + R rho_s) n_s
 * with s the component, o the other component, sgn = +1 for psi_+ and -1 for psi_-. */
void orc_rhs(const orc_params *p, const cplx *psi, const double *n, const double *V,
             const double *P, cplx *f_psi, double *f_n)
{
    const size_t N = cells(p);
    const int C = p->components;
    for (int c = 0; c < C; ++c) {
        const cplx *ps = psi + (size_t)c * N;
        const cplx *po = psi + (size_t)(C - 1 - c) * N;
        const double sgn = (c == 0) ? 1.0 : -1.0;
#pragma omp parallel for schedule(static) if (N >= 16384)
        for (int j = 0; j < p->ny; ++j) {
            for (int i = 0; i < p->nx; ++i) {
                const size_t k = (size_t)j * p->nx + i;
                const cplx v = ps[k];
                const double rho = creal(v) * creal(v) + cimag(v) * cimag(v);
                const double rho_o = (C == 2) ? creal(po[k]) * creal(po[k]) + cimag(po[k]) * cimag(po[k]) : 0.0;
                const double nn = p->reservoir ? n[(size_t)c * N + k] : 0.0;
                const double pot = V ? V[k] : 0.0;
                cplx h = -(p->hbar * p->hbar / (2.0 * p->mass)) * laplacian(p, ps, i, j)
                         + (pot + p->g * rho + p->g_x * rho_o + p->g_r * nn) * v;
                if (C == 2)
                    h += p->delta_lt * (d_xx(p, po, i, j) - d_yy(p, po, i, j)
                                        - 2.0 * sgn * I * d_xy(p, po, i, j));
                f_psi[(size_t)c * N + k] = -(I / p->hbar) * h + 0.5 * (p->R * nn - p->gamma_c) * v;
                if (p->reservoir)
                    f_n[(size_t)c * N + k] = P[(size_t)c * N + k] - (p->gamma_r + p->R * rho) * nn;
            }
        }
    }
}

/* Right-hand side at time t: orc_rhs plus the coherent drive -(i/hbar) E_s(r) e^{-i omega t}. */
static void rhs_at(const orc_params *p, const cplx *psi, const double *n, const double *V,
                   const double *P, double t, cplx *f_psi, double *f_n)
{
    orc_rhs(p, psi, n, V, P, f_psi, f_n);
    if (!p->E) return;
    const size_t M = cells(p) * (size_t)p->components;
    const cplx phase = cexp(-I * p->omega * t);
    for (size_t q = 0; q < M; ++q) f_psi[q] += -(I / p->hbar) * (p->E[q] * phase);
}

/* Right-hand side at time p->t0 (the drive's phase); orc_rhs without a drive. */
void orc_rhs_t(const orc_params *p, const cplx *psi, const double *n, const double *V,
               const double *P, cplx *f_psi, double *f_n)
{
    rhs_at(p, psi, n, V, P, p->t0, f_psi, f_n);
}

/* ------------------------------------------------------------------------ RK4 */

static void *xmalloc(size_t bytes)
{
    void *q = malloc(bytes ? bytes : 1);
    if (!q) abort();
    return q;
}

/* n_steps classical RK4 steps, Eqs. (rk4_K1)-(rk4_final), applied in place to the
 * coupled state (psi, n):
 *   K1 = f(y), K2 = f(y + dt/2 K1), K3 = f(y + dt/2 K2), K4 = f(y + dt K3),
 *   y <- y + (1/6)(K1 + 2 K2 + 2 K3 + K4) dt. */
void orc_rk4(const orc_params *p, cplx *psi, double *n, const double *V, const double *P,
             double dt, int64_t n_steps)
{
    const size_t M = cells(p) * (size_t)p->components;
    const size_t Mn = p->reservoir ? M : 0;
    cplx *k[4], *y = xmalloc(M * sizeof(cplx));
    double *kn[4], *yn = xmalloc((Mn ? Mn : 1) * sizeof(double));
    for (int s = 0; s < 4; ++s) {
        k[s] = xmalloc(M * sizeof(cplx));
        kn[s] = xmalloc((Mn ? Mn : 1) * sizeof(double));
    }
    const double a[4] = {0.0, 0.5, 0.5, 1.0}; /* stage argument and time offsets, Eqs. rk4_K2-K4 */
    for (int64_t step = 0; step < n_steps; ++step) {
        const double t = p->t0 + (double)step * dt;
        for (int s = 0; s < 4; ++s) {
            if (s == 0) {
                rhs_at(p, psi, n, V, P, t, k[0], kn[0]);
                continue;
            }
            for (size_t q = 0; q < M; ++q) y[q] = psi[q] + a[s] * dt * k[s - 1][q];
            for (size_t q = 0; q < Mn; ++q) yn[q] = n[q] + a[s] * dt * kn[s - 1][q];
            rhs_at(p, y, yn, V, P, t + a[s] * dt, k[s], kn[s]);
        }
        for (size_t q = 0; q < M; ++q)
            psi[q] = psi[q] + (1.0 / 6.0) * (k[0][q] + 2.0 * k[1][q] + 2.0 * k[2][q] + k[3][q]) * dt;
        for (size_t q = 0; q < Mn; ++q)
            n[q] = n[q] + (1.0 / 6.0) * (kn[0][q] + 2.0 * kn[1][q] + 2.0 * kn[2][q] + kn[3][q]) * dt;
    }
    for (int s = 0; s < 4; ++s) { free(k[s]); free(kn[s]); }
    free(y); free(yn);
}

/* Total norm dxdy sum |psi|^2 over all components. */
static double total_norm(const orc_params *p, const cplx *psi)
{
    const size_t M = cells(p) * (size_t)p->components;
    double s = 0.0;
    for (size_t q = 0; q < M; ++q) s += creal(psi[q]) * creal(psi[q]) + cimag(psi[q]) * cimag(psi[q]);
    return p->dx * p->dy * s;
}

/* n_steps imaginary-time steps (t -> -i tau) of the conservative equation (no
 * reservoir, gamma_c = R = 0, no drive): classical RK4 on d psi/d tau = -(1/hbar) H psi,
 * whose right-hand side is -i times the real-time one, and after every step psi is
 * scaled by sqrt(N0 / N) so that its total norm N returns to the value N0 it had when
 * the call began. */
void orc_rk4_imag(const orc_params *p, cplx *psi, const double *V, double dt, int64_t n_steps)
{
    const size_t M = cells(p) * (size_t)p->components;
    cplx *k[4], *y = xmalloc(M * sizeof(cplx));
    for (int s = 0; s < 4; ++s) k[s] = xmalloc(M * sizeof(cplx));
    const double a[4] = {0.0, 0.5, 0.5, 1.0};
    const double N0 = total_norm(p, psi);
    for (int64_t step = 0; step < n_steps; ++step) {
        for (int s = 0; s < 4; ++s) {
            const cplx *arg = psi;
            if (s > 0) {
                for (size_t q = 0; q < M; ++q) y[q] = psi[q] + a[s] * dt * k[s - 1][q];
                arg = y;
            }
            orc_rhs(p, arg, NULL, V, NULL, k[s], NULL);
            for (size_t q = 0; q < M; ++q) k[s][q] *= -I;
        }
        for (size_t q = 0; q < M; ++q)
            psi[q] = psi[q] + (1.0 / 6.0) * (k[0][q] + 2.0 * k[1][q] + 2.0 * k[2][q] + k[3][q]) * dt;
        const double scale = sqrt(N0 / total_norm(p, psi));
        for (size_t q = 0; q < M; ++q) psi[q] *= scale;
    }
    for (int s = 0; s < 4; ++s) free(k[s]);
    free(y);
}

/* ------------------------------------------------------- Dormand-Prince 5(4) */

/* Butcher tableau of Dormand & Prince (1980), method RK5(4)7M. */
static const double DP_A[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5.0, 0, 0, 0, 0, 0},
    {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0, 0},
    {44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0, 0, 0, 0},
    {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0, 0, 0},
    {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0, 0},
    {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0},
};
/* fifth-order weights (equal to the last row of A: first same as last) */
static const double DP_B[7] = {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0,
                               -2187.0 / 6784.0, 11.0 / 84.0, 0.0};
/* embedded fourth-order weights */
static const double DP_BHAT[7] = {5179.0 / 57600.0, 0.0, 7571.0 / 16695.0, 393.0 / 640.0,
                                  -92097.0 / 339200.0, 187.0 / 2100.0, 1.0 / 40.0};
/* stage times (nodes) of the same tableau */
static const double DP_C[7] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 4.0 / 5.0, 8.0 / 9.0, 1.0, 1.0};

/* One Dormand-Prince step of size dt from (psi, n), written to (psi_out, n_out), with
 * the embedded error e = y5 - y4 = dt sum_j (b_j - bhat_j) K_j written to (e_psi, e_n).
 * Seven stage evaluations; the seventh is f(y5); stage s is evaluated at time
 * p->t0 + c_s dt.  Any output may alias nothing. */
void orc_dopri5_step(const orc_params *p, const cplx *psi, const double *n, const double *V,
                     const double *P, double dt, cplx *psi_out, double *n_out, cplx *e_psi,
                     double *e_n)
{
    const size_t M = cells(p) * (size_t)p->components;
    const size_t Mn = p->reservoir ? M : 0;
    cplx *k[7], *y = xmalloc(M * sizeof(cplx));
    double *kn[7], *yn = xmalloc((Mn ? Mn : 1) * sizeof(double));
    for (int s = 0; s < 7; ++s) {
        k[s] = xmalloc(M * sizeof(cplx));
        kn[s] = xmalloc((Mn ? Mn : 1) * sizeof(double));
    }
    for (int s = 0; s < 7; ++s) {
        /* stage argument y_s = y + dt sum_{j<s} a_sj K_j */
        for (size_t q = 0; q < M; ++q) {
            cplx acc = 0.0;
            for (int j = 0; j < s; ++j) acc += DP_A[s][j] * k[j][q];
            y[q] = psi[q] + dt * acc;
        }
        for (size_t q = 0; q < Mn; ++q) {
            double acc = 0.0;
            for (int j = 0; j < s; ++j) acc += DP_A[s][j] * kn[j][q];
            yn[q] = n[q] + dt * acc;
        }
        rhs_at(p, y, yn, V, P, p->t0 + DP_C[s] * dt, k[s], kn[s]);
    }
    for (size_t q = 0; q < M; ++q) {
        cplx acc = 0.0, err = 0.0;
        for (int j = 0; j < 7; ++j) {
            acc += DP_B[j] * k[j][q];
            err += (DP_B[j] - DP_BHAT[j]) * k[j][q];
        }
        psi_out[q] = psi[q] + dt * acc;
        e_psi[q] = dt * err;
    }
    for (size_t q = 0; q < Mn; ++q) {
        double acc = 0.0, err = 0.0;
        for (int j = 0; j < 7; ++j) {
            acc += DP_B[j] * kn[j][q];
            err += (DP_B[j] - DP_BHAT[j]) * kn[j][q];
        }
        n_out[q] = n[q] + dt * acc;
        e_n[q] = dt * err;
    }
    for (int s = 0; s < 7; ++s) { free(k[s]); free(kn[s]); }
    free(y); free(yn);
}

/* Weighted RMS error of an attempted step (Hairer-Norsett-Wanner II.4):
 *   err = sqrt( (1/M_real) sum |e|^2 / (atol + rtol max(|y_old|, |y_new|))^2 )
 * where the complex entries use their modulus for the scale and count as two real
 * unknowns, reservoir entries count as one. */
double orc_error_norm(const orc_params *p, const cplx *psi, const double *n, const cplx *psi_new,
                      const double *n_new, const cplx *e_psi, const double *e_n, double rtol,
                      double atol)
{
    const size_t M = cells(p) * (size_t)p->components;
    const size_t Mn = p->reservoir ? M : 0;
    double sum = 0.0;
    for (size_t q = 0; q < M; ++q) {
        const double sc = atol + rtol * fmax(cabs(psi[q]), cabs(psi_new[q]));
        const double e2 = creal(e_psi[q]) * creal(e_psi[q]) + cimag(e_psi[q]) * cimag(e_psi[q]);
        sum += e2 / (sc * sc);
    }
    for (size_t q = 0; q < Mn; ++q) {
        const double sc = atol + rtol * fmax(fabs(n[q]), fabs(n_new[q]));
        sum += e_n[q] * e_n[q] / (sc * sc);
    }
    return sqrt(sum / (double)(2 * M + Mn));
}

typedef struct {
    double t, dt;           /* time reached and next step size to try             */
    int64_t accepted, rejected;
    int32_t last_rejected;  /* 1 if the most recent attempt was rejected            */
    int32_t status;         /* 0 ok, -5 step size fell below dt_min                 */
} orc_ctrl;

/* Adaptive Dormand-Prince integration until n_accept more steps are accepted.
 * Controller: accept when err <= 1; next dt = dt * clamp(0.9 err^(-1/5), 0.2, fmax)
 * with fmax = 5, or 1 for the step right after a rejection; a non-finite err is a
 * rejection with factor 0.2; dt is capped at dt_max and the run stops with status -5
 * when dt < dt_min.  The attempted dt of every
 * attempt and its error are appended to hist (pairs), when hist is not NULL and
 * hist_cap allows. */
void orc_dopri5(const orc_params *p, cplx *psi, double *n, const double *V, const double *P,
                double rtol, double atol, double dt_min, double dt_max, int64_t n_accept,
                orc_ctrl *ctrl, double *hist, int64_t hist_cap)
{
    const size_t M = cells(p) * (size_t)p->components;
    const size_t Mn = p->reservoir ? M : 0;
    cplx *y5 = xmalloc(M * sizeof(cplx)), *e = xmalloc(M * sizeof(cplx));
    double *n5 = xmalloc((Mn ? Mn : 1) * sizeof(double)), *en = xmalloc((Mn ? Mn : 1) * sizeof(double));
    int64_t done = 0, h = 0;
    ctrl->status = 0;
    while (done < n_accept) {
        const double dt = ctrl->dt;
        if (!(dt >= dt_min)) { ctrl->status = -5; break; }
        orc_params pt = *p;  /* the attempt starts at the time reached */
        pt.t0 = ctrl->t;
        orc_dopri5_step(&pt, psi, n, V, P, dt, y5, n5, e, en);
        const double err = orc_error_norm(p, psi, n, y5, n5, e, en, rtol, atol);
        if (hist && h < hist_cap) { hist[2 * h] = dt; hist[2 * h + 1] = err; ++h; }
        const double fmaxf = ctrl->last_rejected ? 1.0 : 5.0;
        double fac;
        if (!isfinite(err)) fac = 0.2;           /* non-finite estimate: reject, shrink most */
        else if (err > 0.0) fac = 0.9 * pow(err, -0.2);
        else fac = fmaxf;
        if (fac < 0.2) fac = 0.2;
        if (fac > fmaxf) fac = fmaxf;
        if (err <= 1.0) {
            memcpy(psi, y5, M * sizeof(cplx));
            if (Mn) memcpy(n, n5, Mn * sizeof(double));
            ctrl->t += dt;
            ctrl->accepted += 1;
            ctrl->last_rejected = 0;
            ++done;
        } else {
            ctrl->rejected += 1;
            ctrl->last_rejected = 1;
        }
        ctrl->dt = fmin(dt * fac, dt_max);
    }
    free(y5); free(e); free(n5); free(en);
}

/* ---------------------------------------------------------------- observables */

/* Discrete observables.  The kinetic energy is the sum over all grid links of
 * (hbar^2/2m)|forward difference|^2; with a zero boundary the links to the ghost
 * cells on both sides count, so that e_kin = -(hbar^2/2m) dxdy sum Re(psi* Lap psi)
 * holds exactly (summation by parts).  e_tetm = dxdy sum 2 Re(psi_+* J_+ psi_-).
 * The steady residuals use the right-hand side at time p->t0 (drive included). */
void orc_observables(const orc_params *p, const cplx *psi, const double *n, const double *V,
                     const double *P, orc_obs *o)
{
    const size_t N = cells(p);
    const int C = p->components;
    const double dA = p->dx * p->dy;
    const double kin = p->hbar * p->hbar / (2.0 * p->mass);
    memset(o, 0, sizeof(*o));
    cplx *fp = xmalloc(N * C * sizeof(cplx));
    double *fn = xmalloc((p->reservoir ? N * C : 1) * sizeof(double));
    rhs_at(p, psi, n, V, P, p->t0, fp, fn);
    double s_kin = 0, s_pot = 0, s_int = 0, s_cross = 0, s_tetm = 0, s_res = 0, s_nr = 0;
    double s_drho2 = 0, s_rho2 = 0, s_fn2 = 0, s_p2 = 0;
    for (int c = 0; c < C; ++c) {
        const cplx *ps = psi + (size_t)c * N;
        const int ilo = (p->bc_x == ORC_BC_ZERO) ? -1 : 0;
        const int jlo = (p->bc_y == ORC_BC_ZERO) ? -1 : 0;
        double s_norm = 0;
        for (int j = jlo; j < p->ny; ++j)
            for (int i = ilo; i < p->nx; ++i) {
                if (j >= 0) {
                    const cplx d = (at(p, ps, i + 1, j) - at(p, ps, i, j)) / p->dx;
                    s_kin += creal(d) * creal(d) + cimag(d) * cimag(d);
                }
                if (i >= 0) {
                    const cplx d = (at(p, ps, i, j + 1) - at(p, ps, i, j)) / p->dy;
                    s_kin += creal(d) * creal(d) + cimag(d) * cimag(d);
                }
            }
        for (size_t k = 0; k < N; ++k) {
            const double rho = creal(ps[k]) * creal(ps[k]) + cimag(ps[k]) * cimag(ps[k]);
            s_norm += rho;
            s_pot += (V ? V[k] : 0.0) * rho;
            s_int += rho * rho;
            s_rho2 += rho * rho;
            if (rho > o->max_density) o->max_density = rho;
            const cplx f = fp[(size_t)c * N + k];
            const double drho = 2.0 * (creal(ps[k]) * creal(f) + cimag(ps[k]) * cimag(f));
            s_drho2 += drho * drho;
            if (!isfinite(creal(ps[k])) || !isfinite(cimag(ps[k]))) o->nonfinite += 1;
            if (p->reservoir) {
                const double nn = n[(size_t)c * N + k];
                s_nr += nn;
                s_res += nn * rho;
                s_fn2 += fn[(size_t)c * N + k] * fn[(size_t)c * N + k];
                s_p2 += P[(size_t)c * N + k] * P[(size_t)c * N + k];
                if (!isfinite(nn)) o->nonfinite += 1;
            }
        }
        o->norm[c] = dA * s_norm;
    }
    if (C == 2) {
        const cplx *pp = psi, *pm = psi + N;
        for (int j = 0; j < p->ny; ++j)
            for (int i = 0; i < p->nx; ++i) {
                const size_t k = (size_t)j * p->nx + i;
                const double rp = creal(pp[k]) * creal(pp[k]) + cimag(pp[k]) * cimag(pp[k]);
                const double rm = creal(pm[k]) * creal(pm[k]) + cimag(pm[k]) * cimag(pm[k]);
                s_cross += rp * rm;
                const cplx jp = p->delta_lt * (d_xx(p, pm, i, j) - d_yy(p, pm, i, j)
                                               - 2.0 * I * d_xy(p, pm, i, j));
                s_tetm += 2.0 * creal(conj(pp[k]) * jp);
            }
    }
    o->e_kin = kin * dA * s_kin;
    o->e_pot = dA * s_pot;
    o->e_int = 0.5 * p->g * dA * s_int;
    o->e_cross = p->g_x * dA * s_cross;
    o->e_tetm = dA * s_tetm;
    o->e_res = p->g_r * dA * s_res;
    o->energy = o->e_kin + o->e_pot + o->e_int + o->e_cross + o->e_tetm + o->e_res;
    o->reservoir = dA * s_nr;
    o->steady_res_density = (s_rho2 > 0) ? sqrt(s_drho2) / sqrt(s_rho2) : 0.0;
    o->steady_res_reservoir = (p->reservoir && s_p2 > 0) ? sqrt(s_fn2) / sqrt(s_p2) : 0.0;
    free(fp); free(fn);
}

/* ------------------------------------------------- stochastic (Wiener) noise */

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
 * 1, 2, 3", SC'11): ten rounds of the Philox S-box on a 4 x 32-bit counter with a
 * 2 x 32-bit key.  One round multiplies words 0 and 2 by the two round constants,
 * takes the 64-bit products apart, and forms the new counter from their high words
 * xor-ed with words 1 and 3 and the key, and their low words; the key is bumped by
 * the two Weyl constants between rounds. */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;  /* multipliers of the paper */
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;  /* key schedule (Weyl) */
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)M0 * c0, p1 = (uint64_t)M1 * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Two standard normal numbers for (cell q of component s, step) and a 64-bit seed.
 * One Philox4x32-10 call serves the two cells 2p and 2p + 1: the counter is
 * (p = q / 2, s, step low word, step high word), the key (seed low word, seed high
 * word); cell 2p takes output words (x0, x1), cell 2p + 1 words (x2, x3).  The two
 * words become uniforms u = (x + 1/2) 2^-32 in (0, 1), and the Box-Muller transform
 * (Box & Muller, Ann. Math. Statist. 29 (1958) 610) gives r cos(2 pi u2),
 * r sin(2 pi u2) with r = sqrt(-2 ln u1). */
void orc_gauss_pair(uint32_t q, uint32_t s, int64_t step, uint64_t seed, double out[2])
{
    const uint32_t ctr[4] = {q >> 1, s, (uint32_t)(uint64_t)step, (uint32_t)((uint64_t)step >> 32)};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    orc_philox(ctr, key, x);
    const uint32_t *w = x + 2 * (q & 1);
    const double u1 = ((double)w[0] + 0.5) / 4294967296.0;
    const double u2 = ((double)w[1] + 0.5) / 4294967296.0;
    const double r = sqrt(-2.0 * log(u1));
    const double two_pi = 6.283185307179586476925286766559;
    out[0] = r * cos(two_pi * u2);
    out[1] = r * sin(two_pi * u2);
}

/* The complex Wiener increment of step `step` added to every cell (Sec. 5, truncated
 * Wigner): <dW dW> = 0 and <dW dW*> = nu (R n + gamma_c) dt / (2 dV) per cell, with
 * dV = dx dy the cell area and n the reservoir value of the cell (0 without the
 * reservoir); dW = sqrt(nu (R n + gamma_c) dt / (4 dV)) (xi1 + i xi2). */
void orc_noise(const orc_params *p, cplx *psi, const double *n, double dt, double nu, uint64_t seed,
               int64_t step)
{
    const size_t N = cells(p);
    const double dV = p->dx * p->dy;
    for (int s = 0; s < p->components; ++s) {
#pragma omp parallel for schedule(static) if (N >= 16384)
        for (size_t q = 0; q < N; ++q) {
            const double nn = p->reservoir ? n[(size_t)s * N + q] : 0.0;
            const double var = nu * (p->R * nn + p->gamma_c) * dt / (4.0 * dV);
            double xi[2];
            orc_gauss_pair((uint32_t)q, (uint32_t)s, step, seed, xi);
            psi[(size_t)s * N + q] += sqrt(var > 0.0 ? var : 0.0) * (xi[0] + I * xi[1]);
        }
    }
}

/* n_steps RK4 steps, each followed by the Wiener increment of its step index
 * step0, step0 + 1, ... (the noise amplitude uses the reservoir after the step). */
void orc_rk4_noise(const orc_params *p, cplx *psi, double *n, const double *V, const double *P, double dt,
                   int64_t n_steps, double nu, uint64_t seed, int64_t step0)
{
    for (int64_t k = 0; k < n_steps; ++k) {
        orc_params pk = *p;  /* step k starts at t0 + k dt (drive phase) */
        pk.t0 = p->t0 + (double)k * dt;
        orc_rk4(&pk, psi, n, V, P, dt, 1);
        orc_noise(p, psi, n, dt, nu, seed, step0 + k);
    }
}

/* Threads the OpenMP loops above use (reported beside timings of this oracle), and
   a setter for timing it on fewer threads (n >= 1). */
int orc_num_threads(void) { return omp_get_max_threads(); }
void orc_set_num_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
