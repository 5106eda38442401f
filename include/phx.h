/*
 * phx.h -- C interface of libphx, an MI355X (gfx950) solver for the 2D dissipative
 * nonlinear Schroedinger / Gross-Pitaevskii equation of arXiv 2411.18341 (PHOENIX):
 * fixed-step RK4 and adaptive Dormand-Prince 5(4) time stepping of Eq. (1) and of
 * its extended form, Eqs. (PULSE_psi) and (PULSE_res) of Sec. 5 (spinor components,
 * cross interaction, TE-TM coupling, pump-fed reservoir), on a uniform grid with the
 * five-point Laplacian of Sec. 3.2.8 and periodic or zero boundaries (Sec. 5).
 *
 * Conventions shared by every call:
 *   - Units are the caller's: hbar and mass are parameters.
 *   - Grid cell (i, j), i in [0, nx) along x, j in [0, ny); storage index j*nx + i
 *     (x fastest), row-major, contiguous.
 *   - psi is interleaved complex: {re, im} pairs of float (PHX_C64) or double
 *     (PHX_C128), shaped [components][ny][nx].  n and P (reservoir) are real
 *     [components][ny][nx]; V is real [ny][nx] and shared by both components.
 *     Real arrays are float for PHX_C64 and double for PHX_C128.
 *   - All device pointers are HIP device memory owned by the caller, 256-byte
 *     aligned.  The library never allocates or frees device memory: scratch space
 *     is the caller's workspace, sized by phx_workspace_bytes.  It allocates only
 *     host memory (handles, a small pinned read-back buffer).
 *   - All device work is enqueued on the caller's HIP stream (hipStream_t passed as
 *     void*; NULL is the null stream).  Calls return after enqueueing unless a
 *     call's description says it synchronizes; then it waits on that stream only.
 *   - Every call returns a phx_status; no C++ exception crosses this interface.
 *     phx_last_error() gives a message for the calling thread's last failure.
 *   - A handle is not thread-safe; distinct handles may be used concurrently from
 *     distinct threads and streams.
 */
#ifndef PHX_H
#define PHX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum phx_status {
    PHX_OK = 0,
    PHX_EINVAL = -1,        /* invalid configuration, pointer, size or alignment        */
    PHX_EWORKSPACE = -2,    /* workspace missing or smaller than phx_workspace_bytes     */
    PHX_EHIP = -3,          /* a HIP runtime call failed (message has the HIP error)     */
    PHX_ENONFINITE = -4,    /* a non-finite value appeared in the state                  */
    PHX_EDTMIN = -5,        /* adaptive step size fell below dt_min                      */
    PHX_EUNSUPPORTED = -6,  /* valid combination this build does not implement           */
    PHX_ESTATE = -7         /* call not valid in the handle's current state              */
} phx_status;

enum { PHX_BC_PERIODIC = 0, PHX_BC_ZERO = 1 };  /* zero: ghost cells outside hold 0      */
enum { PHX_C64 = 0, PHX_C128 = 1 };             /* complex64 + float32 / complex128 + float64 */
enum { PHX_RK4 = 0, PHX_RK45 = 1 };             /* Eqs. rk4_K1-rk4_final / Dormand-Prince 5(4) */
enum { PHX_KERNEL_AUTO = 0, PHX_KERNEL_STAGE = 1, PHX_KERNEL_STEP = 2 };

/* Equation, grid and integrator parameters.  All real values are given in double
 * precision; the library forms every derived coefficient (hbar/2m/dx^2, dt/2, dt/6,
 * ...) in double and rounds it once to the kernel precision.
 *
 * Right-hand side advanced by the integrators, per component s (o = other component,
 * sgn = +1 for psi_+, -1 for psi_-; Eq. 1 for one component, Eqs. PULSE_psi/res):
 *   d psi_s/dt = -(i/hbar) [ -(hbar^2/2m) Lap psi_s + (V + g|psi_s|^2 + g_x|psi_o|^2
 *                + g_r n_s) psi_s + delta_lt (Dxx - Dyy - 2 i sgn Dxy) psi_o ]
 *                + (R n_s - gamma_c) psi_s / 2
 *   d n_s/dt   = P_s - (gamma_r + R |psi_s|^2) n_s
 * Lap = Dxx + Dyy, Dxx/Dyy the 3-point second differences, Dxy the 4-corner cross
 * difference (psi[i+1,j+1] - psi[i+1,j-1] - psi[i-1,j+1] + psi[i-1,j-1])/(4 dx dy). */
typedef struct phx_config {
    int32_t nx, ny;         /* grid size, >= 1 each; nx*ny*components < 2^31          */
    double dx, dy;          /* grid spacing, > 0                                        */
    int32_t bc_x, bc_y;     /* PHX_BC_PERIODIC or PHX_BC_ZERO, independently             */
    int32_t components;     /* 1 scalar, 2 spinor                                        */
    int32_t reservoir;      /* 0 or 1: evolve n with pump P                              */
    int32_t precision;      /* PHX_C64 or PHX_C128                                       */
    int32_t integrator;     /* PHX_RK4 or PHX_RK45                                       */
    double hbar, mass;      /* > 0                                                       */
    double g, g_x, g_r;     /* self, cross and reservoir interaction                     */
    double R, gamma_c, gamma_r; /* gain, condensate loss, reservoir loss                 */
    double delta_lt;        /* TE-TM splitting (spinor only)                             */
    double dt;              /* RK4: fixed step.  RK45: first step to try                 */
    double rtol, atol;      /* RK45 tolerances (>= 0, not both 0)                        */
    double dt_min, dt_max;  /* RK45 step bounds (0 < dt_min <= dt_max; dt_max may be inf) */
    int32_t kernel;         /* PHX_KERNEL_AUTO picks the fastest applicable kernel family */
    int32_t tile_wx;        /* 0 = automatic; stage-fused kernels: waves across x (1, 2, 4);
                               whole-step kernel: waves per workgroup of the region form
                               (4, 8, 12, 16), 1 for the streaming form, 2 or 3 for the wide
                               streaming form (two columns per lane; complex64, one
                               component, no drive, even nx; 2: 8-row input ring, 3: 12-row
                               ring; with the noise on periodic grids the increment is
                               drawn in the step, with imaginary time the norm partials are
                               written per wave)                                           */
    int32_t tile_rows;      /* rows per wave (stage-fused: 1..64); streaming form: rows per
                               band (40, 64, 88, 112); wide streaming form: rows per band
                               (8..4096), or 0 for the height that fills the device with
                               one wave per band; streaming forms need a state under 2 GiB;
                               0 with tile_wx 0 = automatic                                 */
    int32_t graph_steps;    /* RK4 steps per captured hipGraph chunk replayed by phx_step:
                               0 = default (64), < 0 = launch every kernel directly        */
    double noise;           /* intensity nu of the complex Wiener noise dW (Sec. 5, truncated
                               Wigner); 0 = deterministic.  RK4 only (PHX_EUNSUPPORTED
                               otherwise): after every step each cell of each component gets
                               dW = sqrt(nu (R n + gamma_c) dt / (4 dx dy)) (xi1 + i xi2),
                               <dW dW*> = nu (R n + gamma_c) dt / (2 dx dy), n the cell's
                               reservoir after the step (0 without the reservoir)          */
    uint64_t seed;          /* noise key: xi1, xi2 are the Box-Muller pair of the first two
                               words of Philox4x32-10 (Salmon et al., SC'11) of the counter
                               (j nx + i, component, step low word, step high word) under the
                               key (seed low word, seed high word), u = (x + 1/2) 2^-32; the
                               step index is phx_info.steps_accepted before the step        */
    double drive_omega;     /* frequency omega of the coherent drive                        */
    int32_t drive;          /* 1: add the coherent drive of Eq. (PULSE_psi), the term
                               -(i/hbar) E_s(r) exp(-i omega t) in d psi_s/dt, with the profile
                               E_s(r) from phx_fields.E, evaluated at every stage's own time
                               (RK4: t + {0, 1/2, 1/2, 1} dt; Dormand-Prince: its nodes c_s);
                               t is phx_info.t (a step taken k steps after the last
                               phx_set_info or phx_create starts at t_set + k dt).  RK4 on
                               the streaming whole-step kernel (one component, or two
                               without reservoirs; bands of 40 or 64 rows; PHX_KERNEL_AUTO
                               picks it when the state is under 2 GiB) or the stage-fused
                               kernels (two components with reservoirs, or on
                               request), and RK45; batches: PHX_EUNSUPPORTED.  0: none      */
    int32_t imag_time;      /* 1: imaginary-time propagation (t -> -i tau, named in Sec. 6)
                               of the conservative equation (reservoir, gamma_c, R, noise and
                               drive all off, else PHX_EINVAL): RK4 steps of
                               d psi/d tau = -(1/hbar) H psi (the streaming whole-step
                               kernel when the state is under 2 GiB: one component on the
                               one-column or wide walk, two on the spinor walk; else, or
                               on request, the stage-fused kernels), each
                               followed by scaling psi so that its total norm
                               dx dy sum_s,cells |psi_s|^2 equals the value it had when the
                               phx_step call began (deterministic FP64 reduction on the
                               device).  dt is the tau step; RK4 only.  0: real time         */
} phx_config;

/* Caller-owned device arrays bound to a handle (borrowed until phx_destroy). */
typedef struct phx_fields {
    void *psi;              /* [components][ny][nx] complex, read and written            */
    void *n;                /* [components][ny][nx] real, read and written (reservoir)   */
    const void *V;          /* [ny][nx] real potential, or NULL for V = 0                */
    const void *P;          /* [components][ny][nx] real pump (required with reservoir)  */
    void *workspace;        /* scratch of at least phx_workspace_bytes, 256-B aligned    */
    size_t workspace_bytes;
    const void *E;          /* [components][ny][nx] complex drive profile E_s(r), read only;
                               required with cfg.drive = 1, NULL otherwise                  */
} phx_fields;

/* Observables of the current state, all accumulated in double precision over the
 * whole grid (A = dx*dy the cell area, rho_s = |psi_s|^2):
 *   norm[s]   = A sum rho_s                 reservoir = A sum n
 *   e_kin     = (hbar^2/2m) A sum over all grid links |forward difference|^2 (with a
 *               zero boundary the links to the ghost cells count), which equals
 *               -(hbar^2/2m) A sum Re(psi* Lap psi)
 *   e_pot     = A sum V rho                 e_int  = (g/2) A sum rho_s^2
 *   e_cross   = g_x A sum rho_+ rho_-        e_tetm = A sum 2 Re(psi_+* J_+ psi_-)
 *   e_res     = g_r A sum n_s rho_s          energy = sum of the six terms
 *   max_density = max rho_s
 *   steady_res_density   = ||2 Re(psi* dpsi/dt)||_2 / ||rho||_2   (d rho/dt residual)
 *   steady_res_reservoir = ||dn/dt||_2 / ||P||_2 (0 without reservoir or pump)
 *   nonfinite = number of non-finite entries in psi and n
 *   norm_renorm[s] = norm[s] - nu Nx Ny / 2: the renormalized density of the truncated
 *               Wigner form (Sec. 5) integrated over the grid, A sum (rho_s - nu/(2A)),
 *               i.e. minus the share nu/(2A) per cell that the noise alone holds in a
 *               lossy empty cell (half a quantum per mode); equals norm[s] without noise
 *               (0 for an absent second component). */
typedef struct phx_obs {
    double norm[2];
    double reservoir;
    double energy, e_kin, e_pot, e_int, e_cross, e_tetm, e_res;
    double max_density;
    double steady_res_density, steady_res_reservoir;
    int64_t nonfinite;
    double norm_renorm[2];
} phx_obs;

/* Integrator progress of a handle. */
typedef struct phx_info {
    double t;               /* simulated time reached                                   */
    double dt;              /* RK4: the fixed step.  RK45: next step size to try        */
    int64_t steps_accepted; /* RK4 steps, or accepted RK45 steps                        */
    int64_t steps_rejected; /* rejected RK45 attempts                                   */
    int32_t last_rejected;  /* RK45: 1 if the last attempt was rejected                 */
    int32_t nonfinite;      /* 1 once a non-finite state was detected                   */
} phx_info;

typedef struct phx_handle phx_handle;

/* Bytes of device workspace a handle with this configuration needs.
 * Host-only; no device access.  PHX_EINVAL on an invalid configuration. */
phx_status phx_workspace_bytes(const phx_config *cfg, size_t *out);

/* Validate cfg and fields, form the coefficients and bind the caller's arrays and
 * stream to a new handle (*out).  Host-only apart from querying the current device;
 * no kernel runs.  The stage arguments of Eqs. rk4_K2-rk4_K4 and the Dormand-Prince
 * stage values live in the workspace.  Errors: PHX_EINVAL (bad value, NULL required
 * pointer, misalignment, RK4 dt beyond the linear stability bound of the kinetic
 * term, |lambda| dt > 2 sqrt(2)), PHX_EWORKSPACE, PHX_EUNSUPPORTED, PHX_EHIP. */
phx_status phx_create(const phx_config *cfg, const phx_fields *fields, void *hip_stream,
                      phx_handle **out);

/* Advance the bound state.  RK4: n_steps steps of Eqs. rk4_K1-rk4_final (Sec. 2),
 * enqueued asynchronously; runs of graph_steps steps are captured once into a
 * hipGraph (on a private stream of default priority) and replayed on the caller's
 * stream, the rest is launched directly (also while kernel timing is on).
 * RK45: attempts Dormand-Prince steps until n_steps are accepted; each attempt
 * reads its error norm back to the host, so the call synchronizes the stream once
 * per attempt.  n_steps >= 0.  *out_or_null receives
 * the progress when not NULL (for RK4 without waiting for the device).
 * PHX_ENONFINITE is returned by the first call that finds the device-side
 * non-finite flag set by an earlier step; PHX_EDTMIN when RK45 cannot meet the
 * tolerance with dt >= dt_min (the state then holds the last accepted step). */
phx_status phx_step(phx_handle *h, int64_t n_steps, phx_info *out_or_null);

/* Compute phx_obs for the current state.  Two-pass deterministic FP64 reduction
 * (fixed block partition and fixed summation order), then a read-back: the call
 * synchronizes the handle's stream. */
phx_status phx_observables(phx_handle *h, phx_obs *out);

/* Read or overwrite the integrator progress (checkpoint and restore: the caller
 * saves psi and n itself and restores them together with this record). */
phx_status phx_get_info(const phx_handle *h, phx_info *out);
phx_status phx_set_info(phx_handle *h, const phx_info *in);

/* RK45 only: log every later Dormand-Prince attempt (Sec. 2) into the caller's host
 * array log[3k], log[3k+1], log[3k+2] = (dt of the attempt, its error norm, 1.0 if it
 * was accepted else 0.0) for k = *count .. cap-1; *count (caller-owned, host) counts
 * the attempts logged so far and is advanced by phx_step; attempts beyond cap are
 * not logged.  log = NULL stops logging.  The arrays stay owned by the caller and
 * must stay valid while logging is on.  Host-only.  Errors: PHX_EINVAL (NULL
 * handle, cap < 0, NULL count with a log), PHX_EUNSUPPORTED (RK4 handle). */
phx_status phx_log_attempts(phx_handle *h, double *log, int64_t cap, int64_t *count);

/* Release host resources of a handle (NULL is a no-op).  Does not synchronize;
 * the caller keeps its arrays alive until enqueued work has finished. */
void phx_destroy(phx_handle *h);

/* Message of the calling thread's last failed call ("" if none). */
const char *phx_last_error(void);

/* ---------------------------------------------------------------- kernel timing
 * Per-kernel GPU time of a handle's own launches, measured with HIP events
 * recorded on the handle's stream around every kernel launch while timing is on
 * (the per-kernel view of Sec. 4.4).  Kernel kinds are named, e.g. "rk4_stage2". */
#define PHX_MAX_KERNEL_KINDS 24
typedef struct phx_timing {
    int32_t count;                          /* kinds with at least one launch            */
    int32_t reserved;
    char name[PHX_MAX_KERNEL_KINDS][32];    /* NUL-terminated kernel kind names          */
    int64_t launches[PHX_MAX_KERNEL_KINDS]; /* launches timed since timing was enabled   */
    double ms_total[PHX_MAX_KERNEL_KINDS];  /* summed GPU time in milliseconds           */
} phx_timing;

/* Turn timing on (enable = 1, also resets the totals) or off (0).  Host-only. */
phx_status phx_set_timing(phx_handle *h, int32_t enable);

/* Totals since timing was enabled; synchronizes the handle's stream. */
phx_status phx_kernel_times(phx_handle *h, phx_timing *out);

/* ---------------------------------------------------------------- tuning
 * Tile-shape search for the handle's RK4 kernel family.  Each candidate shape is
 * timed with HIP events over `reps` launches on the handle's stream; the trial
 * launches read the bound state and write only workspace buffers, so the state is
 * unchanged.  The fastest shape is adopted for later phx_step calls and reported
 * in the phx_config encoding (stage-fused: tile_wx = waves across x, tile_rows =
 * rows per wave; whole-step: tile_wx = waves per workgroup, tile_rows = rows per
 * wave, or tile_wx = 1, 2, 3 and tile_rows = band rows for the streaming forms), so that a
 * caller can cache it and pass it to phx_create next time.
 * Synchronizes the stream.  PHX_EUNSUPPORTED for RK45 handles. */
typedef struct phx_tune_result {
    int32_t family;         /* PHX_KERNEL_STAGE or PHX_KERNEL_STEP                         */
    int32_t tile_wx, tile_rows;  /* adopted shape                                         */
    int32_t candidates;     /* shapes timed                                               */
    double best_us;         /* mean launch time of the adopted shape                      */
    double default_us;      /* mean launch time of the shape in use before the call      */
} phx_tune_result;

phx_status phx_autotune(phx_handle *h, int32_t reps, phx_tune_result *out);

/* ---------------------------------------------------------------- batches
 * Many independent one-component instances (Eq. 1, optionally with the pump-fed
 * reservoir of Eqs. PULSE_psi / PULSE_res) on grids of different sizes, advanced
 * together by one persistent whole-step RK4 kernel launch per step: workgroups
 * walk a list of (instance, region) work items.  Instance k uses
 * params[instances[k].param_index] for its physics, boundaries and dt (the nx,
 * ny, components, precision, integrator, kernel and tile fields of the params are
 * ignored), on its own slice of packed caller-owned device arrays. */
typedef struct phx_instance {
    int32_t nx, ny;         /* grid of this instance, >= 1                              */
    int32_t param_index;    /* index into phx_batch_desc.params                         */
    int32_t reserved;       /* must be 0                                                */
    int64_t offset;         /* element offset of this instance in psi, n, P and V       */
    uint64_t seed;          /* Wiener-noise key of this instance (used when its params
                               have noise > 0): it draws what a single-grid handle with
                               this seed draws                                           */
} phx_instance;

typedef struct phx_batch_desc {
    int32_t count;          /* number of instances, >= 1                                */
    int32_t precision;      /* PHX_C64 or PHX_C128 for all instances                    */
    const phx_instance *instances;  /* host array [count]; slices must not overlap     */
    const phx_config *params;       /* host array [n_params]; all with the same reservoir flag */
    int32_t n_params;
    int32_t check_finite;   /* 1: wait for the stream at the end and report non-finite  */
    int64_t total_cells;    /* length of each packed array in cells                     */
    void *psi;              /* packed complex [total_cells], read and written           */
    void *n;                /* packed real [total_cells] (reservoir), read and written  */
    const void *P;          /* packed real pump [total_cells] (reservoir)               */
    const void *V;          /* packed real potential [total_cells], or NULL for V = 0   */
    void *workspace;        /* scratch of at least phx_batch_workspace_bytes, 256-B aligned */
    size_t workspace_bytes;
    int64_t step0;          /* noise step index of the first step of this call (step k of
                               the call draws index step0 + k, like a single-grid handle
                               whose steps_accepted is step0); the caller advances it      */
} phx_batch_desc;

/* Workspace bytes phx_batch_step needs for this descriptor (host-only). */
phx_status phx_batch_workspace_bytes(const phx_batch_desc *desc, size_t *out);

/* Advance every instance by n_steps RK4 steps (Eqs. rk4_K1-rk4_final), enqueued on
 * hip_stream.  Uploads the instance table (synchronizing the stream once), then
 * one persistent launch per step.  With check_finite = 1 it waits for the stream
 * at the end and returns PHX_ENONFINITE if any stored value was not finite.
 * Errors: PHX_EINVAL (bad descriptor, slice outside total_cells or overlapping,
 * unstable dt), PHX_EWORKSPACE, PHX_EUNSUPPORTED, PHX_EHIP, PHX_ENONFINITE. */
phx_status phx_batch_step(const phx_batch_desc *desc, int64_t n_steps, void *hip_stream);

/* ---------------------------------------------------------------- learned corrector
 * A coarse grid (block means of a fine grid, larger time step) stands in for the
 * fine grid when a small convolutional network adds a learned correction after
 * every coarse step.  The network: four 3x3 convolutions with circular padding,
 * in_channels -> hidden -> hidden -> hidden -> out_channels, ReLU between them.  It
 * runs on BF16 MFMA with FP32 accumulation; master parameters and Adam moments are
 * FP32.  Inputs and outputs are FP32 NHWC: x[batch][height][width][in_channels],
 * y[batch][height][width][out_channels].
 *
 * Parameter layout (FP32, n_params entries, padded entries must be 0): for each
 * layer l, weights W_l[c_out_pad][K_pad] at w_off[l] with K index
 * k = tap * c_in_pad + c_in, tap = (dy + 1) * 3 + (dx + 1) for the input pixel
 * (y + dy, x + dx), then biases b_l[c_out_pad] at b_off[l]
 * (phx_cnn_param_offsets gives the offsets and padded sizes). */
typedef struct phx_cnn_config {
    int32_t in_channels;    /* 4                                                       */
    int32_t hidden;         /* 32                                                      */
    int32_t out_channels;   /* 3                                                       */
    int32_t height, width;  /* grid of every sample; width a multiple of 32             */
    int32_t max_batch;      /* samples per call, >= 1                                  */
} phx_cnn_config;

typedef struct phx_cnn_buffers {
    float *params;          /* [n_params] FP32 master parameters (caller-owned)        */
    float *adam_m, *adam_v; /* [n_params] Adam moments, zero before the first update   */
    void *workspace;        /* at least the workspace_bytes of phx_cnn_sizes            */
    size_t workspace_bytes;
} phx_cnn_buffers;

typedef struct phx_cnn phx_cnn;

phx_status phx_cnn_sizes(const phx_cnn_config *cfg, int64_t *n_params, size_t *workspace_bytes);
phx_status phx_cnn_param_offsets(const phx_cnn_config *cfg, int64_t *w_off /*[4]*/, int64_t *b_off /*[4]*/,
                                 int32_t *k_pad /*[4]*/, int32_t *c_in_pad /*[4]*/, int32_t *c_out_pad /*[4]*/);
phx_status phx_cnn_create(const phx_cnn_config *cfg, const phx_cnn_buffers *buf, void *hip_stream, phx_cnn **out);
void phx_cnn_destroy(phx_cnn *h);

/* y = network(x) for `batch` samples (enqueued on the handle's stream). */
phx_status phx_cnn_forward(phx_cnn *h, const float *x, int32_t batch, float *y);

/* Mean-squared-error loss of network(x) against target ([batch][height][width]
 * [out_channels]) and its gradient with respect to every parameter, written to
 * grads[n_params] (same layout as the parameters); *loss (device double) receives
 * the loss.  Backward passes: data gradients through the flipped weights times
 * the ReLU masks, weight gradients reduced over pixels in a fixed order. */
phx_status phx_cnn_gradients(phx_cnn *h, const float *x, const float *target, int32_t batch, float *grads,
                             double *loss);

/* One Adam step (Kingma & Ba 2015, Algorithm 1) at step t >= 1 on the master
 * parameters with moment buffers adam_m / adam_v. */
phx_status phx_cnn_adam(phx_cnn *h, const float *grads, int32_t t, float lr, float beta1, float beta2, float eps);

/* phx_cnn_gradients followed by phx_cnn_adam (beta1 0.9, beta2 0.999, eps 1e-8). */
phx_status phx_cnn_train_step(phx_cnn *h, const float *x, const float *target, int32_t batch, int32_t t, float lr,
                              double *loss);

/* Block means over factor x factor cells of a fine grid (nx_f, ny_f multiples of
 * factor): psi_c, n_c, P_c on the (nx_f/factor) x (ny_f/factor) grid.  n_f, P_f may
 * be NULL. */
phx_status phx_coarsen(int32_t precision, const void *psi_f, const void *n_f, const void *P_f, int32_t nx_f,
                       int32_t ny_f, int32_t factor, void *psi_c, void *n_c, void *P_c, void *hip_stream);

/* Network input x[cell] = (Re psi/s_psi, Im psi/s_psi, n/s_n, P/s_p) (n, P may be NULL: 0). */
phx_status phx_corrector_features(int32_t precision, const void *psi, const void *n, const void *P, int32_t nx,
                                  int32_t ny, double s_psi, double s_n, double s_p, float *x, void *hip_stream);

/* Training target r[cell] = ((psi_ref - psi)/s_psi as re, im, (n_ref - n)/s_n). */
phx_status phx_corrector_residual(int32_t precision, const void *psi_ref, const void *n_ref, const void *psi,
                                  const void *n, int32_t nx, int32_t ny, double s_psi, double s_n, float *r,
                                  void *hip_stream);

/* Correction: psi += s_psi (y0 + i y1), n += s_n y2 (n may be NULL). */
phx_status phx_corrector_apply(int32_t precision, void *psi, void *n, const float *y, int32_t nx, int32_t ny,
                               double s_psi, double s_n, void *hip_stream);

/* ---------------------------------------------------------------- without allocation
 * phx_observables for callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the observables of
 * the given fields (bound as in phx_create; workspace ignored) for configuration
 * cfg, at time t (the drive's phase in the steady residual).  The same kernels,
 * block partition and summation order as phx_observables, so the results agree bit
 * for bit; the per-workgroup partials (at most PHX_STATIC_OBS_BLOCKS workgroups, 128
 * KiB) live in one array of static device memory per GPU that the library holds
 * until the process ends.  Calls no allocator.  Calls that overlap on one GPU race
 * on that array (serialize them, e.g. on one stream).  Synchronizes hip_stream.
 * PHX_EINVAL on bad arguments, PHX_EWORKSPACE if the grid needs more partials than
 * the array holds, PHX_EHIP on a runtime failure. */
#define PHX_STATIC_OBS_BLOCKS 1024
phx_status phx_observables_static(const phx_config *cfg, const phx_fields *f, double t, void *hip_stream,
                                  phx_obs *out);

/* ---------------------------------------------------------------- measurement
 * Copies `bytes` from src to dst (device arrays, 16-byte aligned, bytes a multiple
 * of 16, not overlapping) with a streaming copy kernel, enqueued on hip_stream.  It
 * is the attainable-bandwidth reference beside which the solver kernels' HBM rates
 * are reported (2 * bytes moved per call); it plays no part in the solver.
 * PHX_EINVAL on bad arguments, PHX_EHIP if the launch fails. */
phx_status phx_stream_copy(void *dst, const void *src, size_t bytes, void *hip_stream);

/* Replays the memory traffic of the complex64 wide whole-step walk (tile_wx 2: one wave
 * per band of a 120-column strip, an 8-row input ring filled 3 rows ahead) with none of
 * its arithmetic, enqueued on hip_stream: psi_out = psi_in and n_out = n_in + P on
 * every cell of a periodic nx x ny grid (psi interleaved complex64, n and P float32,
 * [ny][nx], caller-owned device arrays, 256-byte aligned, outputs not overlapping the
 * inputs or each other).  Its 28 bytes per point in the step kernel's access pattern
 * time the floor that pattern sets for that kernel (the RK4 step of Eqs. rk4_K1 to
 * rk4_final moves the same bytes); it plays no part in the solver.  band_rows: 8..4096,
 * or 0 for the height the step kernel picks for this grid.  PHX_EINVAL on bad arguments
 * (odd nx, psi of 2 GiB or more, overlap), PHX_EHIP if the launch fails. */
phx_status phx_walk_pattern(void *psi_out, void *n_out, const void *psi_in, const void *n_in, const void *P,
                            int32_t nx, int32_t ny, int32_t band_rows, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* PHX_H */
