// Host side of libphx: validation, workspace layout, coefficients, launch plans and
// the C-ABI entry points declared in include/phx.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>

#include "phx_kernels.h"
#include "runtime.h"

namespace phx {

static thread_local std::string g_err;

phx_status fail(phx_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

void clear_error() { g_err.clear(); }
const char* last_error() { return g_err.c_str(); }

static bool finite_pos(double x) { return isfinite(x) && x > 0.0; }
static bool aligned(const void* p) { return ((uintptr_t)p & 255u) == 0; }

size_t align_up(size_t x) { return (x + 255u) & ~(size_t)255u; }

phx_status validate_config(const phx_config* c)
{
    if (!c) return fail(PHX_EINVAL, "config is NULL");
    if (c->nx < 1 || c->ny < 1) return fail(PHX_EINVAL, "nx=%d ny=%d must be >= 1", c->nx, c->ny);
    if (c->components != 1 && c->components != 2)
        return fail(PHX_EINVAL, "components=%d must be 1 or 2", c->components);
    if ((int64_t)c->nx * c->ny * c->components >= ((int64_t)1 << 31))
        return fail(PHX_EINVAL, "nx*ny*components must be < 2^31");
    if (!finite_pos(c->dx) || !finite_pos(c->dy)) return fail(PHX_EINVAL, "dx, dy must be finite and > 0");
    if ((c->bc_x != PHX_BC_PERIODIC && c->bc_x != PHX_BC_ZERO) ||
        (c->bc_y != PHX_BC_PERIODIC && c->bc_y != PHX_BC_ZERO))
        return fail(PHX_EINVAL, "bc_x=%d bc_y=%d must be PHX_BC_PERIODIC or PHX_BC_ZERO", c->bc_x, c->bc_y);
    if (c->reservoir != 0 && c->reservoir != 1) return fail(PHX_EINVAL, "reservoir must be 0 or 1");
    if (c->precision != PHX_C64 && c->precision != PHX_C128)
        return fail(PHX_EINVAL, "precision=%d must be PHX_C64 or PHX_C128", c->precision);
    if (c->integrator != PHX_RK4 && c->integrator != PHX_RK45)
        return fail(PHX_EINVAL, "integrator=%d must be PHX_RK4 or PHX_RK45", c->integrator);
    if (c->kernel < PHX_KERNEL_AUTO || c->kernel > PHX_KERNEL_STEP)
        return fail(PHX_EINVAL, "kernel=%d is not a PHX_KERNEL_* value", c->kernel);
    if (c->kernel == PHX_KERNEL_STEP &&
        (c->integrator != PHX_RK4 || (c->components == 2 && c->drive && c->reservoir)))
        return fail(PHX_EUNSUPPORTED, "the whole-step kernel covers RK4 with one component, or two (with the "
                                      "drive: without reservoirs)");
    if ((c->tile_wx == 0) != (c->tile_rows == 0) && !(wide_shape(c->tile_wx) && c->kernel != PHX_KERNEL_STAGE))
        return fail(PHX_EINVAL, "tile_wx and tile_rows: both 0 or both set (tile_rows 0 with tile_wx 2 or 3: "
                                "the wide streaming form with the device-filling band height)");
    if (c->tile_wx != 0) {
        if (c->integrator == PHX_RK4 && rk4_family(*c) == PHX_KERNEL_STEP) {
            if ((c->drive || c->components == 2) && c->tile_wx != 1)
                return fail(PHX_EINVAL, "the drive and the spinor on the whole-step kernel use the streaming shapes "
                                        "(tile_wx 1)");
            if (c->imag_time && c->tile_wx != 1 && !wide_shape(c->tile_wx))
                return fail(PHX_EINVAL, "imaginary time on the whole-step kernel uses the streaming shapes (tile_wx "
                                        "1, 2 or 3)");
            if ((c->drive || c->components == 2) && !drive_stream_rows(c->tile_rows))
                return fail(PHX_EINVAL, "the drive and the spinor on the whole-step kernel use bands of 40 or 64 rows");
            if (!valid_step_shape(c->precision, c->tile_wx, c->tile_rows))
                return fail(PHX_EINVAL, "tile %d x %d is not a whole-step kernel shape", c->tile_wx, c->tile_rows);
            if (!step_shape_fits(*c, c->tile_wx))
                return fail(PHX_EINVAL, "streaming shapes (tile_wx 1, 2, 3) need a state array under 2 GiB; the "
                                        "wide ones (tile_wx 2, 3) complex64 and an even nx");
        } else if ((c->tile_wx != 1 && c->tile_wx != 2 && c->tile_wx != 4) || c->tile_rows < 1 || c->tile_rows > 64) {
            return fail(PHX_EINVAL, "tile_wx must be 1, 2 or 4 and tile_rows 1..64");
        }
    }
    if (!finite_pos(c->hbar) || !finite_pos(c->mass)) return fail(PHX_EINVAL, "hbar, mass must be finite and > 0");
    const double coefs[] = {c->g, c->g_x, c->g_r, c->R, c->gamma_c, c->gamma_r, c->delta_lt};
    for (double x : coefs)
        if (!isfinite(x)) return fail(PHX_EINVAL, "equation parameters must be finite");
    if (!finite_pos(c->dt)) return fail(PHX_EINVAL, "dt must be finite and > 0");
    if (!isfinite(c->noise) || c->noise < 0.0) return fail(PHX_EINVAL, "noise must be finite and >= 0");
    if (c->drive != 0 && c->drive != 1) return fail(PHX_EINVAL, "drive must be 0 or 1");
    if (!isfinite(c->drive_omega)) return fail(PHX_EINVAL, "drive_omega must be finite");
    if (c->imag_time != 0 && c->imag_time != 1) return fail(PHX_EINVAL, "imag_time must be 0 or 1");
    if (c->imag_time) {
        if (c->reservoir || c->gamma_c != 0.0 || c->R != 0.0 || c->noise != 0.0 || c->drive)
            return fail(PHX_EINVAL, "imaginary time needs the conservative equation "
                                    "(no reservoir, gamma_c = R = 0, no noise, no drive)");
        if (c->integrator != PHX_RK4) return fail(PHX_EUNSUPPORTED, "imaginary time is implemented for RK4 only");
    }

    if (c->noise > 0.0 && c->integrator != PHX_RK4)
        return fail(PHX_EUNSUPPORTED, "Wiener noise is implemented for RK4 only");
    if (c->integrator == PHX_RK4) {
        // Largest |lambda| of the kinetic term on the grid: (hbar/2m) 4 (1/dx^2 + 1/dy^2);
        // RK4 is unstable on the imaginary axis beyond |lambda dt| = 2 sqrt(2), and on
        // the negative real axis (imaginary time) beyond 2.785.
        const double lam = c->hbar / (2.0 * c->mass) * 4.0 * (1.0 / (c->dx * c->dx) + 1.0 / (c->dy * c->dy));
        const double bound = c->imag_time ? 2.78 : 2.0 * sqrt(2.0);
        if (lam * c->dt > bound)
            return fail(PHX_EINVAL, "dt=%g exceeds the RK4 stability bound %g of the kinetic term",
                        c->dt, bound / lam);
    } else {
        if (!(c->rtol >= 0.0) || !(c->atol >= 0.0) || !isfinite(c->rtol) || !isfinite(c->atol) ||
            c->rtol + c->atol <= 0.0)
            return fail(PHX_EINVAL, "rtol, atol must be finite, >= 0 and not both 0");
        if (!finite_pos(c->dt_min) || !(c->dt_max >= c->dt_min))
            return fail(PHX_EINVAL, "need 0 < dt_min <= dt_max");
    }
    return PHX_OK;
}

bool uses_step_index(const phx_config& c) { return c.noise > 0.0 || (c.drive && c.integrator == PHX_RK4); }

Layout make_layout(const phx_config& c)
{
    Layout L{};
    const size_t rs = c.precision == PHX_C64 ? 4 : 8;
    const size_t cells = (size_t)c.nx * c.ny * c.components;
    const size_t cb = align_up(cells * 2 * rs), rb = align_up(cells * rs);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align_up(bytes); return o; };
    L.flag = take(256);
    L.obs = take(OBS_SLOTS * sizeof(double));
    const bool stage_tiles = c.integrator == PHX_RK4 && rk4_family(c) == PHX_KERNEL_STAGE;
    L.tiles = plan_tiles(c.nx, c.ny, stage_tiles ? c.tile_wx : 0, stage_tiles ? c.tile_rows : 0);
    L.obs_blocks = L.tiles.tiles < 1024 ? L.tiles.tiles : 1024;
    L.partials = take((size_t)L.obs_blocks * OBS_SLOTS * sizeof(double));
    if (uses_step_index(c)) L.noise = take(sizeof(uint64_t));
    if (c.drive && c.integrator == PHX_RK4) L.drive_ph = take(4 * 2 * rs);
    if (c.imag_time) {
        // partials: one per workgroup of the stage-family reduction, or one per wave of
        // the streaming kernel (bands of at least 40 rows)
        L.imag = take(2 * sizeof(double));
        const int64_t stream_waves = 4 * (int64_t)((c.nx + 56 * 4 - 1) / (56 * 4)) * ((c.ny + 39) / 40);
        // the wide walk: one wave per band of one strip, bands of at least 8 rows
        const int64_t wide_waves = (int64_t)wide_strips(c.nx) * ((c.ny + 7) / 8);
        const int64_t blocks = imag_norm_blocks(c.nx * (int64_t)c.ny * c.components);
        int64_t slots = stream_waves > blocks ? stream_waves : blocks;
        if (wide_waves > slots) slots = wide_waves;
        L.imag_partials = take((size_t)slots * sizeof(double));
    }
    if (c.integrator == PHX_RK4) {
        L.family = rk4_family(c);
        if (L.family == PHX_KERNEL_STEP) {
            L.alt = take(cb);
            if (c.reservoir) L.alt_n = take(rb);
            L.alt2 = take(cb);
            if (c.reservoir) L.alt2_n = take(rb);
        } else {
            L.y[0] = take(cb);
            L.y[1] = take(cb);
            L.acc = take(cb);
            if (c.reservoir) {
                L.yn[0] = take(rb);
                L.yn[1] = take(rb);
                L.accn = take(rb);
            }
        }
    }
    if (c.integrator == PHX_RK45) {
        // K_1..K_7, two stage arguments and a second state, for psi and n
        L.k[0] = take(10 * cb + (c.reservoir ? 10 * rb : 0));
        L.err_blocks = L.tiles.tiles;
        L.err = take((size_t)L.tiles.tiles * sizeof(double));
    }
    L.total = off;
    return L;
}

// The streaming shapes (waves 1, and 2 or 3 for the wide form) address their arrays
// through 32-bit buffer offsets: the complex state array must stay below 2 GiB.  The
// wide form runs complex64 with one component (no drive; imaginary time allowed) on grids
// of even width.
bool step_shape_fits(const phx_config& c, int waves)
{
    const double bytes = (double)c.nx * c.ny * c.components * (c.precision == PHX_C64 ? 8.0 : 16.0);
    if ((c.drive || c.components == 2) && waves != 1) return false;  // streaming form only
    if (c.imag_time && waves != 1 && !wide_shape(waves)) return false;
    if (wide_shape(waves) && (c.precision != PHX_C64 || c.nx % 2 != 0)) return false;
    return waves > 3 || bytes < 2147483648.0 - 256.0;
}

bool wide_shape(int waves) { return waves == 2 || waves == 3; }

bool noise_in_step(const phx_config& c, const StepShapeId& sh)
{
    return wide_shape(sh.waves) && c.precision == PHX_C64 && c.components == 1 && c.bc_x == PHX_BC_PERIODIC &&
           c.bc_y == PHX_BC_PERIODIC && !c.drive && !c.imag_time && c.nx % 2 == 0;
}

int wide_strips(int nx) { return (nx + 119) / 120; }

// Band height of a wide shape.  rows > 0 is taken as given; rows = 0 picks the
// smallest height whose bands, one wave each, fit on the device at once (at the
// kernel's waves per SIMD), at least 16 rows.
int wide_band_rows(const phx_config& c, const StepShapeId& sh, bool has_v, int cus)
{
    if (sh.rows > 0) return sh.rows;
    const bool ghosts = c.bc_x == PHX_BC_ZERO || c.bc_y == PHX_BC_ZERO;
    const bool noise = c.noise > 0.0 && noise_in_step(c, sh);
    const int per_simd = wide_waves_per_simd(sh.waves == 2 ? 8 : 12, c.reservoir != 0, has_v, ghosts, noise);
    const int slots = (cus > 0 ? cus : 256) * 4 * per_simd;
    const int per_strip = slots / wide_strips(c.nx);
    const int bands = per_strip > 0 ? per_strip : 1;
    const int b = (c.ny + bands - 1) / bands;
    return b < 16 ? 16 : b;
}

bool step_shape_allowed(const phx_config& c, const StepShapeId& sh)
{
    if (!step_shape_fits(c, sh.waves)) return false;
    return (!c.drive && c.components == 1) || drive_stream_rows(sh.rows);
}

bool valid_step_shape(int precision, int waves, int rows)
{
    if (wide_shape(waves)) return precision == PHX_C64 && (rows == 0 || (rows >= 8 && rows <= 4096));
    const StepShapeId* sh;
    const int n = step_shapes(precision, &sh);
    for (int k = 0; k < n; ++k)
        if (sh[k].waves == waves && sh[k].rows == rows) return true;
    return false;
}

// RK4 kernel family: the whole-step kernel (one launch per step, state read and
// written once) for one component and for the spinor (its streaming form), also with
// the drive (the spinor without reservoirs) or in imaginary time, the stage-fused
// kernels otherwise or on request.
int rk4_family(const phx_config& c)
{
    if (c.kernel == PHX_KERNEL_STAGE) return PHX_KERNEL_STAGE;
    if (c.drive)  // the streaming form when it fits, else the stage-fused kernels
        return ((c.components == 1 || !c.reservoir) && step_shape_fits(c, 1)) ? PHX_KERNEL_STEP : PHX_KERNEL_STAGE;
    if (c.imag_time)  // one component or the spinor: the streaming form when it fits
        return step_shape_fits(c, 1) ? PHX_KERNEL_STEP : PHX_KERNEL_STAGE;
    if (c.components == 1) return PHX_KERNEL_STEP;
    if (step_shape_fits(c, 1)) return PHX_KERNEL_STEP;  // spinor: streaming form
    return PHX_KERNEL_STAGE;
}

// Tile plan for a grid: waves across x chosen from the width; rows per wave halved
// until the launch has enough workgroups to cover the 256 CUs several times.
TilePlan plan_tiles(int nx, int ny, int wx, int rows)
{
    TilePlan t{};
    if (wx > 0) {
        t.ts.wx = wx;
        t.ts.rows = rows;
        t.tiles_x = (nx + 64 * wx - 1) / (64 * wx);
        const int th = rows * (4 / wx);
        t.tiles = t.tiles_x * ((ny + th - 1) / th);
        return t;
    }
    t.ts.wx = nx >= 192 ? 4 : (nx >= 96 ? 2 : 1);
    t.tiles_x = (nx + 64 * t.ts.wx - 1) / (64 * t.ts.wx);
    t.ts.rows = 16;
    for (;;) {
        const int th = t.ts.rows * (4 / t.ts.wx);
        t.tiles = t.tiles_x * ((ny + th - 1) / th);
        if (t.tiles >= 2048 || t.ts.rows == 1) break;
        t.ts.rows >>= 1;
    }
    return t;
}

template <typename R>
Coef<R> make_coef(const phx_config& c)
{
    Coef<R> k;
    k.ax = (R)(c.hbar / (2.0 * c.mass * c.dx * c.dx));
    k.ay = (R)(c.hbar / (2.0 * c.mass * c.dy * c.dy));
    k.inv_hbar = (R)(1.0 / c.hbar);
    k.gh = (R)(c.g / c.hbar);
    k.gxh = (R)(c.g_x / c.hbar);
    k.grh = (R)(c.g_r / c.hbar);
    k.half_R = (R)(0.5 * c.R);
    k.half_gamma = (R)(0.5 * c.gamma_c);
    k.R_ = (R)c.R;
    k.gamma_r = (R)c.gamma_r;
    k.bx = (R)(c.delta_lt / (c.hbar * c.dx * c.dx));
    k.by = (R)(c.delta_lt / (c.hbar * c.dy * c.dy));
    k.bxy = (R)(c.delta_lt / (2.0 * c.hbar * c.dx * c.dy));
    return k;
}

template Coef<float> make_coef<float>(const phx_config&);
template Coef<double> make_coef<double>(const phx_config&);

}  // namespace phx

using namespace phx;

#define HIP_OR_FAIL(call)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) return fail(PHX_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)


phx_status phx_workspace_bytes(const phx_config* cfg, size_t* out)
{
    clear_error();
    if (!out) return fail(PHX_EINVAL, "out is NULL");
    phx_status s = validate_config(cfg);
    if (s != PHX_OK) return s;
    *out = make_layout(*cfg).total;
    return PHX_OK;
}

phx_status phx_create(const phx_config* cfg, const phx_fields* f, void* stream,
                                 phx_handle** out)
{
    clear_error();
    if (!out) return fail(PHX_EINVAL, "out is NULL");
    *out = nullptr;
    phx_status s = validate_config(cfg);
    if (s != PHX_OK) return s;
    if (!f) return fail(PHX_EINVAL, "fields is NULL");
    if (!f->psi) return fail(PHX_EINVAL, "psi is NULL");
    if (cfg->reservoir && (!f->n || !f->P)) return fail(PHX_EINVAL, "reservoir needs n and P");
    if (cfg->drive ? !f->E : f->E != nullptr)
        return fail(PHX_EINVAL, cfg->drive ? "drive needs the profile E" : "E given without drive");
    const void* ptrs[] = {f->psi, f->n, f->V, f->P, f->workspace, f->E};
    for (const void* p : ptrs)
        if (p && !aligned(p)) return fail(PHX_EINVAL, "device pointers must be 256-byte aligned");
    const Layout L = make_layout(*cfg);
    if (!f->workspace || f->workspace_bytes < L.total)
        return fail(PHX_EWORKSPACE, "workspace of %zu bytes needed, %zu given", L.total,
                    f->workspace ? f->workspace_bytes : (size_t)0);
    phx_handle* h = new (std::nothrow) phx_handle();
    if (!h) return fail(PHX_EINVAL, "out of host memory");
    h->cfg = *cfg;
    h->f = *f;
    h->stream = (hipStream_t)stream;
    h->L = L;
    h->ws = (char*)f->workspace;
    h->info.t = 0.0;
    h->info.dt = cfg->dt;
    hipError_t e = hipHostMalloc((void**)&h->host, (OBS_SLOTS + 2) * sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->flag_ready, hipEventDisableTiming);
    h->drive_t0 = 0.0;
    h->drive_k0 = 0;
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            h->cus = cus;
        else
            h->cus = 256;
    }
    if (e == hipSuccess) e = hipMemsetAsync(h->ws + L.flag, 0, 256, h->stream);
    if (e == hipSuccess && uses_step_index(*cfg)) e = set_noise_step(h, 0, h->stream);
    if (e == hipSuccess && cfg->drive && cfg->integrator == PHX_RK4)  // valid phasors before any launch
        e = cfg->precision == PHX_C64 ? launch_drive_phasors<float>(h, 0, h->stream)
                                      : launch_drive_phasors<double>(h, 0, h->stream);
    if (e == hipSuccess && cfg->imag_time)  // valid norm target and scale before any launch
        e = cfg->precision == PHX_C64 ? launch_imag_norm<float>(h, f->psi, 0, h->stream)
                                      : launch_imag_norm<double>(h, f->psi, 0, h->stream);
    if (e != hipSuccess) {
        if (h->host) (void)hipHostFree(h->host);
        if (h->flag_ready) (void)hipEventDestroy(h->flag_ready);
        delete h;
        return fail(PHX_EHIP, "phx_create: %s", hipGetErrorString(e));
    }
    memset(h->host, 0, (OBS_SLOTS + 2) * sizeof(double));
    h->cur = f->psi;
    h->stage_tiles = L.tiles;
    {
        const StepShapeId* shapes;
        step_shapes(cfg->precision, &shapes);
        h->step_shape = shapes[0];
        if (cfg->imag_time || cfg->drive || cfg->components == 2) h->step_shape = StepShapeId{1, 40};  // streaming
        if (cfg->tile_wx != 0 && L.family == PHX_KERNEL_STEP) h->step_shape = StepShapeId{cfg->tile_wx, cfg->tile_rows};
    }
    if (cfg->integrator == PHX_RK45) {
        s = create_rk45(h);
        if (s != PHX_OK) {
            phx_destroy(h);
            return s;
        }
    }
    *out = h;
    return PHX_OK;
}

// Reads the non-finite flag copied back by an earlier phx_step, if that copy has
// completed; never blocks.
static void poll_flag(phx_handle* h)
{
    if (!h->flag_pending) return;
    if (hipEventQuery(h->flag_ready) != hipSuccess) return;
    h->flag_pending = false;
    unsigned int v;
    memcpy(&v, &h->host[OBS_SLOTS], sizeof(v));
    if (v) h->info.nonfinite = 1;
}

namespace phx {
template <typename R>
phx_status rk4_stage_launches(phx_handle* h, int64_t n, hipStream_t stream)
{
    const phx_config& c = h->cfg;
    const Layout& L = h->L;
    using C = typename cvec<R>::type;
    Rk4Args<R> a{};
    a.nx = c.nx;
    a.ny = c.ny;
    a.bcx = c.bc_x;
    a.bcy = c.bc_y;
    a.comps = c.components;
    a.tiles_x = h->stage_tiles.tiles_x;
    a.tiles = h->stage_tiles.tiles;
    a.ts = h->stage_tiles.ts;
    a.cstride = (int64_t)c.nx * c.ny;
    a.c = make_coef<R>(c);
    a.V = (const R*)h->f.V;
    a.P = (const R*)h->f.P;
    a.flag = (unsigned int*)(h->ws + L.flag);
    C* psi = (C*)h->f.psi;
    R* n0 = (R*)h->f.n;
    C* Y[2] = {(C*)(h->ws + L.y[0]), (C*)(h->ws + L.y[1])};
    R* YN[2] = {c.reservoir ? (R*)(h->ws + L.yn[0]) : nullptr, c.reservoir ? (R*)(h->ws + L.yn[1]) : nullptr};
    a.acc = (C*)(h->ws + L.acc);
    a.accn = c.reservoir ? (R*)(h->ws + L.accn) : nullptr;
    a.psi = psi;
    a.n = n0;
    a.psi_io = psi;
    a.n_io = n0;
    a.E = c.drive ? (const C*)h->f.E : nullptr;
    a.drive_ph = c.drive ? (const C*)(h->ws + L.drive_ph) : nullptr;
    a.imag = c.imag_time;
    const R half_dt = (R)(0.5 * c.dt), full_dt = (R)c.dt;
    a.dt6 = (R)(c.dt / 6.0);
    const bool res = c.reservoir != 0, hv = h->f.V != nullptr;
    for (int64_t k = 0; k < n; ++k) {
        if (c.drive && launch_drive_phasors<R>(h, k, stream) != hipSuccess)
            return fail(PHX_EHIP, "drive phasor launch failed");
        // stage 1: argument = state; stage s reads y written by stage s-1
        const C* yin[4] = {psi, Y[0], Y[1], Y[0]};
        const R* ynin[4] = {n0, YN[0], YN[1], YN[0]};
        C* yout[4] = {Y[0], Y[1], Y[0], nullptr};
        R* ynout[4] = {YN[0], YN[1], YN[0], nullptr};
        const R adt[4] = {half_dt, half_dt, full_dt, (R)0};
        for (int s = 0; s < 4; ++s) {
            a.y = yin[s];
            a.yn = ynin[s];
            a.y_out = yout[s];
            a.yn_out = ynout[s];
            a.a_dt = adt[s];
            hipEvent_t t0 = nullptr;
            hipError_t e = timing_begin(h, &t0);
            if (e == hipSuccess) e = launch_rk4_stage<R>(s + 1, res, hv, a, stream);
            if (e == hipSuccess) e = timing_end(h, t0, K_RK4_S1 + s);
            if (e != hipSuccess) return fail(PHX_EHIP, "RK4 stage %d launch: %s", s + 1, hipGetErrorString(e));
        }
        if (c.imag_time) {  // restore the call's starting norm
            hipEvent_t t0 = nullptr;
            hipError_t e = timing_begin(h, &t0);
            if (e == hipSuccess) e = launch_imag_norm<R>(h, psi, 1, stream);
            if (e == hipSuccess) e = timing_end(h, t0, K_IMAG_NORM);
            if (e == hipSuccess) e = timing_begin(h, &t0);
            if (e == hipSuccess) e = launch_imag_scale<R>(h, psi, stream);
            if (e == hipSuccess) e = timing_end(h, t0, K_IMAG_SCALE);
            if (e != hipSuccess) return fail(PHX_EHIP, "imaginary-time norm launch: %s", hipGetErrorString(e));
        }
        if (c.noise > 0.0) {
            hipEvent_t t0 = nullptr;
            hipError_t e = timing_begin(h, &t0);
            if (e == hipSuccess) e = launch_noise<R>(h, psi, n0, k, stream);
            if (e == hipSuccess) e = timing_end(h, t0, K_NOISE);
            if (e != hipSuccess) return fail(PHX_EHIP, "noise launch: %s", hipGetErrorString(e));
        }
    }
    if (uses_step_index(c) && n > 0 && advance_noise_step(h, n, stream) != hipSuccess)
        return fail(PHX_EHIP, "step index advance launch failed");
    return PHX_OK;
}

}  // namespace phx

// Trial launches of the stage-fused kernels for the tuner: stage 1 from the state
// into the workspace, then stage 2 between workspace buffers with shape ts.  The
// caller's arrays are only read.
namespace phx {
template <typename R>
hipError_t rk4_stage_trial(phx_handle* h, const TileShape& ts)
{
    using C = typename cvec<R>::type;
    const phx_config& c = h->cfg;
    const Layout& L = h->L;
    Rk4Args<R> a{};
    a.nx = c.nx;
    a.ny = c.ny;
    a.bcx = c.bc_x;
    a.bcy = c.bc_y;
    a.comps = c.components;
    const TilePlan tp = plan_tiles(c.nx, c.ny, ts.wx, ts.rows);
    a.tiles_x = tp.tiles_x;
    a.tiles = tp.tiles;
    a.ts = tp.ts;
    a.cstride = (int64_t)c.nx * c.ny;
    a.c = make_coef<R>(c);
    a.V = (const R*)h->f.V;
    a.P = (const R*)h->f.P;
    a.flag = (unsigned int*)(h->ws + L.flag);
    a.psi = (const C*)h->f.psi;
    a.n = (const R*)h->f.n;
    a.acc = (C*)(h->ws + L.acc);
    a.accn = c.reservoir ? (R*)(h->ws + L.accn) : nullptr;
    a.y = (const C*)(h->ws + L.y[0]);
    a.yn = c.reservoir ? (const R*)(h->ws + L.yn[0]) : nullptr;
    a.y_out = (C*)(h->ws + L.y[1]);
    a.yn_out = c.reservoir ? (R*)(h->ws + L.yn[1]) : nullptr;
    a.a_dt = (R)(0.5 * c.dt);
    return launch_rk4_stage<R>(2, c.reservoir != 0, h->f.V != nullptr, a, h->stream);
}

template hipError_t rk4_stage_trial<float>(phx_handle*, const TileShape&);
template hipError_t rk4_stage_trial<double>(phx_handle*, const TileShape&);
}  // namespace phx

namespace phx {
int graph_chunk(const phx_config& c)
{
    if (c.graph_steps < 0) return 0;
    const int g = c.graph_steps == 0 ? 64 : c.graph_steps;
    return (g + 1) & ~1;  // even, so that a replay of the whole-step family ends in the same buffer
}

// Enqueues n RK4 steps on the handle's stream: whole chunks as replays of one
// captured graph, the remainder directly.  With kernel timing on, everything is
// launched directly so that each kernel is bracketed by events.
template <typename R>
static phx_status rk4_run(phx_handle* h, int64_t n)
{
    const bool step = h->L.family == PHX_KERNEL_STEP;
    auto direct = [&](hipStream_t s, int64_t k) {
        return step ? rk4_fused_launches<R>(h, k, s) : rk4_stage_launches<R>(h, k, s);
    };
    const int G = graph_chunk(h->cfg);
    if (h->timing || G == 0 || n < G) return direct(h->stream, n);
    if (!h->graph || h->graph_dirty) {
        if (h->graph) {
            (void)hipGraphExecDestroy(h->graph);
            h->graph = nullptr;
        }
        if (!h->cap_stream && hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess)
            return fail(PHX_EHIP, "capture stream creation failed");
        // the capture stream must not run ahead of work already queued on the caller's stream
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return fail(PHX_EHIP, "graph capture: %s", hipGetErrorString(e));
        phx_status st = direct(h->cap_stream, G);
        e = hipStreamEndCapture(h->cap_stream, &g);
        if (st != PHX_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (e != hipSuccess) return fail(PHX_EHIP, "graph instantiation: %s", hipGetErrorString(e));
        h->graph_dirty = false;
    }
    for (int64_t k = 0; k < n / G; ++k) {
        hipError_t e = hipGraphLaunch(h->graph, h->stream);
        if (e != hipSuccess) return fail(PHX_EHIP, "graph launch: %s", hipGetErrorString(e));
    }
    return direct(h->stream, n % G);
}

}  // namespace phx

namespace phx {
template <typename R> phx_status rk4_run_graph(phx_handle* h, int64_t n) { return rk4_run<R>(h, n); }
template phx_status rk4_run_graph<float>(phx_handle*, int64_t);
template phx_status rk4_run_graph<double>(phx_handle*, int64_t);
template phx_status rk4_stage_launches<float>(phx_handle*, int64_t, hipStream_t);
template phx_status rk4_stage_launches<double>(phx_handle*, int64_t, hipStream_t);
}  // namespace phx

phx_status phx_step(phx_handle* h, int64_t n_steps, phx_info* out)
{
    clear_error();
    if (!h) return fail(PHX_EINVAL, "handle is NULL");
    if (n_steps < 0) return fail(PHX_EINVAL, "n_steps must be >= 0");
    if (h->cfg.integrator == PHX_RK45) return step_rk45(h, n_steps, out);
    poll_flag(h);
    if (h->info.nonfinite) {
        if (out) *out = h->info;
        return fail(PHX_ENONFINITE, "a non-finite value appeared in the state before step %lld",
                    (long long)h->info.steps_accepted);
    }
    if (n_steps > 0) {
        phx_status s;
        const bool c64 = h->cfg.precision == PHX_C64;
        if (h->cfg.imag_time) {  // the norm every step of this call returns to (scale 1 to start)
            const hipError_t e = c64 ? launch_imag_norm<float>(h, h->f.psi, 0, h->stream)
                                     : launch_imag_norm<double>(h, h->f.psi, 0, h->stream);
            if (e != hipSuccess) return fail(PHX_EHIP, "imaginary-time norm launch: %s", hipGetErrorString(e));
        }
        if (h->L.family == PHX_KERNEL_STEP)
            s = c64 ? rk4_fused_steps<float>(h, n_steps) : rk4_fused_steps<double>(h, n_steps);
        else
            s = c64 ? rk4_run<float>(h, n_steps) : rk4_run<double>(h, n_steps);
        if (s != PHX_OK) return s;
        if (h->cfg.imag_time && h->L.family == PHX_KERNEL_STEP) {
            // the streaming kernel applies each step's restoring scale to its input; the
            // last one is applied here so that the state ends normalized
            const hipError_t e = c64 ? launch_imag_scale<float>(h, h->f.psi, h->stream)
                                     : launch_imag_scale<double>(h, h->f.psi, h->stream);
            if (e != hipSuccess) return fail(PHX_EHIP, "imaginary-time scale launch: %s", hipGetErrorString(e));
        }
        HIP_OR_FAIL(hipMemcpyAsync(&h->host[OBS_SLOTS], h->ws + h->L.flag, sizeof(unsigned int),
                                   hipMemcpyDeviceToHost, h->stream));
        HIP_OR_FAIL(hipEventRecord(h->flag_ready, h->stream));
        h->flag_pending = true;
        h->info.steps_accepted += n_steps;
        h->info.t += (double)n_steps * h->cfg.dt;
    }
    if (out) *out = h->info;
    return PHX_OK;
}

namespace phx {

template <typename R>
ObsArgs<R> obs_args(const phx_config& c, const TilePlan& tiles, const void* psi, const void* n, const void* V,
                    const void* P, const void* E, double t, double* partials, double* out)
{
    ObsArgs<R> a{};
    a.nx = c.nx;
    a.ny = c.ny;
    a.bcx = c.bc_x;
    a.bcy = c.bc_y;
    a.comps = c.components;
    a.reservoir = c.reservoir;
    a.tiles_x = tiles.tiles_x;
    a.tiles = tiles.tiles;
    a.ts = tiles.ts;
    a.cstride = (int64_t)c.nx * c.ny;
    a.c = make_coef<R>(c);
    a.inv_dx2 = 1.0 / (c.dx * c.dx);
    a.inv_dy2 = 1.0 / (c.dy * c.dy);
    a.delta_lt = c.delta_lt;
    a.inv_4dxdy = 1.0 / (4.0 * c.dx * c.dy);
    a.gamma_r_d = c.gamma_r;
    a.R_d = c.R;
    a.psi = (const typename cvec<R>::type*)psi;
    a.n = (const R*)n;
    a.V = (const R*)V;
    a.P = (const R*)P;
    a.partials = partials;
    a.out = out;
    if (c.drive) {  // the residual's right-hand side at time t
        a.E = (const typename cvec<R>::type*)E;
        const double th = c.drive_omega * t;
        a.drive_ph = typename cvec<R>::type{(R)cos(th), (R)-sin(th)};
    }
    return a;
}

template ObsArgs<float> obs_args<float>(const phx_config&, const TilePlan&, const void*, const void*, const void*,
                                        const void*, const void*, double, double*, double*);
template ObsArgs<double> obs_args<double>(const phx_config&, const TilePlan&, const void*, const void*, const void*,
                                          const void*, const void*, double, double*, double*);

void obs_from_slots(const phx_config& c, const double* q, phx_obs* out)
{
    const double A = c.dx * c.dy;
    memset(out, 0, sizeof(*out));
    out->norm[0] = A * q[O_NORM0];
    out->norm[1] = A * q[O_NORM1];
    out->reservoir = A * q[O_NSUM];
    out->e_kin = c.hbar * c.hbar / (2.0 * c.mass) * A * q[O_KIN];
    out->e_pot = A * q[O_POT];
    out->e_int = 0.5 * c.g * A * q[O_RHO2];
    out->e_cross = c.g_x * A * q[O_CROSS];
    out->e_tetm = A * q[O_TETM];
    out->e_res = c.g_r * A * q[O_RES];
    out->energy = out->e_kin + out->e_pot + out->e_int + out->e_cross + out->e_tetm + out->e_res;
    out->max_density = q[O_MAXRHO];
    out->steady_res_density = q[O_RHO2] > 0 ? sqrt(q[O_DRHO2]) / sqrt(q[O_RHO2]) : 0.0;
    out->steady_res_reservoir = (c.reservoir && q[O_P2] > 0) ? sqrt(q[O_FN2]) / sqrt(q[O_P2]) : 0.0;
    out->nonfinite = (int64_t)q[O_NONFINITE];
    const double vacuum = 0.5 * c.noise * (double)c.nx * (double)c.ny;  // nu/(2A) per cell, times A
    for (int s = 0; s < c.components; ++s) out->norm_renorm[s] = out->norm[s] - vacuum;
}

}  // namespace phx

template <typename R>
static phx_status observables_t(phx_handle* h)
{
    const ObsArgs<R> a = obs_args<R>(h->cfg, h->L.tiles, state_psi(h), state_n(h), h->f.V, h->f.P, h->f.E,
                                     h->info.t, (double*)(h->ws + h->L.partials), (double*)(h->ws + h->L.obs));
    hipEvent_t t0 = nullptr;
    hipError_t e = timing_begin(h, &t0);
    if (e == hipSuccess) e = launch_observables<R>(a, h->L.obs_blocks, h->stream);
    if (e == hipSuccess) e = timing_end(h, t0, K_OBS);
    if (e != hipSuccess) return fail(PHX_EHIP, "observables launch: %s", hipGetErrorString(e));
    return PHX_OK;
}

phx_status phx_observables(phx_handle* h, phx_obs* out)
{
    clear_error();
    if (!h || !out) return fail(PHX_EINVAL, "handle or out is NULL");
    phx_status s = h->cfg.precision == PHX_C64 ? observables_t<float>(h) : observables_t<double>(h);
    if (s != PHX_OK) return s;
    HIP_OR_FAIL(hipMemcpyAsync(h->host, h->ws + h->L.obs, OBS_SLOTS * sizeof(double),
                               hipMemcpyDeviceToHost, h->stream));
    HIP_OR_FAIL(hipStreamSynchronize(h->stream));
    obs_from_slots(h->cfg, h->host, out);
    poll_flag(h);
    return PHX_OK;
}

phx_status phx_get_info(const phx_handle* h, phx_info* out)
{
    clear_error();
    if (!h || !out) return fail(PHX_EINVAL, "handle or out is NULL");
    poll_flag(const_cast<phx_handle*>(h));
    *out = h->info;
    return PHX_OK;
}

phx_status phx_set_info(phx_handle* h, const phx_info* in)
{
    clear_error();
    if (!h || !in) return fail(PHX_EINVAL, "handle or in is NULL");
    if (!isfinite(in->t) || !finite_pos(in->dt) || in->steps_accepted < 0 || in->steps_rejected < 0)
        return fail(PHX_EINVAL, "invalid info record");
    if (h->cfg.integrator == PHX_RK4 && in->dt != h->cfg.dt)
        return fail(PHX_EINVAL, "RK4 dt is fixed by the configuration");
    if (h->cfg.integrator == PHX_RK45) return set_info_rk45(h, in);
    if (!in->nonfinite) {
        // the caller restored a good state: clear the device flag and any pending read
        HIP_OR_FAIL(hipStreamSynchronize(h->stream));
        HIP_OR_FAIL(hipMemsetAsync(h->ws + h->L.flag, 0, 256, h->stream));
        h->flag_pending = false;
    }
    // the next Wiener increment continues the restored run's sequence; the drive's
    // clock restarts at (t, steps_accepted), which captured graphs hold as arguments
    if (uses_step_index(h->cfg)) HIP_OR_FAIL(set_noise_step(h, in->steps_accepted, h->stream));
    if (h->cfg.drive) {
        h->drive_t0 = in->t;
        h->drive_k0 = in->steps_accepted;
        h->graph_dirty = true;
    }
    h->info = *in;
    return PHX_OK;
}

// ---------------------------------------------------------------- kernel timing

namespace phx {

const char* kernel_kind_name(int k)
{
    static const char* names[K_KINDS_] = {
        "rk4_stage1", "rk4_stage2", "rk4_stage3", "rk4_stage4", "observables",
        "dp_stage1", "dp_stage2", "dp_stage3", "dp_stage4", "dp_stage5", "dp_stage6",
        "dp_stage7", "dp_error", "batch_stage", "rk4_step", "wiener_noise", "imag_norm", "imag_scale"};
    return (k >= 0 && k < K_KINDS_) ? names[k] : "unknown";
}

static hipError_t get_event(phx_handle* h, hipEvent_t* ev)
{
    if (!h->free_events.empty()) {
        *ev = h->free_events.back();
        h->free_events.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(ev);
}

hipError_t timing_begin(phx_handle* h, hipEvent_t* start)
{
    *start = nullptr;
    if (!h->timing) return hipSuccess;
    hipError_t e = get_event(h, start);
    if (e != hipSuccess) return e;
    return hipEventRecord(*start, h->stream);
}

hipError_t timing_end(phx_handle* h, hipEvent_t start, int kind)
{
    if (!h->timing || !start) return hipSuccess;
    hipEvent_t stop;
    hipError_t e = get_event(h, &stop);
    if (e != hipSuccess) return e;
    e = hipEventRecord(stop, h->stream);
    if (e != hipSuccess) return e;
    h->pending.push_back({start, stop, kind});
    return hipSuccess;
}

}  // namespace phx

phx_status phx_log_attempts(phx_handle* h, double* log, int64_t cap, int64_t* count)
{
    clear_error();
    if (!h) return fail(PHX_EINVAL, "handle is NULL");
    if (h->cfg.integrator != PHX_RK45) return fail(PHX_EUNSUPPORTED, "the attempt log is for RK45 handles");
    if (log && (cap < 0 || !count)) return fail(PHX_EINVAL, "attempt log needs cap >= 0 and a count");
    h->att_log = log;
    h->att_cap = log ? cap : 0;
    h->att_count = log ? count : nullptr;
    return PHX_OK;
}

phx_status phx_set_timing(phx_handle* h, int32_t enable)
{
    clear_error();
    if (!h) return fail(PHX_EINVAL, "handle is NULL");
    if (enable != 0 && enable != 1) return fail(PHX_EINVAL, "enable must be 0 or 1");
    h->timing = enable != 0;
    for (int k = 0; k < PHX_MAX_KERNEL_KINDS; ++k) {
        h->kind_ms[k] = 0.0;
        h->kind_launches[k] = 0;
    }
    return PHX_OK;
}

phx_status phx_kernel_times(phx_handle* h, phx_timing* out)
{
    clear_error();
    if (!h || !out) return fail(PHX_EINVAL, "handle or out is NULL");
    HIP_OR_FAIL(hipStreamSynchronize(h->stream));
    for (const auto& t : h->pending) {
        float ms = 0.f;
        HIP_OR_FAIL(hipEventElapsedTime(&ms, t.start, t.stop));
        h->kind_ms[t.kind] += ms;
        h->kind_launches[t.kind] += 1;
        h->free_events.push_back(t.start);
        h->free_events.push_back(t.stop);
    }
    h->pending.clear();
    memset(out, 0, sizeof(*out));
    for (int k = 0; k < K_KINDS_ && k < PHX_MAX_KERNEL_KINDS; ++k) {
        if (!h->kind_launches[k]) continue;
        const int c = out->count++;
        snprintf(out->name[c], sizeof(out->name[c]), "%s", kernel_kind_name(k));
        out->launches[c] = h->kind_launches[k];
        out->ms_total[c] = h->kind_ms[k];
    }
    return PHX_OK;
}

void phx_destroy(phx_handle* h)
{
    if (!h) return;
    if (!h->pending.empty()) (void)hipStreamSynchronize(h->stream);
    for (const auto& t : h->pending) {
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    for (hipEvent_t e : h->free_events) (void)hipEventDestroy(e);
    if (h->graph) (void)hipGraphExecDestroy(h->graph);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->host) (void)hipHostFree(h->host);
    (void)hipEventDestroy(h->flag_ready);
    delete h;
}

const char* phx_last_error(void) { return last_error(); }

// Accessors used by the other translation units.
namespace phx {
const void* state_psi(const phx_handle* h) { return h->cur ? h->cur : h->f.psi; }
const void* state_n(const phx_handle* h) { return h->f.n; }
}  // namespace phx
