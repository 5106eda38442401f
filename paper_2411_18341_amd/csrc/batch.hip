// Batched whole-step RK4 over many independent one-component instances on grids of
// different sizes: one persistent launch per step.  The work list is the
// concatenation of every instance's regions (56 x (H-8) output cells each, H the
// region height of the step kernel); a workgroup takes items w = blockIdx.x,
// blockIdx.x + gridDim.x, ..., finds the instance by binary search over the
// instances' first item, and runs the same device code as the single-grid
// whole-step kernel on that instance's slice of the packed arrays.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "philox.h"
#include "runtime.h"
#include "step_body.h"
#include "stream_body.h"
#include "stream_wide.h"

namespace phx {

template <typename R>
struct BatchInst {
    int nx, ny, bcx, bcy;
    int tiles_x, tile0;  // regions across x; first work item of this instance (region form)
    int s_tile0;         // first work item of this instance in the streaming form
    int w_strips;        // wide streaming form (complex64): strips of 120 columns, else 0
    int w_band;          // wide streaming form: rows per band
    int w_tile0;         // first work item of this instance in the wide streaming form
    int64_t offset;      // element offset in the packed arrays
    Coef<R> c;
    R half_dt, dt, dt6;
    // Wiener noise: amplitude^2 = noise_a n + noise_b, key, first workgroup of this
    // instance in the noise pass (each instance's cell pairs fill whole workgroups)
    R noise_a, noise_b;
    uint32_t key0, key1;
    int block0;
};

// Wiener increments of one batched step: one thread per cell pair, each instance's
// pairs in whole workgroups (block_inst maps a workgroup to its instance), the same
// counters and transform as a single-grid handle with the instance's seed.
template <typename R, bool RES>
__global__ __launch_bounds__(256) void batch_noise_kernel(const BatchInst<R>* __restrict__ inst,
                                                          const int* __restrict__ block_inst,
                                                          typename cvec<R>::type* psi, const R* n, uint64_t step)
{
    const BatchInst<R>& I = inst[block_inst[blockIdx.x]];
    if (I.noise_a == (R)0 && I.noise_b == (R)0) return;
    const int64_t p = (int64_t)(blockIdx.x - I.block0) * 256 + threadIdx.x;
    const int64_t q = 2 * p;
    const int64_t cells = (int64_t)I.nx * I.ny;
    if (q >= cells) return;
    const noise::Philox4 x = noise::philox4x32_10((uint32_t)p, 0u, (uint32_t)step, (uint32_t)(step >> 32), I.key0,
                                                  I.key1);
    const int64_t k = I.offset + q;
    noise::noise_pair<R, RES>(psi + k, RES ? n + k : nullptr, q + 1 < cells, (k & 1) == 0, I.noise_a, I.noise_b, x);
}

template <typename R, bool RES, bool HASV, bool GHOSTS, int WAVES, int ROWS>
__global__ __launch_bounds__(WAVES * 64) void batch_step_kernel(
    const BatchInst<R>* __restrict__ inst, int count, int total,
    const typename cvec<R>::type* psi_in, const R* n_in, typename cvec<R>::type* psi_out, R* n_out,
    const R* V, const R* P, unsigned int* flag)
{
    __shared__ typename cvec<R>::type edge[2][WAVES][2][64];
    bool bad = false;
    for (int w = blockIdx.x; w < total; w += gridDim.x) {
        const int t = xcd_tile(w, total);
        int lo = 0, hi = count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (inst[mid].tile0 <= t) lo = mid; else hi = mid - 1;
        }
        const BatchInst<R>& I = inst[lo];
        StepArgs<R> a;
        a.nx = I.nx;
        a.ny = I.ny;
        a.bcx = I.bcx;
        a.bcy = I.bcy;
        a.tiles_x = I.tiles_x;
        a.tiles = 0;
        a.c = I.c;
        a.half_dt = I.half_dt;
        a.dt = I.dt;
        a.dt6 = I.dt6;
        a.psi_in = psi_in + I.offset;
        a.n_in = RES ? n_in + I.offset : nullptr;
        a.psi_out = psi_out + I.offset;
        a.n_out = RES ? n_out + I.offset : nullptr;
        a.V = HASV ? V + I.offset : nullptr;
        a.P = RES ? P + I.offset : nullptr;
        a.flag = flag;
        bad = step_region<R, RES, HASV, GHOSTS, WAVES, ROWS>(a, t - I.tile0, edge) || bad;
    }
    if (bad) flag[0] = 1u;  // benign race: every writer stores 1
}

// region shape of the batched kernel per precision (8 waves x 4 rows)
constexpr int BW = 8, BR = 4;

// Streaming form of the batched step (the band walk of stream_body.h): a work item is
// one band of SB rows of SG adjacent strips of one instance, one workgroup per item
// (consecutive items on one XCD); tiles_x counts an instance's strips of 56 columns.
// Single-strip items (one wave each) measured 1 % faster on the batched workload than
// groups of 2 or 4 strips, whose waves share nothing.  YZERO: every instance has a
// zero y boundary (else every one is periodic in y).
constexpr int SB = 40, SG = 1;

template <typename R, bool RES, bool HASV, bool GHOSTS, bool YZERO>
__global__ __launch_bounds__(64 * SG) void batch_stream_kernel(
    const BatchInst<R>* __restrict__ inst, int count, const typename cvec<R>::type* psi_in, const R* n_in,
    typename cvec<R>::type* psi_out, R* n_out, const R* V, const R* P, unsigned int* flag)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (inst[mid].s_tile0 <= t) lo = mid; else hi = mid - 1;
    }
    const BatchInst<R>& I = inst[lo];
    const int lt = t - I.s_tile0;
    const int gx = (I.tiles_x + SG - 1) / SG;
    const int band = lt / gx, strip = (lt - band * gx) * SG + wave;
    if (strip >= I.tiles_x) return;
    StepArgs<R> a{};
    a.nx = I.nx;
    a.ny = I.ny;
    a.bcx = I.bcx;
    a.bcy = I.bcy;
    a.tiles_x = I.tiles_x;
    a.c = I.c;
    a.half_dt = I.half_dt;
    a.dt = I.dt;
    a.dt6 = I.dt6;
    a.psi_in = psi_in + I.offset;
    a.n_in = RES ? n_in + I.offset : nullptr;
    a.psi_out = psi_out + I.offset;
    a.n_out = RES ? n_out + I.offset : nullptr;
    a.V = HASV ? V + I.offset : nullptr;
    a.P = RES ? P + I.offset : nullptr;
    a.comps = 1;
    if (stream_band<R, RES, HASV, GHOSTS, YZERO, SB>(a, strip, band, (band & 1) ? -1 : 1))
        flag[0] = 1u;  // benign race: every writer stores 1
}

template <typename R, bool RES, bool HASV, bool GHOSTS, bool YZERO>
static hipError_t launch_batch_stream_t(int total, const BatchInst<R>* inst, int count, const void* pi,
                                        const void* ni, void* po, void* no, const void* V, const void* P,
                                        unsigned int* flag, hipStream_t s)
{
    using C = typename cvec<R>::type;
    batch_stream_kernel<R, RES, HASV, GHOSTS, YZERO><<<total, 64 * SG, 0, s>>>(
        inst, count, (const C*)pi, (const R*)ni, (C*)po, (R*)no, (const R*)V, (const R*)P, flag);
    return hipGetLastError();
}

template <typename R>
static hipError_t launch_batch_stream(bool res, bool hv, bool ghosts, bool yzero, int total, const BatchInst<R>* inst,
                                      int count, const void* pi, const void* ni, void* po, void* no, const void* V,
                                      const void* P, unsigned int* flag, hipStream_t s)
{
#define PHX_BS(RS, HV, G, Y) \
    if (res == RS && hv == HV && ghosts == G && yzero == Y) \
        return launch_batch_stream_t<R, RS, HV, G, Y>(total, inst, count, pi, ni, po, no, V, P, flag, s)
    PHX_BS(true, false, false, false); PHX_BS(true, true, false, false);
    PHX_BS(false, false, false, false); PHX_BS(false, true, false, false);
    PHX_BS(true, false, true, false); PHX_BS(true, true, true, false);
    PHX_BS(false, false, true, false); PHX_BS(false, true, true, false);
    PHX_BS(true, false, true, true); PHX_BS(true, true, true, true);
    PHX_BS(false, false, true, true); PHX_BS(false, true, true, true);
#undef PHX_BS
    return hipErrorInvalidValue;
}

// Wide streaming form of the batched step (the two-column walk of stream_wide.h) for
// complex64 instances of even width: a work item is one band of an instance's w_band
// rows of one 120-column strip, one single-wave workgroup per item (consecutive items
// on one XCD).  The register budget per wave and the testing variant (CHECK, the last
// step of a call) follow the single-grid wide kernel with the 8-row ring.
template <bool RES, bool HASV, bool GHOSTS, bool YZERO, int WPE, bool CHECK>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE)))
void batch_wide_kernel(const BatchInst<float>* __restrict__ inst, int count, const float2* psi_in, const float* n_in,
                       float2* psi_out, float* n_out, const float* V, const float* P, unsigned int* flag)
{
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (inst[mid].w_tile0 <= t) lo = mid; else hi = mid - 1;
    }
    const BatchInst<float>& I = inst[lo];
    const int lt = t - I.w_tile0;
    const int band = lt / I.w_strips, strip = lt - band * I.w_strips;
    StepArgs<float> a{};
    a.nx = I.nx;
    a.ny = I.ny;
    a.bcx = I.bcx;
    a.bcy = I.bcy;
    a.tiles_x = I.w_strips;
    a.c = I.c;
    a.half_dt = I.half_dt;
    a.dt = I.dt;
    a.dt6 = I.dt6;
    a.psi_in = psi_in + I.offset;
    a.n_in = RES ? n_in + I.offset : nullptr;
    a.psi_out = psi_out + I.offset;
    a.n_out = RES ? n_out + I.offset : nullptr;
    a.V = HASV ? V + I.offset : nullptr;
    a.P = RES ? P + I.offset : nullptr;
    a.comps = 1;
    a.band_rows = I.w_band;
    if (stream_band_wide<RES, HASV, GHOSTS, YZERO, 8, 3, CHECK>(a, strip, band, I.w_band, (band & 1) ? -1 : 1))
        flag[0] = 1u;  // benign race: every writer stores 1
}

template <bool RES, bool HASV, bool GHOSTS, bool YZERO>
static hipError_t launch_batch_wide_t(int total, const BatchInst<float>* inst, int count, const void* pi,
                                      const void* ni, void* po, void* no, const void* V, const void* P,
                                      unsigned int* flag, bool check, hipStream_t s)
{
    constexpr int WPE = !(RES && (HASV || GHOSTS)) ? 3 : 2;
    constexpr int WPE_CHECK = RES ? 2 : WPE;
    if (check)
        batch_wide_kernel<RES, HASV, GHOSTS, YZERO, WPE_CHECK, true><<<total, 64, 0, s>>>(
            inst, count, (const float2*)pi, (const float*)ni, (float2*)po, (float*)no, (const float*)V,
            (const float*)P, flag);
    else
        batch_wide_kernel<RES, HASV, GHOSTS, YZERO, WPE, false><<<total, 64, 0, s>>>(
            inst, count, (const float2*)pi, (const float*)ni, (float2*)po, (float*)no, (const float*)V,
            (const float*)P, flag);
    return hipGetLastError();
}

static hipError_t launch_batch_wide(bool res, bool hv, bool ghosts, bool yzero, int total,
                                    const BatchInst<float>* inst, int count, const void* pi, const void* ni, void* po,
                                    void* no, const void* V, const void* P, unsigned int* flag, bool check,
                                    hipStream_t s)
{
#define PHX_BW(RS, HV, G, Y) \
    if (res == RS && hv == HV && ghosts == G && yzero == Y) \
        return launch_batch_wide_t<RS, HV, G, Y>(total, inst, count, pi, ni, po, no, V, P, flag, check, s)
    PHX_BW(true, false, false, false); PHX_BW(true, true, false, false);
    PHX_BW(false, false, false, false); PHX_BW(false, true, false, false);
    PHX_BW(true, false, true, false); PHX_BW(true, true, true, false);
    PHX_BW(false, false, true, false); PHX_BW(false, true, true, false);
    PHX_BW(true, false, true, true); PHX_BW(true, true, true, true);
    PHX_BW(false, false, true, true); PHX_BW(false, true, true, true);
#undef PHX_BW
    return hipErrorInvalidValue;
}

// Band height of the batched wide walk: about 48 rows, evened out over an instance's
// bands (the walk's 8 halo rows per band then cover no empty rows).
constexpr int kBatchWideRows = 48;
static int batch_wide_band(int ny)
{
    const int bands = (ny + kBatchWideRows - 1) / kBatchWideRows;
    const int b = (ny + bands - 1) / bands;
    return b < 8 ? 8 : b;
}

template <typename R, bool RES, bool HASV, bool GHOSTS>
static hipError_t launch_batch_t(int grid, const BatchInst<R>* inst, int count, int total, const void* pi,
                                 const void* ni, void* po, void* no, const void* V, const void* P,
                                 unsigned int* flag, hipStream_t s)
{
    using C = typename cvec<R>::type;
    batch_step_kernel<R, RES, HASV, GHOSTS, BW, BR><<<grid, BW * 64, 0, s>>>(
        inst, count, total, (const C*)pi, (const R*)ni, (C*)po, (R*)no, (const R*)V, (const R*)P, flag);
    return hipGetLastError();
}

template <typename R>
static hipError_t launch_batch(bool res, bool hv, bool ghosts, int grid, const BatchInst<R>* inst, int count,
                               int total, const void* pi, const void* ni, void* po, void* no, const void* V,
                               const void* P, unsigned int* flag, hipStream_t s)
{
#define PHX_B(RS, HV, G) \
    if (res == RS && hv == HV && ghosts == G) \
        return launch_batch_t<R, RS, HV, G>(grid, inst, count, total, pi, ni, po, no, V, P, flag, s)
    PHX_B(true, false, false); PHX_B(true, true, false); PHX_B(false, false, false); PHX_B(false, true, false);
    PHX_B(true, false, true); PHX_B(true, true, true); PHX_B(false, false, true); PHX_B(false, true, true);
#undef PHX_B
    return hipErrorInvalidValue;
}

struct BatchLayout {
    size_t table, block_inst, alt, alt_n, flag, total;
};

// Workgroups of the noise pass: each instance's cell pairs in whole workgroups of 256.
static int64_t noise_blocks_bound(const phx_batch_desc& d) { return d.total_cells / 512 + d.count + 1; }

static BatchLayout batch_layout(const phx_batch_desc& d)
{
    const size_t rs = d.precision == PHX_C64 ? 4 : 8;
    const size_t inst_bytes = d.precision == PHX_C64 ? sizeof(BatchInst<float>) : sizeof(BatchInst<double>);
    BatchLayout L{};
    size_t off = 0;
    auto take = [&](size_t b) { size_t o = off; off += align_up(b); return o; };
    L.flag = take(256);
    L.table = take((size_t)d.count * inst_bytes);
    L.block_inst = take((size_t)noise_blocks_bound(d) * sizeof(int));
    L.alt = take((size_t)d.total_cells * 2 * rs);
    const bool res = d.params && d.n_params > 0 && d.params[0].reservoir;
    L.alt_n = res ? take((size_t)d.total_cells * rs) : 0;
    L.total = off;
    return L;
}

static phx_status validate_batch(const phx_batch_desc* d)
{
    if (!d) return fail(PHX_EINVAL, "descriptor is NULL");
    if (d->count < 1) return fail(PHX_EINVAL, "count must be >= 1");
    if (d->precision != PHX_C64 && d->precision != PHX_C128) return fail(PHX_EINVAL, "bad precision");
    if (!d->instances || !d->params || d->n_params < 1) return fail(PHX_EINVAL, "instances and params required");
    if (d->check_finite != 0 && d->check_finite != 1) return fail(PHX_EINVAL, "check_finite must be 0 or 1");
    if (d->total_cells < 1 || d->total_cells >= ((int64_t)1 << 40)) return fail(PHX_EINVAL, "bad total_cells");
    if (d->step0 < 0) return fail(PHX_EINVAL, "step0 must be >= 0");
    const int res = d->params[0].reservoir;
    for (int k = 0; k < d->n_params; ++k) {
        phx_config c = d->params[k];
        c.nx = c.ny = 1;
        c.components = 1;
        c.precision = d->precision;
        c.integrator = PHX_RK4;
        c.kernel = PHX_KERNEL_AUTO;
        c.tile_wx = c.tile_rows = 0;
        phx_status s = validate_config(&c);
        if (s != PHX_OK) return s;
        if (c.drive != 0) return fail(PHX_EUNSUPPORTED, "the coherent drive is not implemented for batches");
        if (c.imag_time != 0) return fail(PHX_EUNSUPPORTED, "imaginary time is not implemented for batches");
        if (c.reservoir != res) return fail(PHX_EINVAL, "all params must share the reservoir flag");
    }
    std::vector<std::pair<int64_t, int64_t>> spans;
    spans.reserve(d->count);
    int64_t tiles = 0;
    for (int k = 0; k < d->count; ++k) {
        const phx_instance& I = d->instances[k];
        if (I.nx < 1 || I.ny < 1 || (int64_t)I.nx * I.ny >= ((int64_t)1 << 31))
            return fail(PHX_EINVAL, "instance %d: bad grid %d x %d", k, I.nx, I.ny);
        if (I.param_index < 0 || I.param_index >= d->n_params || I.reserved != 0)
            return fail(PHX_EINVAL, "instance %d: bad param_index or reserved field", k);
        if (I.offset < 0 || I.offset + (int64_t)I.nx * I.ny > d->total_cells)
            return fail(PHX_EINVAL, "instance %d: slice outside the packed arrays", k);
        phx_config c = d->params[I.param_index];
        c.nx = I.nx;
        c.ny = I.ny;
        c.components = 1;
        c.precision = d->precision;
        c.integrator = PHX_RK4;
        c.kernel = PHX_KERNEL_AUTO;
        c.tile_wx = c.tile_rows = 0;
        phx_status s = validate_config(&c);  // stability of dt on this grid
        if (s != PHX_OK) return s;
        spans.push_back({I.offset, I.offset + (int64_t)I.nx * I.ny});
        tiles += (int64_t)((I.nx + 55) / 56) * ((I.ny + BW * BR - 9) / (BW * BR - 8));
    }
    if (tiles >= ((int64_t)1 << 31)) return fail(PHX_EINVAL, "too many work items");
    std::sort(spans.begin(), spans.end());
    for (size_t k = 1; k < spans.size(); ++k)
        if (spans[k].first < spans[k - 1].second) return fail(PHX_EINVAL, "instance slices overlap");
    if (!d->psi || (res && (!d->n || !d->P))) return fail(PHX_EINVAL, "psi (and n, P with the reservoir) required");
    const void* ptrs[] = {d->psi, d->n, d->P, d->V, d->workspace};
    for (const void* p : ptrs)
        if (p && ((uintptr_t)p & 255u)) return fail(PHX_EINVAL, "device pointers must be 256-byte aligned");
    return PHX_OK;
}

// When a batch has instances on both walks, the one-column launch of each step runs on
// a second stream of the device (created once, default priority), forked from the
// caller's stream before the step and joined back into it after, so that the two
// launches fill the device together rather than one after the other.
static hipStream_t side_stream(int dev)
{
    static std::mutex mu;
    static hipStream_t streams[64];
    if (dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess)
        streams[dev] = nullptr;
    return streams[dev];
}

// fork / join events of one call; they are released only after the last join has
// completed (the call then returns with its work finished)
struct ForkJoin {
    hipEvent_t fork = nullptr, join = nullptr;
    bool used = false;
    ~ForkJoin()
    {
        if (used && join) (void)hipEventSynchronize(join);
        if (fork) (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
    }
};

template <typename R>
static phx_status batch_run(const phx_batch_desc* d, int64_t n, hipStream_t stream)
{
    const BatchLayout L = batch_layout(*d);
    char* ws = (char*)d->workspace;
    const int res = d->params[0].reservoir;
    std::vector<BatchInst<R>> table(d->count);
    int tile0 = 0;
    int64_t s_tile0 = 0;
    std::vector<int> block_inst;
    bool ghosts = false, noisy = false;
    // the streaming form needs every instance's state under 2 GiB (32-bit buffer
    // offsets) and one y boundary rule for all instances
    bool use_stream = true, all_zero_y = true, all_periodic_y = true;
    int64_t w_tile0 = 0;  // work items of the wide streaming form (complex64 instances of even width)
    for (int k = 0; k < d->count; ++k) {
        const phx_instance& I = d->instances[k];
        phx_config c = d->params[I.param_index];
        c.nx = I.nx;
        c.ny = I.ny;
        BatchInst<R>& b = table[k];
        b.nx = I.nx;
        b.ny = I.ny;
        b.bcx = c.bc_x;
        b.bcy = c.bc_y;
        b.tiles_x = (I.nx + 55) / 56;
        b.tile0 = tile0;
        b.offset = I.offset;
        b.c = make_coef<R>(c);
        b.half_dt = (R)(0.5 * c.dt);
        b.dt = (R)c.dt;
        b.dt6 = (R)(c.dt / 6.0);
        tile0 += b.tiles_x * ((I.ny + BW * BR - 9) / (BW * BR - 8));
        // the one-column and the wide work lists give each instance a range in one of
        // them and an empty range in the other
        // complex64 instances of even width take the wide walk, the others the
        // one-column walk (on a second stream when both occur)
        const bool wide = sizeof(R) == 4 && I.nx % 2 == 0;
        b.w_strips = wide ? wide_strips(I.nx) : 0;
        b.w_band = batch_wide_band(I.ny);
        b.s_tile0 = (int)std::min<int64_t>(s_tile0, INT32_MAX);
        b.w_tile0 = (int)std::min<int64_t>(w_tile0, INT32_MAX);
        if (wide)
            w_tile0 += (int64_t)b.w_strips * ((I.ny + b.w_band - 1) / b.w_band);
        else
            s_tile0 += (int64_t)((b.tiles_x + SG - 1) / SG) * ((I.ny + SB - 1) / SB);
        use_stream = use_stream && (double)I.nx * I.ny * 2.0 * sizeof(R) < 2147483648.0 - 256.0;
        all_zero_y = all_zero_y && c.bc_y == PHX_BC_ZERO;
        all_periodic_y = all_periodic_y && c.bc_y == PHX_BC_PERIODIC;
        ghosts = ghosts || c.bc_x == PHX_BC_ZERO || c.bc_y == PHX_BC_ZERO;
        const double scale = c.noise * c.dt / (4.0 * c.dx * c.dy);  // as the single-grid pass forms it
        b.noise_a = (R)(scale * c.R);
        b.noise_b = (R)(scale * c.gamma_c);
        b.key0 = (uint32_t)I.seed;
        b.key1 = (uint32_t)(I.seed >> 32);
        b.block0 = (int)block_inst.size();
        const int64_t nb = (((int64_t)I.nx * I.ny + 1) / 2 + 255) / 256;
        block_inst.insert(block_inst.end(), (size_t)nb, k);
        noisy = noisy || c.noise > 0.0;
    }
    const int total = tile0;
    use_stream = use_stream && (all_zero_y || all_periodic_y) && s_tile0 < INT32_MAX && w_tile0 < INT32_MAX;
    const int s_total = (int)std::min<int64_t>(s_tile0, INT32_MAX);
    const int w_total = (int)std::min<int64_t>(w_tile0, INT32_MAX);
    hipError_t e = hipMemcpyAsync(ws + L.table, table.data(), table.size() * sizeof(BatchInst<R>),
                                  hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && noisy)
        e = hipMemcpyAsync(ws + L.block_inst, block_inst.data(), block_inst.size() * sizeof(int),
                           hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemsetAsync(ws + L.flag, 0, 256, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);  // the host table may go out of scope
    if (e != hipSuccess) return fail(PHX_EHIP, "batch table upload: %s", hipGetErrorString(e));

    // persistent grid: as many workgroups as fit on the device at once, a multiple
    // of 8 so that every workgroup stays on one XCD's share of the work list
    int dev = 0, cus = 256, per_cu = 1;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    }
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_step_kernel<R, true, false, false, BW, BR>,
                                                     BW * 64, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int grid = cus * per_cu;
    grid = std::min(grid, (total + 7) / 8 * 8);
    grid = (grid + 7) / 8 * 8;

    const size_t rs = sizeof(R);
    void* S[2] = {d->psi, ws + L.alt};
    void* SN[2] = {d->n, res ? ws + L.alt_n : nullptr};
    int cur = 0;
    if (n & 1) {
        e = hipMemcpyAsync(S[1], S[0], (size_t)d->total_cells * 2 * rs, hipMemcpyDeviceToDevice, stream);
        if (e == hipSuccess && res)
            e = hipMemcpyAsync(SN[1], SN[0], (size_t)d->total_cells * rs, hipMemcpyDeviceToDevice, stream);
        if (e != hipSuccess) return fail(PHX_EHIP, "batch state copy: %s", hipGetErrorString(e));
        cur = 1;
    }
    const BatchInst<R>* dtab = (const BatchInst<R>*)(ws + L.table);
    unsigned int* flag = (unsigned int*)(ws + L.flag);
    // both walks in use: the one-column launch goes to the device's second stream
    hipStream_t side = nullptr;
    ForkJoin fj;
    if (use_stream && w_total > 0 && s_total > 0) {
        side = side_stream(dev);
        if (side && (hipEventCreateWithFlags(&fj.fork, hipEventDisableTiming) != hipSuccess ||
                     hipEventCreateWithFlags(&fj.join, hipEventDisableTiming) != hipSuccess))
            side = nullptr;
    }
    for (int64_t k = 0; k < n; ++k) {
        if (use_stream) {
            e = hipSuccess;
            hipStream_t s_narrow = stream;
            if (side) {
                fj.used = true;
                e = hipEventRecord(fj.fork, stream);
                if (e == hipSuccess) e = hipStreamWaitEvent(side, fj.fork, 0);
                s_narrow = side;
            }
            if constexpr (sizeof(R) == 4) {
                if (e == hipSuccess && w_total > 0)
                    e = launch_batch_wide(res != 0, d->V != nullptr, ghosts, all_zero_y, w_total,
                                          (const BatchInst<float>*)dtab, d->count, S[cur], SN[cur], S[cur ^ 1],
                                          SN[cur ^ 1], d->V, d->P, flag, k == n - 1, stream);
            }
            if (e == hipSuccess && s_total > 0)
                e = launch_batch_stream<R>(res != 0, d->V != nullptr, ghosts, all_zero_y, s_total, dtab, d->count,
                                           S[cur], SN[cur], S[cur ^ 1], SN[cur ^ 1], d->V, d->P, flag, s_narrow);
            if (e == hipSuccess && side) {
                e = hipEventRecord(fj.join, side);
                if (e == hipSuccess) e = hipStreamWaitEvent(stream, fj.join, 0);
            }
        } else
            e = launch_batch<R>(res != 0, d->V != nullptr, ghosts, grid, dtab, d->count, total, S[cur], SN[cur],
                                S[cur ^ 1], SN[cur ^ 1], d->V, d->P, flag, stream);
        if (e != hipSuccess) return fail(PHX_EHIP, "batch step launch: %s", hipGetErrorString(e));
        cur ^= 1;
        if (noisy) {
            using C = typename cvec<R>::type;
            const unsigned blocks = (unsigned)block_inst.size();
            const int* bi = (const int*)(ws + L.block_inst);
            const uint64_t step = (uint64_t)(d->step0 + k);
            if (res)
                batch_noise_kernel<R, true><<<blocks, 256, 0, stream>>>(dtab, bi, (C*)S[cur], (const R*)SN[cur],
                                                                        step);
            else
                batch_noise_kernel<R, false><<<blocks, 256, 0, stream>>>(dtab, bi, (C*)S[cur], nullptr, step);
            e = hipGetLastError();
            if (e != hipSuccess) return fail(PHX_EHIP, "batch noise launch: %s", hipGetErrorString(e));
        }
    }
    if (d->check_finite) {
        unsigned int v = 0;
        e = hipMemcpyAsync(&v, flag, sizeof(v), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return fail(PHX_EHIP, "batch flag read: %s", hipGetErrorString(e));
        if (v) return fail(PHX_ENONFINITE, "a non-finite value appeared in the batch");
    }
    return PHX_OK;
}

}  // namespace phx

using namespace phx;

phx_status phx_batch_workspace_bytes(const phx_batch_desc* desc, size_t* out)
{
    clear_error();
    if (!out) return fail(PHX_EINVAL, "out is NULL");
    phx_status s = validate_batch(desc);
    if (s != PHX_OK) return s;
    *out = batch_layout(*desc).total;
    return PHX_OK;
}

phx_status phx_batch_step(const phx_batch_desc* desc, int64_t n_steps, void* hip_stream)
{
    clear_error();
    phx_status s = validate_batch(desc);
    if (s != PHX_OK) return s;
    if (n_steps < 0) return fail(PHX_EINVAL, "n_steps must be >= 0");
    const BatchLayout L = batch_layout(*desc);
    if (!desc->workspace || desc->workspace_bytes < L.total)
        return fail(PHX_EWORKSPACE, "workspace of %zu bytes needed", L.total);
    if (n_steps == 0) return PHX_OK;
    hipStream_t st = (hipStream_t)hip_stream;
    return desc->precision == PHX_C64 ? batch_run<float>(desc, n_steps, st) : batch_run<double>(desc, n_steps, st);
}
