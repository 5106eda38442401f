// Streaming copy kernel: the attainable HBM bandwidth that the solver's kernels are
// measured beside (read + write of a large buffer, no arithmetic).  Each workgroup
// moves one contiguous chunk of 1024 16-byte words: each lane loads four words 4 KiB
// apart, then stores them, all non-temporal (on this part contiguous chunks per
// workgroup stream faster than a grid-stride loop over the whole buffer).
//
// Walk-pattern kernel: the loads and stores of the wide whole-step walk (one wave per
// band of a 120-column strip, psi read as 16 bytes per lane and row, n and P as 8,
// an 8-row input ring filled 3 rows ahead, the finished row stored 4 rows behind the
// newest one) with none of its arithmetic: each row of psi is copied and n + P
// written for n.  Its time is the floor that this access pattern sets for the step
// kernel's 28 bytes per point.
#include "runtime.h"
#include "stream_wide.h"

namespace phx {

typedef unsigned int cw4 __attribute__((ext_vector_type(4)));  // one 16-byte word

__global__ __launch_bounds__(256) void stream_copy_kernel(const cw4* __restrict__ src, cw4* __restrict__ dst,
                                                          size_t words)
{
    const size_t base = (size_t)blockIdx.x * 1024 + threadIdx.x;
    cw4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (base + 256 * k < words) v[k] = __builtin_nontemporal_load(src + base + 256 * k);
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (base + 256 * k < words) __builtin_nontemporal_store(v[k], dst + base + 256 * k);
}

// Tile t: band t / strips, strip t % strips (consecutive tiles on one XCD); odd
// bands walk upwards, as in the step kernel.  Periodic rows and columns.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3)))
void walk_pattern_kernel(const float2* psi_in, const float* n_in, const float* P, float2* psi_out, float* n_out,
                         int nx, int ny, int strips, int B)
{
    constexpr int K = 8, PF = 3;
    const int lane = threadIdx.x & 63;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int band = t / strips, strip = t - band * strips;
    const int dir = (band & 1) ? -1 : 1;
    const int b0 = band * B, npos = B + 8;
    const int gi = strip * kWideCols - 4 + 2 * lane;
    const int ci = ((gi % nx) + nx) % nx;
    const size_t cells = (size_t)nx * ny;
    const __amdgpu_buffer_rsrc_t rpi = buffer_of(psi_in, cells * 8), rni = buffer_of(n_in, cells * 4);
    const __amdgpu_buffer_rsrc_t rP = buffer_of(P, cells * 4);
    const __amdgpu_buffer_rsrc_t rpo = buffer_of(psi_out, cells * 8), rno = buffer_of(n_out, cells * 4);
    const __amdgpu_buffer_rsrc_t rnull = buffer_of(psi_out, 0);
    const int v8 = ci * 8, v4 = ci * 4;
    const bool out_col = lane >= 2 && lane < 62 && gi < nx;
    const int o8 = out_col ? gi * 8 : kOutOfRange, o4 = out_col ? gi * 4 : kOutOfRange;
    const int row8 = nx * 8, row4 = nx * 4;
    wf4 sp[K];
    wf2 sn[K], sP[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        sp[k] = wf4{0.f, 0.f, 0.f, 0.f};
        sn[k] = sP[k] = wf2{0.f, 0.f};
    }
    const int start = dir > 0 ? b0 - 4 : b0 + B + 3;
    int rw = ((start % ny) + ny) % ny;
    auto fetch = [&](int k, bool use) {
        sp[k] = wload4(rpi, v8, rw * row8);
        sn[k] = wload2(rni, v4, rw * row4);
        sP[k] = wload2(rP, v4, rw * row4);
        int nr = rw + dir;
        nr = nr == ny ? 0 : (nr < 0 ? ny - 1 : nr);
        rw = use ? nr : rw;
    };
#pragma unroll
    for (int k = 0; k < PF; ++k) fetch(k, true);
    for (int base = 0; base < npos; base += 24) {
#pragma unroll
        for (int u = 0; u < 24; ++u) {
            if (base + u >= npos) break;
            const int j = start + dir * (base + u);
            fetch(slot<K>(u, -PF), base + u + PF < npos);
            const int s4 = slot<K>(u, 4);
            const int r = j - 4 * dir;  // the row that leaves the ring
            const bool st = r >= b0 && r < b0 + B && r < ny;
            const int rr = st ? r : 0;
            wstore4(sp[s4], st ? rpo : rnull, o8, rr * row8);
            wstore2(sn[s4] + sP[s4], st ? rno : rnull, o4, rr * row4);
        }
    }
}

}  // namespace phx

extern "C" phx_status phx_walk_pattern(void* psi_out, void* n_out, const void* psi_in, const void* n_in,
                                       const void* P, int32_t nx, int32_t ny, int32_t band_rows, void* stream)
{
    using namespace phx;
    clear_error();
    if (!psi_out || !n_out || !psi_in || !n_in || !P) return fail(PHX_EINVAL, "a pointer is NULL");
    const void* ptrs[] = {psi_out, n_out, psi_in, n_in, P};
    for (const void* p : ptrs)
        if (((uintptr_t)p & 255u) != 0) return fail(PHX_EINVAL, "device pointers must be 256-byte aligned");
    if (nx < 2 || nx % 2 != 0 || ny < 1) return fail(PHX_EINVAL, "nx must be even and >= 2, ny >= 1 (%d x %d)", nx, ny);
    const double bytes = (double)nx * ny * 8.0;
    if (bytes >= 2147483648.0) return fail(PHX_EINVAL, "psi must stay below 2 GiB (32-bit buffer offsets)");
    if (band_rows != 0 && (band_rows < 8 || band_rows > 4096))
        return fail(PHX_EINVAL, "band_rows must be 0 or 8..4096 (got %d)", band_rows);
    const size_t cells = (size_t)nx * ny;
    const char* ins[] = {(const char*)psi_in, (const char*)n_in, (const char*)P};
    const size_t in_bytes[] = {cells * 8, cells * 4, cells * 4};
    const char* outs[] = {(const char*)psi_out, (const char*)n_out};
    const size_t out_bytes[] = {cells * 8, cells * 4};
    for (int o = 0; o < 2; ++o)
        for (int i = 0; i < 3; ++i)
            if (outs[o] < ins[i] + in_bytes[i] && ins[i] < outs[o] + out_bytes[o])
                return fail(PHX_EINVAL, "outputs must not overlap the inputs");
    if (psi_out < (char*)n_out + cells * 4 && n_out < (char*)psi_out + cells * 8)
        return fail(PHX_EINVAL, "psi_out and n_out overlap");
    int B = band_rows;
    if (B == 0) {  // the device-filling height of the step kernel's 8-row ring
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 256;
        phx_config c{};
        c.nx = nx;
        c.ny = ny;
        c.reservoir = 1;
        c.bc_x = c.bc_y = PHX_BC_PERIODIC;
        B = wide_band_rows(c, StepShapeId{2, 0}, false, cus);
    }
    const int strips = wide_strips(nx);
    const int64_t tiles = (int64_t)strips * ((ny + B - 1) / B);
    if (tiles > 0x7fffffff) return fail(PHX_EINVAL, "too many tiles");
    walk_pattern_kernel<<<(unsigned)tiles, 64, 0, (hipStream_t)stream>>>(
        (const float2*)psi_in, (const float*)n_in, (const float*)P, (float2*)psi_out, (float*)n_out, nx, ny, strips, B);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(PHX_EHIP, "walk-pattern launch: %s", hipGetErrorString(e));
    return PHX_OK;
}

extern "C" phx_status phx_stream_copy(void* dst, const void* src, size_t bytes, void* stream)
{
    using namespace phx;
    clear_error();
    if (!dst || !src) return fail(PHX_EINVAL, "dst and src must not be NULL");
    if (bytes % 16 != 0 || ((uintptr_t)dst | (uintptr_t)src) % 16 != 0)
        return fail(PHX_EINVAL, "bytes and both pointers must be multiples of 16");
    const char* d = (const char*)dst;
    const char* s = (const char*)src;
    if (d < s + bytes && s < d + bytes) return fail(PHX_EINVAL, "src and dst overlap");
    if (bytes == 0) return PHX_OK;
    const size_t words = bytes / 16;
    const size_t blocks = (words + 1023) / 1024;
    if (blocks > 0x7fffffff) return fail(PHX_EINVAL, "copy of %zu bytes is too large", bytes);
    stream_copy_kernel<<<(unsigned)blocks, 256, 0, (hipStream_t)stream>>>((const cw4*)src, (cw4*)dst, words);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(PHX_EHIP, "copy launch: %s", hipGetErrorString(e));
    return PHX_OK;
}
