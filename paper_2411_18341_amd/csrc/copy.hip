// Streaming copy kernel: the attainable HBM bandwidth that the solver's kernels are
// measured beside (read + write of a large buffer, no arithmetic).  Each workgroup
// moves one contiguous chunk of 1024 16-byte words: each lane loads four words 4 KiB
// apart, then stores them, all non-temporal (on this part contiguous chunks per
// workgroup stream faster than a grid-stride loop over the whole buffer).
#include "runtime.h"

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

}  // namespace phx

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
