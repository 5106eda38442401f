// Streaming copy kernel: the attainable HBM bandwidth that the solver's kernels are
// measured beside (read + write of a large buffer, no arithmetic).  Each lane moves
// four independent 16-byte words per iteration with non-temporal loads and stores;
// the grid strides over the buffer.
#include "runtime.h"

namespace phx {

typedef unsigned int cw4 __attribute__((ext_vector_type(4)));  // one 16-byte word

__global__ __launch_bounds__(256) void stream_copy_kernel(const cw4* __restrict__ src, cw4* __restrict__ dst,
                                                          size_t words)
{
    const size_t lanes = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * lanes < words; i += 4 * lanes) {
        const cw4 a = __builtin_nontemporal_load(src + i);
        const cw4 b = __builtin_nontemporal_load(src + i + lanes);
        const cw4 c = __builtin_nontemporal_load(src + i + 2 * lanes);
        const cw4 d = __builtin_nontemporal_load(src + i + 3 * lanes);
        __builtin_nontemporal_store(a, dst + i);
        __builtin_nontemporal_store(b, dst + i + lanes);
        __builtin_nontemporal_store(c, dst + i + 2 * lanes);
        __builtin_nontemporal_store(d, dst + i + 3 * lanes);
    }
    for (; i < words; i += lanes) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
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
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                 hipSuccess || cus <= 0)
        cus = 256;
    const size_t words = bytes / 16;
    size_t blocks = (words + 1023) / 1024;
    const size_t cap = (size_t)cus * 16;
    if (blocks > cap) blocks = cap;
    stream_copy_kernel<<<(unsigned)blocks, 256, 0, (hipStream_t)stream>>>((const cw4*)src, (cw4*)dst, words);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(PHX_EHIP, "copy launch: %s", hipGetErrorString(e));
    return PHX_OK;
}
