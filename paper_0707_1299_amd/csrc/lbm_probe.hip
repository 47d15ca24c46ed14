// Streaming-copy probe: a plain device-to-device copy, 16 bytes per thread with
// non-temporal loads and stores.  Its measured rate is the practical HBM
// ceiling the fused step kernel is compared with, beside the vendor peak; it
// computes nothing of the method.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lbm.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_copy16(const f4* __restrict__ a, f4* __restrict__ b, int64_t n)
{
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(a + i), b + i);
}

}  // namespace

extern "C" int lb_copy_probe(const void* d_src, void* d_dst, size_t bytes, void* hip_stream)
{
    if (!d_src || !d_dst || bytes == 0 || bytes % 16) return LB_ERR_ARG;
    if ((uintptr_t(d_src) | uintptr_t(d_dst)) % 16) return LB_ERR_ARG;
    const uintptr_t s = uintptr_t(d_src), d = uintptr_t(d_dst);
    if (s < d + bytes && d < s + bytes) return LB_ERR_ARG;      // overlapping ranges
    const int64_t n = int64_t(bytes / 16);
    const int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7FFFFFFF) return LB_ERR_SIZE;
    hipLaunchKernelGGL(k_copy16, dim3(unsigned(blocks)), dim3(256), 0, hipStream_t(hip_stream),
                       static_cast<const f4*>(d_src), static_cast<f4*>(d_dst), n);
    return hipGetLastError() == hipSuccess ? LB_OK : LB_ERR_HIP;
}
