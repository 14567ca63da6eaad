/*
 * plain_baseline.hip -- the "plain" baseline: each thread calls the HIP
 * runtime's own device malloc / free (the vendor allocator the paper calls
 * slow and unreliable for CUDA, Introduction).  Called and timed as a black
 * box; nothing here depends on how it works.
 */
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "hbheap.h"

namespace {
constexpr uint32_t kBlock = 256;

uint32_t grid_for(uint64_t n)
{
    const uint64_t g = (n + kBlock - 1) / kBlock;
    return (uint32_t)(g ? g : 1);
}
}  // namespace

__global__ void __launch_bounds__(kBlock) k_plain_alloc(const uint64_t* sizes, void** ptrs, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    ptrs[i] = malloc(sizes[i]);
}

__global__ void __launch_bounds__(kBlock) k_plain_free(void* const* ptrs, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    if (ptrs[i]) free(ptrs[i]);
}

extern "C" {

int hb_plain_set_heap(size_t bytes)
{
    return hipDeviceSetLimit(hipLimitMallocHeapSize, bytes) == hipSuccess ? HBHEAP_OK : HBHEAP_E_UNSUP;
}

int hb_plain_alloc(const size_t* sizes, void** ptrs, size_t n, hipStream_t stream)
{
    if (n && (!sizes || !ptrs)) return HBHEAP_E_INVAL;
    if (!n) return HBHEAP_OK;
    hipLaunchKernelGGL(k_plain_alloc, dim3(grid_for(n)), dim3(kBlock), 0, stream, (const uint64_t*)sizes, ptrs,
                       (uint64_t)n);
    return hipGetLastError() == hipSuccess ? HBHEAP_OK : HBHEAP_E_HIP;
}

int hb_plain_free(void* const* ptrs, size_t n, hipStream_t stream)
{
    if (n && !ptrs) return HBHEAP_E_INVAL;
    if (!n) return HBHEAP_OK;
    hipLaunchKernelGGL(k_plain_free, dim3(grid_for(n)), dim3(kBlock), 0, stream, ptrs, (uint64_t)n);
    return hipGetLastError() == hipSuccess ? HBHEAP_OK : HBHEAP_E_HIP;
}

}  // extern "C"
