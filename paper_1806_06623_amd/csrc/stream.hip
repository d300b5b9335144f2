// Streaming device copy: the bandwidth reference of the memory-bound kernels
// (declared in spp_reference.h).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "internal.h"
#include "spp_reference.h"

namespace {

constexpr int THREADS = 256, UNROLL = 4, MAX_BLOCKS = 8192;
using d2 = __attribute__((ext_vector_type(2))) double;

// Grid-stride copy of n 16-byte elements; each thread has UNROLL loads in
// flight before its stores.
__global__ __launch_bounds__(THREADS) void k_stream_copy(const d2* __restrict__ src, d2* __restrict__ dst, size_t n)
{
    const size_t stride = size_t(gridDim.x) * THREADS * UNROLL;
    for (size_t base = size_t(blockIdx.x) * THREADS * UNROLL + threadIdx.x; base < n; base += stride) {
        d2 v[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const size_t i = base + size_t(u) * THREADS;
            if (i < n) v[u] = src[i];
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const size_t i = base + size_t(u) * THREADS;
            if (i < n) dst[i] = v[u];
        }
    }
}

}  // namespace

extern "C" spp_status spp_stream_copy(const void* src_dev, void* dst_dev, size_t bytes, void* stream)
{
    if (bytes == 0) return SPP_OK;
    if (!src_dev || !dst_dev) return spp_fail(SPP_EINVAL, "spp_stream_copy: NULL pointer");
    if ((reinterpret_cast<uintptr_t>(src_dev) | reinterpret_cast<uintptr_t>(dst_dev) | bytes) % 16 != 0)
        return spp_fail(SPP_EINVAL, "spp_stream_copy: pointers and size must be multiples of 16 bytes");
    const size_t n = bytes / 16;
    const size_t per_block = size_t(THREADS) * UNROLL;
    const size_t want = (n + per_block - 1) / per_block;
    const unsigned blocks = unsigned(want < size_t(MAX_BLOCKS) ? want : size_t(MAX_BLOCKS));
    hipLaunchKernelGGL(k_stream_copy, dim3(blocks), dim3(THREADS), 0, static_cast<hipStream_t>(stream),
                       static_cast<const d2*>(src_dev), static_cast<d2*>(dst_dev), n);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return spp_fail(SPP_EDEVICE, std::string("spp_stream_copy: ") + hipGetErrorString(e));
    return SPP_OK;
}
