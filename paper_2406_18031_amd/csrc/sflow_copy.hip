// A plain streaming device-to-device copy (sf_copy_probe in include/sflow.h): the yardstick
// for the HBM bandwidth this GPU reaches in practice, against which the filter kernels'
// bandwidth is reported, and a copy of known size for scaling the HBM byte counters.
//
// Each thread moves 16-byte vectors in a grid-stride loop, four in flight per iteration;
// loads and stores are non-temporal (streamed past the caches, as a copy far larger than the
// last-level cache would be anyway).  The grid is a whole number of waves per CU.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sflow.h"

namespace {

constexpr int kCopyThreads = 256;
constexpr int kUnroll = 4;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(kCopyThreads) k_copy(const u32x4* __restrict__ src,
                                                      u32x4* __restrict__ dst, size_t n) {
    const size_t stride = (size_t)gridDim.x * kCopyThreads;
    size_t i = (size_t)blockIdx.x * kCopyThreads + threadIdx.x;
    for (; i + (kUnroll - 1) * stride < n; i += kUnroll * stride) {
        u32x4 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) __builtin_nontemporal_store(v[u], dst + i + u * stride);
    }
    for (; i < n; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

__global__ void k_copy_tail(const uint8_t* src, uint8_t* dst, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

}  // namespace

extern "C" sf_status sf_copy_probe(const void* src, void* dst, size_t bytes, void* hip_stream) {
    if (bytes == 0) return SF_OK;
    if (!src || !dst) return SF_ERR_INVALID_ARG;
    hipPointerAttribute_t as, ad;
    if (hipPointerGetAttributes(&as, src) != hipSuccess ||
        hipPointerGetAttributes(&ad, dst) != hipSuccess) {
        (void)hipGetLastError();
        return SF_ERR_INVALID_ARG;
    }
    if (as.type != hipMemoryTypeDevice || ad.type != hipMemoryTypeDevice) return SF_ERR_INVALID_ARG;
    if (((uintptr_t)src | (uintptr_t)dst) & 15) return SF_ERR_INVALID_ARG;
    const char* s8 = (const char*)src;
    char* d8 = (char*)dst;
    if ((s8 < d8 + bytes) && (d8 < s8 + bytes)) return SF_ERR_INVALID_ARG;   // overlap
    hipStream_t s = (hipStream_t)hip_stream;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return SF_ERR_HIP;
    }
    const size_t n = bytes / 16;
    if (n > 0) {
        const size_t want = (n + kCopyThreads - 1) / kCopyThreads;
        const size_t blocks = want < (size_t)cus * 8 ? want : (size_t)cus * 8;
        hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(kCopyThreads), 0, s,
                           (const u32x4*)src, (u32x4*)dst, n);
    }
    const size_t tail = bytes - n * 16;
    if (tail > 0)
        hipLaunchKernelGGL(k_copy_tail, dim3(1), dim3(16), 0, s, (const uint8_t*)s8 + n * 16,
                           (uint8_t*)d8 + n * 16, tail);
    return hipGetLastError() == hipSuccess ? SF_OK : SF_ERR_HIP;
}
