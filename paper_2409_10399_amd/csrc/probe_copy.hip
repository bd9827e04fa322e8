// Plain device-to-device copy kernels of known size: the bandwidth reference
// for the step kernel's roofline and the scale of the HBM traffic counters.
// Variant 0: one 16-byte element per thread and iteration.  Variant 1: four
// independent 16-byte elements in flight per thread.  Variant 2: as 1 with
// nontemporal loads and stores.
#include <hip/hip_runtime.h>

#include <cstddef>

typedef float v4f __attribute__((ext_vector_type(4)));

template <int U, bool NT>
__global__ void __launch_bounds__(256) k_copy(const v4f* __restrict__ src, v4f* __restrict__ dst, size_t n4) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (U - 1) * stride < n4; i += U * stride) {
        v4f v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = NT ? __builtin_nontemporal_load(src + i + u * stride) : src[i + u * stride];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (NT)
                __builtin_nontemporal_store(v[u], dst + i + u * stride);
            else
                dst[i + u * stride] = v[u];
        }
    }
    for (; i < n4; i += stride) dst[i] = src[i];
}

extern "C" int eelbm_probe_copy(const void* src, void* dst, size_t bytes, int blocks, int variant, void* stream) {
    if (bytes % 16 != 0 || blocks < 1) return -1;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const v4f* a = static_cast<const v4f*>(src);
    v4f* b = static_cast<v4f*>(dst);
    const size_t n4 = bytes / 16;
    switch (variant) {
        case 0: hipLaunchKernelGGL((k_copy<1, false>), dim3(blocks), dim3(256), 0, s, a, b, n4); break;
        case 1: hipLaunchKernelGGL((k_copy<4, false>), dim3(blocks), dim3(256), 0, s, a, b, n4); break;
        case 2: hipLaunchKernelGGL((k_copy<4, true>), dim3(blocks), dim3(256), 0, s, a, b, n4); break;
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}
