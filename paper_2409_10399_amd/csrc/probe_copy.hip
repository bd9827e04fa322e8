// Plain device-to-device copy kernels of known size: the bandwidth reference
// for the step kernel's roofline and the scale of the HBM traffic counters.
// Variants: 0 one 16-byte element per lane and iteration; 1 four independent
// 16-byte elements in flight per lane; 2 as 1 with nontemporal loads and
// stores; 3 four 4-byte elements per lane (one dword per lane and
// instruction, like an SoA population stream); 4 four 8-byte elements per lane.
#include <hip/hip_runtime.h>

#include <cstddef>

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));

template <class V, int U, bool NT>
__global__ void __launch_bounds__(256) k_copy(const V* __restrict__ src, V* __restrict__ dst, size_t nv) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (U - 1) * stride < nv; i += U * stride) {
        V v[U];
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
    for (; i < nv; i += stride) dst[i] = src[i];
}

template <class V, int U, bool NT>
static void go(const void* a, void* b, size_t bytes, int blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_copy<V, U, NT>), dim3(blocks), dim3(256), 0, s, static_cast<const V*>(a), static_cast<V*>(b),
                       bytes / sizeof(V));
}

extern "C" int eelbm_probe_copy(const void* src, void* dst, size_t bytes, int blocks, int variant, void* stream) {
    if (bytes % 16 != 0 || blocks < 1) return -1;
    hipStream_t s = static_cast<hipStream_t>(stream);
    switch (variant) {
        case 0: go<v4f, 1, false>(src, dst, bytes, blocks, s); break;
        case 1: go<v4f, 4, false>(src, dst, bytes, blocks, s); break;
        case 2: go<v4f, 4, true>(src, dst, bytes, blocks, s); break;
        case 3: go<float, 4, false>(src, dst, bytes, blocks, s); break;
        case 4: go<v2f, 4, false>(src, dst, bytes, blocks, s); break;
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}
