// Micro-benchmark kernels: fp32 VALU instruction rate and HBM copy bandwidth
// (include/trig_probe.h).  Built into libtrig.so with the same flags as the
// selection kernels (no contraction, no packed fp32).
#include <hip/hip_runtime.h>

#include "trig_probe.h"

namespace {

__global__ __launch_bounds__(256) void k_probe_valu(int iters, float seed, float* out) {
    const unsigned gid = blockIdx.x * 256u + threadIdx.x;
    float a[8], b[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        a[k] = seed + (float)(gid & 7) * 0.125f + (float)k;
        b[k] = 1.0f - seed * (float)(k + 1) * 1e-3f;
    }
    const float m = 0.999f + seed * 1e-6f, s = 1e-7f * seed;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            a[k] = a[k] * m;   // v_mul_f32
            b[k] = b[k] + s;   // v_add_f32
        }
    }
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) acc += a[k] + b[k];
    out[gid] = acc;
}

__global__ __launch_bounds__(256) void k_probe_copy(const float4* __restrict__ src,
                                                    float4* __restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

}  // namespace

extern "C" {

int trig_probe_valu(int32_t n_blocks, int32_t iters, float seed, float* out, void* stream) {
    if (n_blocks <= 0 || iters < 0 || !out) return -1;
    hipLaunchKernelGGL(k_probe_valu, dim3(n_blocks), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                       iters, seed, out);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int trig_probe_copy(const void* src, void* dst, int64_t n_vec4, int32_t n_blocks, void* stream) {
    if (n_vec4 < 0 || n_blocks <= 0 || (n_vec4 > 0 && (!src || !dst))) return -1;
    if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15) return -1;
    if (n_vec4 == 0) return 0;
    hipLaunchKernelGGL(k_probe_copy, dim3(n_blocks), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                       static_cast<const float4*>(src), static_cast<float4*>(dst), n_vec4);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // extern "C"
