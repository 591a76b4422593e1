// Exclusive scan of int64 workgroup totals, one workgroup (included by the
// station filter and the event builder; each translation unit has its own
// copy).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

// In-place exclusive scan of partials[0..n) (int64); partials[n] = total.
// One workgroup of kScanThreads: thread t sums its run of ceil(n / threads)
// consecutive partials (loads issued kScanUnroll at a time); a wave scan of
// those sums (shuffles) and one barrier to add the totals of the waves
// before; then each thread rewrites its run from its prefix, again
// kScanUnroll loads before their stores.
constexpr int kScanThreads = 1024;
constexpr int kScanWaves = kScanThreads / 64;
constexpr int kScanUnroll = 8;

// Inclusive sum over the lanes of a wave (lanes 0..lane).
__device__ __forceinline__ int64_t scan_wave_incl(int64_t v) {
    const int lane = (int)(threadIdx.x & 63);
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t o = __shfl_up(v, (unsigned)d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_i64(int64_t* partials, int64_t n) {
    __shared__ int64_t wave_total[kScanWaves];
    const int t = (int)threadIdx.x, w = t / 64;
    const int64_t per = (n + kScanThreads - 1) / kScanThreads;
    const int64_t lo = min(n, (int64_t)t * per), hi = min(n, lo + per);
    int64_t sum = 0;
    for (int64_t i0 = lo; i0 < hi; i0 += kScanUnroll) {
        int64_t v[kScanUnroll];
#pragma unroll
        for (int u = 0; u < kScanUnroll; ++u) v[u] = i0 + u < hi ? partials[i0 + u] : 0;
#pragma unroll
        for (int u = 0; u < kScanUnroll; ++u) sum += v[u];
    }
    const int64_t incl = scan_wave_incl(sum);
    if ((t & 63) == 63) wave_total[w] = incl;
    __syncthreads();
    int64_t before = 0;
    for (int k = 0; k < w; ++k) before += wave_total[k];
    int64_t run = before + incl - sum;  // exclusive prefix of this run
    for (int64_t i0 = lo; i0 < hi; i0 += kScanUnroll) {
        // a batch's loads go out together, before its stores
        int64_t v[kScanUnroll];
#pragma unroll
        for (int u = 0; u < kScanUnroll; ++u) v[u] = i0 + u < hi ? partials[i0 + u] : 0;
#pragma unroll
        for (int u = 0; u < kScanUnroll; ++u)
            if (i0 + u < hi) {
                partials[i0 + u] = run;
                run += v[u];
            }
    }
    if (t == kScanThreads - 1) partials[n] = before + incl;
}

}  // namespace
