// Exclusive scan of int64 workgroup totals, one workgroup (included by the
// station filter and the event builder; each translation unit has its own
// copy).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

// In-place exclusive scan of partials[0..n) (int64); partials[n] = total.
// One workgroup of kScanThreads: thread t sums its run of ceil(n / threads)
// consecutive partials (loads issued kScanUnroll at a time), one block scan of
// those sums (Hillis-Steele in LDS), then each thread rewrites its run from
// its prefix, again kScanUnroll loads before their stores.
constexpr int kScanThreads = 1024;
constexpr int kScanUnroll = 8;

__global__ __launch_bounds__(kScanThreads) void k_scan_i64(int64_t* partials, int64_t n) {
    __shared__ int64_t buf[kScanThreads];
    const int t = (int)threadIdx.x;
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
    buf[t] = sum;
    __syncthreads();
    for (int d = 1; d < kScanThreads; d <<= 1) {  // inclusive
        const int64_t o = t >= d ? buf[t - d] : 0;
        __syncthreads();
        buf[t] += o;
        __syncthreads();
    }
    int64_t run = buf[t] - sum;  // exclusive prefix of this run
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
    if (t == kScanThreads - 1) partials[n] = buf[t];
}

}  // namespace
