// Trigger-station filtering on the device (include/trig_filter.h): every
// event's hits of the three trigger layers, in input order per layer, as the
// CSR offsets and fp32 x/y arrays the selection reads.  The paper does this
// on the host before the transfer (Sec. 5.3, implementation i3); here the
// station numbers are streamed once to count and once to scatter.
//
// Partition: a workgroup of 4 waves owns kFilterEvents consecutive events;
// wave w takes events w, w + 4, ...  A wave reads an event's station numbers
// four per lane (one 32-bit load of 4 consecutive hits; 256 hits per step),
// so the hits of lane L precede those of lane L + 1 in a step.  Counts come
// from wave sums; in the scatter, a hit's rank in its layer is the exclusive
// prefix over lanes of the per-lane counts plus the count of the lane's
// earlier hits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "trig.h"
#include "trig_device.hpp"
#include "trig_filter.h"

namespace {

constexpr int kFilterThreads = 256;
constexpr int kFilterWaves = kFilterThreads / trig::kWave;
constexpr int kFilterEvents = 64;  // events per workgroup (one per lane of a wave in the block scan)

struct Range {
    int64_t a, b;
    bool ok;
};

__device__ __forceinline__ Range event_range(const int64_t* __restrict__ off, int e, int64_t n_hits) {
    Range r;
    r.a = off[e];
    r.b = off[e + 1];
    r.ok = 0 <= r.a && r.a <= r.b && r.b <= n_hits && r.b - r.a <= (int64_t)INT32_MAX;
    return r;
}

// Station numbers of hits h0 .. h0 + 3 (h0 a multiple of 4 when vec), 0xFF
// bytes where a hit is past the array; the caller masks hits outside the
// event.  A padding byte can equal a trigger layer only if the layer number
// is 255; the event mask excludes those hits anyway.
__device__ __forceinline__ uint32_t station_word(const uint8_t* __restrict__ st, int64_t h0, int64_t n_hits,
                                                 bool vec) {
    if (vec && h0 + 3 < n_hits) return *reinterpret_cast<const uint32_t*>(st + h0);
    uint32_t w = 0xFFFFFFFFu;
    for (int k = 0; k < 4; ++k)
        if (h0 + k < n_hits) w = (w & ~(0xFFu << (8 * k))) | ((uint32_t)st[h0 + k] << (8 * k));
    return w;
}

// Per lane: which of its four hits (bits 0..3) belong to layer l, for l = 0, 1, 2.
struct LaneMatch {
    uint32_t m[3];
};

__device__ __forceinline__ LaneMatch match_word(uint32_t w, int64_t h0, int64_t a, int64_t b, uint32_t layers) {
    LaneMatch r{{0u, 0u, 0u}};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t h = h0 + k;
        const uint32_t s = (w >> (8 * k)) & 0xFFu;
        const bool in = h >= a && h < b;
#pragma unroll
        for (int l = 0; l < 3; ++l) r.m[l] |= (uint32_t)(in && s == ((layers >> (8 * l)) & 0xFFu)) << k;
    }
    return r;
}

__global__ __launch_bounds__(kFilterThreads) void k_filter_count(const int64_t* __restrict__ off, int n_events,
                                                                   int64_t n_hits, const uint8_t* __restrict__ st,
                                                                   uint32_t layers, int vec,
                                                                   int32_t* __restrict__ counts,
                                                                   int64_t* __restrict__ partials,
                                                                   uint32_t* status) {
    __shared__ int64_t wave_total[kFilterWaves];
    const int w = trig::uniform_i((int)(threadIdx.x / trig::kWave));
    const int lane = (int)trig::lane_id();
    const int e_first = (int)blockIdx.x * kFilterEvents;
    int64_t total = 0;
    for (int j = w; j < kFilterEvents; j += kFilterWaves) {
        const int e = e_first + j;
        if (e >= n_events) break;
        const Range r = event_range(off, e, n_hits);
        uint32_t c[3] = {0u, 0u, 0u};
        if (r.ok) {
            for (int64_t base = r.a & ~(int64_t)3; base < r.b; base += 4 * trig::kWave) {
                const int64_t h0 = base + 4 * lane;
                const LaneMatch m = match_word(station_word(st, h0, n_hits, vec != 0), h0, r.a, r.b, layers);
#pragma unroll
                for (int l = 0; l < 3; ++l) c[l] += (uint32_t)__builtin_popcount(m.m[l]);
            }
        } else if (lane == 0 && status) {
            atomicOr(status, TRIG_FILTER_MALFORMED);
        }
        const uint32_t s0 = trig::wave_sum_u(c[0]), s1 = trig::wave_sum_u(c[1]), s2 = trig::wave_sum_u(c[2]);
        if (lane == 0) {
            counts[3 * (int64_t)e] = (int32_t)s0;
            counts[3 * (int64_t)e + 1] = (int32_t)s1;
            counts[3 * (int64_t)e + 2] = (int32_t)s2;
        }
        total += (int64_t)s0 + s1 + s2;
    }
    if (lane == 0) wave_total[w] = total;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int k = 0; k < kFilterWaves; ++k) t += wave_total[k];
        partials[blockIdx.x] = t;
    }
}

// In-place exclusive scan of partials[0..n) (int64); partials[n] = total.
// One workgroup, kFilterThreads values per step.
__global__ __launch_bounds__(kFilterThreads) void k_filter_scan(int64_t* partials, int n) {
    __shared__ int64_t buf[kFilterThreads];
    int64_t carry = 0;
    const int t = (int)threadIdx.x;
    for (int base = 0; base < n; base += kFilterThreads) {
        const int i = base + t;
        const int64_t v = i < n ? partials[i] : 0;
        buf[t] = v;
        __syncthreads();
        for (int d = 1; d < kFilterThreads; d <<= 1) {  // inclusive Hillis-Steele scan
            const int64_t o = t >= d ? buf[t - d] : 0;
            __syncthreads();
            buf[t] += o;
            __syncthreads();
        }
        if (i < n) partials[i] = carry + buf[t] - v;
        carry += buf[kFilterThreads - 1];
        __syncthreads();
    }
    if (t == 0) partials[n] = carry;
}

__global__ __launch_bounds__(kFilterThreads) void k_filter_scatter(
    const int64_t* __restrict__ off, int n_events, int64_t n_hits, const uint8_t* __restrict__ st,
    const float* __restrict__ x, const float* __restrict__ y, uint32_t layers, int vec,
    const int32_t* __restrict__ counts, const int64_t* __restrict__ partials, int n_blocks, int32_t capacity,
    int32_t* __restrict__ out_off, float* __restrict__ out_x, float* __restrict__ out_y, uint32_t* status) {
    __shared__ int64_t ev_start[kFilterEvents];
    const int w = trig::uniform_i((int)(threadIdx.x / trig::kWave));
    const int lane = (int)trig::lane_id();
    const int e_first = (int)blockIdx.x * kFilterEvents;
    const int64_t cap = capacity;
    if (w == 0) {
        // Starts of the workgroup's events: its base plus an exclusive scan of
        // the events' totals, one event per lane.
        const int e = e_first + lane;
        int32_t tot = 0;
        if (e < n_events)
            tot = counts[3 * (int64_t)e] + counts[3 * (int64_t)e + 1] + counts[3 * (int64_t)e + 2];
        const int32_t excl = trig::wave_inclusive_sum(tot) - tot;
        ev_start[lane] = partials[blockIdx.x] + excl;
    }
    if ((int)blockIdx.x == n_blocks - 1 && threadIdx.x == 0) {
        const int64_t total = partials[n_blocks];
        if (total > cap && status) atomicOr(status, TRIG_FILTER_CAPACITY);
        out_off[3 * (int64_t)n_events] = (int32_t)std::min<int64_t>(total, cap);
    }
    __syncthreads();
    for (int j = w; j < kFilterEvents; j += kFilterWaves) {
        const int e = e_first + j;
        if (e >= n_events) break;
        const int64_t c0 = counts[3 * (int64_t)e], c1 = counts[3 * (int64_t)e + 1];
        int64_t s[3];
        s[0] = ev_start[j];
        s[1] = s[0] + c0;
        s[2] = s[1] + c1;
        if (lane < 3) {
            const int64_t v = lane == 0 ? s[0] : (lane == 1 ? s[1] : s[2]);
            out_off[3 * (int64_t)e + lane] = (int32_t)std::min<int64_t>(v, cap);
        }
        const Range r = event_range(off, e, n_hits);
        if (!r.ok) continue;
        for (int64_t base = r.a & ~(int64_t)3; base < r.b; base += 4 * trig::kWave) {
            const int64_t h0 = base + 4 * lane;
            const LaneMatch m = match_word(station_word(st, h0, n_hits, vec != 0), h0, r.a, r.b, layers);
            int64_t pos[3];
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                const int n = __builtin_popcount(m.m[l]);
                const int incl = trig::wave_inclusive_sum(n);
                pos[l] = s[l] + (incl - n);
                s[l] += __builtin_amdgcn_readlane(incl, 63);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
#pragma unroll
                for (int l = 0; l < 3; ++l) {
                    if ((m.m[l] >> k) & 1u) {
                        const int64_t p = pos[l]++;
                        if (p >= 0 && p < cap) {  // positions past an int32 block prefix are never written
                            out_x[p] = x[h0 + k];
                            out_y[p] = y[h0 + k];
                        }
                    }
                }
            }
        }
    }
}

__global__ void k_filter_zero(int32_t* p) { *p = 0; }

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

size_t trig_filter_workspace_bytes(int32_t n_events) {
    if (n_events < 0) return 0;
    const int64_t nb = std::max<int64_t>(1, ((int64_t)n_events + kFilterEvents - 1) / kFilterEvents);
    return align256(sizeof(int32_t) * 3 * (size_t)n_events) + align256(sizeof(int64_t) * (size_t)(nb + 1));
}

int trig_filter_stations(const trig_raw_events* ev, const trig_filter_params* p, void* stream) {
    if (!ev || !p || ev->n_events < 0 || ev->n_hits < 0 || !ev->offsets || !p->out_layer_offsets ||
        p->out_capacity < 0 || p->reserved != 0)
        return TRIG_EINVAL;
    if (ev->n_hits > 0 && (!ev->station || !ev->x || !ev->y)) return TRIG_EINVAL;
    if (p->out_capacity > 0 && (!p->out_x || !p->out_y)) return TRIG_EINVAL;
    if (p->layers[0] == p->layers[1] || p->layers[0] == p->layers[2] || p->layers[1] == p->layers[2])
        return TRIG_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int n = ev->n_events;
    if (n == 0) {
        hipLaunchKernelGGL(k_filter_zero, dim3(1), dim3(1), 0, s, p->out_layer_offsets);
        return hipGetLastError() == hipSuccess ? TRIG_OK : TRIG_EHIP;
    }
    const size_t need = trig_filter_workspace_bytes(n);
    if (!p->workspace || p->workspace_bytes < need || (reinterpret_cast<uintptr_t>(p->workspace) & 255))
        return TRIG_EINVAL;
    const int nb = (int)(((int64_t)n + kFilterEvents - 1) / kFilterEvents);
    auto* counts = static_cast<int32_t*>(p->workspace);
    auto* partials =
        reinterpret_cast<int64_t*>(static_cast<char*>(p->workspace) + align256(sizeof(int32_t) * 3 * (size_t)n));
    const uint32_t layers = (uint32_t)p->layers[0] | ((uint32_t)p->layers[1] << 8) | ((uint32_t)p->layers[2] << 16);
    const int vec = (reinterpret_cast<uintptr_t>(ev->station) & 3) == 0;
    hipLaunchKernelGGL(k_filter_count, dim3(nb), dim3(kFilterThreads), 0, s, ev->offsets, n, ev->n_hits,
                       ev->station, layers, vec, counts, partials, p->out_status);
    if (hipGetLastError() != hipSuccess) return TRIG_EHIP;
    hipLaunchKernelGGL(k_filter_scan, dim3(1), dim3(kFilterThreads), 0, s, partials, nb);
    if (hipGetLastError() != hipSuccess) return TRIG_EHIP;
    hipLaunchKernelGGL(k_filter_scatter, dim3(nb), dim3(kFilterThreads), 0, s, ev->offsets, n, ev->n_hits,
                       ev->station, ev->x, ev->y, layers, vec, counts, partials, nb, p->out_capacity,
                       p->out_layer_offsets, p->out_x, p->out_y, p->out_status);
    return hipGetLastError() == hipSuccess ? TRIG_OK : TRIG_EHIP;
}

}  // extern "C"
