// Event building from a time-ordered hit stream (include/trig_events.h):
// time-gap clustering, the reading this library takes of the paper's outlook
// on free-streaming data (Sec. 8), which gives no algorithm.
//
// Partition: a workgroup of 4 waves owns kEbHits consecutive hits; wave w
// takes the kEbRounds * 64 hits from (4 b + w) * kEbWaveHits on, 64 per
// round, lane L on hit 64 r + L.  A hit's predecessor is the previous lane's
// hit (a shuffle), lane 0's the previous round's lane 63 (or, for a
// wave's first round, one scalar load).  The count kernel writes each
// round's ballot of event starts to a bit mask in the workspace (one bit per
// hit), the wave's count and the workgroup's total; the scan turns the
// totals into positions; the scatter kernel gives each of a wave's rounds
// (one lane per round) its first position by a wave scan of the masks'
// popcounts and writes the hit index of every set bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "scan_i64.hpp"
#include "trig.h"
#include "trig_device.hpp"
#include "trig_events.h"

namespace {

constexpr int kEbWaves = 4;
constexpr int kEbThreads = kEbWaves * trig::kWave;
constexpr int kEbRounds = 64;  // rounds of 64 hits per wave (lane r holds round r's mask)
static_assert(kEbRounds <= trig::kWave, "one lane per round's mask");
constexpr int64_t kEbWaveHits = (int64_t)kEbRounds * trig::kWave;
constexpr int64_t kEbHits = kEbWaveHits * kEbWaves;  // hits per workgroup
constexpr int64_t kEbMaxHits = (int64_t)1 << 40;

// Does hit h (time tc, predecessor's time tp) start an event: h == 0, or a
// later time by more than gap (the exact difference: for tc > tp the
// unsigned difference of the two int64 values is the true one).
__device__ __forceinline__ bool starts(int64_t h, int64_t tc, int64_t tp, uint64_t gap) {
    return h == 0 || (tc > tp && (uint64_t)tc - (uint64_t)tp > gap);
}

// The previous lane's int64 value (lane 0 gets `first`).
__device__ __forceinline__ int64_t from_lane_below(int64_t v, int64_t first) {
    const int lane = (int)trig::lane_id();
    const int lo = __shfl_up((int)(uint32_t)v, 1), hi = __shfl_up((int)(uint32_t)((uint64_t)v >> 32), 1);
    const int64_t below = (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
    return lane == 0 ? first : below;
}

__global__ __launch_bounds__(kEbThreads) void k_eb_count(const int64_t* __restrict__ t, int64_t n, uint64_t gap,
                                                         uint64_t* __restrict__ masks, int32_t* __restrict__ wcount,
                                                         int64_t* __restrict__ partials, uint32_t* status) {
    __shared__ int32_t wave_total[kEbWaves];
    const int w = trig::uniform_i((int)(threadIdx.x / trig::kWave));
    const int lane = (int)trig::lane_id();
    const int64_t gw = (int64_t)blockIdx.x * kEbWaves + w;
    const int64_t h0 = gw * kEbWaveHits;
    // the hit before the wave's first (scalar load)
    int64_t carry = (h0 > 0 && h0 - 1 < n) ? t[h0 - 1] : 0;
    uint64_t mine = 0u;  // lane r: round r's mask
    int32_t cnt = 0;
    bool bad = false;
    constexpr int kBatch = 8;  // rounds whose loads are in flight together
#pragma unroll 1
    for (int r0 = 0; r0 < kEbRounds; r0 += kBatch) {
        if (h0 + (int64_t)r0 * trig::kWave >= n) break;  // wave-uniform
        int64_t tv[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const int64_t h = h0 + (int64_t)(r0 + k) * trig::kWave + lane;
            tv[k] = h < n ? t[h] : 0;
        }
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const int64_t h = h0 + (int64_t)(r0 + k) * trig::kWave + lane;
            const bool valid = h < n;
            const int64_t tp = from_lane_below(tv[k], carry);
            bad |= valid && h > 0 && tv[k] < tp;
            const uint64_t m = trig::lanes(valid && starts(h, tv[k], tp, gap));
            cnt += (int32_t)__builtin_popcountll(m);
            mine = lane == r0 + k ? m : mine;
            const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)tv[k], 63);
            const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)tv[k] >> 32), 63);
            carry = (int64_t)(((uint64_t)hi << 32) | lo);
        }
    }
    if (lane < kEbRounds) masks[gw * kEbRounds + lane] = mine;
    if (trig::wave_any(bad) && lane == 0 && status) atomicOr(status, TRIG_EVENTS_UNSORTED);
    if (lane == 0) {
        wcount[gw] = cnt;
        wave_total[w] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t s = 0;
        for (int k = 0; k < kEbWaves; ++k) s += wave_total[k];
        partials[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(kEbThreads) void k_eb_scatter(int64_t n, const uint64_t* __restrict__ masks,
                                                           const int32_t* __restrict__ wcount,
                                                           const int64_t* __restrict__ partials, int n_blocks,
                                                           int64_t* __restrict__ out, int64_t cap,
                                                           int64_t* __restrict__ out_n, uint32_t* status) {
    const int w = trig::uniform_i((int)(threadIdx.x / trig::kWave));
    const int lane = (int)trig::lane_id();
    const int64_t gw = (int64_t)blockIdx.x * kEbWaves + w;
    const int64_t h0 = gw * kEbWaveHits;
    int64_t base = partials[blockIdx.x];
    for (int k = 0; k < w; ++k) base += wcount[(int64_t)blockIdx.x * kEbWaves + k];
    const uint64_t m = lane < kEbRounds ? masks[gw * kEbRounds + lane] : 0u;
    const int pc = __builtin_popcountll(m);
    int64_t pos = base + (trig::wave_inclusive_sum(pc) - pc);
    for (uint64_t bits = m; bits; bits &= bits - 1u) {  // event starts are sparse
        if (pos < cap) out[pos] = h0 + (int64_t)trig::kWave * lane + __builtin_ctzll(bits);
        ++pos;
    }
    if ((int)blockIdx.x == n_blocks - 1 && threadIdx.x == 0) {
        const int64_t e = partials[n_blocks];
        if (e < cap) out[e] = n;
        if (e + 1 > cap && status) atomicOr(status, TRIG_EVENTS_CAPACITY);
        *out_n = e;
    }
}

__global__ void k_eb_empty(int64_t* out, int64_t* out_n) {
    out[0] = 0;
    *out_n = 0;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int64_t eb_blocks(int64_t n) { return (n + kEbHits - 1) / kEbHits; }

}  // namespace

extern "C" {

size_t trig_build_events_workspace_bytes(int64_t n_hits) {
    if (n_hits < 0 || n_hits > kEbMaxHits) return 0;
    const int64_t nb = std::max<int64_t>(1, eb_blocks(n_hits));
    return align256(sizeof(uint64_t) * (size_t)(nb * kEbWaves * kEbRounds)) +
           align256(sizeof(int32_t) * (size_t)(nb * kEbWaves)) + align256(sizeof(int64_t) * (size_t)(nb + 1));
}

int trig_build_events(const int64_t* t, int64_t n_hits, int64_t gap, int64_t* out_offsets, int64_t out_capacity,
                      int64_t* out_n_events, uint32_t* out_status, void* workspace, size_t workspace_bytes,
                      void* stream) {
    if (n_hits < 0 || n_hits > kEbMaxHits || gap < 0 || out_capacity < 1 || !out_offsets || !out_n_events)
        return TRIG_EINVAL;
    if (n_hits > 0 && !t) return TRIG_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (n_hits == 0) {
        hipLaunchKernelGGL(k_eb_empty, dim3(1), dim3(1), 0, s, out_offsets, out_n_events);
        return hipGetLastError() == hipSuccess ? TRIG_OK : TRIG_EHIP;
    }
    const size_t need = trig_build_events_workspace_bytes(n_hits);
    if (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255)) return TRIG_EINVAL;
    const int64_t nb = eb_blocks(n_hits);  // <= 2^40 / 16384 = 2^26
    char* ws = static_cast<char*>(workspace);
    auto* masks = reinterpret_cast<uint64_t*>(ws);
    const size_t mask_bytes = align256(sizeof(uint64_t) * (size_t)(nb * kEbWaves * kEbRounds));
    auto* wcount = reinterpret_cast<int32_t*>(ws + mask_bytes);
    auto* partials = reinterpret_cast<int64_t*>(ws + mask_bytes + align256(sizeof(int32_t) * (size_t)(nb * kEbWaves)));
    hipLaunchKernelGGL(k_eb_count, dim3((unsigned)nb), dim3(kEbThreads), 0, s, t, n_hits, (uint64_t)gap, masks,
                       wcount, partials, out_status);
    if (hipGetLastError() != hipSuccess) return TRIG_EHIP;
    hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(kScanThreads), 0, s, partials, nb);
    if (hipGetLastError() != hipSuccess) return TRIG_EHIP;
    hipLaunchKernelGGL(k_eb_scatter, dim3((unsigned)nb), dim3(kEbThreads), 0, s, n_hits, masks, wcount, partials,
                       (int)nb, out_offsets, out_capacity, out_n_events, out_status);
    return hipGetLastError() == hipSuccess ? TRIG_OK : TRIG_EHIP;
}

}  // extern "C"
