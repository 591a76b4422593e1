// Trigger-station filtering on the device (include/trig_filter.h): every
// event's hits of the three trigger layers, in input order per layer, as the
// CSR offsets and fp32 x/y arrays the selection reads.  The paper does this
// on the host before the transfer (Sec. 5.3, implementation i3); here the
// station numbers are streamed once.
//
// Partition: a workgroup of 4 waves owns kFilterEvents consecutive events;
// wave w takes events w, w + 4, ...  A wave reads an event's station numbers
// 32 per lane (two 16-byte loads of consecutive hits, 2048 hits per step),
// so the hits of lane L precede those of lane L + 1 in a step.  The count
// kernel sums each layer's hits and writes the positions of the trigger hits
// (with their layer, in input order) to the wave's list in the workspace;
// the scatter kernel ranks the list's entries per layer with ballots and
// moves x and y.  A wave whose events hold more trigger hits than its list
// (or an event of 2^30 hits or more) leaves the list incomplete, and the
// scatter then reads those events' station numbers again: a hit's rank in its
// layer is the exclusive prefix over lanes of the per-lane counts plus the
// count of the lane's earlier hits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "trig.h"
#include "trig_device.hpp"
#include "trig_filter.h"

namespace {

constexpr int kFilterThreads = 256;
constexpr int kFilterWaves = kFilterThreads / trig::kWave;
constexpr int kFilterEvents = 32;  // events per workgroup

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

// Hits per lane and step: a lane reads kLaneHits consecutive station numbers
// (two 16-byte loads, both in flight at once), a wave kLaneHits * 64.
constexpr int kLaneHits = 32;
constexpr int64_t kStepHits = (int64_t)kLaneHits * trig::kWave;

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// Station numbers of hits h0 .. h0 + 31 (h0 a multiple of 16 when vec) as 8
// words of 4; 0xFF bytes where a hit is past the array (the caller masks
// hits outside the event, so a padding byte never counts).
struct LaneStations {
    uint32_t w[kLaneHits / 4];
    __device__ __forceinline__ void load(const uint8_t* __restrict__ st, int64_t h0, int64_t n_hits, bool vec) {
        if (vec && h0 + kLaneHits <= n_hits) {
            const u32x4 a = *reinterpret_cast<const u32x4*>(st + h0);
            const u32x4 b = *reinterpret_cast<const u32x4*>(st + h0 + 16);
            w[0] = a.x; w[1] = a.y; w[2] = a.z; w[3] = a.w;
            w[4] = b.x; w[5] = b.y; w[6] = b.z; w[7] = b.w;
            return;
        }
#pragma unroll
        for (int q = 0; q < kLaneHits / 4; ++q) {
            uint32_t v = 0xFFFFFFFFu;
            for (int k = 0; k < 4; ++k) {
                const int64_t h = h0 + 4 * q + k;
                if (h < n_hits) v = (v & ~(0xFFu << (8 * k))) | ((uint32_t)st[h] << (8 * k));
            }
            w[q] = v;
        }
    }
};

// Per lane: which of its kLaneHits hits (bit j = hit h0 + j) belong to trigger
// layer l, for l = 0, 1, 2, among the hits in [a, b).
struct LaneMatch {
    uint32_t m[3];
};

// Bytes of w equal to the byte v (v4 = v * 0x01010101): bit k set for byte k.
// A byte of x = w ^ v4 is zero where they are equal; adding 0x7F to each
// byte's low seven bits carries into its bit 7 exactly when they are not all
// zero (never into the next byte), so bit 7 of ~(that | x) marks the zero
// bytes, and one multiply gathers the four marks into bits 21..24.
__device__ __forceinline__ uint32_t eq_bytes(uint32_t w, uint32_t v4) {
    const uint32_t x = w ^ v4;
    const uint32_t t = ((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x;
    const uint32_t z = ~t & 0x80808080u;
    return (((z >> 7) * 0x00204081u) >> 21) & 0xFu;
}

__device__ __forceinline__ LaneMatch match_lane(const LaneStations& s, int64_t h0, int64_t a, int64_t b,
                                                 uint32_t layers) {
    // hits of the event: bits [lo, hi) of the lane's window
    const int64_t lo = a - h0 > 0 ? a - h0 : 0, hi = b - h0 < kLaneHits ? b - h0 : kLaneHits;
    uint32_t in = 0;
    if (hi > lo) {
        const uint32_t up = hi >= 32 ? 0xFFFFFFFFu : ((1u << hi) - 1u);
        in = up & ~((1u << lo) - 1u);
    }
    LaneMatch r{{0u, 0u, 0u}};
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const uint32_t v4 = ((layers >> (8 * l)) & 0xFFu) * 0x01010101u;
#pragma unroll
        for (int q = 0; q < kLaneHits / 4; ++q) r.m[l] |= eq_bytes(s.w[q], v4) << (4 * q);
    }
#pragma unroll
    for (int l = 0; l < 3; ++l) r.m[l] &= in;
    return r;
}

// Trigger-hit entries one wave keeps for the scatter (its events' trigger
// hits, input order): (layer << 30) | (hit - event start).
constexpr int kWaveList = 2048;
constexpr int64_t kMaxListEvent = (int64_t)1 << 30;  // events this large are not listed

// Offsets of a step's matched hits in the step's list (per wave, in LDS):
// entry (layer << 11) | (offset of the hit in the step), layer 0's, 1's and
// 2's hits merged in input order (per-lane counts, a wave scan, then each
// lane's hits in bit order).  Returns the step's number of entries.
__device__ __forceinline__ int32_t step_list(const LaneMatch& m, uint16_t* list) {
    const int lane = (int)trig::lane_id();
    const uint32_t all = m.m[0] | m.m[1] | m.m[2];
    const int n = __builtin_popcount(all);
    const int incl = trig::wave_inclusive_sum(n);
    int32_t q = incl - n;
    for (uint32_t bits = all; bits; bits &= bits - 1u) {
        const int b = __builtin_ctz(bits);
        const uint32_t l = (m.m[0] >> b) & 1u ? 0u : ((m.m[1] >> b) & 1u ? 1u : 2u);
        list[q++] = (uint16_t)((l << 11) | (uint32_t)(kLaneHits * lane + b));
    }
    return __builtin_amdgcn_readlane(incl, 63);
}

__global__ __launch_bounds__(kFilterThreads) void k_filter_count(const int64_t* __restrict__ off, int n_events,
                                                                   int64_t n_hits, const uint8_t* __restrict__ st,
                                                                   uint32_t layers, int vec,
                                                                   int32_t* __restrict__ counts,
                                                                   int64_t* __restrict__ partials,
                                                                   uint32_t* __restrict__ wave_lists,
                                                                   uint32_t* status) {
    __shared__ int64_t wave_total[kFilterWaves];
    __shared__ uint16_t lists[kFilterWaves][kStepHits];  // per wave: the step's matched hits
    const int w = trig::uniform_i((int)(threadIdx.x / trig::kWave));
    const int lane = (int)trig::lane_id();
    const int e_first = (int)blockIdx.x * kFilterEvents;
    uint16_t* slist = lists[w];
    uint32_t* wlist = wave_lists + ((int64_t)blockIdx.x * kFilterWaves + w) * kWaveList;
    int32_t used = 0;   // entries of wlist written
    bool keep = true;   // wlist holds every trigger hit of this wave's events so far (wave-uniform)
    int64_t total = 0;
    for (int j = w; j < kFilterEvents; j += kFilterWaves) {
        const int e = e_first + j;
        if (e >= n_events) break;
        const Range r = event_range(off, e, n_hits);
        uint32_t c[3] = {0u, 0u, 0u};
        if (r.ok) {
            if (r.b - r.a >= kMaxListEvent) keep = false;
            // double-buffered: the next step's station numbers are in flight
            // while this step's are matched
            int64_t base = r.a & ~(int64_t)15;
            LaneStations cur, nxt;
            cur.load(st, base + (int64_t)kLaneHits * lane, n_hits, vec != 0);
            for (; base < r.b; base += kStepHits) {
                const int64_t h0 = base + (int64_t)kLaneHits * lane;
                if (base + kStepHits < r.b) nxt.load(st, h0 + kStepHits, n_hits, vec != 0);  // wave-uniform
                const LaneMatch m = match_lane(cur, h0, r.a, r.b, layers);
#pragma unroll
                for (int l = 0; l < 3; ++l) c[l] += (uint32_t)__builtin_popcount(m.m[l]);
                cur = nxt;
                if (keep) {
                    const int32_t nstep = step_list(m, slist);
                    if (used + nstep > kWaveList) {
                        keep = false;
                    } else if (nstep > 0) {
                        trig::wave_lds_sync();
                        // matched hits lie in [r.a, r.b): base - r.a + offset >= 0
                        const int32_t rel0 = (int32_t)(base - r.a);
                        for (int32_t i = lane; i < nstep; i += trig::kWave) {
                            const uint32_t en = slist[i];
                            wlist[used + i] = ((en >> 11) << 30) | (uint32_t)(rel0 + (int32_t)(en & 2047u));
                        }
                        used += nstep;
                    }
                    trig::wave_lds_sync();  // the next step rewrites the list
                }
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
// One workgroup: thread t sums its run of ceil(n / threads) consecutive
// partials, one block scan of those sums (Hillis-Steele in LDS), then each
// thread rewrites its run from its prefix.
__global__ __launch_bounds__(kFilterThreads) void k_filter_scan(int64_t* partials, int n) {
    __shared__ int64_t buf[kFilterThreads];
    const int t = (int)threadIdx.x;
    const int per = (n + kFilterThreads - 1) / kFilterThreads;
    const int lo = min(n, t * per), hi = min(n, lo + per);
    int64_t sum = 0;
    for (int i = lo; i < hi; ++i) sum += partials[i];
    buf[t] = sum;
    __syncthreads();
    for (int d = 1; d < kFilterThreads; d <<= 1) {  // inclusive
        const int64_t o = t >= d ? buf[t - d] : 0;
        __syncthreads();
        buf[t] += o;
        __syncthreads();
    }
    int64_t run = buf[t] - sum;  // exclusive prefix of this run
    for (int i = lo; i < hi; ++i) {
        const int64_t v = partials[i];
        partials[i] = run;
        run += v;
    }
    if (t == kFilterThreads - 1) partials[n] = buf[t];
}

__global__ __launch_bounds__(kFilterThreads) void k_filter_scatter(
    const int64_t* __restrict__ off, int n_events, int64_t n_hits, const uint8_t* __restrict__ st,
    const float* __restrict__ x, const float* __restrict__ y, uint32_t layers, int vec,
    const int32_t* __restrict__ counts, const int64_t* __restrict__ partials,
    const uint32_t* __restrict__ wave_lists, int n_blocks, int32_t capacity, int32_t* __restrict__ out_off,
    float* __restrict__ out_x, float* __restrict__ out_y, uint32_t* status) {
    __shared__ int64_t ev_start[kFilterEvents];
    __shared__ uint16_t lists[kFilterWaves][kStepHits];  // per wave: the step's matched hits (no-list path)
    const int w = trig::uniform_i((int)(threadIdx.x / trig::kWave));
    uint16_t* list = lists[w];
    const int lane = (int)trig::lane_id();
    const int e_first = (int)blockIdx.x * kFilterEvents;
    const int64_t cap = capacity;
    if (threadIdx.x == 0) {
        // Starts of the workgroup's events: its base plus the totals of the
        // events before (int64: three int32 counts per event).
        int64_t at = partials[blockIdx.x];
        for (int j = 0; j < kFilterEvents; ++j) {
            ev_start[j] = at;
            const int e = e_first + j;
            if (e < n_events)
                at += (int64_t)counts[3 * (int64_t)e] + counts[3 * (int64_t)e + 1] + counts[3 * (int64_t)e + 2];
        }
    }
    if ((int)blockIdx.x == n_blocks - 1 && threadIdx.x == 0) {
        const int64_t total = partials[n_blocks];
        if (total > cap && status) atomicOr(status, TRIG_FILTER_CAPACITY);
        out_off[3 * (int64_t)n_events] = (int32_t)std::min<int64_t>(total, cap);
    }
    __syncthreads();
    // The wave's list is complete iff the count kernel never stopped writing
    // it: all its events' trigger hits fit, and none of its events has 2^30
    // hits or more (the same conditions, from the counts and offsets).
    const uint32_t* wlist = wave_lists + ((int64_t)blockIdx.x * kFilterWaves + w) * kWaveList;
    bool listed = true;
    {
        int64_t n_list = 0;
        for (int j = w; j < kFilterEvents; j += kFilterWaves) {
            const int e = e_first + j;
            if (e >= n_events) break;
            const Range r = event_range(off, e, n_hits);
            if (r.ok && r.b - r.a >= kMaxListEvent) listed = false;
            n_list += (int64_t)counts[3 * (int64_t)e] + counts[3 * (int64_t)e + 1] + counts[3 * (int64_t)e + 2];
        }
        if (n_list > kWaveList) listed = false;
    }
    int32_t pos = 0;  // this event's first entry in wlist
    for (int j = w; j < kFilterEvents; j += kFilterWaves) {
        const int e = e_first + j;
        if (e >= n_events) break;
        const int64_t c0 = counts[3 * (int64_t)e], c1 = counts[3 * (int64_t)e + 1];
        const int64_t c2 = counts[3 * (int64_t)e + 2];
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
        if (listed) {
            // 64 entries per round: a lane's rank in its layer is the number
            // of earlier lanes with the same layer (entries are in input order)
            const int32_t tot = (int32_t)(c0 + c1 + c2);
            for (int32_t k0 = 0; k0 < tot; k0 += trig::kWave) {
                const int32_t k = k0 + lane;
                const bool valid = k < tot;
                const uint32_t en = valid ? wlist[pos + k] : 0u;
                const uint32_t l = en >> 30;
                const uint64_t b0 = trig::lanes(valid && l == 0u);
                const uint64_t b1 = trig::lanes(valid && l == 1u);
                const uint64_t b2 = trig::lanes(valid && l == 2u);
                const uint64_t mb = l == 0u ? b0 : (l == 1u ? b1 : b2);
                const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mb >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)mb, 0u));
                const int64_t p = (l == 0u ? s[0] : (l == 1u ? s[1] : s[2])) + rank;
                if (valid && p >= 0 && p < cap) {
                    const int64_t h = r.a + (int64_t)(en & 0x3FFFFFFFu);
                    out_x[p] = x[h];
                    out_y[p] = y[h];
                }
                s[0] += __builtin_popcountll(b0);
                s[1] += __builtin_popcountll(b1);
                s[2] += __builtin_popcountll(b2);
            }
            pos += tot;
            continue;
        }
        int64_t base = r.a & ~(int64_t)15;
        LaneStations cur, nxt;
        cur.load(st, base + (int64_t)kLaneHits * lane, n_hits, vec != 0);
        for (; base < r.b; base += kStepHits) {
            const int64_t h0 = base + (int64_t)kLaneHits * lane;
            if (base + kStepHits < r.b) nxt.load(st, h0 + kStepHits, n_hits, vec != 0);  // wave-uniform
            const LaneMatch m = match_lane(cur, h0, r.a, r.b, layers);
            cur = nxt;
            // Each matched hit's place in the step's list (layer 0's hits, then
            // layer 1's, then layer 2's, each in input order): entry =
            // layer << 11 | offset in the step.  Then every lane copies entries
            // lane, lane + 64, ...: one coalesced round trip per 64 hits,
            // however the trigger hits are spread over the lanes.
            int32_t at = 0;
            int32_t list_off[3], tot[3];
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                const int n = __builtin_popcount(m.m[l]);
                const int incl = trig::wave_inclusive_sum(n);
                tot[l] = __builtin_amdgcn_readlane(incl, 63);
                list_off[l] = at;
                int32_t q = at + (incl - n);
                for (uint32_t bits = m.m[l]; bits; bits &= bits - 1u)
                    list[q++] = (uint16_t)((l << 11) | (kLaneHits * lane + __builtin_ctz(bits)));
                at += tot[l];
            }
            trig::wave_lds_sync();
            for (int32_t i = lane; i < at; i += trig::kWave) {
                const uint32_t entry = list[i];
                const int l = (int)(entry >> 11);
                const int64_t h = base + (entry & 2047u);
                const int64_t p = s[l] + (i - (l == 0 ? list_off[0] : (l == 1 ? list_off[1] : list_off[2])));
                if (p >= 0 && p < cap) {  // positions past an int32 block prefix are never written
                    out_x[p] = x[h];
                    out_y[p] = y[h];
                }
            }
            trig::wave_lds_sync();  // the next step rewrites the list
#pragma unroll
            for (int l = 0; l < 3; ++l) s[l] += tot[l];
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
    return align256(sizeof(int32_t) * 3 * (size_t)n_events) + align256(sizeof(int64_t) * (size_t)(nb + 1)) +
           align256(sizeof(uint32_t) * (size_t)nb * kFilterWaves * kWaveList);
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
    char* ws = static_cast<char*>(p->workspace);
    const size_t counts_bytes = align256(sizeof(int32_t) * 3 * (size_t)n);
    auto* partials = reinterpret_cast<int64_t*>(ws + counts_bytes);
    auto* wave_lists = reinterpret_cast<uint32_t*>(ws + counts_bytes + align256(sizeof(int64_t) * (size_t)(nb + 1)));
    const uint32_t layers = (uint32_t)p->layers[0] | ((uint32_t)p->layers[1] << 8) | ((uint32_t)p->layers[2] << 16);
    const int vec = (reinterpret_cast<uintptr_t>(ev->station) & 15) == 0;
    hipLaunchKernelGGL(k_filter_count, dim3(nb), dim3(kFilterThreads), 0, s, ev->offsets, n, ev->n_hits,
                       ev->station, layers, vec, counts, partials, wave_lists, p->out_status);
    if (hipGetLastError() != hipSuccess) return TRIG_EHIP;
    hipLaunchKernelGGL(k_filter_scan, dim3(1), dim3(kFilterThreads), 0, s, partials, nb);
    if (hipGetLastError() != hipSuccess) return TRIG_EHIP;
    hipLaunchKernelGGL(k_filter_scatter, dim3(nb), dim3(kFilterThreads), 0, s, ev->offsets, n, ev->n_hits,
                       ev->station, ev->x, ev->y, layers, vec, counts, partials, wave_lists, nb, p->out_capacity,
                       p->out_layer_offsets, p->out_x, p->out_y, p->out_status);
    return hipGetLastError() == hipSuccess ? TRIG_OK : TRIG_EHIP;
}

}  // extern "C"
