// HIP kernels and C ABI of the trigger-station triplet selection (gfx950).
//
// Paper Sec. 3.2 "Algorithm": every one-hit-per-layer triplet is fitted by a
// line through the vertex in x-z and y-z, rejected if the mean square
// deviation per degree of freedom is above the plane's cut, and the event is
// selected with at least two passing triplets.  The selected-event list is
// what the paper copies back to the host (Sec. 5.3, step 6).
//
// Kernels
//   k_plain        one wave per event, all pair tiles, layer-2 hits in LDS
//   k_units        persistent form, step 1: per-event validation and the
//                  number of work units (ceil(pair tiles / tile units))
//   k_scan_*       exclusive scans of per-block partial sums
//   k_persistent   persistent grid; workgroups take batches of work units from
//                  one global counter, waves add their counts with integer atomics
//   k_finalize     accept flags from the accumulated counts
//   k_block        batched form: blocks of events staged in LDS, exact pair
//                  pruning (trig_block.hpp); optionally persistent
//   k_binned       binned form: one wave per event, slope-cell binning of
//                  layers 1 and 2 in LDS (trig_binned.hpp); optionally
//                  persistent
//   k_compact_*    ordered list of accepted event ids
#include <hip/hip_runtime.h>

#include <algorithm>
#include <limits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include "trig.h"
#include "trig_binned.hpp"
#include "trig_block.hpp"
#include "trig_bounds.hpp"
#include "trig_device.hpp"

using namespace trig;

namespace {

constexpr int kPlainWaves = 4;      // waves (events) per workgroup, plain form
constexpr int kChunkMsd = 512;      // layer-2 hits per LDS chunk (2 floats each)
constexpr int kChunkFit = 256;      // layer-2 hits per LDS chunk (4 floats each)
constexpr int kChunkZ = 160;        // layer-2 hits per LDS chunk (6 floats each)
constexpr int kScanBlock = 256;     // threads of the scan/compaction kernels
constexpr int kCompactItems = 4;    // events per thread in compaction
constexpr int kPersistWaves = 4;    // waves per workgroup, persistent form
constexpr int kPersistBatch = 4;    // work units taken per atomic
constexpr int kDefaultTileUnits = 8;  // pair tiles (of 64 pairs) per work unit
constexpr int kClaimsPerGroup = 8;    // claims per workgroup (pipelined batched form) or per wave (binned)
constexpr double kRuleFill = 0.85;    // built-in rule: hits per block over the LDS capacity

template <class T>
struct Chunk;
template <>
struct Chunk<MsdBasisTest> { static constexpr int value = kChunkMsd; };
template <>
struct Chunk<WindowTest> { static constexpr int value = kChunkMsd; };
template <>
struct Chunk<MsdFitTest> { static constexpr int value = kChunkFit; };
template <>
struct Chunk<MsdZTest> { static constexpr int value = kChunkZ; };
template <>
struct Chunk<WindowZTest> { static constexpr int value = kChunkMsd; };

__device__ __forceinline__ void write_result(int e, int32_t cnt, const Consts& c,
                                             int32_t* counts, uint8_t* accept,
                                             uint32_t* status) {
    counts[e] = capped(cnt, c);
    accept[e] = (uint8_t)(cnt >= 0 && cnt >= c.min_triplets);
    if (cnt < 0 && status) atomicOr(status, cnt == -1 ? TRIG_STATUS_MALFORMED : TRIG_STATUS_OVERFLOW);
}

// ---------------------------------------------------------------- plain ---

template <class T, int WPB>
__global__ __launch_bounds__(WPB * kWave) void k_plain(const int32_t* __restrict__ off,
                                                       int n_events, const float* __restrict__ x,
                                                       const float* __restrict__ y,
                                                       const float* __restrict__ z, Consts c,
                                                       int32_t* __restrict__ counts,
                                                       uint8_t* __restrict__ accept,
                                                       uint32_t* status) {
    constexpr int KCH = Chunk<T>::value;
    __shared__ __align__(16) float lds_all[WPB][KCH * T::HF];
    const int w = uniform_i(threadIdx.x / kWave);
    const int e = uniform_i(blockIdx.x) * WPB + w;
    if (e >= n_events) return;
    EventRange ev;
    int32_t cnt = load_event(off, e, c.n_hits, ev);
    if (cnt == 0) {
        const uint32_t tiles = pair_tiles(ev);
        if (tiles) cnt = (int32_t)wave_count<T, KCH>(x, y, z, ev, 0, tiles, c, lds_all[w]);
    }
    if (lane_id() == 0) write_result(e, cnt, c, counts, accept, status);
}

// ---------------------------------------------------------------- scans ---

// Exclusive scan of one value per thread over a workgroup of kScanBlock
// threads; also returns the workgroup total.
template <typename V>
__device__ V block_exclusive_scan(V v, V& total) {
    __shared__ V wave_sums[kScanBlock / kWave];
    const unsigned lane = lane_id();
    const int w = threadIdx.x / kWave;
    V incl = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const V o = __shfl_up(incl, d, kWave);
        if ((int)lane >= d) incl += o;
    }
    if (lane == kWave - 1) wave_sums[w] = incl;
    __syncthreads();
    V before = 0, sum = 0;
#pragma unroll
    for (int k = 0; k < kScanBlock / kWave; ++k) {
        const V s = wave_sums[k];
        if (k < w) before += s;
        sum += s;
    }
    __syncthreads();
    total = sum;
    return before + incl - v;
}

// In-place exclusive scan of partials[0..n); partials[n] receives the total.
// One workgroup.
template <typename V>
__global__ __launch_bounds__(kScanBlock) void k_scan_partials(V* partials, int n) {
    V carry = 0;
    for (int base = 0; base < n; base += kScanBlock) {
        const int i = base + (int)threadIdx.x;
        const V v = i < n ? partials[i] : V(0);
        V total;
        const V ex = block_exclusive_scan<V>(v, total);
        if (i < n) partials[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) partials[n] = carry;
}

// ------------------------------------------------------------ compaction ---

__global__ __launch_bounds__(kScanBlock) void k_compact_count(const uint8_t* __restrict__ accept,
                                                              int n_events,
                                                              int32_t* __restrict__ partials) {
    const int64_t base = (int64_t)blockIdx.x * kScanBlock * kCompactItems +
                         (int64_t)threadIdx.x * kCompactItems;
    int32_t c = 0;
#pragma unroll
    for (int k = 0; k < kCompactItems; ++k)
        if (base + k < n_events) c += accept[base + k] != 0;
    int32_t total;
    block_exclusive_scan<int32_t>(c, total);
    if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanBlock) void k_compact_write(const uint8_t* __restrict__ accept,
                                                              int n_events,
                                                              const int32_t* __restrict__ partials,
                                                              int n_blocks,
                                                              int32_t* __restrict__ ids,
                                                              int32_t* __restrict__ n_out) {
    const int64_t base = (int64_t)blockIdx.x * kScanBlock * kCompactItems +
                         (int64_t)threadIdx.x * kCompactItems;
    uint8_t f[kCompactItems];
    int32_t c = 0;
#pragma unroll
    for (int k = 0; k < kCompactItems; ++k) {
        f[k] = (base + k < n_events) ? (accept[base + k] != 0) : 0;
        c += f[k];
    }
    int32_t total;
    int32_t pos = partials[blockIdx.x] + block_exclusive_scan<int32_t>(c, total);
#pragma unroll
    for (int k = 0; k < kCompactItems; ++k)
        if (f[k]) ids[pos++] = (int32_t)(base + k);
    if (blockIdx.x == 0 && threadIdx.x == 0) *n_out = partials[n_blocks];
}

// k_compact_write without the scan kernel before it: each block sums the
// counts of the blocks before it (at most kPrefixBlocks of them, read from
// L2), and the last block writes the total.
constexpr int kPrefixBlocks = 4096;

__global__ __launch_bounds__(kScanBlock) void k_compact_write_prefix(const uint8_t* __restrict__ accept,
                                                                     int n_events,
                                                                     const int32_t* __restrict__ partials,
                                                                     int n_blocks,
                                                                     int32_t* __restrict__ ids,
                                                                     int32_t* __restrict__ n_out) {
    int32_t before = 0;
    for (int i = (int)threadIdx.x; i < (int)blockIdx.x; i += kScanBlock) before += partials[i];
    int32_t prefix;
    block_exclusive_scan<int32_t>(before, prefix);
    const int64_t base = (int64_t)blockIdx.x * kScanBlock * kCompactItems +
                         (int64_t)threadIdx.x * kCompactItems;
    uint8_t f[kCompactItems];
    int32_t c = 0;
#pragma unroll
    for (int k = 0; k < kCompactItems; ++k) {
        f[k] = (base + k < n_events) ? (accept[base + k] != 0) : 0;
        c += f[k];
    }
    int32_t total;
    int32_t pos = prefix + block_exclusive_scan<int32_t>(c, total);
#pragma unroll
    for (int k = 0; k < kCompactItems; ++k)
        if (f[k]) ids[pos++] = (int32_t)(base + k);
    if ((int)blockIdx.x == n_blocks - 1 && threadIdx.x == 0) *n_out = prefix + total;
}

__global__ void k_store_zero(int32_t* p) { *p = 0; }

// ------------------------------------------------------------ persistent ---

// Per event: validation (error counts written here), count initialised to 0,
// number of work units stored in ustart[e]; per-block unit totals.
__global__ __launch_bounds__(kScanBlock) void k_units(const int32_t* __restrict__ off,
                                                      int n_events, Consts c, int tile_units,
                                                      int32_t* __restrict__ counts,
                                                      uint8_t* __restrict__ accept,
                                                      uint32_t* status,
                                                      int64_t* __restrict__ ustart,
                                                      int64_t* __restrict__ partials,
                                                      unsigned long long* counter) {
    const int64_t e = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
    int64_t units = 0;
    if (e < n_events) {
        int32_t cnt = 0;
        const int64_t b = 3 * e;
        const int a0 = off[b], a1 = off[b + 1], a2 = off[b + 2], a3 = off[b + 3];
        if (!(0 <= a0 && a0 <= a1 && a1 <= a2 && a2 <= a3 && a3 <= c.n_hits)) {
            cnt = -1;
        } else {
            const int64_t n0 = a1 - a0, n1 = a2 - a1, n2 = a3 - a2;
            if (n2 > 0 && n0 * n1 > (int64_t)INT32_MAX / n2) {
                cnt = -2;
            } else if (n2 > 0) {
                const int64_t tiles = (n0 * n1 + kWave - 1) / kWave;
                units = (tiles + tile_units - 1) / tile_units;
            }
        }
        counts[e] = cnt;
        if (cnt < 0) {
            accept[e] = 0;
            if (status) atomicOr(status, cnt == -1 ? TRIG_STATUS_MALFORMED : TRIG_STATUS_OVERFLOW);
        }
        ustart[e] = units;
    }
    int64_t total;
    block_exclusive_scan<int64_t>(units, total);
    if (threadIdx.x == 0) partials[blockIdx.x] = total;
    if (e == 0) *counter = 0ull;
}

__global__ __launch_bounds__(kScanBlock) void k_units_apply(int n_events,
                                                            int64_t* __restrict__ ustart,
                                                            const int64_t* __restrict__ partials,
                                                            int n_blocks) {
    const int64_t e = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
    const int64_t units = e < n_events ? ustart[e] : 0;
    int64_t total;
    const int64_t ex = block_exclusive_scan<int64_t>(units, total);
    if (e < n_events) ustart[e] = partials[blockIdx.x] + ex;
    if (blockIdx.x == 0 && threadIdx.x == 0) ustart[n_events] = partials[n_blocks];
}

// Largest event e in [0, n) with ustart[e] <= u, for ustart non-decreasing,
// ustart[0] = 0 <= u < ustart[n].  64-ary search: each round probes 64
// evenly spaced entries with one load per lane.
__device__ int wave_find_event(const int64_t* __restrict__ ustart, int n, int64_t u) {
    const unsigned lane = lane_id();
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int len = hi - lo;
        const int step = (len + kWave - 1) / kWave;
        const int64_t idx = (int64_t)lo + (int64_t)lane * step;
        const bool ok = (idx < hi) && (ustart[idx] <= u);
        const int cnt = __popcll(__ballot(ok));  // lane 0 always true: cnt >= 1
        const int nlo = lo + (cnt - 1) * step;
        const int nhi = (int)min((int64_t)hi, (int64_t)lo + (int64_t)cnt * step);
        lo = uniform_i(nlo);
        hi = uniform_i(nhi);
    }
    return lo;
}

template <class T, int WPB>
__global__ __launch_bounds__(WPB * kWave) void k_persistent(
    const int32_t* __restrict__ off, int n_events, const float* __restrict__ x,
    const float* __restrict__ y, const float* __restrict__ z, Consts c, const int64_t* __restrict__ ustart,
    int tile_units,
    unsigned long long* counter, int32_t* counts) {
    constexpr int KCH = Chunk<T>::value;
    __shared__ __align__(16) float lds_all[WPB][KCH * T::HF];
    __shared__ unsigned long long s_first;
    const int w = uniform_i(threadIdx.x / kWave);
    float* lds = lds_all[w];
    const int64_t total = ustart[n_events];
    for (;;) {
        // The workgroup takes WPB batches at once (thread 0, through LDS);
        // every branch below depends on workgroup-uniform values only.
        if (threadIdx.x == 0) s_first = atomicAdd(counter, (unsigned long long)(WPB * kPersistBatch));
        __syncthreads();
        const unsigned long long wg_first = s_first;
        __syncthreads();
        const int64_t first = (int64_t)(((uint64_t)(uint32_t)uniform_i((int)(uint32_t)(wg_first >> 32)) << 32) |
                                        (uint32_t)uniform_i((int)(uint32_t)wg_first));
        if (first >= total) break;
        const int64_t lo = first + (int64_t)w * kPersistBatch;
        const int64_t hi = min(lo + kPersistBatch, total);
        if (lo < hi) {
            int e = wave_find_event(ustart, n_events, lo);
            for (int64_t u = lo; u < hi; ++u) {
                while (ustart[e + 1] <= u) ++e;  // next non-empty event
                EventRange ev;
                load_event(off, e, c.n_hits, ev);  // valid: only such events own units
                const uint32_t tiles = pair_tiles(ev);
                const uint32_t tb = (uint32_t)((u - ustart[e]) * tile_units);
                const uint32_t te = min(tiles, tb + (uint32_t)tile_units);
                const uint32_t cnt = wave_count<T, KCH>(x, y, z, ev, tb, te, c, lds);
                if (lane_id() == 0 && cnt) atomicAdd(&counts[e], (int32_t)cnt);
            }
        }
    }
}

__global__ __launch_bounds__(kScanBlock) void k_finalize(int n_events, Consts c,
                                                         int32_t* __restrict__ counts,
                                                         uint8_t* __restrict__ accept) {
    const int64_t e = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
    if (e < n_events) {
        const int32_t cnt = counts[e];
        counts[e] = capped(cnt, c);
        accept[e] = (uint8_t)(cnt >= 0 && cnt >= c.min_triplets);
    }
}

// --------------------------------------------------------------- binned ---

constexpr int kBinWaves = 4;     // waves (one event each) per workgroup
constexpr int kBinResident = 8;  // binned workgroups per CU (LDS bound)

// One wave per event.  Non-persistent when block_counter == nullptr:
// workgroup b takes events [4 b, 4 b + 4), one per wave.  Otherwise every
// wave on its own takes runs of `chunk` consecutive events from
// *block_counter (zero at launch; one atomic per run) until none is left:
// no barrier, and no LDS beyond the waves' cells (8 workgroups fit on a CU).
// Events with more than kBinCap hits in layer 1 or 2 take the pair-pruned
// path from HBM.  The register budget is held to kBinResident waves per
// SIMD, the occupancy its LDS allows (one wave per SIMD per workgroup).
template <class B>
__global__ __launch_bounds__(kBinWaves * kWave) __attribute__((amdgpu_waves_per_eu(kBinResident))) void k_binned(
    const int32_t* __restrict__ off, int n_events, const float* __restrict__ x, const float* __restrict__ y,
    Consts c, unsigned* block_counter, int chunk, int32_t* __restrict__ counts, uint8_t* __restrict__ accept,
    uint32_t* status) {
    __shared__ __align__(16) BinLds lds_all[kBinWaves];
    const int w = uniform_i((int)(threadIdx.x / kWave));
    BinLds& L = lds_all[w];
    auto one_event = [&](int e) {
        EventRange ev;
        int32_t cnt = load_event(off, e, c.n_hits, ev);
        if (cnt == 0 && ev.n0 > 0 && ev.n1 > 0 && ev.n2 > 0) {
            if (ev.n1 <= kBinCap && ev.n2 <= kBinCap) {
                cnt = (int32_t)wave_event_binned<B>(c, x, y, ev.o0, ev.n0, ev.o1, ev.n1, ev.o2, ev.n2, L);
            } else {
                using P = typename B::Prune;
                const GlobalHits gh{x, y};
                float M = 0.0f;
                if constexpr (P::kMag) M = layer_mag(gh, ev.o1, ev.n1);
                cnt = (int32_t)wave_event_pruned<P>(c, P::bounds(c, M), gh, ev.o0, ev.n0, ev.o1, ev.n1, ev.o2,
                                                    ev.n2, L.a1, L.b1);
                wave_lds_sync();
            }
        }
        if (lane_id() == 0) write_result(e, cnt, c, counts, accept, status);
    };
    if (!block_counter) {
        const int64_t e = (int64_t)blockIdx.x * kBinWaves + w;
        if (e < n_events) one_event((int)e);
        return;
    }
    for (;;) {
        // every branch below depends on wave-uniform values only
        unsigned claim = 0u;
        if (lane_id() == 0) claim = atomicAdd(block_counter, 1u);
        const int64_t first = (int64_t)(unsigned)uniform_i((int)claim) * chunk;
        if (first >= n_events) break;
        const int last = (int)min(first + chunk, (int64_t)n_events);
        for (int e = (int)first; e < last; ++e) one_event(e);
    }
}

// -------------------------------------------------- two-particle mode ---

// TRIG_ACCEPT_TWO_PARTICLES, after the counting form has flagged the
// candidates (count >= 2): each wave scans the flags of 64 consecutive
// events and decides its candidates one by one (wave_two_particles), writing
// the final flag.  Events without a candidate cost one coalesced read.
constexpr int kTwoWaves = 4;
constexpr int kTwoPartCap = 512;  // layer-0 and layer-1 partials a wave keeps in LDS

template <class P>
__global__ __launch_bounds__(kTwoWaves * kWave) void k_two_particles(const int32_t* __restrict__ off, int n_events,
                                                                     const float* __restrict__ x,
                                                                     const float* __restrict__ y,
                                                                     const float* __restrict__ z, Consts c,
                                                                     uint8_t* __restrict__ accept) {
    const int w = uniform_i((int)(threadIdx.x / kWave));
    const int64_t base = ((int64_t)blockIdx.x * kTwoWaves + w) * kWave;
    if (base >= n_events) return;
    const int64_t e = base + lane_id();
    uint64_t m = lanes(e < n_events && accept[e] != 0);
    __shared__ float2 part_all[kTwoWaves][kTwoPartCap];
    using H = typename std::conditional<P::kZ, SlopeHits, GlobalHits>::type;
    H gh;
    if constexpr (P::kZ)
        gh = SlopeHits{x, y, z};
    else
        gh = GlobalHits{x, y};
    while (m) {
        const int L = __builtin_ctzll(m);
        m &= m - 1;
        const int ev_i = (int)(base + L);
        EventRange ev;
        bool two = false;
        if (load_event(off, ev_i, c.n_hits, ev) == 0 && ev.n0 > 0 && ev.n1 > 0 && ev.n2 > 0)
            two = wave_two_particles<P>(c, gh, ev.o0, ev.n0, ev.o1, ev.n1, ev.o2, ev.n2, part_all[w], kTwoPartCap);
        if (lane_id() == 0) accept[ev_i] = (uint8_t)two;
    }
}

// ------------------------------------------------------------ per-hit z ---

// Per-hit z (trig_hits.z), batched, binned and autotuned forms: one wave per
// event from HBM, pairs pruned on their slopes with the event's bound
// (wave_event_pruned over SlopeHits), or every triplet (wave_count) when the
// event has no valid bound.
template <class P, class T>
__global__ __launch_bounds__(kBinWaves * kWave) void k_event_z(const int32_t* __restrict__ off, int n_events,
                                                               const float* __restrict__ x,
                                                               const float* __restrict__ y,
                                                               const float* __restrict__ z, Consts c,
                                                               int32_t* __restrict__ counts,
                                                               uint8_t* __restrict__ accept, uint32_t* status) {
    constexpr int KCH = Chunk<T>::value;
    static_assert(KCH * T::HF >= 2 * kPBuf, "the pruned path's buffers fit in the staging slice");
    __shared__ __align__(16) float lds_all[kBinWaves][KCH * T::HF];
    const int w = uniform_i((int)(threadIdx.x / kWave));
    const int64_t e64 = (int64_t)blockIdx.x * kBinWaves + w;
    if (e64 >= n_events) return;
    const int e = (int)e64;
    float* lds = lds_all[w];
    EventRange ev;
    int32_t cnt = load_event(off, e, c.n_hits, ev);
    if (cnt == 0 && ev.n0 > 0 && ev.n1 > 0 && ev.n2 > 0) {
        const SlopeHits sh{x, y, z};
        const PairBounds pb = event_bounds<P>(c, sh, ev.o0, ev.n0, ev.o1, ev.n1);
        if (pb.prune) {
            // An event that fits one lane pass and one buffer fill takes the
            // fast path (the prefilter folded over all pairs, one vote); the
            // slope tests are symmetric in the two layers, as the batched
            // form's are.
            int R, TB, S;
            event_layout(ev.n0, ev.n1, R, TB, S);
            if (TB > 0)
                cnt = (int32_t)wave_event_fast<P>(c, pb, sh, ev.o0, ev.n0, ev.o1, ev.n1, ev.o2, ev.n2, R, TB, S,
                                                  recip16(S ? ev.n0 : ev.n1), lds, lds + kPBuf);
            else
                cnt = (int32_t)wave_event_pruned<P>(c, pb, sh, ev.o0, ev.n0, ev.o1, ev.n1, ev.o2, ev.n2, lds,
                                                    lds + kPBuf);
        } else {
            cnt = (int32_t)wave_count<T, KCH>(x, y, z, ev, 0, pair_tiles(ev), c, lds);
        }
    }
    if (lane_id() == 0) write_result(e, cnt, c, counts, accept, status);
}

// ------------------------------------------------------- static scratch ---

// Device scratch of trig_select_noalloc: the workspace of trig_select for
// callers that cannot allocate.  Every GPU the library runs on holds its own
// copy until the process ends; kernels receive its device address (looked up
// once per device), never this host-side name.
static __device__ __align__(256) unsigned char scratch[TRIG_NOALLOC_SCRATCH_BYTES];

// ------------------------------------------------------------------ host ---

thread_local std::string g_detail;
thread_local hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;

// Records the profiling hook's start event before the dominant kernel.
int mark_start(hipStream_t s) {
    if (g_ev_start && hipEventRecord(g_ev_start, s) != hipSuccess) return -1;
    return 0;
}
int mark_stop(hipStream_t s) {
    if (g_ev_stop && hipEventRecord(g_ev_stop, s) != hipSuccess) return -1;
    return 0;
}

int fail(int code, const std::string& why) {
    g_detail = why;
    return code;
}

// Device address of `scratch` on the current device, looked up on the first
// call per device (that device current) and kept.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

int scratch_address(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return fail(TRIG_EHIP, "no current device (or a device index beyond 63)");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(TRIG_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
    return TRIG_OK;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

Consts make_consts(const trig_params* p, int n_hits) {
    using namespace trig_host;
    Consts c;
    const Basis K = basis(p->z[0], p->z[1], p->z[2]);
    c.U0 = K.U0;
    c.U1 = K.U1;
    c.V0 = K.V0;
    c.V1 = K.V1;
    c.V2 = K.V2;
    c.z0 = p->z[0];
    c.z1 = p->z[1];
    c.z2 = p->z[2];
    const float szz = (c.z0 * c.z0 + c.z1 * c.z1) + c.z2 * c.z2;
    c.w = (float)(1.0 / (double)szz);
    c.qmax_x = fold_threshold(p->msd_max[0], p->ndf);
    c.qmax_y = fold_threshold(p->msd_max[1], p->ndf);
    c.beta_x = pair_bound(c.qmax_x);
    c.beta_y = pair_bound(c.qmax_y);
    const FitBounds fx = fit_bounds(c.z0, c.z1, c.z2, c.qmax_x);
    const FitBounds fy = fit_bounds(c.z0, c.z1, c.z2, c.qmax_y);
    c.fit_a0x = fx.a0;
    c.fit_a1x = fx.a1;
    c.fit_a0y = fy.a0;
    c.fit_a1y = fy.a1;
    c.fit_b0x = fx.b0;
    c.fit_b1x = fx.b1;
    const SlopeBounds sx = slope_bounds(c.qmax_x), sy = slope_bounds(c.qmax_y);
    c.zs_a0x = sx.a0;
    c.zs_a1x = sx.a1;
    c.zs_a0y = sy.a0;
    c.zs_a1y = sy.a1;
    c.pre_msd = std::max(c.beta_x, c.beta_y);
    c.pre_win = std::max(p->slope_window[0], p->slope_window[1]);
    c.win_x = p->slope_window[0];
    c.win_y = p->slope_window[1];
    c.bin_r = p->test == TRIG_TEST_SLOPE_WINDOW ? c.win_x : std::nextafter(c.beta_x, INFINITY);
    const bool two = (p->flags & TRIG_ACCEPT_TWO_PARTICLES) != 0;
    c.min_triplets = two ? 2 : p->min_triplets;  // two particles need two passing triplets
    c.count_cap = (p->flags & TRIG_DECISION_ONLY) ? (two ? 2 : p->min_triplets) : INT32_MAX;
    c.n_hits = n_hits;
    return c;
}

int validate_params(const trig_params* p, bool need_outputs);

int validate(const trig_events_csr* ev, const trig_hits* hits, const trig_params* p) {
    if (!ev || !hits || !p) return fail(TRIG_EINVAL, "NULL descriptor");
    if (ev->n_events < 0) return fail(TRIG_EINVAL, "n_events < 0");
    if (hits->n_hits < 0) return fail(TRIG_EINVAL, "n_hits < 0");
    if (ev->n_events > 0 && !ev->layer_offsets) return fail(TRIG_EINVAL, "layer_offsets is NULL");
    if (hits->n_hits > 0 && (!hits->x || !hits->y)) return fail(TRIG_EINVAL, "x or y is NULL");
    if (int r = validate_params(p, true)) return r;
    if (hits->z && p->test == TRIG_TEST_MSD_BASIS)
        return fail(TRIG_EUNSUPPORTED, "per-hit z is not provided for TRIG_TEST_MSD_BASIS");
    return TRIG_OK;
}

int validate_params(const trig_params* p, bool need_outputs) {
    if (!p) return fail(TRIG_EINVAL, "NULL params");
    if (p->abi_version != TRIG_ABI_VERSION) return fail(TRIG_EINVAL, "abi_version mismatch");
    if (p->test != TRIG_TEST_MSD && p->test != TRIG_TEST_MSD_BASIS && p->test != TRIG_TEST_SLOPE_WINDOW)
        return fail(TRIG_EINVAL, "unknown test");
    for (int l = 0; l < 3; ++l)
        if (!std::isfinite(p->z[l]) || !(p->z[l] > 0.0f)) return fail(TRIG_EINVAL, "z must be finite and > 0");
    for (int k = 0; k < 2; ++k) {
        if (!std::isfinite(p->msd_max[k]) || p->msd_max[k] < 0.0f)
            return fail(TRIG_EINVAL, "msd_max must be finite and >= 0");
        if (!std::isfinite(p->slope_window[k]) || p->slope_window[k] < 0.0f)
            return fail(TRIG_EINVAL, "slope_window must be finite and >= 0");
    }
    if (p->ndf < 1) return fail(TRIG_EINVAL, "ndf < 1");
    if (p->min_triplets < 0) return fail(TRIG_EINVAL, "min_triplets < 0");
    if (p->tile_pairs < 0 || p->tile_pairs % kWave) return fail(TRIG_EINVAL, "tile_pairs not a multiple of 64");
    if (p->block_events < 0 || p->block_events > kMaxEB) return fail(TRIG_EINVAL, "block_events outside 0..128");
    if (p->block_hits != 0 && p->block_hits != 1024 && p->block_hits != 2048 && p->block_hits != 4096)
        return fail(TRIG_EINVAL, "block_hits must be 0, 1024, 2048 or 4096");
    if (p->block_waves != 0 && p->block_waves != 1 && p->block_waves != 2 && p->block_waves != 4)
        return fail(TRIG_EINVAL, "block_waves must be 0, 1, 2 or 4");
    for (int r : p->reserved)
        if (r) return fail(TRIG_EINVAL, "reserved fields must be zero");
    const uint32_t known = TRIG_EXEC_PERSISTENT | TRIG_EXEC_PRUNED | TRIG_EXEC_BINNED |
                           TRIG_EXEC_AUTOTUNE | TRIG_OUT_COMPACT | TRIG_ACCEPT_TWO_PARTICLES | TRIG_DECISION_ONLY;
    if (p->flags & ~known) return fail(TRIG_EINVAL, "unknown flag bits");
    if (need_outputs && (p->flags & TRIG_OUT_COMPACT) && (!p->out_accepted_ids || !p->out_n_accepted))
        return fail(TRIG_EINVAL, "TRIG_OUT_COMPACT needs out_accepted_ids and out_n_accepted");
    if ((p->flags & TRIG_EXEC_BINNED) && (p->flags & (TRIG_EXEC_PRUNED | TRIG_EXEC_AUTOTUNE)))
        return fail(TRIG_EUNSUPPORTED, "TRIG_EXEC_BINNED does not combine with TRIG_EXEC_PRUNED or TRIG_EXEC_AUTOTUNE");
    return TRIG_OK;
}

struct Layout {
    size_t compact_off = 0, units_off = 0, upart_off = 0, counter_off = 0, total = 0;
    int compact_blocks = 0, unit_blocks = 0;
};

Layout layout(int n_events, uint32_t flags) {
    Layout L;
    size_t at = 0;
    if (flags & TRIG_OUT_COMPACT) {
        L.compact_blocks = (int)std::max<int64_t>(1, cdiv(n_events, (int64_t)kScanBlock * kCompactItems));
        L.compact_off = at;
        at += align256(sizeof(int32_t) * (size_t)(L.compact_blocks + 1));
    }
    if ((flags & TRIG_EXEC_PERSISTENT) && (flags & (TRIG_EXEC_PRUNED | TRIG_EXEC_BINNED))) {
        L.counter_off = at;  // block counter only
        at += 256;
    } else if (flags & TRIG_EXEC_PERSISTENT) {
        L.unit_blocks = (int)std::max<int64_t>(1, cdiv(n_events, kScanBlock));
        L.counter_off = at;
        at += 256;
        L.units_off = at;
        at += align256(sizeof(int64_t) * ((size_t)n_events + 1));
        L.upart_off = at;
        at += align256(sizeof(int64_t) * (size_t)(L.unit_blocks + 1));
    }
    L.total = at;
    return L;
}

// Flags whose workspace layout covers a call: an autotuned call may run the
// batched or binned form with or without stealing, so it reserves the block
// counter.
uint32_t layout_flags(const trig_params* p) {
    if (!(p->flags & TRIG_EXEC_AUTOTUNE)) return p->flags;
    const uint32_t f = p->flags & ~(uint32_t)TRIG_EXEC_AUTOTUNE;
    return f | TRIG_EXEC_PRUNED | TRIG_EXEC_PERSISTENT;
}

int check_launch(const char* what) {
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return fail(TRIG_EHIP, std::string(what) + ": " + hipGetErrorString(err));
    return TRIG_OK;
}

int device_cus() {
    static std::mutex mu;
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    std::lock_guard<std::mutex> lock(mu);
    if (!cached[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
        cached[dev] = v;
    }
    return cached[dev];
}

template <class T>
int launch_plain(const trig_events_csr* ev, const trig_hits* h, const Consts& c, int32_t* counts,
                 uint8_t* accept, uint32_t* status, hipStream_t s) {
    const int n = ev->n_events;
    const unsigned grid = (unsigned)cdiv(n, kPlainWaves);
    if (mark_start(s)) return fail(TRIG_EHIP, "hipEventRecord(start)");
    hipLaunchKernelGGL((k_plain<T, kPlainWaves>), dim3(grid), dim3(kPlainWaves * kWave), 0, s,
                       ev->layer_offsets, n, h->x, h->y, h->z, c, counts, accept, status);
    if (int r = check_launch("k_plain")) return r;
    if (mark_stop(s)) return fail(TRIG_EHIP, "hipEventRecord(stop)");
    return TRIG_OK;
}

template <class T>
int launch_persistent(const trig_events_csr* ev, const trig_hits* h, const Consts& c, int tile_units,
                      const Layout& L, char* ws, int32_t* counts, uint8_t* accept, uint32_t* status,
                      hipStream_t s) {
    const int n = ev->n_events;
    auto* counter = reinterpret_cast<unsigned long long*>(ws + L.counter_off);
    auto* ustart = reinterpret_cast<int64_t*>(ws + L.units_off);
    auto* upart = reinterpret_cast<int64_t*>(ws + L.upart_off);
    hipLaunchKernelGGL(k_units, dim3(L.unit_blocks), dim3(kScanBlock), 0, s, ev->layer_offsets, n, c,
                       tile_units, counts, accept, status, ustart, upart, counter);
    if (int r = check_launch("k_units")) return r;
    hipLaunchKernelGGL(k_scan_partials<int64_t>, dim3(1), dim3(kScanBlock), 0, s, upart, L.unit_blocks);
    if (int r = check_launch("k_scan_partials")) return r;
    hipLaunchKernelGGL(k_units_apply, dim3(L.unit_blocks), dim3(kScanBlock), 0, s, n, ustart, upart,
                       L.unit_blocks);
    if (int r = check_launch("k_units_apply")) return r;
    // Enough resident waves to fill every CU; each exits once the counter
    // passes the unit total.
    const unsigned grid = (unsigned)device_cus() * 8u;
    if (mark_start(s)) return fail(TRIG_EHIP, "hipEventRecord(start)");
    hipLaunchKernelGGL((k_persistent<T, kPersistWaves>), dim3(grid), dim3(kPersistWaves * kWave), 0, s,
                       ev->layer_offsets, n, h->x, h->y, h->z, c, ustart, tile_units, counter, counts);
    if (int r = check_launch("k_persistent")) return r;
    if (mark_stop(s)) return fail(TRIG_EHIP, "hipEventRecord(stop)");
    hipLaunchKernelGGL(k_finalize, dim3(L.unit_blocks), dim3(kScanBlock), 0, s, n, c, counts, accept);
    return check_launch("k_finalize");
}

__global__ void k_zero_u32(unsigned* p) { *p = 0u; }

// Shape of the batched form: LDS hit capacity (hb), waves per workgroup (nw)
// and events per block (eb).  Given values are used as they are; the
// defaults take the largest capacity whose block holds at least 8 events of
// the batch's mean multiplicity at 60 % fill (fluctuations fit; blocks that
// overflow are split into sub-blocks by the kernel), one wave per 1024 hits.
struct BlockShape {
    int hb, nw, eb;
};
// Events per block that fill `fill` of an hb-hit block at the batch's mean
// event size.
int events_for_fill(double fill, int hb, int nw, int n_events, int n_hits) {
    const double mean = std::max(n_events > 0 ? (double)n_hits / n_events : 1.0, 1.0);
    int eb = (int)std::max(1.0, std::min((double)kMaxEB, std::floor(fill * hb / mean)));
    if (nw > 0 && eb >= nw) eb -= eb % nw;  // whole rounds of events over the waves
    return eb;
}

BlockShape choose_block_shape(const trig_params* p, int n_events, int n_hits) {
    const double mean = std::max(n_events > 0 ? (double)n_hits / n_events : 1.0, 1.0);
    int hb = p->block_hits;
    if (hb <= 0) hb = kRuleFill * 1024 / mean >= 16.0 ? 1024 : kRuleFill * 2048 / mean >= 16.0 ? 2048 : 4096;
    int nw = p->block_waves;
    if (nw <= 0) nw = std::min(4, hb / 512);
    int eb = p->block_events;
    if (eb <= 0) eb = events_for_fill(kRuleFill, hb, nw, n_events, n_hits);
    return {hb, nw, eb};
}

using BlockKernel = void (*)(const int32_t*, int, const float*, const float*, Consts, int, int, unsigned*, int,
                             int32_t*, uint8_t*, uint32_t*);

// Workgroups of `kern` that fit on one CU at once (cached per kernel).
int resident_per_cu(BlockKernel kern, int threads) {
    static std::mutex mu;
    static std::map<BlockKernel, int> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(kern);
    if (it != cache.end()) return it->second;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern), threads, 0) !=
            hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    cache[kern] = per_cu;
    return per_cu;
}

// The kernel for a shape; blocks of at most kSmallEB events at 2048 hits and
// four waves take the small event table (eight workgroups per CU).
template <class P>
BlockKernel block_kernel(int hb, int nw, bool pipelined, int eb) {
    if (!pipelined && hb == 2048 && nw == 4 && eb <= kSmallEB) return k_block<P, 2048, 4, kSmallEB>;
#define TRIG_BLOCK_CASE(H, W) \
    if (hb == H && nw == W) return pipelined ? k_block_pipe<P, H, W> : k_block<P, H, W, kMaxEB>;
    TRIG_BLOCK_CASE(1024, 1) TRIG_BLOCK_CASE(1024, 2) TRIG_BLOCK_CASE(1024, 4)
    TRIG_BLOCK_CASE(2048, 1) TRIG_BLOCK_CASE(2048, 2) TRIG_BLOCK_CASE(2048, 4)
    TRIG_BLOCK_CASE(4096, 1) TRIG_BLOCK_CASE(4096, 2) TRIG_BLOCK_CASE(4096, 4)
#undef TRIG_BLOCK_CASE
    return nullptr;
}

template <class P>
int launch_block(const trig_events_csr* ev, const trig_hits* h, const trig_params* p, const Consts& c,
                 const Layout& L, char* ws, int32_t* counts, uint8_t* accept, hipStream_t s) {
    const int n = ev->n_events;
    const BlockShape bs = choose_block_shape(p, n, h->n_hits);
    const int vec = ((reinterpret_cast<uintptr_t>(h->x) | reinterpret_cast<uintptr_t>(h->y)) & 15) == 0;
    // Block stealing uses the pipelined kernel, which needs 16-byte aligned
    // hit arrays; otherwise one workgroup per block.
    const bool pipelined = (p->flags & TRIG_EXEC_PERSISTENT) && vec;
    const BlockKernel kern = block_kernel<P>(bs.hb, bs.nw, pipelined, bs.eb);
    if (!kern) return fail(TRIG_EINVAL, "block_hits must be 1024, 2048 or 4096 and block_waves 1, 2 or 4");
    const int n_blocks = (int)cdiv(n, bs.eb);
    unsigned* counter = nullptr;
    unsigned grid = (unsigned)n_blocks;
    if (pipelined) {
        counter = reinterpret_cast<unsigned*>(ws + L.counter_off);
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, counter);
        if (int r = check_launch("k_zero_u32")) return r;
        grid = (unsigned)std::min<int64_t>(n_blocks, (int64_t)device_cus() * resident_per_cu(kern, bs.nw * kWave));
    }
    // Pipelined kernel: blocks per claim, about kClaimsPerGroup claims per
    // workgroup (one atomic on one counter per claim).
    const int aux = pipelined ? (int)std::max<int64_t>(1, n_blocks / ((int64_t)grid * kClaimsPerGroup)) : vec;
    if (mark_start(s)) return fail(TRIG_EHIP, "hipEventRecord(start)");
    hipLaunchKernelGGL(kern, dim3(grid), dim3(bs.nw * kWave), 0, s, ev->layer_offsets, n, h->x, h->y, c, bs.eb,
                       n_blocks, counter, aux, counts, accept, p->out_status);
    if (int r = check_launch("k_block")) return r;
    if (mark_stop(s)) return fail(TRIG_EHIP, "hipEventRecord(stop)");
    return TRIG_OK;
}

template <class B>
int launch_binned(const trig_events_csr* ev, const trig_hits* h, const trig_params* p, const Consts& c,
                  const Layout& L, char* ws, int32_t* counts, uint8_t* accept, hipStream_t s) {
    const int n = ev->n_events;
    const int64_t n_blocks = cdiv(n, kBinWaves);
    unsigned* counter = nullptr;
    unsigned grid = (unsigned)n_blocks;
    if (p->flags & TRIG_EXEC_PERSISTENT) {
        counter = reinterpret_cast<unsigned*>(ws + L.counter_off);
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, counter);
        if (int r = check_launch("k_zero_u32")) return r;
        grid = (unsigned)std::min<int64_t>(n_blocks, (int64_t)device_cus() * kBinResident);
    }
    // Persistent: runs of events per claim, about kClaimsPerGroup claims per wave.
    const int chunk =
        counter ? (int)std::max<int64_t>(1, (int64_t)n / ((int64_t)grid * kBinWaves * kClaimsPerGroup)) : 1;
    if (mark_start(s)) return fail(TRIG_EHIP, "hipEventRecord(start)");
    hipLaunchKernelGGL(k_binned<B>, dim3(grid), dim3(kBinWaves * kWave), 0, s, ev->layer_offsets, n, h->x, h->y, c,
                       counter, chunk, counts, accept, p->out_status);
    if (int r = check_launch("k_binned")) return r;
    if (mark_stop(s)) return fail(TRIG_EHIP, "hipEventRecord(stop)");
    return TRIG_OK;
}

template <class P>
int launch_two_particles(const trig_events_csr* ev, const trig_hits* h, const Consts& c, uint8_t* accept,
                         hipStream_t s) {
    const int64_t waves = cdiv(ev->n_events, kWave);
    hipLaunchKernelGGL(k_two_particles<P>, dim3((unsigned)cdiv(waves, kTwoWaves)), dim3(kTwoWaves * kWave), 0, s,
                       ev->layer_offsets, ev->n_events, h->x, h->y, h->z, c, accept);
    return check_launch("k_two_particles");
}

// Per-hit z: brute force as asked, every other form one wave per event with
// slope pruning (k_event_z).
template <class T, class P>
int run_form_z(const trig_events_csr* ev, const trig_hits* h, const trig_params* p, const Consts& c,
               const Layout& L, char* ws, int32_t* counts, uint8_t* accept, hipStream_t s) {
    int r = TRIG_OK;
    if (p->flags & (TRIG_EXEC_PRUNED | TRIG_EXEC_BINNED)) {
        if (mark_start(s)) return fail(TRIG_EHIP, "hipEventRecord(start)");
        hipLaunchKernelGGL((k_event_z<P, T>), dim3((unsigned)cdiv(ev->n_events, kBinWaves)), dim3(kBinWaves * kWave),
                           0, s, ev->layer_offsets, ev->n_events, h->x, h->y, h->z, c, counts, accept, p->out_status);
        if ((r = check_launch("k_event_z"))) return r;
        if (mark_stop(s)) return fail(TRIG_EHIP, "hipEventRecord(stop)");
    } else if (p->flags & TRIG_EXEC_PERSISTENT) {
        const int tile_units = p->tile_pairs ? p->tile_pairs / kWave : kDefaultTileUnits;
        r = launch_persistent<T>(ev, h, c, tile_units, L, ws, counts, accept, p->out_status, s);
    } else {
        r = launch_plain<T>(ev, h, c, counts, accept, p->out_status, s);
    }
    if (r == TRIG_OK && (p->flags & TRIG_ACCEPT_TWO_PARTICLES)) r = launch_two_particles<P>(ev, h, c, accept, s);
    return r;
}

template <class T, class P, class B>
int run_counting_form(const trig_events_csr* ev, const trig_hits* h, const trig_params* p, const Consts& c,
                      const Layout& L, char* ws, int32_t* counts, uint8_t* accept, hipStream_t s) {
    if (p->flags & TRIG_EXEC_BINNED) return launch_binned<B>(ev, h, p, c, L, ws, counts, accept, s);
    if (p->flags & TRIG_EXEC_PRUNED) return launch_block<P>(ev, h, p, c, L, ws, counts, accept, s);
    if (p->flags & TRIG_EXEC_PERSISTENT) {
        const int tile_units = p->tile_pairs ? p->tile_pairs / kWave : kDefaultTileUnits;
        return launch_persistent<T>(ev, h, c, tile_units, L, ws, counts, accept, p->out_status, s);
    }
    return launch_plain<T>(ev, h, c, counts, accept, p->out_status, s);
}

template <class T, class P, class B>
int run_form(const trig_events_csr* ev, const trig_hits* h, const trig_params* p, const Consts& c,
             const Layout& L, char* ws, int32_t* counts, uint8_t* accept, hipStream_t s) {
    int r = run_counting_form<T, P, B>(ev, h, p, c, L, ws, counts, accept, s);
    if (r == TRIG_OK && (p->flags & TRIG_ACCEPT_TWO_PARTICLES)) r = launch_two_particles<P>(ev, h, c, accept, s);
    return r;
}


// ------------------------------------------------------------ autotuner ---

// Multiplicity class of a batch: floor(log2(mean hits per event)), 0..31.
int multiplicity_class(int n_events, int n_hits) {
    const double mean = n_events > 0 ? (double)n_hits / n_events : 1.0;
    int cls = 0;
    while (cls < 31 && mean >= (double)(2u << cls)) ++cls;
    return cls;
}

struct TunedShape {
    int hb, nw;
    double fill;  // events per block = fill * hb / mean hits per event
    bool persistent;
    bool binned;  // the binned form (hb, nw, fill unused)
};


std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, TunedShape> g_tuned;  // (device, test, class)

int current_device() {
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess) d = 0;
    return d;
}

// A device as the autotune cache names it: architecture name and number of
// compute units (a record made on one MI355X holds for another).
bool device_key(int dev, std::string& key) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
    std::string arch(prop.gcnArchName);
    for (char& ch : arch)
        if (ch == ' ') ch = '_';
    key = arch + "/" + std::to_string(prop.multiProcessorCount) + "cu";
    return true;
}

constexpr const char* kCacheHeader = "trig-autotune-cache 1";

// Effective parameters of a TRIG_EXEC_AUTOTUNE call: the recorded form and
// shape of the batch's class, else the batched form with the built-in rule.
// Block fields the caller set explicitly win over the record and select the
// batched form.
trig_params resolve_autotune(const trig_params* p, int n_events, int n_hits) {
    trig_params q = *p;
    q.flags &= ~(uint32_t)TRIG_EXEC_AUTOTUNE;
    q.flags |= TRIG_EXEC_PRUNED;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tuned.find({current_device(), p->test, multiplicity_class(n_events, n_hits)});
    if (it != g_tuned.end()) {
        const TunedShape& t = it->second;
        if (t.binned && !p->block_hits && !p->block_waves && !p->block_events) {
            q.flags = (q.flags & ~(uint32_t)TRIG_EXEC_PRUNED) | TRIG_EXEC_BINNED |
                      (t.persistent ? (uint32_t)TRIG_EXEC_PERSISTENT : 0u);
            return q;
        }
        if (t.binned) return q;
        if (!q.block_hits) q.block_hits = t.hb;
        if (!q.block_waves) q.block_waves = t.nw;
        if (!q.block_events) q.block_events = events_for_fill(t.fill, q.block_hits, q.block_waves, n_events, n_hits);
        if (t.persistent) q.flags |= TRIG_EXEC_PERSISTENT;
    }
    return q;
}

}  // namespace

extern "C" {

int trig_params_init(trig_params* p) {
    if (!p) return fail(TRIG_EINVAL, "NULL params");
    std::memset(p, 0, sizeof(*p));
    p->abi_version = TRIG_ABI_VERSION;
    p->test = TRIG_TEST_MSD;
    p->z[0] = 400.0f;
    p->z[1] = 410.0f;
    p->z[2] = 420.0f;
    p->msd_max[0] = 0.03f;
    p->msd_max[1] = 0.025f;
    p->ndf = 2;
    p->slope_window[0] = 0.005f;
    p->slope_window[1] = 0.005f;
    p->min_triplets = 2;
    p->flags = TRIG_EXEC_PLAIN;
    return TRIG_OK;
}

int trig_params_check(const trig_params* p) {
    const int r = validate_params(p, false);
    if (r == TRIG_OK) g_detail.clear();
    return r;
}

size_t trig_workspace_bytes(const trig_events_csr* ev, const trig_params* p) {
    if (!ev || !p || ev->n_events < 0) return 0;
    return layout(ev->n_events, layout_flags(p)).total;
}

int trig_select(const trig_events_csr* ev, const trig_hits* hits, const trig_params* p_in,
                int32_t* out_counts, uint8_t* out_accept, void* stream) {
    if (int r = validate(ev, hits, p_in)) return r;
    // An autotuned call runs with the effective parameters of its batch's
    // multiplicity class; its workspace was sized by layout_flags().
    trig_params p_eff;
    const trig_params* p = p_in;
    if (p_in->flags & TRIG_EXEC_AUTOTUNE) {
        p_eff = resolve_autotune(p_in, ev->n_events, hits->n_hits);
        p_eff.workspace = p_in->workspace;
        p_eff.workspace_bytes = p_in->workspace_bytes;
        p = &p_eff;
    }
    const int n = ev->n_events;
    if (n > 0 && (!out_counts || !out_accept)) return fail(TRIG_EINVAL, "out_counts or out_accept is NULL");
    const Layout L = layout(n, layout_flags(p_in));
    if (L.total && (!p->workspace || p->workspace_bytes < L.total))
        return fail(TRIG_EWORKSPACE, "workspace smaller than trig_workspace_bytes()");
    if (L.total && (reinterpret_cast<uintptr_t>(p->workspace) & 255))
        return fail(TRIG_EWORKSPACE, "workspace must be 256-byte aligned");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char* ws = static_cast<char*>(p->workspace);
    const Consts c = make_consts(p, hits->n_hits);

    if (n > 0 && hits->z) {
        // per-hit z (validated: not with the basis form)
        const int r = p->test == TRIG_TEST_MSD
                          ? run_form_z<MsdZTest, MsdZPrune>(ev, hits, p, c, L, ws, out_counts, out_accept, s)
                          : run_form_z<WindowZTest, WindowZPrune>(ev, hits, p, c, L, ws, out_counts, out_accept, s);
        if (r) return r;
    } else if (n > 0) {
        int r = TRIG_OK;
        switch (p->test) {
            case TRIG_TEST_MSD:
                r = run_form<MsdFitTest, MsdFitPrune, MsdFitBin>(ev, hits, p, c, L, ws, out_counts, out_accept, s);
                break;
            case TRIG_TEST_MSD_BASIS:
                r = run_form<MsdBasisTest, MsdBasisPrune, MsdBasisBin>(ev, hits, p, c, L, ws, out_counts, out_accept,
                                                                       s);
                break;
            default:
                r = run_form<WindowTest, WindowPrune, WindowBin>(ev, hits, p, c, L, ws, out_counts, out_accept, s);
                break;
        }
        if (r) return r;
    }
    if (p->flags & TRIG_OUT_COMPACT) {
        if (n == 0) {
            hipLaunchKernelGGL(k_store_zero, dim3(1), dim3(1), 0, s, p->out_n_accepted);
            return check_launch("k_store_zero");
        }
        auto* part = reinterpret_cast<int32_t*>(ws + L.compact_off);
        hipLaunchKernelGGL(k_compact_count, dim3(L.compact_blocks), dim3(kScanBlock), 0, s, out_accept, n, part);
        if (int r = check_launch("k_compact_count")) return r;
        if (L.compact_blocks <= kPrefixBlocks) {
            // up to 4M events: no scan launch, each block sums the counts before it
            hipLaunchKernelGGL(k_compact_write_prefix, dim3(L.compact_blocks), dim3(kScanBlock), 0, s, out_accept,
                               n, part, L.compact_blocks, p->out_accepted_ids, p->out_n_accepted);
            if (int r = check_launch("k_compact_write_prefix")) return r;
        } else {
            hipLaunchKernelGGL(k_scan_partials<int32_t>, dim3(1), dim3(kScanBlock), 0, s, part, L.compact_blocks);
            if (int r = check_launch("k_scan_partials")) return r;
            hipLaunchKernelGGL(k_compact_write, dim3(L.compact_blocks), dim3(kScanBlock), 0, s, out_accept, n,
                               part, L.compact_blocks, p->out_accepted_ids, p->out_n_accepted);
            if (int r = check_launch("k_compact_write")) return r;
        }
    }
    g_detail.clear();
    return TRIG_OK;
}

void trig_autotune_reset(void) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tuned.clear();
}

int trig_autotune_save(const char* path) {
    if (!path) return fail(TRIG_EINVAL, "NULL path");
    std::vector<std::string> lines;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        for (const auto& kv : g_tuned) {
            std::string key;
            if (!device_key(std::get<0>(kv.first), key)) return fail(TRIG_EHIP, "hipGetDeviceProperties failed");
            const TunedShape& t = kv.second;
            char buf[256];
            std::snprintf(buf, sizeof buf, "%s %d %d %s %d %d %.17g %d", key.c_str(), std::get<1>(kv.first),
                          std::get<2>(kv.first), t.binned ? "binned" : "batched", t.binned ? 0 : t.hb,
                          t.binned ? 0 : t.nw, t.binned ? 0.0 : t.fill, t.persistent ? 1 : 0);
            lines.push_back(buf);
        }
    }
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(TRIG_EINVAL, std::string("cannot write ") + path);
    bool ok = std::fprintf(f, "%s\n", kCacheHeader) > 0;
    for (const auto& l : lines) ok = ok && std::fprintf(f, "%s\n", l.c_str()) > 0;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return fail(TRIG_EINVAL, std::string("cannot write ") + path);
    g_detail.clear();
    return TRIG_OK;
}

int trig_autotune_load(const char* path, int32_t* n_recorded) {
    if (!path) return fail(TRIG_EINVAL, "NULL path");
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(TRIG_EINVAL, std::string("cannot open ") + path);
    struct Line {
        std::string key;
        int test, cls;
        TunedShape t;
    };
    std::vector<Line> recs;
    char buf[512];
    int line_no = 0;
    bool header = false;
    std::string bad;
    while (std::fgets(buf, sizeof buf, f)) {
        ++line_no;
        std::string line(buf);
        while (!line.empty() && (line.back() == '\n' || line.back() == '\r')) line.pop_back();
        if (!header) {
            if (line != kCacheHeader) { bad = "not an autotune cache (header)"; break; }
            header = true;
            continue;
        }
        if (line.empty()) continue;
        char key[256], form[16];
        int test = -1, cls = -1, hb = -1, nw = -1, pers = -1;
        double fill = -1.0;
        char tail = 0;
        const int n = std::sscanf(line.c_str(), "%255s %d %d %15s %d %d %lf %d %c", key, &test, &cls, form, &hb, &nw,
                                  &fill, &pers, &tail);
        const bool binned = std::strcmp(form, "binned") == 0;
        const bool ok = n == 8 && test >= 0 && test <= 2 && cls >= 0 && cls <= 31 && (pers == 0 || pers == 1) &&
                        (binned ? (hb == 0 && nw == 0 && fill == 0.0)
                                : (std::strcmp(form, "batched") == 0 && (hb == 1024 || hb == 2048 || hb == 4096) &&
                                   (nw == 1 || nw == 2 || nw == 4) && fill > 0.0 && fill <= 1.0));
        if (!ok) { bad = "malformed line " + std::to_string(line_no); break; }
        recs.push_back({key, test, cls, TunedShape{hb, nw, fill, pers == 1, binned}});
    }
    const bool read_error = std::ferror(f) != 0;
    std::fclose(f);
    if (read_error) return fail(TRIG_EINVAL, std::string("cannot read ") + path);
    if (bad.empty() && !header) bad = "empty file";
    if (!bad.empty()) return fail(TRIG_EINVAL, std::string(path) + ": " + bad);
    int n_dev = 0;
    if (hipGetDeviceCount(&n_dev) != hipSuccess) n_dev = 0;
    std::vector<std::string> keys;
    for (int d = 0; d < n_dev; ++d) {
        std::string k;
        keys.push_back(device_key(d, k) ? k : std::string());
    }
    int32_t n = 0;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        for (const Line& r : recs)
            for (int d = 0; d < n_dev; ++d)
                if (!keys[d].empty() && keys[d] == r.key) {
                    g_tuned[{d, r.test, r.cls}] = r.t;
                    ++n;
                }
    }
    if (n_recorded) *n_recorded = n;
    g_detail.clear();
    return TRIG_OK;
}

int trig_autotune_lookup(int32_t test, int32_t mult_class, int32_t* found, trig_autotune_result* out) {
    if (!found || !out) return fail(TRIG_EINVAL, "NULL pointer");
    if (test < 0 || test > 2 || mult_class < 0 || mult_class > 31) return fail(TRIG_EINVAL, "test or class out of range");
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tuned.find({current_device(), test, mult_class});
    *found = it != g_tuned.end();
    *out = trig_autotune_result{};
    out->mult_class = mult_class;
    if (*found) {
        const TunedShape& t = it->second;
        out->block_hits = t.binned ? 0 : t.hb;
        out->block_waves = t.binned ? 0 : t.nw;
        out->persistent = t.persistent ? 1 : 0;
        out->binned = t.binned ? 1 : 0;
    }
    g_detail.clear();
    return TRIG_OK;
}

int trig_autotune(const trig_events_csr* ev, const trig_hits* hits, const trig_params* p,
                  int32_t* out_counts, uint8_t* out_accept, int32_t reps, trig_autotune_result* out,
                  void* stream) {
    if (!p) return fail(TRIG_EINVAL, "NULL params");
    if (!(p->flags & TRIG_EXEC_AUTOTUNE)) return fail(TRIG_EINVAL, "TRIG_EXEC_AUTOTUNE is not set");
    if (reps < 1 || reps > 100) return fail(TRIG_EINVAL, "reps must be in 1..100");
    if (int r = validate(ev, hits, p)) return r;
    trig_autotune_result res{};
    const int n = ev->n_events, n_hits = hits->n_hits;
    res.mult_class = multiplicity_class(n, n_hits);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);

    if (n > 0) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            if (e0) (void)hipEventDestroy(e0);
            return fail(TRIG_EHIP, "hipEventCreate failed");
        }
        // Times one candidate: the whole selection without compaction.
        auto time_shape = [&](const TunedShape& t, float& ms) -> int {
            trig_params q = *p;
            q.flags = (t.binned ? TRIG_EXEC_BINNED : TRIG_EXEC_PRUNED) | (t.persistent ? TRIG_EXEC_PERSISTENT : 0u);
            q.block_hits = t.hb;
            q.block_waves = t.nw;
            q.block_events = t.binned ? 0 : events_for_fill(t.fill, t.hb, t.nw, n, n_hits);
            q.out_accepted_ids = nullptr;
            q.out_n_accepted = nullptr;
            double total = 0.0;
            for (int it = 0; it <= reps; ++it) {
                if (hipEventRecord(e0, s) != hipSuccess) return fail(TRIG_EHIP, "hipEventRecord failed");
                if (int r = trig_select(ev, hits, &q, out_counts, out_accept, stream)) return r;
                if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
                    return fail(TRIG_EHIP, "event synchronisation failed");
                float one = 0.0f;
                if (hipEventElapsedTime(&one, e0, e1) != hipSuccess) return fail(TRIG_EHIP, "hipEventElapsedTime failed");
                if (it > 0) total += one;  // the first run warms up
            }
            ms = (float)(total / reps);
            return TRIG_OK;
        };
        // The built-in rule's shape first.
        trig_params rp = *p;
        rp.block_hits = rp.block_waves = rp.block_events = 0;
        const BlockShape r0 = choose_block_shape(&rp, n, n_hits);
        TunedShape best{r0.hb, r0.nw, kRuleFill, false, false};
        int rc = time_shape(best, res.ms_rule);
        res.ms_best = res.ms_rule;
        if (rc == TRIG_OK) res.n_candidates = 1;
        const int hbs[3] = {1024, 2048, 4096}, nws[2] = {2, 4};
        const double fills[4] = {0.5, 0.7, 0.85, 1.0};
        for (int a = 0; a < 3 && rc == TRIG_OK; ++a)
            for (int b = 0; b < 2 && rc == TRIG_OK; ++b)
                for (int f = 0; f < 4 && rc == TRIG_OK; ++f)
                    for (int ps = 0; ps < 2 && rc == TRIG_OK; ++ps) {
                        const TunedShape t{hbs[a], nws[b], fills[f], ps == 1, false};
                        float ms = 0.0f;
                        rc = time_shape(t, ms);
                        if (rc == TRIG_OK) {
                            ++res.n_candidates;
                            if (ms < res.ms_best) {
                                res.ms_best = ms;
                                best = t;
                            }
                        }
                    }
        for (int ps = 0; ps < 2 && rc == TRIG_OK; ++ps) {
            const TunedShape t{0, 0, 0.0, ps == 1, true};
            float ms = 0.0f;
            rc = time_shape(t, ms);
            if (rc == TRIG_OK) {
                ++res.n_candidates;
                if (ms < res.ms_best) {
                    res.ms_best = ms;
                    best = t;
                }
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc) return rc;
        {
            std::lock_guard<std::mutex> lock(g_tune_mu);
            g_tuned[{current_device(), p->test, res.mult_class}] = best;
        }
    }
    // The caller's outputs: one autotuned call with the new record.
    trig_params q = *p;
    q.block_hits = q.block_waves = q.block_events = 0;
    if (int r = trig_select(ev, hits, &q, out_counts, out_accept, stream)) return r;
    if (n > 0) {
        const trig_params eff = resolve_autotune(&q, n, n_hits);
        res.persistent = (eff.flags & TRIG_EXEC_PERSISTENT) ? 1 : 0;
        res.binned = (eff.flags & TRIG_EXEC_BINNED) ? 1 : 0;
        if (!res.binned) {
            const BlockShape bs = choose_block_shape(&eff, n, n_hits);
            res.block_hits = bs.hb;
            res.block_waves = bs.nw;
            res.block_events = bs.eb;
        }
    }
    if (hipStreamSynchronize(s) != hipSuccess) return fail(TRIG_EHIP, "hipStreamSynchronize failed");
    if (out) *out = res;
    g_detail.clear();
    return TRIG_OK;
}

int trig_select_noalloc(const trig_events_csr* ev, const trig_hits* hits, const trig_params* p,
                        int32_t* out_counts, uint8_t* out_accept, void* stream) {
    if (!ev || !hits || !p) return fail(TRIG_EINVAL, "NULL descriptor");
    if (p->workspace || p->workspace_bytes)
        return fail(TRIG_EINVAL, "trig_select_noalloc uses the library's scratch: workspace must be NULL, "
                                 "workspace_bytes 0");
    const size_t need = trig_workspace_bytes(ev, p);
    if (need > (size_t)TRIG_NOALLOC_SCRATCH_BYTES)
        return fail(TRIG_EWORKSPACE, "this batch and these flags need " + std::to_string(need) +
                                         " bytes of scratch, more than the " +
                                         std::to_string((size_t)TRIG_NOALLOC_SCRATCH_BYTES) +
                                         " of trig_select_noalloc");
    trig_params q = *p;
    if (need) {
        if (int r = scratch_address(&q.workspace)) return r;
        q.workspace_bytes = TRIG_NOALLOC_SCRATCH_BYTES;
    }
    return trig_select(ev, hits, &q, out_counts, out_accept, stream);
}

int trig_set_kernel_events(void* start, void* stop) {
    if ((start == nullptr) != (stop == nullptr)) return fail(TRIG_EINVAL, "give both events or neither");
    g_ev_start = reinterpret_cast<hipEvent_t>(start);
    g_ev_stop = reinterpret_cast<hipEvent_t>(stop);
    return TRIG_OK;
}

const char* trig_strerror(int code) {
    switch (code) {
        case TRIG_OK: return "success";
        case TRIG_EINVAL: return "invalid argument";
        case TRIG_EWORKSPACE: return "workspace missing, too small or misaligned";
        case TRIG_EHIP: return "HIP runtime or kernel launch failure";
        case TRIG_EUNSUPPORTED: return "unsupported test/flag combination";
        default: return "unknown error code";
    }
}

const char* trig_last_error_detail(void) { return g_detail.c_str(); }

}  // extern "C"
