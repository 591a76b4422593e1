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
// kernel sums each layer's hits and writes one record per lane window (32
// consecutive hits) that holds a trigger hit: the window's start and its
// three layer masks, to the wave's list in the workspace.  The scatter kernel
// finds every event's output positions with one lane per event, then each
// wave takes its list 64 records at a time: a wave scan of the records'
// layer counts gives each record's first output position per layer, and two
// records per round, one per half-wave and one lane per hit of the window,
// move x and y (a hit's rank within its record is the bits below it in the
// record's mask).  A wave whose events need more records than its list
// holds leaves the list incomplete, and the scatter then reads those
// events' station numbers again: a hit's rank in its layer is the exclusive
// prefix over lanes of the per-lane counts plus the count of the lane's
// earlier hits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "trig.h"
#include "trig_device.hpp"
#include "trig_filter.h"
#include "scan_i64.hpp"

namespace {

constexpr int kFilterThreads = 256;
constexpr int kFilterWaves = kFilterThreads / trig::kWave;
constexpr int kFilterEvents = 16;  // events per workgroup

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
// words of 4; 0xFF bytes where a hit is past the array, and for a lane whose
// window holds no hit of the event [a, b) (not read: a step's lanes past the
// event's end would otherwise fetch the next event's station numbers).  The
// caller masks hits outside the event, so a padding byte never counts.
struct LaneStations {
    uint32_t w[kLaneHits / 4];
    __device__ __forceinline__ void load(const uint8_t* __restrict__ st, int64_t h0, int64_t a, int64_t b,
                                         int64_t n_hits, bool vec) {
        if (h0 >= b || h0 + kLaneHits <= a) {
#pragma unroll
            for (int q = 0; q < kLaneHits / 4; ++q) w[q] = 0xFFFFFFFFu;
            return;
        }
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

// Bytes of w equal to the byte v (v4 = v * 0x01010101), as bit 7 of each
// byte.  A byte of x = w ^ v4 is zero where they are equal; adding 0x7F to
// each byte's low seven bits carries into its bit 7 exactly when they are
// not all zero (never into the next byte), so bit 7 of ~(that | x) marks the
// zero bytes.
__device__ __forceinline__ uint32_t byte_flags(uint32_t w, uint32_t v4) {
    const uint32_t x = w ^ v4;
    const uint32_t t = ((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x;
    return ~t & 0x80808080u;
}

// The same as bits 0..3 (bit k for byte k): one multiply gathers the four
// marks into bits 21..24.
__device__ __forceinline__ uint32_t eq_bytes(uint32_t w, uint32_t v4) {
    return (((byte_flags(w, v4) >> 7) * 0x00204081u) >> 21) & 0xFu;
}

// Transposed lane masks (the count kernel's records): bit 8 k + q stands for
// hit 4 q + k of a lane's 32-hit window (word q of its eight station words,
// byte k).  Shifting word q's byte flags right by 7 - q puts them at bits
// 8 k + q, so the eight words OR into one mask with a shift and an OR each.
__device__ __forceinline__ uint32_t tpos(int n) { return 8u * (uint32_t)(n & 3) + (uint32_t)(n >> 2); }

// Transposed mask of the hits [0, h) of a window, 0 <= h <= 32: in byte row
// k, the words q with 4 q + k < h, i.e. q < (h - k + 3) / 4.
__device__ __forceinline__ uint32_t tupto(int h) {
    uint32_t m = 0u;
#pragma unroll
    for (int k = 0; k < 4; ++k) m |= ((1u << (uint32_t)((h - k + 3) >> 2)) - 1u) << (8 * k);
    return m;
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

// Transposed layer masks of a lane's window (see tpos), restricted to the
// hits in_t marks.
__device__ __forceinline__ LaneMatch match_lane_t(const LaneStations& s, uint32_t in_t, uint32_t layers) {
    LaneMatch r{{0u, 0u, 0u}};
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const uint32_t v4 = ((layers >> (8 * l)) & 0xFFu) * 0x01010101u;
        uint32_t acc = 0u;
#pragma unroll
        for (int q = 0; q < kLaneHits / 4; ++q) acc |= byte_flags(s.w[q], v4) >> (7 - q);
        r.m[l] = acc & in_t;
    }
    return r;
}

// Records one wave keeps for the scatter: per lane window of kLaneHits
// consecutive hits that holds a trigger hit of its event, the window's start
// relative to the event's first hit and the transposed layer masks (bit
// tpos(b): hit start + b), in input order.
constexpr int kWaveRecords = 128;
typedef unsigned u32x4r __attribute__((ext_vector_type(4)));  // {start, m0, m1, m2}

__global__ __launch_bounds__(kFilterThreads) void k_filter_count(const int64_t* __restrict__ off, int n_events,
                                                                   int64_t n_hits, const uint8_t* __restrict__ st,
                                                                   uint32_t layers, int vec,
                                                                   int32_t* __restrict__ counts,
                                                                   int64_t* __restrict__ partials,
                                                                   u32x4r* __restrict__ wave_recs,
                                                                   int32_t* __restrict__ ev_recs,
                                                                   uint32_t* status) {
    constexpr int kPer = kFilterEvents / kFilterWaves;  // events of a wave
    __shared__ int64_t wave_total[kFilterWaves];
    __shared__ uint32_t tup[kLaneHits + 1];  // tupto(h)
    if (threadIdx.x <= (unsigned)kLaneHits) tup[threadIdx.x] = tupto((int)threadIdx.x);
    __syncthreads();
    const int w = trig::uniform_i((int)(threadIdx.x / trig::kWave));
    const int lane = (int)trig::lane_id();
    const int e_first = (int)blockIdx.x * kFilterEvents;
    u32x4r* wrec = wave_recs + ((int64_t)blockIdx.x * kFilterWaves + w) * kWaveRecords;
    // The wave's events (w, w + 4, ...): ranges; empty and malformed ones are
    // written here, the others while their hits stream by.
    int64_t ra[kPer], rb[kPer];
    bool live[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int e = e_first + w + kFilterWaves * k;
        live[k] = false;
        ra[k] = rb[k] = 0;
        if (e < n_events) {
            const Range r = event_range(off, e, n_hits);
            ra[k] = r.a;
            rb[k] = r.b;
            live[k] = r.ok && r.a < r.b;
            if (!live[k] && lane == 0) {
                counts[3 * (int64_t)e] = 0;
                counts[3 * (int64_t)e + 1] = 0;
                counts[3 * (int64_t)e + 2] = 0;
                ev_recs[e] = 0;
                if (!r.ok && status) atomicOr(status, TRIG_FILTER_MALFORMED);
            }
        }
    }
    // The first step of the wave's next live event after event k (kPer if none).
    auto next_live = [&](int k) {
        int n = kPer;
#pragma unroll
        for (int q = kPer - 1; q >= 0; --q)
            if (q > k && live[q]) n = q;
        return n;
    };
    int32_t used = 0;   // records of wrec written
    bool keep = true;   // wrec holds every record of this wave's events so far (wave-uniform)
    int64_t total = 0;
    // One flat stream over the live events' steps: the next step's station
    // numbers (of this event or the next) are in flight while this step's
    // are matched.
    // k and the step starts are wave-uniform; readfirstlane keeps them in
    // scalar registers (the compiler cannot see it through the loop).
    auto uniform64 = [](int64_t v) {
        const uint32_t lo = (uint32_t)trig::uniform_i((int)(uint32_t)v);
        const uint32_t hi = (uint32_t)trig::uniform_i((int)(uint32_t)((uint64_t)v >> 32));
        return (int64_t)(((uint64_t)hi << 32) | lo);
    };
    int k = trig::uniform_i(next_live(-1));
    if (k < kPer) {
        int64_t base = ra[k] & ~(int64_t)15;
        LaneStations cur, nxt;
        cur.load(st, base + (int64_t)kLaneHits * lane, ra[k], rb[k], n_hits, vec != 0);
        uint32_t c[3] = {0u, 0u, 0u};
        int32_t recs = 0;  // this event's records
        for (;;) {
            // wave-uniform choice of the next step
            int k1 = k;
            int64_t base1 = base + kStepHits;
            if (base1 >= rb[k]) {
                k1 = next_live(k);
                base1 = k1 < kPer ? ra[k1] & ~(int64_t)15 : 0;
            }
            k1 = trig::uniform_i(k1);
            base1 = uniform64(base1);
            if (k1 < kPer) nxt.load(st, base1 + (int64_t)kLaneHits * lane, ra[k1], rb[k1], n_hits, vec != 0);
            const int64_t h0 = base + (int64_t)kLaneHits * lane;
            // the lane's hits of event k: all of them unless the step
            // straddles an end of the event
            uint32_t in_t = 0xFFFFFFFFu;
            if (base < ra[k] || base + kStepHits > rb[k]) {  // wave-uniform
                const int64_t lo = ra[k] - h0, hi = rb[k] - h0;
                const int l0 = lo <= 0 ? 0 : (lo >= kLaneHits ? kLaneHits : (int)lo);
                const int h1 = hi <= 0 ? 0 : (hi >= kLaneHits ? kLaneHits : (int)hi);
                in_t = h1 > l0 ? tup[h1] & ~tup[l0] : 0u;
            }
            const LaneMatch m = match_lane_t(cur, in_t, layers);
#pragma unroll
            for (int l = 0; l < 3; ++l) c[l] += (uint32_t)__builtin_popcount(m.m[l]);
            cur = nxt;
            // one record per lane window with a trigger hit, in lane order
            const bool active = (m.m[0] | m.m[1] | m.m[2]) != 0u;
            const uint64_t am = trig::lanes(active);
            const int32_t nrec = (int32_t)__builtin_popcountll(am);
            recs += nrec;
            if (keep && used + nrec > kWaveRecords) keep = false;
            if (keep && active) {
                const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(am >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)am, 0u));
                // h0 - ra[k] lies in [-15, rb[k] - ra[k]): an int32
                wrec[used + rank] = u32x4r{(uint32_t)(int32_t)(h0 - ra[k]), m.m[0], m.m[1], m.m[2]};
            }
            if (keep) used += nrec;
            if (k1 != k) {
                // event k is complete
                const int e = e_first + w + kFilterWaves * k;
                const uint32_t s0 = trig::wave_sum_u(c[0]), s1 = trig::wave_sum_u(c[1]), s2 = trig::wave_sum_u(c[2]);
                if (lane == 0) {
                    counts[3 * (int64_t)e] = (int32_t)s0;
                    counts[3 * (int64_t)e + 1] = (int32_t)s1;
                    counts[3 * (int64_t)e + 2] = (int32_t)s2;
                    ev_recs[e] = recs;
                }
                total += (int64_t)s0 + s1 + s2;
                c[0] = c[1] = c[2] = 0u;
                recs = 0;
                if (k1 >= kPer) break;
            }
            k = k1;
            base = base1;
        }
    }
    if (lane == 0) wave_total[w] = total;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int k = 0; k < kFilterWaves; ++k) t += wave_total[k];
        partials[blockIdx.x] = t;
    }
}

// Per-event data of the scatter's workgroup, in LDS.
struct ScatterEvent {
    int64_t s[3];   // first output position of the event's layer-l hits
    int64_t d[3];   // s[l] minus the layer-l hits of the wave's earlier events
    int64_t a;      // first hit of the event
    int32_t rec0;   // first record of the event in its wave's list
    int32_t nrec;   // records of the event (0 for a malformed one)
    int32_t ok;     // the event range is well-formed
    int32_t pad;
};

// Record data of one chunk of 64 records of a wave, in LDS.
struct ScatterRec {
    int64_t h0;        // hit of bit 0
    int64_t base[3];   // output position of the record's first layer-l hit
    uint32_t m[3];     // layer masks
    uint32_t pad;
};

__global__ __launch_bounds__(kFilterThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_filter_scatter(
    const int64_t* __restrict__ off, int n_events, int64_t n_hits, const uint8_t* __restrict__ st,
    const float* __restrict__ x, const float* __restrict__ y, uint32_t layers, int vec,
    const int32_t* __restrict__ counts, const int64_t* __restrict__ partials,
    const u32x4r* __restrict__ wave_recs, const int32_t* __restrict__ ev_recs, int n_blocks, int32_t capacity,
    int32_t* __restrict__ out_off, float* __restrict__ out_x, float* __restrict__ out_y, uint32_t* status) {
    static_assert(kFilterEvents <= trig::kWave, "one lane per event in the prologue");
    constexpr int kPer = kFilterEvents / kFilterWaves;  // events of a wave
    // Per wave, its own copies: no wave waits for another.
    __shared__ ScatterEvent ev_all[kFilterWaves][kPer];  // the wave's events w, w + 4, ...
    __shared__ int64_t cnt_all[kFilterWaves][kFilterEvents][3];
    __shared__ int32_t nrec_all[kFilterWaves][kFilterEvents];
    // Per wave: the record data of a chunk (listed path) or the step's
    // matched hits (the other path).
    __shared__ union {
        ScatterRec recs[trig::kWave];
        uint16_t lists[kStepHits];
    } work[kFilterWaves];
    const int w = trig::uniform_i((int)(threadIdx.x / trig::kWave));
    const int lane = (int)trig::lane_id();
    const int e_first = (int)blockIdx.x * kFilterEvents;
    const int64_t cap = capacity;
    ScatterEvent* ev = ev_all[w];
    // The first 64 entries of the wave's list, loaded with the prologue's
    // loads (one round trip for both; entries past the wave's records are
    // not used, and the list holds kWaveRecords >= 64 entries).
    static_assert(kWaveRecords >= trig::kWave, "first chunk inside the list");
    const u32x4r* wrec = wave_recs + ((int64_t)blockIdx.x * kFilterWaves + w) * kWaveRecords;
    const u32x4r first = wrec[lane];
    if ((int)blockIdx.x == n_blocks - 1 && threadIdx.x == 0) {
        const int64_t total = partials[n_blocks];
        if (total > cap && status) atomicOr(status, TRIG_FILTER_CAPACITY);
        out_off[3 * (int64_t)n_events] = (int32_t)std::min<int64_t>(total, cap);
    }
    // Prologue, every wave for itself, one lane per event j of the
    // workgroup: its counts and record count; then, for the wave's own
    // events (j % 4 == w), the output positions, the first record in the
    // wave's list and the offsets out_off[3 e + l].
    int32_t n_rec = 0;  // records of the wave's events
    {
        const int64_t wg_base = partials[blockIdx.x];
        int64_t(*cnt)[3] = cnt_all[w];
        int32_t* nrec = nrec_all[w];
        const int j = lane;
        const int e = e_first + j;
        const bool in = j < kFilterEvents && e < n_events;
        int64_t c[3] = {0, 0, 0};
        int32_t nr = 0;
        Range r{0, 0, false};
        const bool mine = j < kFilterEvents && j % kFilterWaves == w;
        if (in) {
            // every load first (one round trip), then their uses
            const int64_t oa = off[e], ob = off[e + 1];
            const int32_t c0 = counts[3 * (int64_t)e], c1 = counts[3 * (int64_t)e + 1];
            const int32_t c2 = counts[3 * (int64_t)e + 2];
            nr = ev_recs[e];
            c[0] = c0;
            c[1] = c1;
            c[2] = c2;
            r.a = oa;
            r.b = ob;
            r.ok = 0 <= oa && oa <= ob && ob <= n_hits && ob - oa <= (int64_t)INT32_MAX;
        }
        if (j < kFilterEvents) {
            cnt[j][0] = c[0];
            cnt[j][1] = c[1];
            cnt[j][2] = c[2];
            nrec[j] = nr;
        }
        trig::wave_lds_sync();
        if (mine) {
            int64_t before = wg_base, wave_before[3] = {0, 0, 0};
            int32_t rec_before = 0;
            for (int k = 0; k < j; ++k) before += cnt[k][0] + cnt[k][1] + cnt[k][2];
            for (int k = w; k < j; k += kFilterWaves) {
                rec_before += nrec[k];
                wave_before[0] += cnt[k][0];
                wave_before[1] += cnt[k][1];
                wave_before[2] += cnt[k][2];
            }
            ScatterEvent v;
            v.s[0] = before;
            v.s[1] = before + c[0];
            v.s[2] = before + c[0] + c[1];
#pragma unroll
            for (int l = 0; l < 3; ++l) v.d[l] = v.s[l] - wave_before[l];
            v.a = r.a;
            v.rec0 = rec_before;
            v.nrec = nr;
            v.ok = r.ok ? 1 : 0;
            v.pad = 0;
            ev[j / kFilterWaves] = v;
            if (in) {
#pragma unroll
                for (int l = 0; l < 3; ++l) out_off[3 * (int64_t)e + l] = (int32_t)std::min<int64_t>(v.s[l], cap);
            }
        }
        for (int k = w; k < kFilterEvents; k += kFilterWaves) n_rec += nrec[k];  // wave-uniform LDS reads
        n_rec = trig::uniform_i(n_rec);
        trig::wave_lds_sync();  // ev[] written
    }
    if (n_rec <= kWaveRecords) {
        // The wave's list is complete (the count kernel's condition): its
        // records, 64 at a time.  Lane i takes record i: its event (the
        // wave's event whose record range holds i), layer counts and, by a
        // wave scan, its first output position per layer; then two records
        // per round, one per half-wave, lane b of a half on hit h0 + b.
        ScatterRec* rl = work[w].recs;
        int32_t carry[3] = {0, 0, 0};  // layer-l hits of the wave's earlier chunks
        for (int32_t cb = 0; cb < n_rec; cb += trig::kWave) {
            const int32_t i = cb + lane;
            const bool valid = i < n_rec;
            const u32x4r R = !valid ? u32x4r{0u, 0u, 0u, 0u} : (cb == 0 ? first : wrec[i]);
            int j = 0;  // the wave's event (index among its kPer) that holds record i
            for (int k = 1; k < kPer; ++k)
                if (ev[k].nrec > 0 && ev[k].rec0 <= i) j = k;
            const uint32_t m[3] = {R.y, R.z, R.w};
            ScatterRec v;
            v.h0 = ev[j].a + (int64_t)(int32_t)R.x;
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                const int p = __builtin_popcount(m[l]);
                const int incl = trig::wave_inclusive_sum(p);
                v.base[l] = ev[j].d[l] + carry[l] + (incl - p);
                v.m[l] = m[l];
                carry[l] += __builtin_amdgcn_readlane(incl, 63);
            }
            v.pad = 0;
            rl[lane] = v;
            trig::wave_lds_sync();
            const int32_t nc = min(trig::kWave, n_rec - cb);
            const int half = lane >> 5, b = lane & 31;
            const uint32_t bit = 1u << tpos(b), below = tupto(b);  // hit b, hits before b
            // kRoundBatch rounds at a time: every lane's loads of the batch go
            // out together (a lane without a hit to move reads hit 0), then
            // the stores, so that a batch costs one round trip
            constexpr int kRoundBatch = 8;
            for (int32_t q0 = 0; q0 < nc; q0 += 2 * kRoundBatch) {
                float vx[kRoundBatch], vy[kRoundBatch];
                int64_t pos[kRoundBatch];
                bool put[kRoundBatch];
#pragma unroll
                for (int r = 0; r < kRoundBatch; ++r) {
                    const int32_t k = q0 + 2 * r + half;
                    int64_t p = 0, h = 0;
                    bool ok = false;
                    if (k < nc) {
                        const ScatterRec& u = rl[k];
                        const uint32_t m0 = u.m[0], m1 = u.m[1], m2 = u.m[2];
                        if ((m0 | m1 | m2) & bit) {
                            const int l = (m0 & bit) ? 0 : ((m1 & bit) ? 1 : 2);
                            const uint32_t ml = l == 0 ? m0 : (l == 1 ? m1 : m2);
                            p = u.base[l] + __builtin_popcount(ml & below);
                            h = u.h0 + b;
                            ok = p >= 0 && p < cap;  // positions past an int32 block prefix are never written
                        }
                    }
                    const int64_t hh = ok ? h : 0;  // a record exists, so n_hits > 0
                    vx[r] = x[hh];
                    vy[r] = y[hh];
                    pos[r] = p;
                    put[r] = ok;
                }
#pragma unroll
                for (int r = 0; r < kRoundBatch; ++r)
                    if (put[r]) {
                        out_x[pos[r]] = vx[r];
                        out_y[pos[r]] = vy[r];
                    }
            }
            trig::wave_lds_sync();  // the next chunk rewrites rl
        }
        return;
    }
    // The list is incomplete: read the wave's events' station numbers again.
    uint16_t* list = work[w].lists;
    for (int j = w; j < kFilterEvents; j += kFilterWaves) {
        const int e = e_first + j;
        if (e >= n_events) break;
        const ScatterEvent& v = ev[j / kFilterWaves];
        if (!v.ok) continue;
        int64_t s[3] = {v.s[0], v.s[1], v.s[2]};
        const Range r = event_range(off, e, n_hits);
        int64_t base = r.a & ~(int64_t)15;
        LaneStations cur, nxt;
        cur.load(st, base + (int64_t)kLaneHits * lane, r.a, r.b, n_hits, vec != 0);
        for (; base < r.b; base += kStepHits) {
            const int64_t h0 = base + (int64_t)kLaneHits * lane;
            if (base + kStepHits < r.b) nxt.load(st, h0 + kStepHits, r.a, r.b, n_hits, vec != 0);  // wave-uniform
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
           align256(sizeof(int32_t) * (size_t)n_events) + align256(16 * (size_t)nb * kFilterWaves * kWaveRecords);
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
    const size_t partial_bytes = align256(sizeof(int64_t) * (size_t)(nb + 1));
    auto* ev_recs = reinterpret_cast<int32_t*>(ws + counts_bytes + partial_bytes);
    auto* wave_recs = reinterpret_cast<u32x4r*>(ws + counts_bytes + partial_bytes +
                                                align256(sizeof(int32_t) * (size_t)n));
    const uint32_t layers = (uint32_t)p->layers[0] | ((uint32_t)p->layers[1] << 8) | ((uint32_t)p->layers[2] << 16);
    const int vec = (reinterpret_cast<uintptr_t>(ev->station) & 15) == 0;
    hipLaunchKernelGGL(k_filter_count, dim3(nb), dim3(kFilterThreads), 0, s, ev->offsets, n, ev->n_hits,
                       ev->station, layers, vec, counts, partials, wave_recs, ev_recs, p->out_status);
    if (hipGetLastError() != hipSuccess) return TRIG_EHIP;
    hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(kScanThreads), 0, s, partials, (int64_t)nb);
    if (hipGetLastError() != hipSuccess) return TRIG_EHIP;
    hipLaunchKernelGGL(k_filter_scatter, dim3(nb), dim3(kFilterThreads), 0, s, ev->offsets, n, ev->n_hits,
                       ev->station, ev->x, ev->y, layers, vec, counts, partials, wave_recs, ev_recs, nb, p->out_capacity,
                       p->out_layer_offsets, p->out_x, p->out_y, p->out_status);
    return hipGetLastError() == hipSuccess ? TRIG_OK : TRIG_EHIP;
}

}  // extern "C"
