// Block-staged selection with exact pair pruning (the batched form).
//
// A workgroup takes a block of consecutive events, copies their hits (one
// contiguous CSR range) from HBM into LDS with coalesced loads, and counts
// every event's passing triplets from LDS.  The count is the same as the
// brute-force triplet loop (paper Sec. 3.2 steps 1-3), but triplets are only
// completed for pairs (i, j) that can still pass:
//
//   MSD test:  Q = f32(A + f32(b*b)) >= A = f32(a*a) in binary32 (rounding is
//              monotone and b*b >= 0), so a triplet can pass only if
//              f32(a*a) <= Qmax in both planes, i.e. |a| <= beta with beta the
//              largest binary32 value whose rounded square is <= Qmax
//              (f32(a*a) is non-decreasing in |a|).  a = f32(U0*c_i + U1*c_j)
//              depends on (i, j) only.
//   window:    the layer-1 window |s_j - s_i| < W is itself part of the test.
//
// Both conditions are exact consequences of the binary32 test, so pruning
// never changes a count.  Surviving pairs (rare: a is the distance of hit j
// from the line through the vertex and hit i, in cm) are completed against
// every layer-2 hit with the full binary32 test, lanes over k.
//
// Lane layout of the pair scan: lane L holds layer-1 hit j and its constant
// part of a; for n1 <= 32 the 64 lanes hold R = floor(64/n1) copies of the
// layer-1 hits, copy g scanning layer-0 hits i = g, g+R, g+2R, ... so that
// few lanes idle.  The layer-0 part of a (or the layer-0 slope) is computed
// once per hit into a per-wave LDS buffer and read with a broadcast.
#pragma once

#include "trig_device.hpp"

namespace trig {

constexpr int kPBuf = 128;     // per-wave buffer of layer-0 values (float2)
constexpr int kMaxEB = 128;    // events per block at most

// Small exact quotients without integer division: for 0 <= a < 4096 and
// 1 <= n <= 256, a / n = floor(a * rcp(n) + 2^-10), rcp the hardware
// reciprocal.  The computed product is within (a/n) 2^-22 <= 2^-10 of a/n
// (relative error of rcp and of the product below 2^-22 together), so an
// exact quotient q is reached again after adding 2^-10; otherwise a/n lies
// at least 1/n >= 2^-8 below q + 1, and error plus 2^-10 stays below that
// (and far from q + 1 in binary32 spacing, 2^-11 at most here).
__device__ __forceinline__ int div_small(int a, int n) {
    return (int)((float)a * __builtin_amdgcn_rcpf((float)n) + 0.0009765625f);
}

// Hits of the current sub-block in LDS (structure of arrays), indexed
// relative to the staged range's 4-aligned start.
struct LdsHits {
    const float* xs;
    const float* ys;
    __device__ __forceinline__ float2 at(int h) const { return make_float2(xs[h], ys[h]); }
};
// Hits read straight from HBM (events too large for LDS, irregular blocks).
struct GlobalHits {
    const float* x;
    const float* y;
    __device__ __forceinline__ float2 at(int h) const { return make_float2(x[h], y[h]); }
};

__device__ __forceinline__ float2 nan2() {
    const float n = __builtin_nanf("");
    return make_float2(n, n);
}

struct MsdPrune {
    __device__ static __forceinline__ float2 layer0(const Consts& c, float2 h) {
        return make_float2(c.U0 * h.x, c.U0 * h.y);
    }
    __device__ static __forceinline__ float2 layer1(const Consts& c, float2 h) {
        return make_float2(c.U1 * h.x, c.U1 * h.y);
    }
    // Lanes whose pair can still pass: |f32(P + Q)| <= beta in both planes.
    __device__ static __forceinline__ uint64_t pair_mask(const Consts& c, float2 p, float2 q) {
        const float ax = p.x + q.x;
        const float ay = p.y + q.y;
        return lanes(__builtin_fabsf(ax) <= c.beta_x) & lanes(__builtin_fabsf(ay) <= c.beta_y);
    }
    // Prefilter score: pair_mask's lane set is within {score <= bound()}.
    __device__ static __forceinline__ float score(const Consts& c, float2 p, float2 q) {
        const float ax = p.x + q.x;
        const float ay = p.y + q.y;
        return __builtin_fmaxf(__builtin_fabsf(ax), __builtin_fabsf(ay) * c.pre_k_msd);
    }
    __device__ static __forceinline__ float bound(const Consts& c) { return c.beta_x; }
    // Passing triplets of the surviving pair (hi, hj) over layer-2 hits
    // [o2, o2 + n2): lanes over k, the binary32 test of include/trig.h.
    template <class H>
    __device__ static uint32_t complete(const Consts& c, const H& hits, int hi, int hj, int o2, int n2) {
        const float2 ci = hits.at(hi), cj = hits.at(hj);
        const float ax = c.U0 * ci.x + c.U1 * cj.x;
        const float ay = c.U0 * ci.y + c.U1 * cj.y;
        const float ax2 = ax * ax, ay2 = ay * ay;
        const float bx0 = c.V0 * ci.x + c.V1 * cj.x;
        const float by0 = c.V0 * ci.y + c.V1 * cj.y;
        uint32_t cnt = 0;
        for (int k0 = 0; k0 < n2; k0 += kWave) {
            const int k = k0 + (int)lane_id();
            float2 w = nan2();
            if (k < n2) {
                const float2 ck = hits.at(o2 + k);
                w = make_float2(c.V2 * ck.x, c.V2 * ck.y);
            }
            const float bx = bx0 + w.x;
            const float qx = ax2 + bx * bx;
            const float by = by0 + w.y;
            const float qy = ay2 + by * by;
            cnt += (uint32_t)__builtin_popcountll(lanes(qx <= c.qmax_x) & lanes(qy <= c.qmax_y));
        }
        return cnt;
    }
};

struct WindowPrune {
    __device__ static __forceinline__ float2 layer0(const Consts& c, float2 h) {
        return make_float2(h.x / c.z0, h.y / c.z0);
    }
    __device__ static __forceinline__ float2 layer1(const Consts& c, float2 h) {
        return make_float2(h.x / c.z1, h.y / c.z1);
    }
    __device__ static __forceinline__ uint64_t pair_mask(const Consts& c, float2 p, float2 q) {
        return lanes(__builtin_fabsf(q.x - p.x) < c.win_x) & lanes(__builtin_fabsf(q.y - p.y) < c.win_y);
    }
    __device__ static __forceinline__ float score(const Consts& c, float2 p, float2 q) {
        return __builtin_fmaxf(__builtin_fabsf(q.x - p.x), __builtin_fabsf(q.y - p.y) * c.pre_k_win);
    }
    __device__ static __forceinline__ float bound(const Consts& c) { return c.win_x; }
    template <class H>
    __device__ static uint32_t complete(const Consts& c, const H& hits, int hi, int /*hj*/, int o2, int n2) {
        const float2 ci = hits.at(hi);
        const float sxi = ci.x / c.z0, syi = ci.y / c.z0;
        uint32_t cnt = 0;
        for (int k0 = 0; k0 < n2; k0 += kWave) {
            const int k = k0 + (int)lane_id();
            float2 s = nan2();
            if (k < n2) {
                const float2 ck = hits.at(o2 + k);
                s = make_float2(ck.x / c.z2, ck.y / c.z2);
            }
            cnt += (uint32_t)__builtin_popcountll(lanes(__builtin_fabsf(s.x - sxi) < c.win_x) &
                                                  lanes(__builtin_fabsf(s.y - syi) < c.win_y));
        }
        return cnt;
    }
};

// Passing triplets of one event (all layers non-empty), by one wave.
// o0, o1, o2 index `hits`; px/py are this wave's kPBuf-entry LDS buffers
// (16-byte aligned) for the layer-0 partials.
//
// Layout: lane L holds layer-1 hit j and copy number g; with R copies of
// layer 1 (R = min(64 / n1, kPBuf / 4) for n1 <= 32, else 1) copy g scans the
// contiguous layer-0 slice [g T, g T + T) of the current buffer fill, T a
// multiple of 4, so one 16-byte LDS read per coordinate serves four pairs.
// Buffer entries past the event's layer-0 hits hold NaN and fail every test.
template <class P, class H>
__device__ uint32_t wave_event_pruned(const Consts& c, const H& hits, int o0, int n0, int o1, int n1,
                                      int o2, int n2, float* __restrict__ px, float* __restrict__ py) {
    const int lane = (int)lane_id();
    const int R = uniform_i(n1 <= kWave / 2 ? min(div_small(kWave, n1), kPBuf / 4) : 1);
    const int chunk = uniform_i(div_small(kPBuf, 4 * R) * 4 * R);  // a positive multiple of 4R
    uint32_t cnt = 0;
    for (int jc = 0; jc < n1; jc += kWave) {
        int g = 0, j = jc + lane;
        if (R > 1) {
            g = div_small(lane, n1);  // floor(lane / n1)
            j = lane - g * n1;
        }
        const bool jv = (g < R) && (j < n1);
        if (!jv) g = 0;
        const float2 q = jv ? P::layer1(c, hits.at(o1 + j)) : nan2();
        for (int ic = 0; ic < n0; ic += chunk) {
            const int ni = min(chunk, n0 - ic);
            const int T = uniform_i(div_small(ni + 4 * R - 1, 4 * R) * 4);  // per copy, multiple of 4
            const int npad = T * R;                                          // <= chunk <= kPBuf
            for (int t = lane; t < npad; t += kWave) {
                const float2 v = t < ni ? P::layer0(c, hits.at(o0 + ic + t)) : nan2();
                px[t] = v.x;
                py[t] = v.y;
            }
            wave_lds_sync();
            // Survivors among the lanes' pairs (ic + g T + t, j).
            auto finish = [&](uint64_t m, int t) {
                while (m) {
                    const int L = __builtin_ctzll(m);
                    m &= m - 1;
                    const int iL = __builtin_amdgcn_readlane(g, L) * T + t;
                    const int jL = __builtin_amdgcn_readlane(j, L);
                    cnt += P::complete(c, hits, o0 + ic + iL, o1 + jL, o2, n2);
                }
            };
            const float4* ppx = reinterpret_cast<const float4*>(px + g * T);
            const float4* ppy = reinterpret_cast<const float4*>(py + g * T);
            const float bnd = P::bound(c);
            for (int t = 0; t < T; t += 4) {
                const float4 vx = ppx[t >> 2], vy = ppy[t >> 2];
                // Prefilter on the vector unit: does the smallest of the four
                // pairs' scores reach the bound?  (fmin drops NaN scores; all
                // NaN gives NaN, which fails.)
                const float s0 = P::score(c, make_float2(vx.x, vy.x), q);
                const float s1 = P::score(c, make_float2(vx.y, vy.y), q);
                const float s2 = P::score(c, make_float2(vx.z, vy.z), q);
                const float s3 = P::score(c, make_float2(vx.w, vy.w), q);
                const float smin = __builtin_fminf(__builtin_fminf(s0, s1), __builtin_fminf(s2, s3));
                if (wave_any(smin <= bnd)) {
                    finish(P::pair_mask(c, make_float2(vx.x, vy.x), q), t);
                    finish(P::pair_mask(c, make_float2(vx.y, vy.y), q), t + 1);
                    finish(P::pair_mask(c, make_float2(vx.z, vy.z), q), t + 2);
                    finish(P::pair_mask(c, make_float2(vx.w, vy.w), q), t + 3);
                }
            }
            wave_lds_sync();
        }
    }
    return cnt;
}

// Passing triplets of an event with 1 <= n1 <= 64 and n0 <= the buffer fill
// for its lane layout (one layer-1 pass, one buffer fill): the same
// computation as wave_event_pruned with its loops taken once.  R and T come
// from the per-event descriptor (lane_layout).
template <class P, class H>
__device__ uint32_t wave_event_fast(const Consts& c, const H& hits, int o0, int n0, int o1, int n1, int o2,
                                    int n2, int R, int T, float* __restrict__ px, float* __restrict__ py) {
    const int lane = (int)lane_id();
    int g = 0, j = lane;
    if (R > 1) {
        g = div_small(lane, n1);
        j = lane - g * n1;
    }
    const bool jv = (g < R) && (j < n1);
    if (!jv) g = 0;
    const float2 q = jv ? P::layer1(c, hits.at(o1 + j)) : nan2();
    const int npad = T * R;
    for (int t = lane; t < npad; t += kWave) {
        const float2 v = t < n0 ? P::layer0(c, hits.at(o0 + t)) : nan2();
        px[t] = v.x;
        py[t] = v.y;
    }
    wave_lds_sync();
    uint32_t cnt = 0;
    auto finish = [&](uint64_t m, int t) {
        while (m) {
            const int L = __builtin_ctzll(m);
            m &= m - 1;
            const int iL = __builtin_amdgcn_readlane(g, L) * T + t;
            const int jL = __builtin_amdgcn_readlane(j, L);
            cnt += P::complete(c, hits, o0 + iL, o1 + jL, o2, n2);
        }
    };
    const float4* ppx = reinterpret_cast<const float4*>(px + g * T);
    const float4* ppy = reinterpret_cast<const float4*>(py + g * T);
    const float bnd = P::bound(c);
    for (int t = 0; t < T; t += 4) {
        const float4 vx = ppx[t >> 2], vy = ppy[t >> 2];
        const float s0 = P::score(c, make_float2(vx.x, vy.x), q);
        const float s1 = P::score(c, make_float2(vx.y, vy.y), q);
        const float s2 = P::score(c, make_float2(vx.z, vy.z), q);
        const float s3 = P::score(c, make_float2(vx.w, vy.w), q);
        const float smin = __builtin_fminf(__builtin_fminf(s0, s1), __builtin_fminf(s2, s3));
        if (wave_any(smin <= bnd)) {
            finish(P::pair_mask(c, make_float2(vx.x, vy.x), q), t);
            finish(P::pair_mask(c, make_float2(vx.y, vy.y), q), t + 1);
            finish(P::pair_mask(c, make_float2(vx.z, vy.z), q), t + 2);
            finish(P::pair_mask(c, make_float2(vx.w, vy.w), q), t + 3);
        }
    }
    wave_lds_sync();
    return cnt;
}

// Lane layout of wave_event_pruned for one buffer fill: R copies of layer 1
// and T (a multiple of 4) layer-0 entries per copy; T = 0 when the event
// needs more than one layer-1 pass or buffer fill.
__device__ __forceinline__ void lane_layout(int n0, int n1, int& R, int& T) {
    R = n1 <= kWave / 2 ? min(div_small(kWave, n1), kPBuf / 4) : 1;
    const int chunk = div_small(kPBuf, 4 * R) * 4 * R;
    T = (n1 <= kWave && n0 <= chunk) ? div_small(n0 + 4 * R - 1, 4 * R) * 4 : 0;
}

// Count of event e (absolute index) whose CSR range was checked by the
// caller; writes count and flag.  h_base: index of hits.at(0) in the global
// hit arrays (0 for GlobalHits).
template <class P, class H>
__device__ void wave_event(const Consts& c, const H& hits, int h_base, int o0, int o1, int o2, int o3,
                           int e, int32_t* counts, uint8_t* accept, uint32_t* status, float* px, float* py) {
    const int n0 = o1 - o0, n1 = o2 - o1, n2 = o3 - o2;
    int32_t cnt = 0;
    const int64_t n01 = (int64_t)n0 * n1;  // < 2^62; if <= INT32_MAX then n01 * n2 < 2^62
    if (n2 > 0 && (n01 > (int64_t)INT32_MAX || n01 * n2 > (int64_t)INT32_MAX)) {
        cnt = -2;
    } else if (n0 > 0 && n1 > 0 && n2 > 0) {
        cnt = (int32_t)wave_event_pruned<P>(c, hits, o0 - h_base, n0, o1 - h_base, n1, o2 - h_base, n2, px, py);
    }
    if (lane_id() == 0) {
        counts[e] = cnt;
        accept[e] = (uint8_t)(cnt >= 0 && cnt >= c.min_triplets);
        if (cnt < 0 && status) atomicOr(status, TRIG_STATUS_OVERFLOW);
    }
}

// The block kernel.  Non-persistent when block_counter == nullptr (block =
// blockIdx.x); otherwise workgroups take blocks from *block_counter until
// they run out (the counter must be zero at launch).
// Copies hits [base, base + nh) of x and y into xs/ys (LDS) at local index
// (h - a0), a0 = base rounded down to a multiple of 4, with 16-byte loads
// issued together (every thread's loads are in flight before any LDS write).
// The one float4 group that would cross n_hits is copied element by element
// by thread 0.  Needs x and y 16-byte aligned (checked by the host; `vec`
// false otherwise: plain 4-byte loads).
template <int HB, int NT>
__device__ __forceinline__ void stage_hits(const float* __restrict__ x, const float* __restrict__ y,
                                           int base, int nh, int n_hits, bool vec, float* xs, float* ys) {
    constexpr int Q = (HB + 6) / 4 / NT + 1;  // float4 groups per thread, upper bound
    const int a0 = base & ~3;
    const int nq = (base + nh - a0 + 3) >> 2;             // float4 groups to copy
    const int t = (int)threadIdx.x;
    if (vec) {
        const int nq_full = min(nq, (n_hits - a0) >> 2);   // groups entirely below n_hits
        if (nq_full > 0) {
            // Unconditional loads (a group past the end re-reads the last full
            // one), so that all of them are in flight in registers at once.
            float4 vx[Q], vy[Q];
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                const int q = min(t + k * NT, nq_full - 1);
                vx[k] = *reinterpret_cast<const float4*>(x + a0 + 4 * q);
                vy[k] = *reinterpret_cast<const float4*>(y + a0 + 4 * q);
            }
            // Consume every loaded value in an empty asm statement: all loads
            // are issued before it (one wait for the lot), the LDS stores
            // after it, instead of each load sinking next to its store.
#pragma unroll
            for (int k = 0; k < Q; ++k)
                asm volatile("" ::"v"(vx[k].x), "v"(vx[k].y), "v"(vx[k].z), "v"(vx[k].w), "v"(vy[k].x),
                             "v"(vy[k].y), "v"(vy[k].z), "v"(vy[k].w));
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                const int q = t + k * NT;
                if (q < nq_full) {
                    reinterpret_cast<float4*>(xs)[q] = vx[k];
                    reinterpret_cast<float4*>(ys)[q] = vy[k];
                }
            }
        }
        if (t == 0 && nq_full < nq) {
            for (int g = a0 + 4 * nq_full; g < base + nh; ++g) {
                xs[g - a0] = x[g];
                ys[g - a0] = y[g];
            }
        }
    } else {
        for (int h = t; h < nh; h += NT) {
            xs[base - a0 + h] = x[base + h];
            ys[base - a0 + h] = y[base + h];
        }
    }
}

template <class P, int HB, int NW>
__global__ __launch_bounds__(NW * kWave) void k_block(const int32_t* __restrict__ off, int n_events,
                                                         const float* __restrict__ x,
                                                         const float* __restrict__ y, Consts c, int eb,
                                                         int n_blocks, unsigned* block_counter, int vec,
                                                         int32_t* __restrict__ counts,
                                                         uint8_t* __restrict__ accept, uint32_t* status) {
    // HB hits plus up to 3 before the first and 3 after the last (4-aligned copy)
    __shared__ __align__(16) float stage_x[HB + 8];
    __shared__ __align__(16) float stage_y[HB + 8];
    constexpr int NT = NW * kWave;
    __shared__ __align__(16) float pbuf_x[NW][kPBuf];
    __shared__ __align__(16) float pbuf_y[NW][kPBuf];
    __shared__ int32_t soff[3 * kMaxEB + 1];
    __shared__ int4 desc0[kMaxEB], desc1[kMaxEB];
    __shared__ int32_t sres[kMaxEB];
    __shared__ int s_block, s_bad;
    const int w = uniform_i(threadIdx.x / kWave);
    float* px = pbuf_x[w];
    float* py = pbuf_y[w];
    const GlobalHits ghits{x, y};
    int iter = 0;
    for (;; ++iter) {
        if (threadIdx.x == 0) {
            if (block_counter)
                s_block = (int)atomicAdd(block_counter, 1u);
            else
                s_block = iter == 0 ? (int)blockIdx.x : n_blocks;
            s_bad = 0;
        }
        __syncthreads();
        const int b = uniform_i(s_block);
        if (b >= n_blocks) break;
        const int e0 = b * eb;
        const int ne = min(eb, n_events - e0);
        for (int t = threadIdx.x; t <= 3 * ne; t += NT) soff[t] = off[3 * (int64_t)e0 + t];
        __syncthreads();
        // Per-event CSR checks; malformed events get -1 here.
        for (int t = threadIdx.x; t < ne; t += NT) {
            const int a0 = soff[3 * t], a1 = soff[3 * t + 1], a2 = soff[3 * t + 2], a3 = soff[3 * t + 3];
            if (!(0 <= a0 && a0 <= a1 && a1 <= a2 && a2 <= a3 && a3 <= c.n_hits)) {
                counts[e0 + t] = -1;
                accept[e0 + t] = 0;
                if (status) atomicOr(status, TRIG_STATUS_MALFORMED);
                atomicOr(&s_bad, 1);
            }
        }
        __syncthreads();
        if (uniform_i(s_bad)) {
            // Irregular block: every well-formed event straight from HBM.
            for (int t = w; t < ne; t += NW) {
                const int a0 = soff[3 * t], a1 = soff[3 * t + 1], a2 = soff[3 * t + 2], a3 = soff[3 * t + 3];
                if (0 <= a0 && a0 <= a1 && a1 <= a2 && a2 <= a3 && a3 <= c.n_hits)
                    wave_event<P>(c, ghits, 0, a0, a1, a2, a3, e0 + t, counts, accept, status, px, py);
            }
            __syncthreads();
            if (!block_counter) break;
            continue;
        }
        // Well-formed block: offsets are non-decreasing over it.  Stage
        // sub-blocks of consecutive events whose hits fit in LDS.
        int cur = 0;
        while (cur < ne) {
            const int base = soff[3 * cur];
            const int t = (int)threadIdx.x;
            // Events from cur on whose hits still fit: a prefix, counted NT at a time.
            int nfit = 0;
            for (int t0 = 0;; t0 += NT) {
                const int tt = t0 + t;
                const bool fits = (cur + tt < ne) && (soff[3 * (cur + tt + 1)] - base <= HB);
                const int c1 = uniform_i(__syncthreads_count(fits));
                nfit += c1;
                if (c1 < NT) break;
            }
            if (nfit == 0) {
                // One event larger than LDS: wave 0 reads it from HBM.
                if (w == 0)
                    wave_event<P>(c, ghits, 0, soff[3 * cur], soff[3 * cur + 1], soff[3 * cur + 2],
                                  soff[3 * cur + 3], e0 + cur, counts, accept, status, px, py);
                __syncthreads();
                cur += 1;
                continue;
            }
            const int end = cur + nfit;
            const int nh = soff[3 * end] - base;
            const int nsub = end - cur;
            stage_hits<HB, NT>(x, y, base, nh, c.n_hits, vec != 0, stage_x, stage_y);
            // Per-event descriptors, one lane per event: local offsets,
            // sizes, lane layout; events decided without pairs get their
            // result here (0 for an empty layer, -2 for a count beyond int32).
            const int a0 = base & ~3;
            for (int te = t; te < nsub; te += NT) {
                const int ev = cur + te;
                const int b0 = soff[3 * ev], b1 = soff[3 * ev + 1], b2 = soff[3 * ev + 2], b3 = soff[3 * ev + 3];
                const int n0 = b1 - b0, n1 = b2 - b1, n2 = b3 - b2;
                const int64_t n01 = (int64_t)n0 * n1;
                int R = 0, T = 0, res = 0, work = 0;
                if (n2 > 0 && (n01 > (int64_t)INT32_MAX || n01 * n2 > (int64_t)INT32_MAX)) {
                    res = -2;
                } else if (n0 > 0 && n1 > 0 && n2 > 0) {
                    work = 1;
                    lane_layout(n0, n1, R, T);
                }
                desc0[te] = make_int4(b0 - a0, n0, b1 - a0, n1);
                desc1[te] = make_int4(b2 - a0, n2, work ? R : 0, T);
                sres[te] = res;
            }
            __syncthreads();
            // Events round-robin over the waves (a static assignment: no
            // per-wave claim loop).
            const LdsHits lh{stage_x, stage_y};
            for (int te = w; te < nsub; te += NW) {
                const int4 d0 = desc0[te], d1 = desc1[te];
                const int o0 = uniform_i(d0.x), n0 = uniform_i(d0.y), o1 = uniform_i(d0.z), n1 = uniform_i(d0.w);
                const int o2 = uniform_i(d1.x), n2 = uniform_i(d1.y), R = uniform_i(d1.z), T = uniform_i(d1.w);
                if (R == 0) continue;  // decided in the descriptor pass
                const uint32_t cnt = T > 0 ? wave_event_fast<P>(c, lh, o0, n0, o1, n1, o2, n2, R, T, px, py)
                                           : wave_event_pruned<P>(c, lh, o0, n0, o1, n1, o2, n2, px, py);
                if (lane_id() == 0) sres[te] = (int32_t)cnt;
            }
            __syncthreads();
            // Results of the sub-block, one lane per event (coalesced).
            for (int te = t; te < nsub; te += NT) {
                const int32_t r = sres[te];
                counts[e0 + cur + te] = r;
                accept[e0 + cur + te] = (uint8_t)(r >= 0 && r >= c.min_triplets);
                if (r < 0 && status) atomicOr(status, TRIG_STATUS_OVERFLOW);
            }
            __syncthreads();
            cur = end;
        }
        if (!block_counter) break;
    }
}

}  // namespace trig
