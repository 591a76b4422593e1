// Block-staged selection with exact pair pruning (the batched form).
//
// A workgroup takes a block of consecutive events, copies their hits (one
// contiguous CSR range) from HBM into LDS with coalesced loads, and counts
// every event's passing triplets from LDS.  The count is the same as the
// brute-force triplet loop (paper Sec. 3.2 steps 1-3), but triplets are only
// completed for pairs (i, j) that can still pass:
//
//   MSD test (the fit written out): a = f32(U0*c_i + U1*c_j) depends on
//              (i, j) only, and a triplet that passes a plane has
//              |a| <= a0 + a1 M for any M >= |c_j| (csrc/trig_bounds.hpp: a
//              rigorous bound on the fit's binary32 rounding).  M is the
//              largest |x|, |y| among the staged hits (per block, or per event
//              for events read from HBM).
//   MSD_BASIS: Q = f32(A + f32(b*b)) >= A = f32(a*a) in binary32 (rounding is
//              monotone and b*b >= 0), so a triplet can pass only if
//              f32(a*a) <= Qmax in both planes, i.e. |a| <= beta with beta the
//              largest binary32 value whose rounded square is <= Qmax
//              (f32(a*a) is non-decreasing in |a|).
//   window:    the layer-1 window |s_j - s_i| < W is itself part of the test.
//
// All three conditions are exact consequences of the binary32 test, so
// pruning never changes a count.  Surviving pairs (rare: a is the distance of hit j
// from the line through the vertex and hit i, in cm) are completed against
// every layer-2 hit with the full binary32 test, lanes over k.
//
// Lane layout of the pair scan: lane L holds layer-1 hit j and its constant
// part of a; for n1 <= 32 the 64 lanes hold R = floor(64/n1) copies of the
// layer-1 hits, copy g scanning layer-0 hits i = g, g+R, g+2R, ... so that
// few lanes idle.  The layer-0 part of a (or the layer-0 slope) is computed
// once per hit into a per-wave LDS buffer and read with a broadcast.  An
// event that fits one pass takes layer 0 into the lanes instead when that
// needs fewer buffer steps (the pair tests are symmetric in the two layers).
#pragma once

#include "trig_device.hpp"

namespace trig {

constexpr int kPBuf = 64;      // per-wave buffer of layer-0 values (float2)
static_assert(kPBuf == kWave, "the fast path fills the buffer with one entry per lane");
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

// floor(lane / n) for 0 <= lane < 64 and 1 <= n <= 64: (lane * r) >> 16 with
// r = ceil(2^16 / n) (a 24-bit multiply and a shift).  With r n = 2^16 + d,
// 0 <= d < n, the product is 2^16 lane / n + lane d / n, and lane d / n < 64
// < 2^16 / n, which never reaches the next multiple of 2^16 / n.  r is
// computed once per event in the descriptor pass (recip16) and travels with
// the event's descriptor.
__device__ __forceinline__ uint32_t recip16(int n) { return (65536u + (uint32_t)n - 1u) / (uint32_t)n; }
__device__ __forceinline__ int div_lane(int lane, uint32_t r) { return (int)(__umul24((unsigned)lane, r) >> 16); }

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

// Largest |x|, |y| of hits [o, o + n) (NaN ignored, infinities kept), by a
// whole wave; the same value on every lane.
template <class H>
__device__ float layer_mag(const H& hits, int o, int n) {
    float m = 0.0f;
    for (int t = (int)lane_id(); t < n; t += kWave) {
        const float2 h = hits.at(o + t);
        m = __builtin_fmaxf(m, __builtin_fmaxf(__builtin_fabsf(h.x), __builtin_fabsf(h.y)));
    }
    return wave_max_f(m);
}

// Pair test bounds of a block or event: the exact pair test is
// |a_x| <= bx and |a_y| <= by (window: strict), and the prefilter score of a
// pair that passes it is at most pre.  prune = false: no valid bound (per-hit
// z outside (0, inf) in layers 0 or 1): every pair must be completed.
struct PairBounds {
    float bx, by, pre;
    bool prune = true;
};

// Per-hit z: hits read from HBM whose at() gives the slopes (x / z, y / z),
// the partials the per-hit-z pair tests compare; x, y and z stay reachable
// for the completion.
struct SlopeHits {
    const float* x;
    const float* y;
    const float* z;
    __device__ __forceinline__ float2 at(int h) const { return make_float2(x[h] / z[h], y[h] / z[h]); }
};

// TRIG_TEST_MSD_BASIS.
struct MsdBasisPrune {
    static constexpr bool kMag = false;  // bounds do not depend on M
    static constexpr bool kEventBounds = false;
    static constexpr bool kZ = false;
    __device__ static __forceinline__ PairBounds bounds(const Consts& c, float) {
        return PairBounds{c.beta_x, c.beta_y, c.pre_msd};
    }
    __device__ static __forceinline__ float2 layer0(const Consts& c, float2 h) {
        return make_float2(c.U0 * h.x, c.U0 * h.y);
    }
    __device__ static __forceinline__ float2 layer1(const Consts& c, float2 h) {
        return make_float2(c.U1 * h.x, c.U1 * h.y);
    }
    // layer0 (l == 0) or layer1 (l == 1), l wave-uniform: the same product.
    __device__ static __forceinline__ float2 layer(const Consts& c, float2 h, int l) {
        const float u = select_uniform(l, c.U1, c.U0);
        return make_float2(u * h.x, u * h.y);
    }
    // Lanes whose pair can still pass: |f32(P + Q)| <= bound in both planes.
    __device__ static __forceinline__ uint64_t pair_mask(const PairBounds& b, float2 p, float2 q) {
        const float ax = p.x + q.x;
        const float ay = p.y + q.y;
        return lanes(__builtin_fabsf(ax) <= b.bx) & lanes(__builtin_fabsf(ay) <= b.by);
    }
    // Prefilter score: pair_mask's lane set is within {score <= b.pre}
    // (|a_x| <= bx and |a_y| <= by imply max(|a_x|, |a_y|) <= max(bx, by);
    // same binary32 a as the exact test, no rounding of its own).
    __device__ static __forceinline__ float score(float2 p, float2 q) {
        const float ax = p.x + q.x;
        const float ay = p.y + q.y;
        return __builtin_fmaxf(__builtin_fabsf(ax), __builtin_fabsf(ay));
    }
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
    // Lanes k (layer-2 hits o2 + k0 + lane, k < n2) whose triplet with
    // (hi, hj) passes.
    template <class H>
    __device__ static uint64_t complete_mask(const Consts& c, const H& hits, int hi, int hj, int o2, int n2, int k0) {
        const float2 ci = hits.at(hi), cj = hits.at(hj);
        const float ax = c.U0 * ci.x + c.U1 * cj.x;
        const float ay = c.U0 * ci.y + c.U1 * cj.y;
        const float bx0 = c.V0 * ci.x + c.V1 * cj.x;
        const float by0 = c.V0 * ci.y + c.V1 * cj.y;
        const int k = k0 + (int)lane_id();
        float2 w = nan2();
        if (k < n2) {
            const float2 ck = hits.at(o2 + k);
            w = make_float2(c.V2 * ck.x, c.V2 * ck.y);
        }
        const float bx = bx0 + w.x;
        const float qx = ax * ax + bx * bx;
        const float by = by0 + w.y;
        const float qy = ay * ay + by * by;
        return lanes(qx <= c.qmax_x) & lanes(qy <= c.qmax_y);
    }
};

// TRIG_TEST_MSD: the basis-form partials a prune pairs with the bounds of
// the written-out fit (a0 + a1 M), and survivors are completed with the fit
// written out.
struct MsdFitPrune {
    static constexpr bool kMag = true;  // bounds grow with M >= |c_j|
    static constexpr bool kEventBounds = false;
    static constexpr bool kZ = false;
    __device__ static __forceinline__ PairBounds bounds(const Consts& c, float M) {
        const float bx = c.fit_a0x + c.fit_a1x * M;
        const float by = c.fit_a0y + c.fit_a1y * M;
        return PairBounds{bx, by, __builtin_fmaxf(bx, by)};
    }
    __device__ static __forceinline__ float2 layer0(const Consts& c, float2 h) {
        return MsdBasisPrune::layer0(c, h);
    }
    __device__ static __forceinline__ float2 layer1(const Consts& c, float2 h) {
        return MsdBasisPrune::layer1(c, h);
    }
    __device__ static __forceinline__ float2 layer(const Consts& c, float2 h, int l) {
        return MsdBasisPrune::layer(c, h, l);
    }
    __device__ static __forceinline__ uint64_t pair_mask(const PairBounds& b, float2 p, float2 q) {
        return MsdBasisPrune::pair_mask(b, p, q);
    }
    __device__ static __forceinline__ float score(float2 p, float2 q) { return MsdBasisPrune::score(p, q); }
    template <class H>
    __device__ static uint32_t complete(const Consts& c, const H& hits, int hi, int hj, int o2, int n2) {
        const float2 ci = hits.at(hi), cj = hits.at(hj);
        const float sx01 = ci.x * c.z0 + cj.x * c.z1;
        const float sy01 = ci.y * c.z0 + cj.y * c.z1;
        uint32_t cnt = 0;
        for (int k0 = 0; k0 < n2; k0 += kWave) {
            const int k = k0 + (int)lane_id();
            const float2 ck = k < n2 ? hits.at(o2 + k) : nan2();
            const float qx = MsdFitTest::plane_q(c, ci.x, cj.x, sx01, ck.x, ck.x * c.z2);
            const float qy = MsdFitTest::plane_q(c, ci.y, cj.y, sy01, ck.y, ck.y * c.z2);
            cnt += (uint32_t)__builtin_popcountll(lanes(qx <= c.qmax_x) & lanes(qy <= c.qmax_y));
        }
        return cnt;
    }
    template <class H>
    __device__ static uint64_t complete_mask(const Consts& c, const H& hits, int hi, int hj, int o2, int n2, int k0) {
        const float2 ci = hits.at(hi), cj = hits.at(hj);
        const float sx01 = ci.x * c.z0 + cj.x * c.z1;
        const float sy01 = ci.y * c.z0 + cj.y * c.z1;
        const int k = k0 + (int)lane_id();
        const float2 ck = k < n2 ? hits.at(o2 + k) : nan2();
        const float qx = MsdFitTest::plane_q(c, ci.x, cj.x, sx01, ck.x, ck.x * c.z2);
        const float qy = MsdFitTest::plane_q(c, ci.y, cj.y, sy01, ck.y, ck.y * c.z2);
        return lanes(qx <= c.qmax_x) & lanes(qy <= c.qmax_y);
    }
};

struct WindowPrune {
    static constexpr bool kMag = false;
    static constexpr bool kEventBounds = false;
    static constexpr bool kZ = false;
    __device__ static __forceinline__ PairBounds bounds(const Consts& c, float) {
        return PairBounds{c.win_x, c.win_y, c.pre_win};
    }
    __device__ static __forceinline__ float2 layer0(const Consts& c, float2 h) {
        return make_float2(h.x / c.z0, h.y / c.z0);
    }
    __device__ static __forceinline__ float2 layer1(const Consts& c, float2 h) {
        return make_float2(h.x / c.z1, h.y / c.z1);
    }
    __device__ static __forceinline__ float2 layer(const Consts& c, float2 h, int l) {
        const float z = select_uniform(l, c.z1, c.z0);
        return make_float2(h.x / z, h.y / z);
    }
    __device__ static __forceinline__ uint64_t pair_mask(const PairBounds& b, float2 p, float2 q) {
        return lanes(__builtin_fabsf(q.x - p.x) < b.bx) & lanes(__builtin_fabsf(q.y - p.y) < b.by);
    }
    // |d_x| < W_x and |d_y| < W_y imply max(|d_x|, |d_y|) <= the larger window.
    __device__ static __forceinline__ float score(float2 p, float2 q) {
        return __builtin_fmaxf(__builtin_fabsf(q.x - p.x), __builtin_fabsf(q.y - p.y));
    }
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
    // (hj is tested by the pair test: the layer-1 window)
    template <class H>
    __device__ static uint64_t complete_mask(const Consts& c, const H& hits, int hi, int /*hj*/, int o2, int n2,
                                             int k0) {
        const float2 ci = hits.at(hi);
        const float sxi = ci.x / c.z0, syi = ci.y / c.z0;
        const int k = k0 + (int)lane_id();
        float2 s = nan2();
        if (k < n2) {
            const float2 ck = hits.at(o2 + k);
            s = make_float2(ck.x / c.z2, ck.y / c.z2);
        }
        return lanes(__builtin_fabsf(s.x - sxi) < c.win_x) & lanes(__builtin_fabsf(s.y - syi) < c.win_y);
    }
};

// Per-hit z, TRIG_TEST_MSD: pairs pruned on their slopes (SlopeHits gives
// s = c / z): a triplet that passes a plane has |f32(s_j - s_i)| <=
// (a0 + a1 M) / zmin (csrc/trig_bounds.hpp), M and zmin over the event's
// layers 0 and 1; survivors completed with the per-hit-z fit.
struct MsdZPrune {
    static constexpr bool kMag = false;
    static constexpr bool kEventBounds = true;
    static constexpr bool kZ = true;  // reads hits through SlopeHits
    __device__ static __forceinline__ float2 layer0(const Consts&, float2 s) { return s; }
    __device__ static __forceinline__ float2 layer1(const Consts&, float2 s) { return s; }
    __device__ static __forceinline__ float2 layer(const Consts&, float2 s, int) { return s; }
    // M, zmin and zmax over layers 0 and 1 (raw coordinates), by the wave.
    __device__ static PairBounds event_bounds(const Consts& c, const SlopeHits& h, int o0, int n0, int o1, int n1) {
        float m = 0.0f, zlo = __builtin_inff(), zhi = 0.0f;
        bool bad = false;
        for (int t = (int)lane_id(); t < n0 + n1; t += kWave) {
            const int q = t < n0 ? o0 + t : o1 + (t - n0);
            const float z = h.z[q];
            m = __builtin_fmaxf(m, __builtin_fmaxf(__builtin_fabsf(h.x[q]), __builtin_fabsf(h.y[q])));
            bad |= !(z > 0.0f && z < __builtin_inff());
            zlo = __builtin_fminf(zlo, z);
            zhi = __builtin_fmaxf(zhi, z);
        }
        PairBounds b;
        const float M = wave_max_f(m), zmin = wave_min_f(zlo);
        const float inv = 1.0f / zmin;
        // every z of layers 0 and 1 in (0, inf), and no slope that can
        // overflow (|c| / z <= M / zmin < 2^126): otherwise no pruning
        b.prune = !wave_any(bad) && M * inv < 0x1p126f;
        b.bx = (c.zs_a0x + c.zs_a1x * M) * inv + 0x1p-126f;
        b.by = (c.zs_a0y + c.zs_a1y * M) * inv + 0x1p-126f;
        b.pre = __builtin_fmaxf(b.bx, b.by);
        (void)zhi;
        return b;
    }
    __device__ static __forceinline__ uint64_t pair_mask(const PairBounds& b, float2 p, float2 q) {
        return lanes(__builtin_fabsf(q.x - p.x) <= b.bx) & lanes(__builtin_fabsf(q.y - p.y) <= b.by);
    }
    __device__ static __forceinline__ float score(float2 p, float2 q) {
        return __builtin_fmaxf(__builtin_fabsf(q.x - p.x), __builtin_fabsf(q.y - p.y));
    }
    __device__ static __forceinline__ uint64_t triplet_mask(const Consts& c, const SlopeHits& h, int hi, int hj,
                                                          int hk, bool valid) {
        const float xi = h.x[hi], yi = h.y[hi], zi = h.z[hi];
        const float xj = h.x[hj], yj = h.y[hj], zj = h.z[hj];
        const float n = __builtin_nanf("");
        const float xk = valid ? h.x[hk] : n, yk = valid ? h.y[hk] : n, zk = valid ? h.z[hk] : n;
        const MsdZTest::Pair pr = MsdZTest::pair(c, xi, yi, zi, xj, yj, zj);
        const float w = 1.0f / (pr.szz01 + zk * zk);
        const float qx = MsdZTest::plane_q(xi, xj, pr.sx01, xk, xk * zk, zi, zj, zk, w);
        const float qy = MsdZTest::plane_q(yi, yj, pr.sy01, yk, yk * zk, zi, zj, zk, w);
        return lanes(qx <= c.qmax_x) & lanes(qy <= c.qmax_y);
    }
    template <class H>
    __device__ static uint32_t complete(const Consts& c, const H& hits, int hi, int hj, int o2, int n2) {
        uint32_t cnt = 0;
        for (int k0 = 0; k0 < n2; k0 += kWave) {
            const int k = k0 + (int)lane_id();
            cnt += (uint32_t)__builtin_popcountll(triplet_mask(c, hits, hi, hj, o2 + min(k, n2 - 1), k < n2));
        }
        return cnt;
    }
    template <class H>
    __device__ static uint64_t complete_mask(const Consts& c, const H& hits, int hi, int hj, int o2, int n2, int k0) {
        const int k = k0 + (int)lane_id();
        return triplet_mask(c, hits, hi, hj, o2 + min(k, n2 - 1), k < n2);
    }
};

// Per-hit z, window test: the slopes are the test's own quantities, so the
// layer-1 window is exact, as in WindowPrune.
struct WindowZPrune {
    static constexpr bool kMag = false;
    static constexpr bool kEventBounds = false;
    static constexpr bool kZ = true;  // reads hits through SlopeHits
    __device__ static __forceinline__ PairBounds bounds(const Consts& c, float) {
        return PairBounds{c.win_x, c.win_y, c.pre_win};
    }
    __device__ static __forceinline__ float2 layer0(const Consts&, float2 s) { return s; }
    __device__ static __forceinline__ float2 layer1(const Consts&, float2 s) { return s; }
    __device__ static __forceinline__ float2 layer(const Consts&, float2 s, int) { return s; }
    __device__ static __forceinline__ uint64_t pair_mask(const PairBounds& b, float2 p, float2 q) {
        return WindowPrune::pair_mask(b, p, q);
    }
    __device__ static __forceinline__ float score(float2 p, float2 q) { return WindowPrune::score(p, q); }
    template <class H>
    __device__ static uint64_t complete_mask(const Consts& c, const H& hits, int hi, int /*hj*/, int o2, int n2,
                                             int k0) {
        const float2 si = hits.at(hi);
        const int k = k0 + (int)lane_id();
        const float2 sk = k < n2 ? hits.at(o2 + k) : nan2();
        return lanes(__builtin_fabsf(sk.x - si.x) < c.win_x) & lanes(__builtin_fabsf(sk.y - si.y) < c.win_y);
    }
    template <class H>
    __device__ static uint32_t complete(const Consts& c, const H& hits, int hi, int hj, int o2, int n2) {
        uint32_t cnt = 0;
        for (int k0 = 0; k0 < n2; k0 += kWave)
            cnt += (uint32_t)__builtin_popcountll(complete_mask(c, hits, hi, hj, o2, n2, k0));
        return cnt;
    }
};

// Bounds of one event read from HBM: the policy's own event bounds, or its
// block bounds with M = the largest layer-1 |x|, |y| where they depend on it.
template <class P, class H>
__device__ __forceinline__ PairBounds event_bounds(const Consts& c, const H& hits, int o0, int n0, int o1, int n1) {
    if constexpr (P::kEventBounds) {
        return P::event_bounds(c, hits, o0, n0, o1, n1);
    } else {
        float M = 0.0f;
        if constexpr (P::kMag) M = layer_mag(hits, o1, n1);
        return P::bounds(c, M);
    }
}

// Two-particle acceptance: whether an event's passing triplets include two
// with no hit in common (the trigger signature of Sec. 3.1, two particles
// pointing back to the target), decided while the passing triplets stream
// by, in O(1) state.  Let e1 = (a, b, c) be the first passing triplet.  A
// later triplet with no hit of e1 decides at once.  Otherwise two passing
// triplets f, g with no common hit both meet e1, in different hits x != y of
// e1 (they cannot share one), f without y and g without x: for (x, y) =
// (a, b), f = (a, j, k) with j != b and g = (i, b, k') with i != a, and
// they share no hit exactly when k != k'.  So for each of the three pairs of
// e1's hits, it is enough to keep up to two distinct values of the third
// layer's hit among the triplets through x but not y, and among those through
// y but not x: two such triplets differ there iff not both sides hold one
// and the same value.  Wave-uniform (every lane runs the same updates).
struct TwoValues {
    int n, v0, v1;  // up to two distinct values seen (n of them)
};
// t with v added when `when` holds (selects, no branches: the state stays in
// registers).
__device__ __forceinline__ TwoValues two_values_add(TwoValues t, int v, bool when) {
    const bool first = when && t.n == 0, second = when && t.n == 1 && v != t.v0;
    return TwoValues{first ? 1 : (second ? 2 : t.n), first ? v : t.v0, second ? v : t.v1};
}
// some value of a differs from some value of b
__device__ __forceinline__ bool two_values_differ(TwoValues a, TwoValues b) {
    return a.n > 0 && b.n > 0 && !(a.n == 1 && b.n == 1 && a.v0 == b.v0);
}

struct DisjointState {
    bool have, found;
    int a, b, c;
    TwoValues ab_a, ab_b, ac_a, ac_c, bc_b, bc_c;
};

__device__ __forceinline__ DisjointState disjoint_start() {
    const TwoValues z{0, 0, 0};
    return DisjointState{false, false, 0, 0, 0, z, z, z, z, z, z};
}

__device__ __forceinline__ DisjointState disjoint_add(DisjointState s, int i, int j, int k) {
    if (!s.have) {
        s.have = true;
        s.a = i;
        s.b = j;
        s.c = k;
        return s;
    }
    if (i != s.a && j != s.b && k != s.c) {
        s.found = true;
        return s;
    }
    s.ab_a = two_values_add(s.ab_a, k, i == s.a && j != s.b);  // through a, not b: layer-2 hit
    s.ab_b = two_values_add(s.ab_b, k, j == s.b && i != s.a);
    s.ac_a = two_values_add(s.ac_a, j, i == s.a && k != s.c);  // through a, not c: layer-1 hit
    s.ac_c = two_values_add(s.ac_c, j, k == s.c && i != s.a);
    s.bc_b = two_values_add(s.bc_b, i, j == s.b && k != s.c);  // through b, not c: layer-0 hit
    s.bc_c = two_values_add(s.bc_c, i, k == s.c && j != s.b);
    s.found = two_values_differ(s.ab_a, s.ab_b) || two_values_differ(s.ac_a, s.ac_c) ||
              two_values_differ(s.bc_b, s.bc_c);
    return s;
}

// Whether event (o0, n0, o1, n1, o2, n2) (all layers non-empty, n0 n1 n2 in
// int32) has two passing triplets with no hit in common: pairs one per lane
// (the exact pair test of the pruned form), surviving pairs completed over
// layer 2 by lanes, each passing triplet fed to the state above.  Whole wave.
template <class P, class H>
__device__ bool wave_two_particles(const Consts& c, const H& hits, int o0, int n0, int o1, int n1, int o2, int n2,
                                   float2* __restrict__ part, int part_cap) {
    const PairBounds pb = event_bounds<P>(c, hits, o0, n0, o1, n1);
    DisjointState st = disjoint_start();
    // n0 n1 <= INT32_MAX, so pair indices (and p0 + 63) fit 32-bit unsigned
    const uint32_t np = (uint32_t)n0 * (uint32_t)n1, un1 = (uint32_t)n1;
    const uint32_t lane = lane_id();
    // The pair partials of layers 0 and 1 in LDS when they fit (one round
    // trip to HBM instead of one per 64 pairs).
    const bool staged = n0 + n1 <= part_cap;
    if (staged) {
        for (int t = (int)lane; t < n0 + n1; t += kWave)
            part[t] = t < n0 ? P::layer0(c, hits.at(o0 + t)) : P::layer1(c, hits.at(o1 + (t - n0)));
        wave_lds_sync();
    }
    for (uint32_t p0 = 0; p0 < np; p0 += kWave) {
        const uint32_t p = p0 + lane;
        const bool v = p < np;
        const uint32_t q = p / un1;
        const int i = v ? (int)q : 0, j = v ? (int)(p - q * un1) : 0;
        float2 u = nan2(), w = nan2();
        if (v) {
            u = staged ? part[i] : P::layer0(c, hits.at(o0 + i));
            w = staged ? part[n0 + j] : P::layer1(c, hits.at(o1 + j));
        }
        uint64_t m = pb.prune ? P::pair_mask(pb, u, w) : lanes(v);
        while (m) {
            const int L = __builtin_ctzll(m);
            m &= m - 1;
            const int iL = __builtin_amdgcn_readlane(i, L), jL = __builtin_amdgcn_readlane(j, L);
            for (int k0 = 0; k0 < n2; k0 += kWave) {
                uint64_t km = P::complete_mask(c, hits, o0 + iL, o1 + jL, o2, n2, k0);
                while (km) {
                    const int kk = k0 + __builtin_ctzll(km);
                    km &= km - 1;
                    st = disjoint_add(st, iL, jL, kk);
                    if (st.found) break;
                }
                if (st.found) break;
            }
            if (st.found) break;
        }
        if (st.found) break;
    }
    if (staged) wave_lds_sync();  // the next event rewrites the partials
    return st.found;
}

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
__device__ uint32_t wave_event_pruned(const Consts& c, const PairBounds& pb, const H& hits, int o0, int n0, int o1,
                                      int n1, int o2, int n2, float* __restrict__ px, float* __restrict__ py) {
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
                    if (cnt >= (uint32_t)c.count_cap) return;  // the result is capped there
                }
            };
            const float4* ppx = reinterpret_cast<const float4*>(px + g * T);
            const float4* ppy = reinterpret_cast<const float4*>(py + g * T);
            const float bnd = pb.pre;
            for (int t = 0; t < T; t += 4) {
                const float4 vx = ppx[t >> 2], vy = ppy[t >> 2];
                // Prefilter on the vector unit: does the smallest of the four
                // pairs' scores reach the bound?  (fmin drops NaN scores; all
                // NaN gives NaN, which fails.)
                const float s0 = P::score(make_float2(vx.x, vy.x), q);
                const float s1 = P::score(make_float2(vx.y, vy.y), q);
                const float s2 = P::score(make_float2(vx.z, vy.z), q);
                const float s3 = P::score(make_float2(vx.w, vy.w), q);
                const float smin = __builtin_fminf(__builtin_fminf(s0, s1), __builtin_fminf(s2, s3));
                if (wave_any(smin <= bnd)) {
                    finish(P::pair_mask(pb, make_float2(vx.x, vy.x), q), t);
                    finish(P::pair_mask(pb, make_float2(vx.y, vy.y), q), t + 1);
                    finish(P::pair_mask(pb, make_float2(vx.z, vy.z), q), t + 2);
                    finish(P::pair_mask(pb, make_float2(vx.w, vy.w), q), t + 3);
                }
            }
            wave_lds_sync();
        }
    }
    return cnt;
}

// Fast path (one lane pass, one buffer fill of at most kPBuf = kWave
// entries; R, T and the orientation from event_layout).  One of layers 0
// and 1 goes to the lanes (layer l = S ? 0 : 1, offset oL, nL hits), the
// other to the LDS buffer (offset oB, nB hits):
// lane L holds lane-layer hit j of copy g and its partial q; the buffer
// layer's partials go to px/py (NaN past nB).  Both pair tests depend on the
// two partials symmetrically (a sum, or the absolute value of a difference,
// which binary32 gives the same either way round), so the orientation does
// not change a count.
template <class P, class H>
__device__ __forceinline__ void fast_setup(const Consts& c, const H& hits, int oB, int nB, int oL, int nL, int S,
                                           int R, int T, uint32_t r, float* __restrict__ px, float* __restrict__ py,
                                           int& g, int& j, float2& q) {
    const int lane = (int)lane_id();
    // floor(lane / nL) for every R (r = recip16(nL)): with R = 1 (nL > 32)
    // lanes past nL get g = 1 and no hit
    g = div_lane(lane, r);
    j = lane - g * nL;
    const bool jv = (g < R) && (j < nL);
    if (!jv) g = 0;
    // Branch-free: every lane reads an in-range hit (indices clamped) and
    // selects NaN where it has none; the whole kPBuf-entry buffer (>= T R
    // entries) is written.
    const float nan = __builtin_nanf("");
    const float2 hq = P::layer(c, hits.at(oL + min(j, nL - 1)), S ? 0 : 1);
    q = make_float2(jv ? hq.x : nan, jv ? hq.y : nan);
    const float2 v = P::layer(c, hits.at(oB + min(lane, nB - 1)), S ? 1 : 0);
    px[lane] = lane < nB ? v.x : nan;
    py[lane] = lane < nB ? v.y : nan;
}

// m folded with the prefilter scores of the four pairs (g T + t .. g T + t +
// 3, j): fmin drops NaN scores; all NaN leaves m, and NaN fails every bound.
template <class P>
__device__ __forceinline__ float fast_fold(const float4* ppx, const float4* ppy, int t, float2 q, float m) {
    const float4 vx = ppx[t >> 2], vy = ppy[t >> 2];
    const float s0 = P::score(make_float2(vx.x, vy.x), q);
    const float s1 = P::score(make_float2(vx.y, vy.y), q);
    const float s2 = P::score(make_float2(vx.z, vy.z), q);
    const float s3 = P::score(make_float2(vx.w, vy.w), q);
    return __builtin_fminf(__builtin_fminf(__builtin_fminf(__builtin_fminf(m, s0), s1), s2), s3);
}

// Exact pass over all pairs of the fast-path layout (taken only when some
// prefilter score reached the bound): the exact pair test per pair, then the
// surviving pairs completed against layer 2 (layer-0 hit first).
template <class P, class H>
__device__ uint32_t fast_exact(const Consts& c, const PairBounds& pb, const H& hits, int oB, int oL, int S, int o2,
                               int n2, int T, int g, int j, float2 q, const float* px, const float* py) {
    uint32_t cnt = 0;
    auto finish = [&](uint64_t m, int t) {
        while (m) {
            const int L = __builtin_ctzll(m);
            m &= m - 1;
            const int hB = oB + __builtin_amdgcn_readlane(g, L) * T + t;
            const int hL = oL + __builtin_amdgcn_readlane(j, L);
            cnt += S ? P::complete(c, hits, hL, hB, o2, n2) : P::complete(c, hits, hB, hL, o2, n2);
            if (cnt >= (uint32_t)c.count_cap) return;  // the result is capped there
        }
    };
    const float4* ppx = reinterpret_cast<const float4*>(px + g * T);
    const float4* ppy = reinterpret_cast<const float4*>(py + g * T);
    for (int t = 0; t < T; t += 4) {
        const float4 vx = ppx[t >> 2], vy = ppy[t >> 2];
        finish(P::pair_mask(pb, make_float2(vx.x, vy.x), q), t);
        finish(P::pair_mask(pb, make_float2(vx.y, vy.y), q), t + 1);
        finish(P::pair_mask(pb, make_float2(vx.z, vy.z), q), t + 2);
        finish(P::pair_mask(pb, make_float2(vx.w, vy.w), q), t + 3);
    }
    return cnt;
}

// Passing triplets of an event that fits one lane pass and one buffer fill
// in the orientation S (S = 0: layer 1 in the lanes, as wave_event_pruned;
// S = 1: layer 0): the computation of wave_event_pruned with its loops taken
// once, and the prefilter minimum taken over the whole event before one
// vote.  R, T and S come from the per-event descriptor (event_layout).
template <class P, class H>
__device__ uint32_t wave_event_fast(const Consts& c, const PairBounds& pb, const H& hits, int o0, int n0, int o1,
                                    int n1, int o2, int n2, int R, int T, int S, uint32_t r,
                                    float* __restrict__ px, float* __restrict__ py) {
    const int oB = S ? o1 : o0, nB = S ? n1 : n0;
    const int oL = S ? o0 : o1, nL = S ? n0 : n1;
    int g, j;
    float2 q;
    fast_setup<P>(c, hits, oB, nB, oL, nL, S, R, T, r, px, py, g, j, q);
    wave_lds_sync();
    const float4* ppx = reinterpret_cast<const float4*>(px + g * T);
    const float4* ppy = reinterpret_cast<const float4*>(py + g * T);
    float m = __builtin_nanf("");
    int t = 0;
    for (; t + 8 <= T; t += 8) m = fast_fold<P>(ppx, ppy, t + 4, q, fast_fold<P>(ppx, ppy, t, q, m));
    if (t < T) m = fast_fold<P>(ppx, ppy, t, q, m);
    uint32_t cnt = 0;
    if (wave_any(m <= pb.pre)) cnt = fast_exact<P>(c, pb, hits, oB, oL, S, o2, n2, T, g, j, q, px, py);
    wave_lds_sync();
    return cnt;
}

// Lane layout of wave_event_pruned for one buffer fill with nL hits in the
// lanes and nB in the buffer: R copies of the lane layer and T (a multiple
// of 4) buffer entries per copy; T = 0 when the event needs more than one
// lane pass or buffer fill.
__device__ __forceinline__ void lane_layout(int nB, int nL, int& R, int& T) {
    R = nL <= kWave / 2 ? min(div_small(kWave, nL), kPBuf / 4) : 1;
    const int chunk = div_small(kPBuf, 4 * R) * 4 * R;
    T = (nL <= kWave && nB <= chunk) ? div_small(nB + 4 * R - 1, 4 * R) * 4 : 0;
}

// Layout of an event with n0, n1 >= 1: layer 1 in the lanes (S = 0, the
// layout of wave_event_pruned), or layer 0 (S = 1) when only that fits the
// fast path or it takes fewer buffer steps (T).  T = 0: general path.
__device__ __forceinline__ void event_layout(int n0, int n1, int& R, int& T, int& S) {
    int R1, T1;
    lane_layout(n0, n1, R, T);
    lane_layout(n1, n0, R1, T1);
    S = 0;
    if (T1 > 0 && (T == 0 || T1 < T)) {
        R = R1;
        T = T1;
        S = 1;
    }
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
        cnt = (int32_t)wave_event_pruned<P>(c, event_bounds<P>(c, hits, o0 - h_base, n0, o1 - h_base, n1), hits,
                                            o0 - h_base, n0, o1 - h_base, n1, o2 - h_base, n2, px, py);
    }
    if (lane_id() == 0) {
        counts[e] = capped(cnt, c);
        accept[e] = (uint8_t)(cnt >= 0 && cnt >= c.min_triplets);
        if (cnt < 0 && status) atomicOr(status, TRIG_STATUS_OVERFLOW);
    }
}

// Copies hits [base, base + nh) of x and y into xs/ys (LDS) at local index
// (h - a0), a0 = base rounded down to a multiple of 4, with 16-byte loads
// issued together (every thread's loads are in flight before any LDS write).
// The one float4 group that would cross n_hits is copied element by element
// by thread 0.  Needs x and y 16-byte aligned (checked by the host; `vec`
// false otherwise: plain 4-byte loads).
// Largest |x|, |y| of staged values as binary32 bit patterns without the
// sign: for non-negative floats the integer order is the float order, so an
// integer max (no NaN canonicalisation) finds it; a NaN pattern lies above
// +inf and is clamped to +inf (an infinite bound: no pruning), see mag_of.
__device__ __forceinline__ uint32_t abs_bits(float v) { return __builtin_bit_cast(uint32_t, v) & 0x7fffffffu; }
__device__ __forceinline__ uint32_t mag4(uint32_t m, float a, float b, float c, float d) {
    return max(max(m, max(abs_bits(a), abs_bits(b))), max(abs_bits(c), abs_bits(d)));
}
__device__ __forceinline__ float mag_of(uint32_t m) { return __builtin_bit_cast(float, min(m, 0x7f800000u)); }

// Returns the largest |x|, |y| among the hits this thread staged (and a few
// neighbours of the range: only an upper bound is needed).
template <int HB, int NT>
__device__ __forceinline__ uint32_t stage_hits(const float* __restrict__ x, const float* __restrict__ y,
                                               int base, int nh, int n_hits, bool vec, float* xs, float* ys) {
    constexpr int Q = (HB + 6) / 4 / NT + 1;  // float4 groups per thread, upper bound
    const int a0 = base & ~3;
    const int nq = (base + nh - a0 + 3) >> 2;             // float4 groups to copy
    const int t = (int)threadIdx.x;
    uint32_t mag = 0u;
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
                mag = mag4(mag4(mag, vx[k].x, vx[k].y, vx[k].z, vx[k].w), vy[k].x, vy[k].y, vy[k].z, vy[k].w);
            }
        }
        if (t == 0 && nq_full < nq) {
            for (int g = a0 + 4 * nq_full; g < base + nh; ++g) {
                xs[g - a0] = x[g];
                ys[g - a0] = y[g];
                mag = mag4(mag, x[g], y[g], 0.0f, 0.0f);
            }
        }
    } else {
        for (int h = t; h < nh; h += NT) {
            const float hx = x[base + h], hy = y[base + h];
            xs[base - a0 + h] = hx;
            ys[base - a0 + h] = hy;
            mag = mag4(mag, hx, hy, 0.0f, 0.0f);
        }
    }
    return mag;
}

// LDS of the block kernels: HB staged hits, NW waves, an event table of EB
// events (a block holds at most EB events).
template <int HB, int NW, int EB>
struct BlockLds {
    // HB hits plus up to 3 before the first and 3 after the last (4-aligned copy)
    float stage_x[HB + 8];
    float stage_y[HB + 8];
    float pbuf_x[NW][kPBuf];
    float pbuf_y[NW][kPBuf];
    // Event descriptors, 13-bit fields (local hit indices < HB + 8 <= 4104,
    // layer sizes <= HB <= 4096): da = o0 | n0 << 13 | R << 26 (R <= 16) |
    // S << 31, db = o1 | n1 << 13 | (T / 4) << 26 (T <= 64), dc = o2 | n2 << 13.
    // dr = recip16 of the lane layer's size (fast-path events only).
    uint32_t da[EB], db[EB], dc[EB], dr[EB];
    int32_t soff[3 * EB + 1];
    int32_t sres[EB];
    float wmag[NW];  // per wave: largest |x|, |y| it staged (TRIG_TEST_MSD bounds)
    int s_block, s_next, s_bad;
};

// Waves per SIMD that a workgroup's BlockLds allows on a CU (160 KB of LDS,
// at most eight waves per SIMD): the register budget k_block is held to.
template <int HB, int NW, int EB>
constexpr int block_waves_per_simd() {
    int wg = (int)(163840 / sizeof(BlockLds<HB, NW, EB>));
    if (wg * NW > 4 * 8) wg = 4 * 8 / NW;
    const int w = wg * NW / 4;
    return w < 1 ? 1 : w;
}
// An event table small enough that eight 2048-hit workgroups of four waves
// fit on a CU (seven with the full kMaxEB table); blocks of at most kSmallEB
// events use it.
constexpr int kSmallEB = 52;
static_assert(block_waves_per_simd<2048, 4, kSmallEB>() == 8, "eight 2048-hit workgroups per CU");

// Each wave's largest staged |x|, |y| into L.wmag (whole waves; read after
// the next barrier by block_mag).  m: mag4 bits.
template <int HB, int NW, int EB>
__device__ __forceinline__ void publish_mag(BlockLds<HB, NW, EB>& L, uint32_t m) {
    const float wm = wave_max_f(mag_of(m));
    if (lane_id() == 0) L.wmag[threadIdx.x / kWave] = wm;
}
template <int HB, int NW, int EB>
__device__ __forceinline__ float block_mag(const BlockLds<HB, NW, EB>& L) {
    float m = 0.0f;
#pragma unroll
    for (int w = 0; w < NW; ++w) m = __builtin_fmaxf(m, L.wmag[w]);
    return m;
}

// CSR checks of the block's events (offsets in L.soff); malformed events get
// -1 here.  Returns (workgroup-uniform) whether any event was malformed.
template <int HB, int NW, int EB>
__device__ bool block_validate(BlockLds<HB, NW, EB>& L, const Consts& c, int e0, int ne, int32_t* counts,
                               uint8_t* accept, uint32_t* status) {
    constexpr int NT = NW * kWave;
    if (threadIdx.x == 0) L.s_bad = 0;
    __syncthreads();
    for (int t = threadIdx.x; t < ne; t += NT) {
        const int a0 = L.soff[3 * t], a1 = L.soff[3 * t + 1], a2 = L.soff[3 * t + 2], a3 = L.soff[3 * t + 3];
        if (!(0 <= a0 && a0 <= a1 && a1 <= a2 && a2 <= a3 && a3 <= c.n_hits)) {
            counts[e0 + t] = -1;
            accept[e0 + t] = 0;
            if (status) atomicOr(status, TRIG_STATUS_MALFORMED);
            atomicOr(&L.s_bad, 1);
        }
    }
    __syncthreads();
    return uniform_i(L.s_bad) != 0;
}

// Descriptors of events [cur, cur + nsub) of a staged sub-block (local hit
// index = global index - a0), one lane per event; events decided without
// pairs get their result here (0 for an empty layer, -2 for a count beyond
// int32).  Ends with a barrier.
template <int HB, int NW, int EB>
__device__ void block_descriptors(BlockLds<HB, NW, EB>& L, int cur, int nsub, int a0) {
    constexpr int NT = NW * kWave;
    for (int te = threadIdx.x; te < nsub; te += NT) {
        const int ev = cur + te;
        const int b0 = L.soff[3 * ev], b1 = L.soff[3 * ev + 1], b2 = L.soff[3 * ev + 2], b3 = L.soff[3 * ev + 3];
        const int n0 = b1 - b0, n1 = b2 - b1, n2 = b3 - b2;
        const int64_t n01 = (int64_t)n0 * n1;
        int R = 0, T = 0, S = 0, res = 0, work = 0;
        if (n2 > 0 && (n01 > (int64_t)INT32_MAX || n01 * n2 > (int64_t)INT32_MAX)) {
            res = -2;
        } else if (n0 > 0 && n1 > 0 && n2 > 0) {
            work = 1;
            event_layout(n0, n1, R, T, S);
        }
        L.da[te] = (uint32_t)(b0 - a0) | ((uint32_t)n0 << 13) | ((uint32_t)(work ? R : 0) << 26) |
                   ((uint32_t)S << 31);
        L.db[te] = (uint32_t)(b1 - a0) | ((uint32_t)n1 << 13) | ((uint32_t)(T >> 2) << 26);
        L.dc[te] = (uint32_t)(b2 - a0) | ((uint32_t)n2 << 13);
        L.dr[te] = T > 0 ? recip16(S ? n0 : n1) : 0u;
        L.sres[te] = res;
    }
    __syncthreads();
}

// CSR checks and descriptors of the block's events in one pass, one lane per
// event (local hit index = global index - a0): malformed events get -1 and
// set L.s_bad (zero on entry); the descriptors are used only when no event
// is malformed and the block is staged whole.  No barrier.
template <int HB, int NW, int EB>
__device__ __forceinline__ void block_check_describe(BlockLds<HB, NW, EB>& L, const Consts& c, int e0, int ne, int a0,
                                                     int32_t* counts, uint8_t* accept, uint32_t* status) {
    constexpr int NT = NW * kWave;
    for (int te = threadIdx.x; te < ne; te += NT) {
        const int b0 = L.soff[3 * te], b1 = L.soff[3 * te + 1], b2 = L.soff[3 * te + 2], b3 = L.soff[3 * te + 3];
        if (!(0 <= b0 && b0 <= b1 && b1 <= b2 && b2 <= b3 && b3 <= c.n_hits)) {
            counts[e0 + te] = -1;
            accept[e0 + te] = 0;
            if (status) atomicOr(status, TRIG_STATUS_MALFORMED);
            atomicOr(&L.s_bad, 1);
            continue;
        }
        const int n0 = b1 - b0, n1 = b2 - b1, n2 = b3 - b2;
        const int64_t n01 = (int64_t)n0 * n1;
        int R = 0, T = 0, S = 0, res = 0, work = 0;
        if (n2 > 0 && (n01 > (int64_t)INT32_MAX || n01 * n2 > (int64_t)INT32_MAX)) {
            res = -2;
        } else if (n0 > 0 && n1 > 0 && n2 > 0) {
            work = 1;
            event_layout(n0, n1, R, T, S);
        }
        L.da[te] = (uint32_t)(b0 - a0) | ((uint32_t)n0 << 13) | ((uint32_t)(work ? R : 0) << 26) |
                   ((uint32_t)S << 31);
        L.db[te] = (uint32_t)(b1 - a0) | ((uint32_t)n1 << 13) | ((uint32_t)(T >> 2) << 26);
        L.dc[te] = (uint32_t)(b2 - a0) | ((uint32_t)n2 << 13);
        L.dr[te] = T > 0 ? recip16(S ? n0 : n1) : 0u;
        L.sres[te] = res;
    }
}

// Counts of the described events from the staged hits (events round-robin
// over the waves, a static assignment), then the results of events
// [e_first, e_first + nsub) with one lane per event.  Ends with a barrier.
template <class P, int HB, int NW, int EB>
__device__ void block_count(BlockLds<HB, NW, EB>& L, const Consts& c, int e_first, int nsub, int32_t* counts,
                            uint8_t* accept, uint32_t* status) {
    constexpr int NT = NW * kWave;
    const int w = uniform_i(threadIdx.x / kWave);
    float* px = L.pbuf_x[w];
    float* py = L.pbuf_y[w];
    const LdsHits lh{L.stage_x, L.stage_y};
    float M = 0.0f;
    if constexpr (P::kMag) M = block_mag(L);
    const PairBounds pb = P::bounds(c, M);
    // The wave's next descriptor is read while the current event is
    // counted (its LDS round trip off the per-event chain).
    uint32_t nda = 0u, ndb = 0u, ndc = 0u, ndr = 0u;
    if (w < nsub) {
        nda = L.da[w];
        ndb = L.db[w];
        ndc = L.dc[w];
        ndr = L.dr[w];
    }
    for (int te = w; te < nsub; te += NW) {
        const uint32_t da = (uint32_t)uniform_i((int)nda);
        const uint32_t db = (uint32_t)uniform_i((int)ndb);
        const uint32_t dc = (uint32_t)uniform_i((int)ndc);
        const uint32_t dr = (uint32_t)uniform_i((int)ndr);
        if (te + NW < nsub) {
            nda = L.da[te + NW];
            ndb = L.db[te + NW];
            ndc = L.dc[te + NW];
            ndr = L.dr[te + NW];
        }
        constexpr uint32_t kF = (1u << 13) - 1;
        const int o0 = (int)(da & kF), n0 = (int)((da >> 13) & kF), R = (int)((da >> 26) & 31u);
        const int S = (int)(da >> 31);
        const int o1 = (int)(db & kF), n1 = (int)((db >> 13) & kF), T = (int)(db >> 26) * 4;
        const int o2 = (int)(dc & kF), n2 = (int)((dc >> 13) & kF);
        if (R == 0) continue;  // decided in the descriptor pass
        const uint32_t cnt = T > 0 ? wave_event_fast<P>(c, pb, lh, o0, n0, o1, n1, o2, n2, R, T, S, dr, px, py)
                                   : wave_event_pruned<P>(c, pb, lh, o0, n0, o1, n1, o2, n2, px, py);
        L.sres[te] = (int32_t)cnt;  // uniform: every lane stores the same value
    }
    __syncthreads();
    for (int te = threadIdx.x; te < nsub; te += NT) {
        const int32_t r = L.sres[te];
        counts[e_first + te] = capped(r, c);
        accept[e_first + te] = (uint8_t)(r >= 0 && r >= c.min_triplets);
        if (r < 0 && status) atomicOr(status, TRIG_STATUS_OVERFLOW);
    }
    __syncthreads();
}

// Whole block [e0, e0 + ne) with its offsets in L.soff: malformed blocks
// event by event from HBM; otherwise sub-blocks of consecutive events whose
// hits fit in LDS are staged and counted (an event larger than LDS is read
// from HBM by wave 0).  Ends with a barrier.
template <class P, int HB, int NW, int EB>
__device__ void block_general(BlockLds<HB, NW, EB>& L, const Consts& c, const float* __restrict__ x,
                              const float* __restrict__ y, int e0, int ne, bool bad, bool vec, int32_t* counts,
                              uint8_t* accept, uint32_t* status) {
    constexpr int NT = NW * kWave;
    const int w = uniform_i(threadIdx.x / kWave);
    float* px = L.pbuf_x[w];
    float* py = L.pbuf_y[w];
    const GlobalHits ghits{x, y};
    if (bad) {
        for (int t = w; t < ne; t += NW) {
            const int a0 = L.soff[3 * t], a1 = L.soff[3 * t + 1], a2 = L.soff[3 * t + 2], a3 = L.soff[3 * t + 3];
            if (0 <= a0 && a0 <= a1 && a1 <= a2 && a2 <= a3 && a3 <= c.n_hits)
                wave_event<P>(c, ghits, 0, a0, a1, a2, a3, e0 + t, counts, accept, status, px, py);
        }
        __syncthreads();
        return;
    }
    // Well-formed block: offsets are non-decreasing over it.
    int cur = 0;
    while (cur < ne) {
        const int base = L.soff[3 * cur];
        const int t = (int)threadIdx.x;
        // Events from cur on whose hits still fit: a prefix, counted NT at a time.
        int nfit = 0;
        for (int t0 = 0;; t0 += NT) {
            const int tt = t0 + t;
            const bool fits = (cur + tt < ne) && (L.soff[3 * (cur + tt + 1)] - base <= HB);
            const int c1 = uniform_i(__syncthreads_count(fits));
            nfit += c1;
            if (c1 < NT) break;
        }
        if (nfit == 0) {
            // One event larger than LDS: wave 0 reads it from HBM.
            if (w == 0)
                wave_event<P>(c, ghits, 0, L.soff[3 * cur], L.soff[3 * cur + 1], L.soff[3 * cur + 2],
                              L.soff[3 * cur + 3], e0 + cur, counts, accept, status, px, py);
            __syncthreads();
            cur += 1;
            continue;
        }
        const int end = cur + nfit;
        const int nh = L.soff[3 * end] - base;
        const uint32_t mag = stage_hits<HB, NT>(x, y, base, nh, c.n_hits, vec, L.stage_x, L.stage_y);
        if constexpr (P::kMag) publish_mag(L, mag);
        block_descriptors(L, cur, nfit, base & ~3);
        block_count<P>(L, c, e0 + cur, nfit, counts, accept, status);
        cur = end;
    }
}

// Hits of one block held in registers between their load and their LDS
// store: the float4 groups of [a0, a0 + 4 nq) (a0 = base rounded down to a
// multiple of 4) that lie entirely below n_hits, loaded unconditionally
// (clamped), so that every load is in flight at once.  The rest (at most
// three hits below n_hits) is copied by thread 0 at the store.  The groups
// are named members (G<k> holds group k of this thread), not an array, so
// that they stay in registers across the pipeline loop.
typedef float f32x4 __attribute__((ext_vector_type(4)));  // a native vector (float4 copies are memcpys)

template <int K, int NT>
struct HitGroups {
    f32x4 vx, vy;
    HitGroups<K - 1, NT> rest;
    __device__ __forceinline__ void load(const float* __restrict__ x, const float* __restrict__ y, int a0,
                                         int nq_full) {
        const int q = min((int)threadIdx.x + (K - 1) * NT, nq_full - 1);
        vx = *reinterpret_cast<const f32x4*>(x + a0 + 4 * q);
        vy = *reinterpret_cast<const f32x4*>(y + a0 + 4 * q);
        rest.load(x, y, a0, nq_full);
    }
    // Returns the largest |x|, |y| of the groups (and m), as mag4 bits.
    __device__ __forceinline__ uint32_t store(int nq_full, float* xs, float* ys, uint32_t m) const {
        const int q = (int)threadIdx.x + (K - 1) * NT;
        if (q < nq_full) {
            reinterpret_cast<f32x4*>(xs)[q] = vx;
            reinterpret_cast<f32x4*>(ys)[q] = vy;
        }
        m = mag4(mag4(m, vx.x, vx.y, vx.z, vx.w), vy.x, vy.y, vy.z, vy.w);
        return rest.store(nq_full, xs, ys, m);
    }
};
template <int NT>
struct HitGroups<0, NT> {
    __device__ __forceinline__ void load(const float*, const float*, int, int) {}
    __device__ __forceinline__ uint32_t store(int, float*, float*, uint32_t m) const { return m; }
};

template <int HB, int NT>
struct HitPrefetch {
    // Blocks of at most kCap = HB - 4 hits: with base - a0 <= 3 they span at
    // most ceil((kCap + 3) / 4) = HB / 4 float4 groups (HB a multiple of 4),
    // so Q groups per thread hold them; larger blocks take the general path.
    static_assert(HB % 4 == 0, "block capacity a multiple of 4");
    static constexpr int kCap = HB - 4;
    static constexpr int Q = (HB / 4 + NT - 1) / NT;  // float4 groups per thread
    HitGroups<Q, NT> g;
    int nq_full;
    __device__ __forceinline__ void issue(const float* __restrict__ x, const float* __restrict__ y, int base,
                                          int nh, int n_hits) {
        nq_full = full_groups(base, nh, n_hits);
        if (nq_full > 0) g.load(x, y, base & ~3, nq_full);
    }
    // The float4 groups of [base, base + nh) that lie entirely below n_hits.
    __device__ static __forceinline__ int full_groups(int base, int nh, int n_hits) {
        const int a0 = base & ~3;
        return min((base + nh - a0 + 3) >> 2, (n_hits - a0) >> 2);
    }
    // issue() for a block known to have nq = full_groups(...) >= 1 (no branch).
    __device__ __forceinline__ void issue_full(const float* __restrict__ x, const float* __restrict__ y, int base,
                                               int nq) {
        nq_full = nq;
        g.load(x, y, base & ~3, nq);
    }
    // Stores the block's hits; returns the largest |x|, |y| this thread
    // stored (the groups of a block with nq_full <= 0 are not loaded: 0).
    __device__ __forceinline__ uint32_t store(const float* __restrict__ x, const float* __restrict__ y, int base,
                                              int nh, float* xs, float* ys) const {
        const int a0 = base & ~3;
        uint32_t m = nq_full > 0 ? g.store(nq_full, xs, ys, 0u) : 0u;
        if (threadIdx.x == 0)
            for (int h = a0 + 4 * max(nq_full, 0); h < base + nh; ++h) {
                xs[h - a0] = x[h];
                ys[h - a0] = y[h];
                m = mag4(m, x[h], y[h], 0.0f, 0.0f);
            }
        return m;
    }
};

// The block kernel (one block of eb <= EB consecutive events per workgroup;
// EB sizes the event table in LDS, and the registers are held to the waves
// per SIMD that this LDS allows).
// `vec`: x and y are 16-byte aligned (the pipelined kernel's same argument
// slot carries its claim chunk instead).  A block whose hits fit in LDS is
// staged whole: its hit loads are issued first, the events are checked and
// described while they are in flight, and one barrier later the counting
// starts.  Other blocks take the general path.
template <class P, int HB, int NW, int EB>
__global__ __launch_bounds__(NW * kWave) __attribute__((amdgpu_waves_per_eu(block_waves_per_simd<HB, NW, EB>())))
void k_block(const int32_t* __restrict__ off, int n_events,
                                                         const float* __restrict__ x,
                                                         const float* __restrict__ y, Consts c, int eb,
                                                         int n_blocks, unsigned* /*unused*/, int vec,
                                                         int32_t* __restrict__ counts,
                                                         uint8_t* __restrict__ accept, uint32_t* status) {
    __shared__ __align__(16) BlockLds<HB, NW, EB> L;
    constexpr int NT = NW * kWave;
    const int b = blockIdx.x;
    if (b >= n_blocks) return;
    const int e0 = b * eb;
    const int ne = min(eb, n_events - e0);
    // The block's offsets go out into registers first, then (the hit range
    // read by two scalar loads) its hits, so that neither waits for the
    // offsets to pass through LDS and a barrier; the offsets are stored
    // once they arrive, while the hits are still in flight.
    constexpr int OQ = (3 * EB + 1 + NT - 1) / NT;
    int ov[OQ];
#pragma unroll
    for (int k = 0; k < OQ; ++k) {
        const int q = (int)threadIdx.x + k * NT;
        ov[k] = off[3 * (int64_t)e0 + min(q, 3 * ne)];  // clamped: every load in range, no branch
    }
    const int base = uniform_i(off[3 * (int64_t)e0]), end = uniform_i(off[3 * (int64_t)(e0 + ne)]);
    using Prefetch = HitPrefetch<HB, NT>;
    const bool whole = vec && 0 <= base && base <= end && end <= c.n_hits && end - base <= Prefetch::kCap &&
                       Prefetch::full_groups(base, end - base, c.n_hits) > 0;
    auto stage_offsets = [&] {
#pragma unroll
        for (int k = 0; k < OQ; ++k) {
            const int q = (int)threadIdx.x + k * NT;
            if (q <= 3 * ne) L.soff[q] = ov[k];
        }
        if (threadIdx.x == 0) L.s_bad = 0;
        __syncthreads();
    };
    // The two sides share no code after the branch: where they joined, the
    // compiler could only wait for the offsets by waiting for every load,
    // the hits' included.
    if (whole) {
        Prefetch pf;
        pf.issue_full(x, y, base, Prefetch::full_groups(base, end - base, c.n_hits));
        stage_offsets();
        block_check_describe(L, c, e0, ne, base & ~3, counts, accept, status);
        const uint32_t mag = pf.store(x, y, base, end - base, L.stage_x, L.stage_y);
        if constexpr (P::kMag) publish_mag(L, mag);
        __syncthreads();
        const bool bad = uniform_i(L.s_bad) != 0;
        if (!bad)
            block_count<P>(L, c, e0, ne, counts, accept, status);
        else
            block_general<P>(L, c, x, y, e0, ne, true, vec != 0, counts, accept, status);
    } else {
        stage_offsets();
        block_check_describe(L, c, e0, ne, base & ~3, counts, accept, status);
        __syncthreads();
        block_general<P>(L, c, x, y, e0, ne, uniform_i(L.s_bad) != 0, vec != 0, counts, accept, status);
    }
}

// Persistent block kernel with a software pipeline: workgroups take chunks
// of `chunk` consecutive blocks from *block_counter (zero at launch; one
// atomic per chunk, each claimed one chunk ahead), and while a block is
// counted from LDS the next block's offsets have arrived and its hits are in
// flight into registers.  Blocks that are malformed or do not fit in LDS take
// the general path.  Needs x and y 16-byte aligned.
template <class P, int HB, int NW>
__global__ __launch_bounds__(NW * kWave) void k_block_pipe(const int32_t* __restrict__ off, int n_events,
                                                              const float* __restrict__ x,
                                                              const float* __restrict__ y, Consts c, int eb,
                                                              int n_blocks, unsigned* block_counter, int chunk,
                                                              int32_t* __restrict__ counts,
                                                              uint8_t* __restrict__ accept, uint32_t* status) {
    __shared__ __align__(16) BlockLds<HB, NW, kMaxEB> L;
    constexpr int NT = NW * kWave;
    const int t = (int)threadIdx.x;
    HitPrefetch<HB, NT> pf;
    // Prologue: claim two chunks, load the first block's offsets, prefetch its hits.
    if (t == 0) {
        L.s_block = (int)atomicAdd(block_counter, 1u);
        L.s_next = (int)atomicAdd(block_counter, 1u);
    }
    __syncthreads();
    // Block indices as int64 products: chunk * claims may pass int32 range.
    auto chunk_start = [&](int claimed) {
        return (int)min((int64_t)claimed * chunk, (int64_t)n_blocks);
    };
    int b = chunk_start(uniform_i(L.s_block));
    int cur_first = b;
    int cur_end = min(b + chunk, n_blocks);
    int next_first = chunk_start(uniform_i(L.s_next));
    if (b >= n_blocks) return;  // workgroup-uniform, before any further barrier
    {
        const int e0 = b * eb, ne = min(eb, n_events - e0);
        for (int q = t; q <= 3 * ne; q += NT) L.soff[q] = off[3 * (int64_t)e0 + q];
    }
    __syncthreads();
    int pf_ok;  // the hits of block b are in pf
    {
        const int ne = min(eb, n_events - b * eb);
        const int base = L.soff[0], end = L.soff[3 * ne];
        pf_ok = (0 <= base && base <= end && end <= c.n_hits && end - base <= HitPrefetch<HB, NT>::kCap);
        if (pf_ok) pf.issue(x, y, base, end - base, c.n_hits);
    }
    for (;;) {
        const int e0 = b * eb;
        const int ne = min(eb, n_events - e0);
        // At a chunk's first block, claim the chunk after the next one.
        const bool first_of_chunk = b == cur_first;
        unsigned claim = 0;
        if (first_of_chunk && t == 0) claim = atomicAdd(block_counter, 1u);
        const int bn = b + 1 < cur_end ? b + 1 : next_first;
        // Offsets of the next block: issued now, stored after this block's descriptors.
        constexpr int OQ = (3 * kMaxEB + 1 + NT - 1) / NT;
        int on[OQ];
        const bool has_next = bn < n_blocks;
        const int e0n = bn * eb;
        const int nen = has_next ? min(eb, n_events - e0n) : 0;
#pragma unroll
        for (int k = 0; k < OQ; ++k) {
            const int q = t + k * NT;
            on[k] = (has_next && q <= 3 * nen) ? off[3 * (int64_t)e0n + q] : 0;
        }
        const bool bad = block_validate(L, c, e0, ne, counts, accept, status);
        const bool regular = !bad && pf_ok;
        if (regular) {
            const int base = L.soff[0];
            const int nh = L.soff[3 * ne] - base;
            const uint32_t mag = pf.store(x, y, base, nh, L.stage_x, L.stage_y);
            if constexpr (P::kMag) publish_mag(L, mag);
            block_descriptors(L, 0, ne, base & ~3);
        } else {
            block_general<P>(L, c, x, y, e0, ne, bad, true, counts, accept, status);
        }
        // L.soff is free: the next block's offsets, then its hits in flight.
#pragma unroll
        for (int k = 0; k < OQ; ++k) {
            const int q = t + k * NT;
            if (has_next && q <= 3 * nen) L.soff[q] = on[k];
        }
        if (first_of_chunk && t == 0) L.s_next = (int)claim;
        __syncthreads();
        if (has_next) {
            const int base = L.soff[0], end = L.soff[3 * nen];
            pf_ok = (0 <= base && base <= end && end <= c.n_hits && end - base <= HitPrefetch<HB, NT>::kCap);
            if (pf_ok) pf.issue(x, y, base, end - base, c.n_hits);
        }
        const int claimed = uniform_i(L.s_next);  // valid after a first block's barrier above
        if (regular) block_count<P>(L, c, e0, ne, counts, accept, status);
        if (!has_next) break;
        if (b + 1 >= cur_end) {
            // Move on to the next chunk; the one after it was claimed at
            // this chunk's first block (or in the prologue).
            cur_first = next_first;
            cur_end = min(next_first + chunk, n_blocks);
            next_first = chunk_start(claimed);
        }
        b = bn;
    }
}

}  // namespace trig
