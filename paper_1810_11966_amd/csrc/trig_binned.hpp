// Slope-cell binned selection (the binned form) for high-multiplicity events.
//
// The count is the brute-force one (paper Sec. 3.2 steps 1-3) in the binary32
// contract of include/trig.h.  Instead of scanning every (i, j) pair, each
// layer-1 hit is put into a cell by a key that is proportional to its slope
// x/z, and each layer-0 hit looks only at the cells that can hold a partner:
//
//   MSD tests: a triplet passes only if |a| <= A in both planes and
//     |b| <= B in the x-z plane (see the batched form; MSD_BASIS: A = B = beta,
//     MSD: A = a0 + a1 M and B = b0 + b1 M with M the event's largest layer-1
//     |x|, |y|), a = f32(u + v) with u = f32(U0 x_i), v = f32(U1 x_j).  As
//     binary32 rounding is monotone and A_up >= next float above A,
//     |f32(u + v)| <= A implies -A_up < u + v < A_up in real numbers,
//     so v lies in (-u - A_up, -u + A_up).  The layer-1 key is v.  In
//     the same way b = f32(p + w_k) with p = f32(V0 x_i + V1 x_j) and
//     w_k = f32(V2 x_k) needs w_k in (-p - B_up, -p + B_up); the
//     layer-2 key is w_k.
//   window test: |f32(s_j - s_i)| < W implies |s_j - s_i| < W (W is a binary32
//     value), so s_j lies in (s_i - W, s_i + W); the same for s_k.  Here the
//     layer-2 condition depends on i alone, so an i's count is the product of
//     its numbers of layer-1 and layer-2 partners.
//
// The interval ends are rounded outwards (by at least one binary32 step
// past the rounded end point), and the cell of a key is a non-decreasing
// function of the key, so the cells from cell(lower end) to cell(upper end)
// contain every key in the interval whatever the cell width.  Every
// candidate then gets the full binary32 test, so the count is exact; a hit
// whose key is not finite can never pass (its a or b is infinite or NaN) and
// is left out.
//
// One wave per event.  Cells are built in LDS with a counting sort (histogram
// of the cell indices, exclusive scan, scatter); events with more than
// kBinCap hits in layer 1 or 2 take the batched form's pair-pruned path from
// HBM instead.
#pragma once

#include "trig_block.hpp"
#include "trig_device.hpp"

namespace trig {

constexpr int kBinCap = 256;            // layer-1 / layer-2 hits per event in LDS
constexpr int kBinRounds = kBinCap / kWave;

// f moved outwards by d = f32(f32(|f| 2^-22) + 2^-126), at least one binary32
// step for any finite f (a step is at most 2^-23 |f| for normal f and 2^-149
// below), so that the result lies beyond every real number that rounds to f
// (those lie within 2^-24 |f| + 2^-150 of it): the rounding of the sum and
// of the final subtraction stay far below the slack d leaves.  Infinities
// stay infinite (+inf - inf is NaN, which the cell function maps to cell 0:
// still a superset).  Three vector instructions, no branch.
__device__ __forceinline__ float widen_down(float f) {
    return f - (__builtin_fabsf(f) * 0x1p-22f + 0x1p-126f);
}
__device__ __forceinline__ float widen_up(float f) {
    return f + (__builtin_fabsf(f) * 0x1p-22f + 0x1p-126f);
}


// LDS of one wave: cell ends and the two payload floats per hit, in cell
// order, for layers 1 and 2.  Float arrays first (16-byte aligned: the
// fallback path reuses a1/b1 as its layer-0 buffers).  A cell end is at most
// kBinCap = 256, so the ends are 16-bit, two cells per 32-bit word (cell t in
// the half t & 1 of word t >> 1): 5 KB per wave, eight workgroups per CU.
struct BinLds {
    float a1[kBinCap], b1[kBinCap];
    float a2[kBinCap], b2[kBinCap];
    uint32_t end1[kBinCap / 2], end2[kBinCap / 2];
};
static_assert(kBinCap < 65536, "cell ends fit in 16 bits");

// Cell t's 16-bit entry of a packed end array.
__device__ __forceinline__ int cell_end(const uint32_t* end, int t) {
    return (int)reinterpret_cast<const uint16_t*>(end)[t];
}

// Cells over [kmin, kmax] of one layer.  cell(v) is non-decreasing in v
// (binary32 subtraction, multiplication and floor are monotone, the clamps
// too, and fmaxf maps a NaN to cell 0, as for every v when inv_w is 0).
struct Bins {
    float kmin, kmax, inv_w;
    int n_cells;
    __device__ __forceinline__ int cell(float v) const {
        const float t = __builtin_floorf((v - kmin) * inv_w);
        return (int)__builtin_fminf(__builtin_fmaxf(t, 0.0f), (float)(n_cells - 1));
    }
    // Index range [first, last) of the hits in cells cell(lo) .. cell(hi).
    __device__ __forceinline__ void range(const uint32_t* end, float lo, float hi, int& first, int& last) const {
        const int cl = cell(lo), ch = cell(hi);
        first = cl > 0 ? cell_end(end, cl - 1) : 0;
        last = cell_end(end, ch);
    }
};

// The hits [o, o + n) (1 <= n <= kBinCap) of one layer in registers, hit
// r kWave + lane in round r; the loads are issued together and unguarded
// (indices clamped to the layer), so that several layers can be in flight.
struct LayerRegs {
    float x[kBinRounds], y[kBinRounds];
    __device__ __forceinline__ void load(const float* __restrict__ xs, const float* __restrict__ ys, int o, int n) {
        const int lane = (int)lane_id();
#pragma unroll
        for (int r = 0; r < kBinRounds; ++r) {
            x[r] = y[r] = 0.0f;
            if (r * kWave < n) {  // wave-uniform: rounds past the layer are skipped
                const int t = min(r * kWave + lane, n - 1);
                x[r] = xs[o + t];
                y[r] = ys[o + t];
            }
        }
    }
};

// Counting sort of the n hits of one layer (held in h, n <= NR kWave) into
// cells of the key K::key, storing K::payload in cell order.  Whole wave.
template <class K, int NR>
__device__ Bins build_bins_r(const Consts& c, const LayerRegs& h, int n, uint32_t* end, float* pa, float* pb) {
    const int lane = (int)lane_id();
    float key[NR];
    float2 pay[NR];
    float lo = __builtin_inff(), hi = -__builtin_inff();
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int t = r * kWave + lane;
        key[r] = __builtin_nanf("");
        if (t < n) {
            key[r] = K::key(c, h.x[r], h.y[r]);
            pay[r] = K::payload(c, h.x[r], h.y[r]);
        }
        if (__builtin_isfinite(key[r])) {
            lo = __builtin_fminf(lo, key[r]);
            hi = __builtin_fmaxf(hi, key[r]);
        } else {
            key[r] = __builtin_nanf("");  // left out below
        }
    }
    Bins b;
    b.kmin = wave_min_f(lo);
    b.kmax = wave_max_f(hi);
    int nc = 64;
    while (nc < n) nc <<= 1;  // power of two >= n, at most kBinCap
    b.n_cells = uniform_i(nc);
    const float width = b.kmax - b.kmin;
    // Any non-negative scale keeps cell() monotone; the hardware reciprocal
    // is enough to spread the keys over the cells.
    b.inv_w = (width > 0.0f && width < __builtin_inff()) ? __builtin_amdgcn_rcpf(width) * (float)b.n_cells : 0.0f;
    for (int t = lane; t < b.n_cells / 2; t += kWave) end[t] = 0u;
    wave_lds_sync();
    // Histogram: cell t counts in the half t & 1 of word t >> 1 (a half
    // never exceeds kBinCap, so no carry reaches the other half).
    int cell[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        cell[r] = -1;
        if (!__builtin_isnan(key[r])) {
            cell[r] = b.cell(key[r]);
            atomicAdd(&end[cell[r] >> 1], 1u << (16 * (cell[r] & 1)));
        }
    }
    wave_lds_sync();
    // Exclusive scan of the cell sizes: lane L owns cells [L*per, L*per + per)
    // (per = 1, 2 or 4), read and written with one access per lane
    // (consecutive lanes, consecutive addresses: no bank conflicts).
    static_assert(kBinCap <= 4 * kWave, "at most four cells per lane");
    const int per = b.n_cells / kWave;  // n_cells is a multiple of 64
    int4 sz = make_int4(0, 0, 0, 0);
    if (per == 4) {
        const uint2 v = reinterpret_cast<const uint2*>(end)[lane];
        sz = make_int4((int)(v.x & 0xFFFFu), (int)(v.x >> 16), (int)(v.y & 0xFFFFu), (int)(v.y >> 16));
    } else if (per == 2) {
        const uint32_t v = end[lane];
        sz = make_int4((int)(v & 0xFFFFu), (int)(v >> 16), 0, 0);
    } else {
        sz.x = cell_end(end, lane);
    }
    const int local = (sz.x + sz.y) + (sz.z + sz.w);
    const int s0 = wave_inclusive_sum(local) - local;  // starts of the lane's cells
    const int4 st = make_int4(s0, s0 + sz.x, s0 + sz.x + sz.y, s0 + sz.x + sz.y + sz.z);
    if (per == 4)
        reinterpret_cast<uint2*>(end)[lane] =
            make_uint2((uint32_t)st.x | ((uint32_t)st.y << 16), (uint32_t)st.z | ((uint32_t)st.w << 16));
    else if (per == 2)
        end[lane] = (uint32_t)st.x | ((uint32_t)st.y << 16);
    else
        reinterpret_cast<uint16_t*>(end)[lane] = (uint16_t)st.x;
    wave_lds_sync();
    // Scatter; afterwards cell t's entry is the end of cell t.
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        if (cell[r] >= 0) {
            const int sh = 16 * (cell[r] & 1);
            const int pos = (int)((atomicAdd(&end[cell[r] >> 1], 1u << sh) >> sh) & 0xFFFFu);
            pa[pos] = pay[r].x;
            pb[pos] = pay[r].y;
        }
    }
    wave_lds_sync();
    return b;
}

// build_bins_r with the fewest rounds that hold the layer (1, 2 or 4 times
// kWave hits; n <= kBinCap).
template <class K>
__device__ __forceinline__ Bins build_bins(const Consts& c, const LayerRegs& h, int n, uint32_t* end, float* pa,
                                           float* pb) {
    static_assert(kBinRounds == 4, "round counts 1, 2 and 4");
    if (n <= kWave) return build_bins_r<K, 1>(c, h, n, end, pa, pb);
    if (n <= 2 * kWave) return build_bins_r<K, 2>(c, h, n, end, pa, pb);
    return build_bins_r<K, 4>(c, h, n, end, pa, pb);
}

// Bounds of one event: pair test |a_x| <= bx, |a_y| <= by (window: strict,
// with the windows), and the half-widths r1, r2 of the layer-1 and layer-2
// key intervals, each at least the next binary32 value above its bound.
struct BinBounds {
    float bx, by, r1, r2;
};

// ---------------------------------------------------------------- MSD ---

// TRIG_TEST_MSD_BASIS.
struct MsdBasisBin {
    using Prune = MsdBasisPrune;
    static constexpr bool kMag = false;
    __device__ static __forceinline__ BinBounds bounds(const Consts& c, float) {
        return BinBounds{c.beta_x, c.beta_y, c.bin_r, c.bin_r};
    }
    struct Key1 {  // layer 1: key U1 x, payload (x, y)
        __device__ static __forceinline__ float key(const Consts& c, float x, float) { return c.U1 * x; }
        __device__ static __forceinline__ float2 payload(const Consts&, float x, float y) {
            return make_float2(x, y);
        }
    };
    struct Key2 {  // layer 2: key V2 x, payload (V2 x, V2 y)
        __device__ static __forceinline__ float key(const Consts& c, float x, float) { return c.V2 * x; }
        __device__ static __forceinline__ float2 payload(const Consts& c, float x, float y) {
            return make_float2(c.V2 * x, c.V2 * y);
        }
    };
    // Passing triplets with layer-0 hit (xi, yi).
    __device__ static uint32_t count_i(const Consts& c, const BinBounds& bb, float xi, float yi, const Bins& b1,
                                       const Bins& b2, const BinLds& L) {
        const float ux = c.U0 * xi;
        const float r = bb.r1;
        if (!__builtin_isfinite(ux)) return 0;
        const float lo = widen_down(-ux - r), hi = widen_up(-ux + r);
        if (hi < b1.kmin || lo > b1.kmax) return 0;
        int j0, j1;
        b1.range(L.end1, lo, hi, j0, j1);
        uint32_t cnt = 0;
        for (int j = j0; j < j1; ++j) {
            const float xj = L.a1[j], yj = L.b1[j];
            const float ax = c.U0 * xi + c.U1 * xj;
            const float ay = c.U0 * yi + c.U1 * yj;
            if (!(__builtin_fabsf(ax) <= bb.bx && __builtin_fabsf(ay) <= bb.by)) continue;
            const float ax2 = ax * ax, ay2 = ay * ay;
            const float bx0 = c.V0 * xi + c.V1 * xj;
            const float by0 = c.V0 * yi + c.V1 * yj;
            if (!__builtin_isfinite(bx0)) continue;
            const float lo2 = widen_down(-bx0 - bb.r2), hi2 = widen_up(-bx0 + bb.r2);
            if (hi2 < b2.kmin || lo2 > b2.kmax) continue;
            int k0, k1;
            b2.range(L.end2, lo2, hi2, k0, k1);
            for (int k = k0; k < k1; ++k) {
                const float bx = bx0 + L.a2[k];
                const float qx = ax2 + bx * bx;
                const float by = by0 + L.b2[k];
                const float qy = ay2 + by * by;
                cnt += (uint32_t)((qx <= c.qmax_x) & (qy <= c.qmax_y));
            }
        }
        return cnt;
    }
};

// TRIG_TEST_MSD: cells and pair test from the written-out fit's bounds
// (a0 + a1 M, b0 + b1 M), candidates completed with the fit written out.
// A pair whose b partial is infinite has no passing triplet: with
// M = |x_j| (finite for a hit in a cell) the bound on |b| is finite.
struct MsdFitBin {
    using Prune = MsdFitPrune;
    static constexpr bool kMag = true;
    __device__ static __forceinline__ BinBounds bounds(const Consts& c, float M) {
        // 1 + 2^-20: fl(A (1 + 2^-20)) >= A (1 + 2^-23), above the next
        // binary32 value after any A >= 2^-126 (the bounds are normal)
        constexpr float kUp = 1.00000095367431640625f;
        const float bx = c.fit_a0x + c.fit_a1x * M;
        const float by = c.fit_a0y + c.fit_a1y * M;
        const float B = c.fit_b0x + c.fit_b1x * M;
        return BinBounds{bx, by, bx * kUp, B * kUp};
    }
    struct Key1 {  // layer 1: key U1 x, payload (x, y)
        __device__ static __forceinline__ float key(const Consts& c, float x, float) { return c.U1 * x; }
        __device__ static __forceinline__ float2 payload(const Consts&, float x, float y) {
            return make_float2(x, y);
        }
    };
    struct Key2 {  // layer 2: key V2 x, payload (x, y)
        __device__ static __forceinline__ float key(const Consts& c, float x, float) { return c.V2 * x; }
        __device__ static __forceinline__ float2 payload(const Consts&, float x, float y) {
            return make_float2(x, y);
        }
    };
    __device__ static uint32_t count_i(const Consts& c, const BinBounds& bb, float xi, float yi, const Bins& b1,
                                       const Bins& b2, const BinLds& L) {
        const float ux = c.U0 * xi;
        if (!__builtin_isfinite(ux)) return 0;  // x_i not finite: the fit fails
        const float lo = widen_down(-ux - bb.r1), hi = widen_up(-ux + bb.r1);
        if (hi < b1.kmin || lo > b1.kmax) return 0;
        int j0, j1;
        b1.range(L.end1, lo, hi, j0, j1);
        const float pxi = xi * c.z0, pyi = yi * c.z0;
        uint32_t cnt = 0;
        for (int j = j0; j < j1; ++j) {
            const float xj = L.a1[j], yj = L.b1[j];
            const float ax = c.U0 * xi + c.U1 * xj;
            const float ay = c.U0 * yi + c.U1 * yj;
            if (!(__builtin_fabsf(ax) <= bb.bx && __builtin_fabsf(ay) <= bb.by)) continue;
            const float bx0 = c.V0 * xi + c.V1 * xj;
            if (!__builtin_isfinite(bx0)) continue;
            const float lo2 = widen_down(-bx0 - bb.r2), hi2 = widen_up(-bx0 + bb.r2);
            if (hi2 < b2.kmin || lo2 > b2.kmax) continue;
            int k0, k1;
            b2.range(L.end2, lo2, hi2, k0, k1);
            const float sx01 = pxi + xj * c.z1;
            const float sy01 = pyi + yj * c.z1;
            for (int k = k0; k < k1; ++k) {
                const float xk = L.a2[k], yk = L.b2[k];
                const float qx = MsdFitTest::plane_q(c, xi, xj, sx01, xk, xk * c.z2);
                const float qy = MsdFitTest::plane_q(c, yi, yj, sy01, yk, yk * c.z2);
                cnt += (uint32_t)((qx <= c.qmax_x) & (qy <= c.qmax_y));
            }
        }
        return cnt;
    }
};

// ------------------------------------------------------------- window ---

struct WindowBin {
    using Prune = WindowPrune;
    static constexpr bool kMag = false;
    __device__ static __forceinline__ BinBounds bounds(const Consts& c, float) {
        return BinBounds{c.win_x, c.win_y, c.bin_r, c.bin_r};
    }
    struct Key1 {  // layer 1: slopes (x / z1, y / z1), key the x slope
        __device__ static __forceinline__ float key(const Consts& c, float x, float) { return x / c.z1; }
        __device__ static __forceinline__ float2 payload(const Consts& c, float x, float y) {
            return make_float2(x / c.z1, y / c.z1);
        }
    };
    struct Key2 {
        __device__ static __forceinline__ float key(const Consts& c, float x, float) { return x / c.z2; }
        __device__ static __forceinline__ float2 payload(const Consts& c, float x, float y) {
            return make_float2(x / c.z2, y / c.z2);
        }
    };
    __device__ static uint32_t count_i(const Consts& c, const BinBounds& bb, float xi, float yi, const Bins& b1,
                                       const Bins& b2, const BinLds& L) {
        const float sxi = xi / c.z0, syi = yi / c.z0;
        if (!__builtin_isfinite(sxi)) return 0;
        const float lo = widen_down(sxi - bb.r1), hi = widen_up(sxi + bb.r1);
        uint32_t nj = 0, nk = 0;
        if (!(hi < b1.kmin || lo > b1.kmax)) {
            int j0, j1;
            b1.range(L.end1, lo, hi, j0, j1);
            for (int j = j0; j < j1; ++j)
                nj += (uint32_t)((__builtin_fabsf(L.a1[j] - sxi) < c.win_x) &
                                 (__builtin_fabsf(L.b1[j] - syi) < c.win_y));
        }
        if (nj == 0 || hi < b2.kmin || lo > b2.kmax) return 0;
        int k0, k1;
        b2.range(L.end2, lo, hi, k0, k1);
        for (int k = k0; k < k1; ++k)
            nk += (uint32_t)((__builtin_fabsf(L.a2[k] - sxi) < c.win_x) &
                             (__builtin_fabsf(L.b2[k] - syi) < c.win_y));
        return nj * nk;
    }
};

// Passing triplets of one event with 1 <= n0 and 1 <= n1, n2 <= kBinCap,
// hits straight from HBM (x, y absolute arrays).  Whole wave; the same count
// on every lane.
template <class B>
__device__ uint32_t wave_event_binned(const Consts& c, const float* __restrict__ x, const float* __restrict__ y,
                                      int o0, int n0, int o1, int n1, int o2, int n2, BinLds& L) {
    // The loads of layers 1 and 2 and of layer 0's first round in flight at
    // once (one HBM latency, not three); later layer-0 rounds are loaded one
    // round ahead.  Indices are clamped to the layers (n0, n1, n2 >= 1).
    const int lane = (int)lane_id();
    LayerRegs h1, h2;
    h1.load(x, y, o1, n1);
    h2.load(x, y, o2, n2);
    float xi = x[o0 + min(lane, n0 - 1)], yi = y[o0 + min(lane, n0 - 1)];
    float M = 0.0f;  // largest layer-1 |x|, |y| (rounds past the layer hold 0 or a layer-1 hit)
    if constexpr (B::kMag) {
        uint32_t m = 0u;
#pragma unroll
        for (int r = 0; r < kBinRounds; ++r)
            if (r * kWave < n1) m = max(m, max(abs_bits(h1.x[r]), abs_bits(h1.y[r])));
        M = wave_max_f(mag_of(m));
    }
    const BinBounds bb = B::bounds(c, M);
    const Bins b1 = build_bins<typename B::Key1>(c, h1, n1, L.end1, L.a1, L.b1);
    const Bins b2 = build_bins<typename B::Key2>(c, h2, n2, L.end2, L.a2, L.b2);
    uint32_t cnt = 0;
    for (int i0 = 0; i0 < n0; i0 += kWave) {
        float xn = 0.0f, yn = 0.0f;
        if (i0 + kWave < n0) {  // wave-uniform
            const int in = min(i0 + kWave + lane, n0 - 1);
            xn = x[o0 + in];
            yn = y[o0 + in];
        }
        if (i0 + lane < n0) cnt += B::count_i(c, bb, xi, yi, b1, b2, L);
        xi = xn;
        yi = yn;
        // decision only: stop once the (capped) result is known
        if (c.count_cap != INT32_MAX && i0 + kWave < n0 && wave_sum_u(cnt) >= (uint32_t)c.count_cap) break;
    }
    cnt = wave_sum_u(cnt);
    wave_lds_sync();  // the next event rebuilds the cells
    return cnt;
}

}  // namespace trig
