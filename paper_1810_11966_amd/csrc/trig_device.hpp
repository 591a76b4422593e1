// Device-side building blocks of the trigger-station triplet selection:
// per-plane test policies, per-event CSR loading and the wave-level triplet
// loop shared by the plain and the persistent kernels.
//
// Method: paper Sec. 3.2 "Algorithm" - all one-hit-per-layer triplets (step
// 1), straight-line fit through the vertex in x-z and y-z and a cut on its
// mean square deviation per degree of freedom (step 2), event selected with at
// least two passing triplets (step 3).  The binary32 operation order is the
// one fixed in include/trig.h; this file must be compiled with
// -ffp-contract=off and without flushing fp32 subnormals.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace trig {

constexpr int kWave = 64;

// Everything a kernel needs from the parameters, derived on the host
// (csrc/trig_bounds.hpp holds the derivations).
struct Consts {
    // Orthonormal basis of the plane orthogonal to (z0, z1, z2): the
    // TRIG_TEST_MSD_BASIS evaluation, and the partial sums a, b that the
    // pruned and binned forms of both MSD tests look at
    float U0, U1, V0, V1, V2;
    // TRIG_TEST_MSD (the fit written out): layer positions and w = 1 / sum z^2
    float z0, z1, z2, w;
    // MSD tests: largest binary32 Q with f32(Q / ndf) <= msd_max, per plane
    float qmax_x, qmax_y;
    // TRIG_TEST_MSD_BASIS pair bound: largest binary32 b >= 0 with
    // f32(b * b) <= qmax, per plane
    float beta_x, beta_y;
    // Per-hit z, pruned form: a triplet that passes a plane has
    // |f32(s_j - s_i)| <= (a0 + a1 M) / zmin for the hits' slopes s = c / z
    // (M >= |c_i|, |c_j|, zmin <= z_i, z_j), per plane
    float zs_a0x, zs_a1x, zs_a0y, zs_a1y;
    // TRIG_TEST_MSD: a triplet that passes a plane has |a| <= a0 + a1 M and
    // |b| <= b0 + b1 M (device evaluation order, M >= |c1| the plane's
    // layer-1 coordinate), per plane for a, x-z plane for b
    float fit_a0x, fit_a1x, fit_a0y, fit_a1y, fit_b0x, fit_b1x;
    // Pair prefilter of the batched form: (|u| <= bx and |v| <= by) implies
    // max(|u|, |v|) <= max(bx, by).  MSD_BASIS: the larger beta; window: the
    // larger window.
    float pre_msd, pre_win;
    // TRIG_TEST_SLOPE_WINDOW
    float win_x, win_y;
    // Binned form, MSD_BASIS and window: half-width of the key interval
    // around a hit's centre (MSD_BASIS: the binary32 value above beta_x;
    // window: win_x).
    float bin_r;
    // accept iff count >= min_triplets (two-particle mode: the candidates,
    // count >= 2)
    int32_t min_triplets;
    // counts are written as min(count, count_cap) (INT32_MAX unless the
    // caller asked for the decision only); an event's search may stop once
    // its count reaches the cap
    int32_t count_cap;
    int32_t n_hits;
};

// The count an event's result holds (errors, negative, unchanged).
__device__ __forceinline__ int32_t capped(int32_t cnt, const Consts& c) { return cnt < c.count_cap ? cnt : c.count_cap; }

__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }
// cond ? a : b for wave-uniform operands, on the scalar unit (a compare
// and a scalar select; the compiler would otherwise select per lane).
__device__ __forceinline__ float select_uniform(int cond, float a, float b) {
    const int c = uniform_i(cond);
    const int ia = uniform_i(__builtin_bit_cast(int, a)), ib = uniform_i(__builtin_bit_cast(int, b));
    int r;
    asm("s_cmp_lg_u32 %1, 0\n\ts_cselect_b32 %0, %2, %3" : "=s"(r) : "s"(c), "s"(ia), "s"(ib) : "scc");
    return __builtin_bit_cast(float, r);
}

__device__ __forceinline__ unsigned lane_id() { return threadIdx.x & (kWave - 1); }

// Order this wave's LDS writes before its later LDS reads, and its reads
// before later writes, across lanes of the wave.  The LDS performs one
// wave's operations in issue order, so nothing has to drain (no s_waitcnt:
// the LDS counter only orders LDS against other memory and other waves);
// only the compiler must be kept from moving memory operations across.
// Global loads in flight, such as the next block's prefetch, keep flying.
__device__ __forceinline__ void wave_lds_sync() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
}

// Number of lanes of the wave with pred set (the lane mask goes straight to
// scalar registers: one compare per predicate, popcount on the scalar unit).
__device__ __forceinline__ uint32_t wave_popc(bool pred) {
    return (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(pred));
}

__device__ __forceinline__ bool wave_any(bool pred) { return __builtin_amdgcn_ballot_w64(pred) != 0ull; }

// Cross-lane steps on the vector unit (DPP, gfx9 controls) for whole-wave
// code (all 64 lanes active).  dpp_i<C, ROWS>(old, v): lanes of the rows of 16
// in the mask ROWS take v from the lane that control C names; other lanes,
// and lanes whose source lies outside their row, keep `old`.
constexpr int kDppQuadXor1 = 0xB1;     // quad_perm [1, 0, 3, 2]
constexpr int kDppQuadXor2 = 0x4E;     // quad_perm [2, 3, 0, 1]
constexpr int kDppRowShr = 0x110;      // row_shr:n = kDppRowShr + n
constexpr int kDppRowMirror = 0x140;   // lane i of a row takes lane 15 - i
constexpr int kDppHalfMirror = 0x141;  // lane i of a half row takes lane 7 - i
constexpr int kDppBcast15 = 0x142;     // with rows 0xA: rows 1, 3 take lane 15 of the row before
constexpr int kDppBcast31 = 0x143;     // with rows 0xC: rows 2, 3 take lane 31

template <int C, int ROWS = 0xF>
__device__ __forceinline__ int dpp_i(int old, int v) {
    return __builtin_amdgcn_update_dpp(old, v, C, ROWS, 0xF, false);
}
template <int C, int ROWS = 0xF>
__device__ __forceinline__ float dpp_f(float old, float v) {
    return __builtin_bit_cast(float, dpp_i<C, ROWS>(__builtin_bit_cast(int, old), __builtin_bit_cast(int, v)));
}

// Wave-wide min, max and sum (result in every lane's return value, taken
// from lane 63): butterflies within quads, mirrors within rows of 16 (every
// lane then holds its row's result), then the row broadcasts carry rows 0-2
// into row 3.  fminf/fmaxf drop NaN as the scalar functions do.
__device__ __forceinline__ float wave_min_f(float v) {
    v = __builtin_fminf(v, dpp_f<kDppQuadXor1>(v, v));
    v = __builtin_fminf(v, dpp_f<kDppQuadXor2>(v, v));
    v = __builtin_fminf(v, dpp_f<kDppHalfMirror>(v, v));
    v = __builtin_fminf(v, dpp_f<kDppRowMirror>(v, v));
    v = __builtin_fminf(v, dpp_f<kDppBcast15, 0xA>(v, v));
    v = __builtin_fminf(v, dpp_f<kDppBcast31, 0xC>(v, v));
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}
__device__ __forceinline__ float wave_max_f(float v) {
    v = __builtin_fmaxf(v, dpp_f<kDppQuadXor1>(v, v));
    v = __builtin_fmaxf(v, dpp_f<kDppQuadXor2>(v, v));
    v = __builtin_fmaxf(v, dpp_f<kDppHalfMirror>(v, v));
    v = __builtin_fmaxf(v, dpp_f<kDppRowMirror>(v, v));
    v = __builtin_fmaxf(v, dpp_f<kDppBcast15, 0xA>(v, v));
    v = __builtin_fmaxf(v, dpp_f<kDppBcast31, 0xC>(v, v));
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}
__device__ __forceinline__ uint32_t wave_sum_u(uint32_t v) {
    int x = (int)v;
    x += dpp_i<kDppQuadXor1>(0, x);
    x += dpp_i<kDppQuadXor2>(0, x);
    x += dpp_i<kDppHalfMirror>(0, x);
    x += dpp_i<kDppRowMirror>(0, x);
    x += dpp_i<kDppBcast15, 0xA>(0, x);
    x += dpp_i<kDppBcast31, 0xC>(0, x);
    return (uint32_t)__builtin_amdgcn_readlane(x, 63);
}
// Inclusive prefix sum over the lanes: shifts by 1, 2, 4, 8 within rows
// (lanes without a source add 0), then the row broadcasts add the totals of
// the rows before.
__device__ __forceinline__ int wave_inclusive_sum(int x) {
    x += dpp_i<kDppRowShr + 1>(0, x);
    x += dpp_i<kDppRowShr + 2>(0, x);
    x += dpp_i<kDppRowShr + 4>(0, x);
    x += dpp_i<kDppRowShr + 8>(0, x);
    x += dpp_i<kDppBcast15, 0xA>(0, x);
    x += dpp_i<kDppBcast31, 0xC>(0, x);
    return x;
}

// Lane mask of a single comparison.  Combining two comparisons with a scalar
// AND of their masks (rather than a ballot of `a & b`) keeps each predicate a
// plain vector compare writing scalar registers.
__device__ __forceinline__ uint64_t lanes(bool cmp) { return __builtin_amdgcn_ballot_w64(cmp); }

// ----------------------------------------------------------------------------
// Test policies.  HF = floats staged in LDS per layer-2 hit; Pair = the part
// of the test that depends on (i, j) only; pass() completes it with hit k and
// returns the mask of lanes whose triplet passes.
// Staged padding and invalid pairs are NaN, which fails every comparison.
// ----------------------------------------------------------------------------

// TRIG_TEST_MSD_BASIS: Q = a^2 + b^2 in the basis (u, v).
struct MsdBasisTest {
    static constexpr int HF = 2;
    static constexpr bool kZ = false;  // layer positions from the parameters
    struct Pair {
        float ax2, bx0, ay2, by0;
    };
    __device__ static __forceinline__ void stage(const Consts& c, float x, float y, float* h) {
        h[0] = c.V2 * x;
        h[1] = c.V2 * y;
    }
    __device__ static __forceinline__ void pad(float* h) {
        h[0] = __builtin_nanf("");
        h[1] = __builtin_nanf("");
    }
    __device__ static __forceinline__ Pair pair(const Consts& c, float xi, float yi, float xj,
                                                float yj) {
        Pair p;
        const float ax = c.U0 * xi + c.U1 * xj;
        const float ay = c.U0 * yi + c.U1 * yj;
        p.ax2 = ax * ax;
        p.ay2 = ay * ay;
        p.bx0 = c.V0 * xi + c.V1 * xj;
        p.by0 = c.V0 * yi + c.V1 * yj;
        return p;
    }
    __device__ static __forceinline__ Pair invalid() {
        const float n = __builtin_nanf("");
        return Pair{n, n, n, n};
    }
    __device__ static __forceinline__ uint64_t pass(const Consts& c, const Pair& p, const float* h) {
        const float bx = p.bx0 + h[0];
        const float qx = p.ax2 + bx * bx;
        const float by = p.by0 + h[1];
        const float qy = p.ay2 + by * by;
        return lanes(qx <= c.qmax_x) & lanes(qy <= c.qmax_y);
    }
};

// TRIG_TEST_MSD: the fit through the vertex written out (slope, residuals,
// their sum of squares), the paper's definition of the test.
struct MsdFitTest {
    static constexpr int HF = 4;
    static constexpr bool kZ = false;  // layer positions from the parameters
    struct Pair {
        float xi, xj, sx01, yi, yj, sy01;
    };
    __device__ static __forceinline__ void stage(const Consts& c, float x, float y, float* h) {
        h[0] = x;
        h[1] = y;
        h[2] = x * c.z2;
        h[3] = y * c.z2;
    }
    __device__ static __forceinline__ void pad(float* h) {
        const float n = __builtin_nanf("");
        h[0] = n; h[1] = n; h[2] = n; h[3] = n;
    }
    __device__ static __forceinline__ Pair pair(const Consts& c, float xi, float yi, float xj,
                                                float yj) {
        Pair p;
        p.xi = xi; p.xj = xj; p.yi = yi; p.yj = yj;
        p.sx01 = xi * c.z0 + xj * c.z1;
        p.sy01 = yi * c.z0 + yj * c.z1;
        return p;
    }
    __device__ static __forceinline__ Pair invalid() {
        const float n = __builtin_nanf("");
        return Pair{n, n, n, n, n, n};
    }
    __device__ static __forceinline__ float plane_q(const Consts& c, float ci, float cj, float s01,
                                                    float ck, float pk) {
        const float m = (s01 + pk) * c.w;
        const float r0 = ci - m * c.z0;
        const float r1 = cj - m * c.z1;
        const float r2 = ck - m * c.z2;
        return (r0 * r0 + r1 * r1) + r2 * r2;
    }
    __device__ static __forceinline__ uint64_t pass(const Consts& c, const Pair& p, const float* h) {
        const float qx = plane_q(c, p.xi, p.xj, p.sx01, h[0], h[2]);
        const float qy = plane_q(c, p.yi, p.yj, p.sy01, h[1], h[3]);
        return lanes(qx <= c.qmax_x) & lanes(qy <= c.qmax_y);
    }
};

struct WindowTest {
    static constexpr int HF = 2;
    static constexpr bool kZ = false;  // layer positions from the parameters
    struct Pair {
        float sxi, syi;  // NaN when the layer-1 window already fails
    };
    __device__ static __forceinline__ void stage(const Consts& c, float x, float y, float* h) {
        h[0] = x / c.z2;
        h[1] = y / c.z2;
    }
    __device__ static __forceinline__ void pad(float* h) {
        h[0] = __builtin_nanf("");
        h[1] = __builtin_nanf("");
    }
    __device__ static __forceinline__ Pair pair(const Consts& c, float xi, float yi, float xj,
                                                float yj) {
        const float sxi = xi / c.z0, syi = yi / c.z0;
        const float sxj = xj / c.z1, syj = yj / c.z1;
        const bool ok = (__builtin_fabsf(sxj - sxi) < c.win_x) & (__builtin_fabsf(syj - syi) < c.win_y);
        const float n = __builtin_nanf("");
        return Pair{ok ? sxi : n, ok ? syi : n};
    }
    __device__ static __forceinline__ Pair invalid() {
        const float n = __builtin_nanf("");
        return Pair{n, n};
    }
    __device__ static __forceinline__ uint64_t pass(const Consts& c, const Pair& p, const float* h) {
        return lanes(__builtin_fabsf(h[0] - p.sxi) < c.win_x) & lanes(__builtin_fabsf(h[1] - p.syi) < c.win_y);
    }
};

// Per-hit z (trig_hits.z): the fit written out with each hit's own z, its
// Szz and reciprocal per triplet (one binary32 division shared by both
// planes):  Szz = (zi*zi + zj*zj) + zk*zk,  w = 1 / Szz,
// m = ((ci*zi + cj*zj) + ck*zk) * w,  r_l = c_l - m*z_l.
struct MsdZTest {
    static constexpr int HF = 6;
    static constexpr bool kZ = true;
    struct Pair {
        float xi, xj, sx01, yi, yj, sy01, zi, zj, szz01;
    };
    __device__ static __forceinline__ void stage(const Consts&, float x, float y, float z, float* h) {
        h[0] = x;
        h[1] = y;
        h[2] = z;
        h[3] = x * z;
        h[4] = y * z;
        h[5] = z * z;
    }
    __device__ static __forceinline__ void pad(float* h) {
        const float n = __builtin_nanf("");
        h[0] = n; h[1] = n; h[2] = n; h[3] = n; h[4] = n; h[5] = n;
    }
    __device__ static __forceinline__ Pair pair(const Consts&, float xi, float yi, float zi, float xj, float yj,
                                                float zj) {
        Pair p;
        p.xi = xi; p.xj = xj; p.yi = yi; p.yj = yj; p.zi = zi; p.zj = zj;
        p.sx01 = xi * zi + xj * zj;
        p.sy01 = yi * zi + yj * zj;
        p.szz01 = zi * zi + zj * zj;
        return p;
    }
    __device__ static __forceinline__ Pair invalid() {
        const float n = __builtin_nanf("");
        return Pair{n, n, n, n, n, n, n, n, n};
    }
    __device__ static __forceinline__ float plane_q(float ci, float cj, float s01, float ck, float pk, float zi,
                                                    float zj, float zk, float w) {
        const float m = (s01 + pk) * w;
        const float r0 = ci - m * zi;
        const float r1 = cj - m * zj;
        const float r2 = ck - m * zk;
        return (r0 * r0 + r1 * r1) + r2 * r2;
    }
    __device__ static __forceinline__ uint64_t pass(const Consts& c, const Pair& p, const float* h) {
        const float w = 1.0f / (p.szz01 + h[5]);
        const float qx = plane_q(p.xi, p.xj, p.sx01, h[0], h[3], p.zi, p.zj, h[2], w);
        const float qy = plane_q(p.yi, p.yj, p.sy01, h[1], h[4], p.zi, p.zj, h[2], w);
        return lanes(qx <= c.qmax_x) & lanes(qy <= c.qmax_y);
    }
};

// Per-hit z, window test: slopes c / z with each hit's own z.
struct WindowZTest {
    static constexpr int HF = 2;
    static constexpr bool kZ = true;
    struct Pair {
        float sxi, syi;  // NaN when the layer-1 window already fails
    };
    __device__ static __forceinline__ void stage(const Consts&, float x, float y, float z, float* h) {
        h[0] = x / z;
        h[1] = y / z;
    }
    __device__ static __forceinline__ void pad(float* h) {
        h[0] = __builtin_nanf("");
        h[1] = __builtin_nanf("");
    }
    __device__ static __forceinline__ Pair pair(const Consts& c, float xi, float yi, float zi, float xj, float yj,
                                                float zj) {
        const float sxi = xi / zi, syi = yi / zi;
        const float sxj = xj / zj, syj = yj / zj;
        const bool ok = (__builtin_fabsf(sxj - sxi) < c.win_x) & (__builtin_fabsf(syj - syi) < c.win_y);
        const float n = __builtin_nanf("");
        return Pair{ok ? sxi : n, ok ? syi : n};
    }
    __device__ static __forceinline__ Pair invalid() {
        const float n = __builtin_nanf("");
        return Pair{n, n};
    }
    __device__ static __forceinline__ uint64_t pass(const Consts& c, const Pair& p, const float* h) {
        return lanes(__builtin_fabsf(h[0] - p.sxi) < c.win_x) & lanes(__builtin_fabsf(h[1] - p.syi) < c.win_y);
    }
};

// ----------------------------------------------------------------------------
// Events
// ----------------------------------------------------------------------------

struct EventRange {
    int o0, o1, o2;
    int n0, n1, n2;
};

// Reads and checks the CSR range of event e (wave-uniform).  Returns 0, or
// the per-event error count (-1 malformed, -2 count not representable).
__device__ __forceinline__ int load_event(const int32_t* __restrict__ off, int e, int n_hits,
                                          EventRange& ev) {
    const int64_t b = 3 * (int64_t)e;
    const int a0 = uniform_i(off[b]), a1 = uniform_i(off[b + 1]);
    const int a2 = uniform_i(off[b + 2]), a3 = uniform_i(off[b + 3]);
    if (!(0 <= a0 && a0 <= a1 && a1 <= a2 && a2 <= a3 && a3 <= n_hits)) return -1;
    ev.o0 = a0; ev.o1 = a1; ev.o2 = a2;
    ev.n0 = a1 - a0; ev.n1 = a2 - a1; ev.n2 = a3 - a2;
    if (ev.n2 > 0 && (int64_t)ev.n0 * ev.n1 > (int64_t)INT32_MAX / ev.n2) return -2;
    return 0;
}

__device__ __forceinline__ uint32_t pair_tiles(const EventRange& ev) {
    const uint64_t np = (uint64_t)ev.n0 * (uint64_t)ev.n1;
    return (ev.n2 == 0) ? 0u : (uint32_t)((np + kWave - 1) / kWave);
}

// Passing triplets of one event over pair tiles [t_begin, t_end); each tile
// is 64 consecutive (i, j) pairs in row-major order (pair p -> i = p / n1,
// j = p % n1), one pair per lane, looping over every layer-2 hit staged in
// this wave's LDS slice (KCH hits per chunk).  Called by a whole wave with
// uniform arguments; returns the same count on every lane.
template <class T, int KCH>
__device__ uint32_t wave_count(const float* __restrict__ x, const float* __restrict__ y,
                               const float* __restrict__ z, const EventRange& ev, uint32_t t_begin,
                               uint32_t t_end, const Consts& c, float* __restrict__ lds) {
    const uint32_t stop = (uint32_t)c.count_cap;  // enough: the result is capped there
    static_assert(KCH % 4 == 0, "chunk must hold whole float4 groups");
    const unsigned lane = lane_id();
    const uint32_t n0 = (uint32_t)ev.n0, n1 = (uint32_t)ev.n1;
    const uint32_t dq = kWave / n1, dr = kWave % n1;
    uint32_t cnt = 0;
    for (int k0 = 0; k0 < ev.n2; k0 += KCH) {
        const int nk = min(KCH, ev.n2 - k0);
        const int nk_pad = (nk + 3) & ~3;
        for (int t = (int)lane; t < nk_pad; t += kWave) {
            float* h = lds + t * T::HF;
            if (t < nk) {
                if constexpr (T::kZ)
                    T::stage(c, x[ev.o2 + k0 + t], y[ev.o2 + k0 + t], z[ev.o2 + k0 + t], h);
                else
                    T::stage(c, x[ev.o2 + k0 + t], y[ev.o2 + k0 + t], h);
            } else {
                T::pad(h);
            }
        }
        wave_lds_sync();
        const uint32_t p0 = t_begin * (uint32_t)kWave + lane;
        uint32_t i = p0 / n1, j = p0 - (p0 / n1) * n1;
        for (uint32_t t = t_begin; t < t_end; ++t) {
            typename T::Pair pr = T::invalid();
            if (i < n0) {
                if constexpr (T::kZ)
                    pr = T::pair(c, x[ev.o0 + i], y[ev.o0 + i], z[ev.o0 + i], x[ev.o1 + j], y[ev.o1 + j],
                                 z[ev.o1 + j]);
                else
                    pr = T::pair(c, x[ev.o0 + i], y[ev.o0 + i], x[ev.o1 + j], y[ev.o1 + j]);
            }
            // nk_pad is a multiple of 4: four layer-2 hits per iteration
            for (int k = 0; k < nk_pad; k += 4) {
                const float* h = lds + k * T::HF;
                const uint64_t m0 = T::pass(c, pr, h);
                const uint64_t m1 = T::pass(c, pr, h + T::HF);
                const uint64_t m2 = T::pass(c, pr, h + 2 * T::HF);
                const uint64_t m3 = T::pass(c, pr, h + 3 * T::HF);
                cnt += (uint32_t)(__builtin_popcountll(m0) + __builtin_popcountll(m1) +
                                  __builtin_popcountll(m2) + __builtin_popcountll(m3));
            }
            j += dr;
            i += dq;
            if (j >= n1) {
                j -= n1;
                ++i;
            }
            if (cnt >= stop) break;  // wave-uniform
        }
        wave_lds_sync();
        if (cnt >= stop) break;
    }
    return cnt;
}

}  // namespace trig
