// Host-side constants of the selection that every MSD decision depends on:
// the threshold folded into a bound on the residual sum of squares, and the
// necessary conditions on partial sums that the pruned and binned forms use
// to skip pairs and cells without changing a count.
//
// Plain C++ (no HIP): the library's host code and a CPU test (g++) compile
// the same file.  Every function is deterministic and exact in the sense its
// comment states; the fit bounds are rigorous upper bounds derived below.
//
// Notation (paper Sec. 3.2, step 2: a line through the vertex, c = m z, per
// plane c in {x, y}; hits c0, c1, c2 of layers 0, 1, 2 at z0, z1, z2).  The
// fit written out, one binary32 rounding per operation (u = 2^-24):
//     s = fl(fl(fl(c0 z0) + fl(c1 z1)) + fl(c2 z2)),   m = fl(s w)
//     t_l = fl(m z_l),   r_l = fl(c_l - t_l),
//     Q = fl(fl(fl(r0^2) + fl(r1^2)) + fl(r2^2)),   pass <=> Q <= Qmax.
// The pruned and binned forms look at partial sums of the same Q written in
// an orthonormal basis (u*, v*) of the plane orthogonal to z:
//     a* = u* . c = (z1 c0 - z0 c1) / |(z0, z1)|,     b* = v* . c,
// computed with binary32 coefficients U0, U1, V0, V1, V2:
//     a~ = fl(fl(U0 c0) + fl(U1 c1)),   b~ = fl(fl(fl(V0 c0) + fl(V1 c1)) + fl(V2 c2)).
//
// Claim: if the written-out fit passes, then |a~| <= A(M) and |b~| <= B(M)
// for any M >= |c1|, with A and B affine in M (fit_bounds).  Derivation:
//  (1) Q <= Qmax forces every intermediate to be finite, and since the
//      partial sums of non-negative terms are monotone,
//      r0^2 + r1^2 + r2^2 <= Qmax / (1-u)^3 + 3 2^-150 =: Rr^2.
//  (2) For the computed (finite) slope m, let rho_l = c_l - m z_l exactly.
//      c_l - t_l = r_l / (1 + d) and |t_l - m z_l| <= u |m z_l| + 2^-150
//      with |m z_l| <= |c_l| + |rho_l|, hence, as vectors over any set of
//      layers,  |rho| <= (|r| / (1-u) + u |c| + k^.5 2^-150) / (1-u).
//  (3) u* and v* are unit vectors orthogonal to z, so u* . c = u* . rho and
//      v* . c = v* . rho for every m: |a*| <= |(rho0, rho1)|, |b*| <= |rho|.
//      This is where the fit's own rounding drops out: m need not be
//      accurate at all.
//  (4) |c_l| <= |m| z_l + |rho_l| and |m| z1 <= |c1| + |rho1| bound every
//      coordinate of a passing triplet by the layer-1 one:
//      |c_l| <= C_l = [(z_l/z1)(M (1+u') + rho_R) + rho_R] / (1-u'),
//      u' = u/(1-u), rho_R = Rr/(1-u)^2 + 2^-150/(1-u).
//  (5) The binary32 coefficients and products: with eU, eV the relative
//      errors of U_l, V_l against u*, v*,
//      |a~| <= (1+u) (|a*| + (eU + u(1+eU)) (|u*_0| C0 + |u*_1| C1) + 2^-149),
//      |b~| <= (1+u) (|b*| + (eV + 2u(1+u)(1+eV)) sum_l |v*_l| C_l + 2^-147).
// Everything is evaluated in long double with upward slack and rounded up
// to binary32; the device evaluates fl(a0 + fl(a1 M)) with a1, a0 inflated
// so that this never falls below the real A(M) (fit_bounds).
#pragma once

#include <cmath>
#include <cstdint>
#include <cstring>

namespace trig_host {

inline uint32_t bits_of(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return u;
}
inline float float_of(uint32_t u) {
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// Largest non-negative binary32 v (bit pattern search over [0, +inf]) with
// pred(v) true, for pred non-increasing in v and pred(0) true.
template <class Pred>
float largest_with(Pred pred) {
    uint32_t lo = 0u, hi = 0x7f800000u;  // pred(lo) true
    if (pred(float_of(hi))) return float_of(hi);
    while (hi - lo > 1u) {  // pred(hi) false
        const uint32_t mid = lo + (hi - lo) / 2u;
        if (pred(float_of(mid))) lo = mid; else hi = mid;
    }
    return float_of(lo);
}

// Largest binary32 q with f32(q / ndf) <= t.  f32(q / ndf) is non-decreasing
// in q, so {q >= 0 : f32(q / ndf) <= t} is exactly {0 <= q <= Qmax}, and
// "MSD per degree of freedom <= t" becomes "Q <= Qmax" without a division.
inline float fold_threshold(float t, int ndf) {
    const float n = (float)ndf;
    return largest_with([&](float q) {
        volatile float d = q / n;
        return (float)d <= t;
    });
}

// Largest binary32 b >= 0 with f32(b * b) <= qmax (f32(b * b) is
// non-decreasing in b >= 0): "f32(a * a) <= qmax" becomes "|a| <= beta".
inline float pair_bound(float qmax) {
    return largest_with([&](float b) {
        volatile float sq = b * b;
        return (float)sq <= qmax;
    });
}

// Binary32 coefficients of the orthonormal basis (u*, v*) of the plane
// orthogonal to (z0, z1, z2): u* = (z1, -z0, 0) / n01,
// v* = (z0 z2, z1 z2, -s01) / (n01 |z|), s01 = z0^2 + z1^2, n01 = sqrt(s01);
// each evaluated in binary64 in the order written, rounded once.
struct Basis {
    float U0, U1, V0, V1, V2;
};
inline Basis basis(float z0f, float z1f, float z2f) {
    const double z0 = z0f, z1 = z1f, z2 = z2f;
    const double s01 = z0 * z0 + z1 * z1;
    const double n01 = std::sqrt(s01);
    const double d = n01 * std::sqrt(s01 + z2 * z2);
    return Basis{(float)(z1 / n01), (float)(-z0 / n01), (float)((z0 * z2) / d), (float)((z1 * z2) / d),
                 (float)(-s01 / d)};
}

// Smallest binary32 >= v (v >= 0 finite long double), or +inf.
inline float round_up_f32(long double v) {
    float f = (float)v;
    if ((long double)f < v) f = std::nextafter(f, INFINITY);
    return f;
}

// Coefficients of the written-out fit's necessary conditions on one plane
// (threshold qmax): the device computes
//     A = fl(a0 + fl(a1 M)),   B = fl(b0 + fl(b1 M))
// for a bound M >= |c1| on the triplet's layer-1 coordinate in that plane,
// and then every triplet that passes the plane has |a~| <= A, |b~| <= B
// (see the derivation above).  M = +inf gives +inf (no pruning).
struct FitBounds {
    float a0, a1, b0, b1;
};

inline FitBounds fit_bounds(float z0f, float z1f, float z2f, float qmax) {
    typedef long double LD;
    const LD u = std::ldexp((LD)1, -24);
    const LD up = u / (1 - u);
    const LD tiny = std::ldexp((LD)1, -147);
    const LD z0 = z0f, z1 = z1f, z2 = z2f;
    // basis coefficients exactly (long double) and as the library rounds them
    const LD n01 = std::sqrt(z0 * z0 + z1 * z1);
    const LD nz = std::sqrt(z0 * z0 + z1 * z1 + z2 * z2);
    const LD us0 = z1 / n01, us1 = z0 / n01;                       // |u*_l|
    const LD vs0 = z0 * z2 / (n01 * nz), vs1 = z1 * z2 / (n01 * nz), vs2 = n01 / nz;  // |v*_l|
    const Basis K = basis(z0f, z1f, z2f);
    const float U0 = K.U0, U1 = K.U1, V0 = K.V0, V1 = K.V1, V2 = K.V2;
    // relative errors of the coefficients, plus slack for long double rounding
    const LD slack = std::ldexp((LD)1, -50);
    const LD eU = std::fmax(std::fabs((LD)U0 / us0 - 1), std::fabs(-(LD)U1 / us1 - 1)) + slack;
    const LD eV = std::fmax(std::fmax(std::fabs((LD)V0 / vs0 - 1), std::fabs((LD)V1 / vs1 - 1)),
                            std::fabs(-(LD)V2 / vs2 - 1)) + slack;
    // (1)-(2): residual norm and rho_R
    const LD Rr = std::sqrt((LD)qmax / ((1 - u) * (1 - u) * (1 - u)) + 3 * std::ldexp((LD)1, -150)) * (1 + slack);
    const LD rhoR = Rr / ((1 - u) * (1 - u)) + std::ldexp((LD)1, -150) / (1 - u);
    // (4): C_l = g_l M + h_l
    const LD r0 = z0 / z1 * (1 + slack), r2 = z2 / z1 * (1 + slack);
    const LD g0 = r0 * (1 + up) / (1 - up), h0 = (r0 * rhoR + rhoR) / (1 - up);
    const LD g2 = r2 * (1 + up) / (1 - up), h2 = (r2 * rhoR + rhoR) / (1 - up);
    // (2)-(3): |a*| <= (Rr/(1-u) + u |(c0, c1)| + 2^-149.5)/(1-u),
    //          |(c0, c1)| <= sqrt(g0^2 + 1) M + h0
    const LD n01g = std::sqrt(g0 * g0 + 1) * (1 + slack);
    const LD a_star0 = (Rr / (1 - u) + u * h0 + tiny) / (1 - u);
    const LD a_star1 = u * n01g / (1 - u);
    // (5)
    const LD kU = eU + u * (1 + eU);
    const LD A0 = (1 + u) * (a_star0 + kU * us0 * h0 + tiny);
    const LD A1 = (1 + u) * (a_star1 + kU * (us0 * g0 + us1));
    const LD n3g = std::sqrt(g0 * g0 + 1 + g2 * g2) * (1 + slack);
    const LD b_star0 = (Rr / (1 - u) + u * (h0 + h2) + tiny) / (1 - u);
    const LD b_star1 = u * n3g / (1 - u);
    const LD kV = eV + 2 * u * (1 + u) * (1 + eV);
    const LD B0 = (1 + u) * (b_star0 + kV * (vs0 * h0 + vs2 * h2) + tiny);
    const LD B1 = (1 + u) * (b_star1 + kV * (vs0 * g0 + vs1 + vs2 * g2));
    // Device evaluation fl(x0 + fl(x1 M)) >= x0 + x1 M when x1 is inflated
    // by 1/(1-u)^2 and x0 by 1/(1-u) plus 2^-126 (which also covers an
    // underflowing product and keeps the bound a normal number).
    const LD n126 = std::ldexp((LD)1, -126);
    FitBounds f;
    f.a0 = round_up_f32(A0 / (1 - u) * (1 + slack) + n126);
    f.a1 = round_up_f32(A1 / ((1 - u) * (1 - u)) * (1 + slack));
    f.b0 = round_up_f32(B0 / (1 - u) * (1 + slack) + n126);
    f.b1 = round_up_f32(B1 / ((1 - u) * (1 - u)) * (1 + slack));
    return f;
}

// Per-hit z (each hit at its own z_h > 0): the pruned form compares the
// hits' slopes s_h = f32(c_h / z_h).  For the computed slope m of the fit,
// c_i/z_i - c_j/z_j = rho_i/z_i - rho_j/z_j exactly (rho_l = c_l - m z_l, as
// above, whatever m's rounding), so a triplet that passes a plane has
//   |c_j/z_j - c_i/z_i| <= sqrt(2) |(rho_i, rho_j)| / zmin,
//   |(rho_i, rho_j)| <= (Rr/(1-u) + u sqrt(2) M + 2^-149.5) / (1-u),
// with zmin <= z_i, z_j and M >= |c_i|, |c_j|; the two divisions and the
// difference add (1+u) and 2u M / zmin:
//   |f32(s_j - s_i)| <= (a0 + a1 M) / zmin + (1+u) 2^-149.
// The device evaluates D = f32(f32(f32(a0 + f32(a1 M)) * f32(1 / zmin)) + 2^-126)
// (four roundings more, covered by the inflation below), for each plane.
struct SlopeBounds {
    float a0, a1;
};

inline SlopeBounds slope_bounds(float qmax) {
    typedef long double LD;
    const LD u = std::ldexp((LD)1, -24);
    const LD slack = std::ldexp((LD)1, -50);
    const LD Rr = std::sqrt((LD)qmax / ((1 - u) * (1 - u) * (1 - u)) + 3 * std::ldexp((LD)1, -150)) * (1 + slack);
    const LD r2 = std::sqrt((LD)2) * (1 + slack);
    const LD A0 = (1 + u) * r2 * (Rr / (1 - u) + std::ldexp((LD)1, -149)) / (1 - u);
    const LD A1 = (1 + u) * (r2 * r2 * u / (1 - u) + 2 * u);
    const LD up = 1 / ((1 - u) * (1 - u) * (1 - u) * (1 - u) * (1 - u));
    return SlopeBounds{round_up_f32(A0 * up * (1 + slack)), round_up_f32(A1 * up * (1 + slack))};
}

}  // namespace trig_host
