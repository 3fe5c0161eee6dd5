// FP64 elementary functions for the per-bin kernels (gfx950).
//
// Each is a textbook construction written for this project: Cody-Waite argument
// reduction with split constants and fused multiply-adds, then a polynomial on the
// reduced interval.  The atan and exp polynomial coefficients are Chebyshev interpolants
// computed in 60-digit arithmetic and rounded to double, and the sin/cos and arc tangent tables
// hold correctly rounded values (fit_elementary.py, next to this file, writes them); the
// measured worst error of each function is about 1 ulp.
//
//   pd_sincos  |x| <= 2^24: q = rint(512x/pi), r = x - q pi/512 (two-part pi/512), short
//              polynomials on |r| <= pi/1024 combined with a 1024-entry (sin, cos) table.
//              Larger |x| falls back to the device library's sincos.  pd_rotate_data applies
//              the same pieces to a complex number directly.
//   pd_atan    |u| > 1 uses pi/2 - atan(1/u); t > tan(pi/12) uses atan(t) = pi/6 +
//              atan((sqrt3 t - 1)/(t + sqrt3)); both reductions share one division.
//   pd_atan_tab_*  atan c + atan((|u| - c)/(1 + |u| c)) with c from a 321-entry table indexed
//              by the exponent and top mantissa bits of |u|; no branches.
//   pd_exp     y = k ln2 + r (two-part ln2), |r| <= ln2/2, exp(y) = 2^k exp(r).
#pragma once
#include <hip/hip_runtime.h>

#include "pd_atan_table.h"
#include "pd_sincos_table.h"

namespace pd {

// A polynomial coefficient materialised in scalar registers where it is used.  FP64
// literals cannot be instruction operands; left alone the compiler hoists every
// coefficient out of the bin loops into vector registers (two per coefficient), which
// costs occupancy.  The empty asm pins the value to an SGPR pair at the use.
__device__ __forceinline__ double sk(double c) {
    asm volatile("" : "+s"(c));
    return c;
}

// Table-driven sin and cos of one argument: x = q pi/512 + r with |r| <= pi/1024 (two-part
// pi/512, fused multiply-adds), j = q mod 1024, and
//   sin x = S_j + (S_j (cos r - 1) + C_j sin r),  cos x = C_j + (C_j (cos r - 1) - S_j sin r)
// with (S_j, C_j) = (sin, cos)(j pi/512) correctly rounded (pd_sincos_table.h) and Taylor
// polynomials on the small interval: sin r through r^5 (the first omitted term is below 1.7e-19
// of sin r) and cos r - 1 through r^4 (the omitted r^6/720 is below 1.2e-18, and enters cos x
// times C_j).  About 1 ulp.  |x| > 2^24 uses the device library.  Two parts of pi/512 suffice:
// the first is pi/512 rounded to double and the second the rounded remainder, so the part left
// out is below 5.9e-36 and |q| <= 2^24 * 512/pi < 2.8e9 puts at most 1.6e-26 into r, where an ulp
// of r (|r| <= pi/1024) is about 3.4e-19.  (The 1024-entry table, against 512, is what lets
// cos r - 1 stop at r^4: one multiply-add whose constant -1/2 is an inline operand.)
constexpr double kTs1 = -1.0 / 6.0, kTs2 = 1.0 / 120.0;
constexpr double kTc2 = 1.0 / 24.0;

// TAB: the (sin, cos) table, in constant memory (default) or a copy staged in LDS by the caller.
// The quotient is rounded with the 1.5 * 2^52 shift: fma(x, 512/pi, 1.5 * 2^52) rounds x 512/pi to
// the nearest integer (ties to even, the product unrounded) and leaves it in the low mantissa bits,
// so the table index is a bit mask of the low word; |x| <= 2^24 keeps it far inside 2^51.
constexpr double kRoundShift = 6755399441055744.0;   // 1.5 * 2^52

// The pieces of the table construction for |x| <= 2^24: the table entry (S, C) and the small-angle
// values sr = sin r and cm = cos r - 1.  Callers that rotate a complex number by the angle combine
// them with it directly (one multiply-add per piece) instead of forming sin x and cos x first.
struct SinCosParts {
    double s, c, sr, cm;
};

__device__ __forceinline__ SinCosParts pd_sincos_parts(double x, const double2* __restrict__ tab) {
    const double qs = fma(x, sk(kInvPiStep), sk(kRoundShift));
    const double q = qs - sk(kRoundShift);
    double r = fma(-q, sk(kPiStep_1), x);
    r = fma(-q, sk(kPiStep_2), r);
    const unsigned j = static_cast<unsigned>(__builtin_bit_cast(unsigned long long, qs)) &
                       static_cast<unsigned>(kSinCosN - 1);
    const double2 sc = tab[j];
    const double z = r * r;
    SinCosParts p;
    p.s = sc.x;
    p.c = sc.y;
    p.sr = fma(r * z, fma(sk(kTs2), z, sk(kTs1)), r);
    p.cm = z * fma(z, sk(kTc2), -0.5);
    return p;
}

__device__ __forceinline__ void pd_sincos(double x, double* s_out, double* c_out,
                                          const double2* __restrict__ tab = reinterpret_cast<const double2*>(kSinCosTab)) {
    if (!(fabs(x) <= sk(16777216.0))) {
        sincos(x, s_out, c_out);
        return;
    }
    const SinCosParts p = pd_sincos_parts(x, tab);
    *s_out = p.s + fma(p.c, p.sr, p.s * p.cm);
    *c_out = p.c + fma(-p.s, p.sr, p.c * p.cm);
}

// A exp(-i x) multiplied by conj(D), D = dr + i di: returns Re and Im of conj(D) A exp(-i x)
// negated in the imaginary part as the likelihood loops use them,
//   px = A (dr cos x - di sin x),  py = -A (dr sin x + di cos x).
// With P + iQ = D (C + i S) (the data rotated by the table angle) and exp(i r) = 1 + cm + i sr:
//   dr cos x - di sin x = P (1 + cm) - Q sr,  dr sin x + di cos x = Q (1 + cm) + P sr.
__device__ __forceinline__ void pd_rotate_data(double x, double a, double dr, double di,
                                               const double2* __restrict__ tab, double& px, double& py) {
    SinCosParts p;
    if (!(fabs(x) <= sk(16777216.0))) {
        sincos(x, &p.s, &p.c);   // the whole angle from the library: r = 0
        p.sr = 0.0;
        p.cm = 0.0;
    } else {
        p = pd_sincos_parts(x, tab);
    }
    const double P = fma(dr, p.c, -di * p.s);
    const double Q = fma(dr, p.s, di * p.c);
    px = a * fma(P, p.cm, fma(-Q, p.sr, P));
    py = -a * fma(Q, p.cm, fma(P, p.sr, Q));
}

// Copy of the (sin, cos) table in LDS, filled cooperatively by a block.
__device__ __forceinline__ void stage_sincos_table(double2* __restrict__ lds) {
    for (unsigned i = threadIdx.x; i < static_cast<unsigned>(kSinCosN); i += blockDim.x)
        lds[i] = reinterpret_cast<const double2*>(kSinCosTab)[i];
}

// Reciprocal and quotient for normal-range operands: hardware reciprocal estimate, two
// Newton-Raphson steps (each doubles the correct bits), and one residual correction of
// the quotient.  Used where an IEEE-exact division is not needed.
__device__ __forceinline__ double pd_rcp(double d) {
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    r = fma(r, fma(-d, r, 1.0), r);
    return r;
}

__device__ __forceinline__ double pd_div(double n, double d) {
    const double r = pd_rcp(d);
    const double q = n * r;
    return fma(fma(-d, q, n), r, q);
}

// atan(t) = t + t^3 A(t^2) on 0 <= t <= tan(pi/12)
constexpr double kA0 = -3.3333333333333333333e-1, kA1 = 1.9999999999999998823e-1,
                 kA2 = -1.428571428571362931e-1, kA3 = 1.1111111110968117452e-1,
                 kA4 = -9.0909090749114103638e-2, kA5 = 7.6923066462929323875e-2,
                 kA6 = -6.6666239162237077212e-2, kA7 = 5.8812262311286723732e-2,
                 kA8 = -5.2439452451309842015e-2, kA9 = 4.5555660614712361532e-2,
                 kA10 = -3.0511307549049541046e-2;
constexpr double kTanPi12 = 0.2679491924311227;
constexpr double kSqrt3 = 1.7320508075688772;
constexpr double kPi6_hi = 0.5235987755982989, kPi6_lo = -5.360408832255455e-17;
constexpr double kPi2_hi = 1.5707963267948966, kPi2_lo = 6.123233995736766e-17;

// atan split around its one division: pd_atan_reduce gives the reduced quotient's numerator
// and denominator, pd_atan_finish takes the quotient t = num / den (computed by the caller,
// possibly sharing a reciprocal with other divisions) and returns atan(u).
struct AtanParts {
    double num, den;
    double u;   // the argument: its sign is copied onto atan(|u|) (one bit-field insert)
    bool hi, inv;
};

__device__ __forceinline__ AtanParts pd_atan_reduce(double u) {
    const double a = fabs(u);
    AtanParts p;
    p.inv = a > 1.0;
    const double num = p.inv ? 1.0 : a;
    const double den = p.inv ? a : 1.0;
    p.hi = num > sk(kTanPi12) * den;
    p.num = p.hi ? fma(sk(kSqrt3), num, -den) : num;
    p.den = p.hi ? fma(sk(kSqrt3), den, num) : den;
    p.u = u;
    return p;
}

__device__ __forceinline__ double pd_atan_finish(const AtanParts& p, double t) {
    const double z = t * t;
    double q = fma(sk(kA10), z, sk(kA9));
    q = fma(q, z, sk(kA8));
    q = fma(q, z, sk(kA7));
    q = fma(q, z, sk(kA6));
    q = fma(q, z, sk(kA5));
    q = fma(q, z, sk(kA4));
    q = fma(q, z, sk(kA3));
    q = fma(q, z, sk(kA2));
    q = fma(q, z, sk(kA1));
    q = fma(q, z, sk(kA0));
    double r = fma(t * z, q, t);
    if (p.hi) r = (r + sk(kPi6_lo)) + sk(kPi6_hi);
    if (p.inv) r = (sk(kPi2_hi) - r) + sk(kPi2_lo);
    return copysign(r, p.u);   // r >= 0 here
}

__device__ __forceinline__ double pd_atan(double u) {
    const double a = fabs(u);
    const bool inv = a > 1.0;
    const double num = inv ? 1.0 : a;
    const double den = inv ? a : 1.0;
    const bool hi = num > sk(kTanPi12) * den;
    const double n2 = hi ? fma(sk(kSqrt3), num, -den) : num;
    const double d2 = hi ? fma(sk(kSqrt3), den, num) : den;
    const double t = pd_div(n2, d2);
    const double z = t * t;
    double p = fma(sk(kA10), z, sk(kA9));
    p = fma(p, z, sk(kA8));
    p = fma(p, z, sk(kA7));
    p = fma(p, z, sk(kA6));
    p = fma(p, z, sk(kA5));
    p = fma(p, z, sk(kA4));
    p = fma(p, z, sk(kA3));
    p = fma(p, z, sk(kA2));
    p = fma(p, z, sk(kA1));
    p = fma(p, z, sk(kA0));
    double r = fma(t * z, p, t);
    if (hi) r = (r + sk(kPi6_lo)) + sk(kPi6_hi);
    if (inv) r = (sk(kPi2_hi) - r) + sk(kPi2_lo);
    return (u < 0.0) ? -r : r;
}

// Table-reduced arc tangent.  With c the table centre nearest |u| (pd_atan_table.h: 16 buckets
// per octave of |u| from 2^-10 to 2^10, indexed by the exponent and top mantissa bits of |u|;
// c = 0 below, the last centre above),
//   atan|u| = atan c + atan t,  t = (|u| - c) / (1 + |u| c),  |t| <= 1/64,
// and atan t = t + t^3 B(t^2) with the Taylor terms through t^7: the first omitted term, t^9/9, is
// below 6.9e-18 of atan|u| over the whole range (|t| <= |u| / (32 (1 + |u| c)); at most 1/64, and
// then atan|u| is of order one).  The quotient's one division is left to the caller (shared with
// other reciprocals), as in the split form above; no branches, and about 1 ulp (atan c correctly
// rounded, one rounding in the final sum).
constexpr double kB0 = -1.0 / 3.0, kB1 = 1.0 / 5.0, kB2 = -1.0 / 7.0;

struct AtanTabParts {
    double num, den;   // t = num / den
    double atc;        // atan c
    double u;          // the argument (its sign goes onto the result)
};

// TAB: (c_j, atan c_j) pairs, in constant memory (default) or a copy staged in LDS by the caller.
__device__ __forceinline__ AtanTabParts pd_atan_tab_reduce(double u, const double2* __restrict__ tab =
                                                                        reinterpret_cast<const double2*>(kAtanTab)) {
    const unsigned hw = static_cast<unsigned>(__builtin_bit_cast(unsigned long long, u) >> 32) & 0x7fffffffu;
    const int j = min(max(static_cast<int>(hw >> kAtanShift) - kAtanBase, 0), kAtanN - 1);
    const double2 e = tab[j];
    const double a = fabs(u);
    AtanTabParts p;
    p.num = a - e.x;
    p.den = fma(a, e.x, 1.0);
    p.atc = e.y;
    p.u = u;
    return p;
}

__device__ __forceinline__ double pd_atan_tab_finish(const AtanTabParts& p, double t) {
    const double z = t * t;
    double q = fma(sk(kB2), z, sk(kB1));
    q = fma(q, z, sk(kB0));
    return copysign(p.atc + fma(t * z, q, t), p.u);   // the sum is atan|u| >= 0
}

// Copy of the arc tangent table in LDS, filled cooperatively by a block.
__device__ __forceinline__ void stage_atan_table(double2* __restrict__ lds) {
    for (unsigned i = threadIdx.x; i < static_cast<unsigned>(kAtanN); i += blockDim.x)
        lds[i] = reinterpret_cast<const double2*>(kAtanTab)[i];
}

// exp(r) = 1 + r + r^2 E(r) on |r| <= ln2/2
constexpr double kE0 = 5.0e-1, kE1 = 1.6666666666666670986e-1, kE2 = 4.1666666666666669752e-2,
                 kE3 = 8.3333333333261408264e-3, kE4 = 1.3888888888883752376e-3,
                 kE5 = 1.9841269874800693264e-4, kE6 = 2.4801587325533507557e-5,
                 kE7 = 2.7557255425491072157e-6, kE8 = 2.7557273661166279923e-7,
                 kE9 = 2.5105206480259365425e-8, kE10 = 2.0914679452495193751e-9;
constexpr double kLn2_hi = 0.6931471805599453, kLn2_lo = 2.3190468138462996e-17;
constexpr double kLog2e = 1.4426950408889634;

__device__ __forceinline__ double pd_exp(double y) {
    if (!(fabs(y) < sk(700.0))) return exp(y);
    const double k = rint(y * sk(kLog2e));
    double r = fma(-k, sk(kLn2_hi), y);
    r = fma(-k, sk(kLn2_lo), r);
    double p = fma(sk(kE10), r, sk(kE9));
    p = fma(p, r, sk(kE8));
    p = fma(p, r, sk(kE7));
    p = fma(p, r, sk(kE6));
    p = fma(p, r, sk(kE5));
    p = fma(p, r, sk(kE4));
    p = fma(p, r, sk(kE3));
    p = fma(p, r, sk(kE2));
    p = fma(p, r, sk(kE1));
    p = fma(p, r, sk(kE0));
    const double e = 1.0 + fma(r * r, p, r);
    return ldexp(e, static_cast<int>(k));
}

}  // namespace pd
