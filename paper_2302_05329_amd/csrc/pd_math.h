// FP64 elementary functions for the per-bin kernels (gfx950).
//
// Each is a textbook construction written for this project: Cody-Waite argument
// reduction with split constants and fused multiply-adds, then a polynomial on the
// reduced interval.  The polynomial coefficients are Chebyshev interpolants computed in
// 60-digit arithmetic and rounded to double (fit_elementary.py, next to this file); the
// measured worst error of each polynomial on its interval is about 1 ulp.
//
//   pd_sincos  |x| <= 1e8 : q = rint(2x/pi), r = x - q pi/2 (three-part pi/2), sin/cos
//              polynomials on |r| <= pi/4, quadrant by q mod 4.  Larger |x| falls back to
//              the device library's sincos.
//   pd_atan    |u| > 1 uses pi/2 - atan(1/u); t > tan(pi/12) uses atan(t) = pi/6 +
//              atan((sqrt3 t - 1)/(t + sqrt3)); both reductions share one division.
//   pd_exp     y = k ln2 + r (two-part ln2), |r| <= ln2/2, exp(y) = 2^k exp(r).
#pragma once
#include <hip/hip_runtime.h>

namespace pd {

constexpr double kPio2_1 = 1.5707963267948966;
constexpr double kPio2_2 = 6.123233995736766e-17;
constexpr double kPio2_3 = -1.4973849048591698e-33;
constexpr double kTwoOverPi = 0.6366197723675814;

// sin(r) = r + r^3 S(r^2), cos(r) = 1 - r^2/2 + r^4 C(r^2) on |r| <= pi/4
constexpr double kS0 = -1.6666666666666666666e-1, kS1 = 8.3333333333333314921e-3,
                 kS2 = -1.9841269841265064899e-4, kS3 = 2.7557319219339129399e-6,
                 kS4 = -2.5052106232434683791e-8, kS5 = 1.6058531616942477437e-10,
                 kS6 = -7.5866969972366332944e-13;
constexpr double kC0 = 4.1666666666666666666e-2, kC1 = -1.3888888888888887865e-3,
                 kC2 = 2.4801587301584646402e-5, kC3 = -2.7557319221402803758e-7,
                 kC4 = 2.08767557910732553e-9, kC5 = -1.1470460886473720733e-11,
                 kC6 = 4.7458718350640028856e-14;

__device__ __forceinline__ void pd_sincos(double x, double* s_out, double* c_out) {
    if (!(fabs(x) <= 1e8)) {
        sincos(x, s_out, c_out);
        return;
    }
    const double q = rint(x * kTwoOverPi);
    double r = fma(-q, kPio2_1, x);
    r = fma(-q, kPio2_2, r);
    r = fma(-q, kPio2_3, r);
    const double z = r * r;
    double ps = fma(kS6, z, kS5);
    ps = fma(ps, z, kS4);
    ps = fma(ps, z, kS3);
    ps = fma(ps, z, kS2);
    ps = fma(ps, z, kS1);
    ps = fma(ps, z, kS0);
    const double sr = fma(r * z, ps, r);
    double pc = fma(kC6, z, kC5);
    pc = fma(pc, z, kC4);
    pc = fma(pc, z, kC3);
    pc = fma(pc, z, kC2);
    pc = fma(pc, z, kC1);
    pc = fma(pc, z, kC0);
    const double hz = 0.5 * z;
    const double w = 1.0 - hz;
    const double cr = w + (((1.0 - w) - hz) + z * z * pc);
    const int j = static_cast<int>(static_cast<long long>(q) & 3);
    const double a = (j & 1) ? cr : sr;
    const double b = (j & 1) ? sr : cr;
    *s_out = (j & 2) ? -a : a;
    *c_out = ((j + 1) & 2) ? -b : b;
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

__device__ __forceinline__ double pd_atan(double u) {
    const double a = fabs(u);
    const bool inv = a > 1.0;
    const double num = inv ? 1.0 : a;
    const double den = inv ? a : 1.0;
    const bool hi = num > kTanPi12 * den;
    const double n2 = hi ? fma(kSqrt3, num, -den) : num;
    const double d2 = hi ? fma(kSqrt3, den, num) : den;
    const double t = n2 / d2;
    const double z = t * t;
    double p = fma(kA10, z, kA9);
    p = fma(p, z, kA8);
    p = fma(p, z, kA7);
    p = fma(p, z, kA6);
    p = fma(p, z, kA5);
    p = fma(p, z, kA4);
    p = fma(p, z, kA3);
    p = fma(p, z, kA2);
    p = fma(p, z, kA1);
    p = fma(p, z, kA0);
    double r = fma(t * z, p, t);
    if (hi) r = (r + kPi6_lo) + kPi6_hi;
    if (inv) r = (kPi2_hi - r) + kPi2_lo;
    return (u < 0.0) ? -r : r;
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
    if (!(fabs(y) < 700.0)) return exp(y);
    const double k = rint(y * kLog2e);
    double r = fma(-k, kLn2_hi, y);
    r = fma(-k, kLn2_lo, r);
    double p = fma(kE10, r, kE9);
    p = fma(p, r, kE8);
    p = fma(p, r, kE7);
    p = fma(p, r, kE6);
    p = fma(p, r, kE5);
    p = fma(p, r, kE4);
    p = fma(p, r, kE3);
    p = fma(p, r, kE2);
    p = fma(p, r, kE1);
    p = fma(p, r, kE0);
    const double e = 1.0 + fma(r * r, p, r);
    return ldexp(e, static_cast<int>(k));
}

}  // namespace pd
