// Per-bin evaluation of the model from a coefficient record, and the "basis visitor"
// that exposes, for every record entry that influences the bin, the partial derivative
// of the phase Psi or of ln(amplitude) with respect to that entry.
//
// The same visitor drives three reductions:
//   * likelihood gradient and mismatch adjoint: moments  sum_k weight_k * partial_k
//     (later contracted with the record's tangents per point);
//   * Fisher matrix: per-bin tangents  sum_j tangent_j * partial_j  along 7 directions.
#pragma once
#include <hip/hip_runtime.h>

#include "pd_model.h"

namespace pd {

struct GridArgs {
    double f0, df, fmin, fref;
    int64_t nb;
};

constexpr double kPi76 = 3.80196561521497470042;  // pi^(7/6)

// Frequency of bin k, rounded exactly as f0 + k*df (two roundings, no fused multiply-add).
__device__ __forceinline__ double bin_freq(const GridArgs& g, int64_t k) {
    return __dadd_rn(g.f0, __dmul_rn(static_cast<double>(k), g.df));
}

// Conservative range [klo, khi) of bins that can carry signal for a source of mass Ms;
// the exact test (f >= f_min and Ms f <= 0.2) is still applied to every bin.
__device__ __forceinline__ void active_range(double ms, const GridArgs& g, int64_t& klo, int64_t& khi) {
    const double kh = floor((kFCut / ms - g.f0) / g.df) + 2.0;
    const double kl = ceil((g.fmin - g.f0) / g.df) - 1.0;
    khi = (kh < 0.0) ? 0 : ((kh > static_cast<double>(g.nb)) ? g.nb : static_cast<int64_t>(kh));
    klo = (kl < 0.0) ? 0 : ((kl > static_cast<double>(g.nb)) ? g.nb : static_cast<int64_t>(kl));
    if (klo > khi) klo = khi;
}

__device__ __forceinline__ bool bin_active(const GridArgs& g, double f, double mf) {
    return (f >= g.fmin) && (mf <= kFCut);
}

// Everything one bin computes on the way to A and Psi, kept for the visitors.
struct BinVals {
    double mf;
    int preg, areg;          // phase / amplitude region: 1 inspiral, 2 intermediate, 3 merger-ringdown
    double v, w, lv;         // v = (pi Mf)^(1/3), w = 1/v, ln v        (phase region 1)
    double lnf, invf;        // ln Mf, 1/Mf                              (phase regions 2, 3)
    double f34, u, at, iu2;  // Mf^(3/4), (Mf - q)/d, atan(u), 1/(1+u^2) (phase region 3)
    double x, den;           // Mf - f_RD, x^2 + g^2                     (amplitude region 3)
    double ahat;             // amplitude ratio
    double pf;               // Mf^(-7/6)
    double psi;              // phase
};

__device__ __forceinline__ void eval_bin(const double* __restrict__ rec, double mf, BinVals& b) {
    b.mf = mf;
    b.preg = (mf < kFPhaseJoin) ? 1 : ((mf < rec[R_FP2]) ? 2 : 3);
    b.areg = (mf < kFAmpJoin) ? 1 : ((mf < rec[R_FA2]) ? 2 : 3);
    const double* c = rec;
    if (b.preg == 1) {
        const double v = cbrt(kPi * mf);
        const double w = 1.0 / v;
        const double lv = log(v);
        b.v = v;
        b.w = w;
        b.lv = lv;
        const double w2 = w * w;
        const double neg = w * (c[R_PH1 + 3] + w * (c[R_PH1 + 2] + w * (c[R_PH1 + 1] + w2 * c[R_PH1 + 0])));
        const double pos =
            c[R_PH1 + 4] +
            v * (c[R_PH1 + 6] +
                 v * (c[R_PH1 + 8] +
                      v * (c[R_PH1 + 9] + v * (c[R_PH1 + 10] + v * (c[R_PH1 + 11] + v * c[R_PH1 + 12])))));
        b.psi = neg + pos + lv * (c[R_PH1 + 5] + c[R_PH1 + 7] * v);
        b.pf = kPi76 * (w2 * w) * sqrt(w);
    } else if (b.preg == 2) {
        const double lnf = log(mf);
        const double invf = 1.0 / mf;
        b.lnf = lnf;
        b.invf = invf;
        b.psi = c[R_PH2 + 0] + c[R_PH2 + 1] * mf + c[R_PH2 + 2] * lnf + c[R_PH2 + 3] * (invf * invf * invf);
        b.pf = exp(-(7.0 / 6.0) * lnf);
    } else {
        const double invf = 1.0 / mf;
        const double s = sqrt(mf);
        const double f34 = s * sqrt(s);
        const double u = (mf - c[R_PH3 + 5]) / c[R_PH3 + 6];
        const double at = atan(u);
        b.invf = invf;
        b.f34 = f34;
        b.u = u;
        b.at = at;
        b.iu2 = 1.0 / (1.0 + u * u);
        b.psi = c[R_PH3 + 0] + c[R_PH3 + 1] * mf + c[R_PH3 + 2] * invf + c[R_PH3 + 3] * f34 + c[R_PH3 + 4] * at;
        b.lnf = log(mf);
        b.pf = exp(-(7.0 / 6.0) * b.lnf);
    }
    if (b.areg == 1) {
        const double v = b.v;
        double a = c[R_AM1 + 9];
#pragma unroll
        for (int i = 8; i >= 0; --i) a = a * v + c[R_AM1 + i];
        b.ahat = a;
    } else if (b.areg == 2) {
        b.ahat = c[R_AM2 + 0] + mf * (c[R_AM2 + 1] + mf * (c[R_AM2 + 2] + mf * (c[R_AM2 + 3] + mf * c[R_AM2 + 4])));
    } else {
        const double x = mf - c[R_AM3 + 1];
        const double g = c[R_AM3 + 2];
        const double den = x * x + g * g;
        b.x = x;
        b.den = den;
        b.ahat = c[R_AM3 + 0] / den * exp(-c[R_AM3 + 3] * x);
    }
}

// Visit d Psi / d rec[s] (vis.ph), d ln A / d rec[s] (vis.am) and the explicit
// Mf-dependence: Mf dPsi/dMf and Mf d lnA/dMf (vis.fd), for one bin.
template <class V>
__device__ __forceinline__ void visit_bin(const double* __restrict__ rec, const BinVals& b, V& vis) {
    const double* c = rec;
    double fpsi;
    if (b.preg == 1) {
        const double v = b.v, w = b.w, lv = b.lv;
        const double w2 = w * w, w3 = w2 * w, w5 = w3 * w2;
        const double v2 = v * v, v3 = v2 * v, v4 = v3 * v, v5 = v4 * v, v6 = v5 * v;
        const double bs[13] = {w5, w3, w2, w, 1.0, lv, v, v * lv, v2, v3, v4, v5, v6};
        const double pw[13] = {-5, -3, -2, -1, 0, 0, 1, 1, 2, 3, 4, 5, 6};
        fpsi = (c[R_PH1 + 5] + c[R_PH1 + 7] * v) * (1.0 / 3.0);
#pragma unroll
        for (int j = 0; j < 13; ++j) {
            vis.ph(R_PH1 + j, bs[j]);
            fpsi += c[R_PH1 + j] * bs[j] * (pw[j] * (1.0 / 3.0));
        }
    } else if (b.preg == 2) {
        const double i3 = b.invf * b.invf * b.invf;
        vis.ph(R_PH2 + 0, 1.0);
        vis.ph(R_PH2 + 1, b.mf);
        vis.ph(R_PH2 + 2, b.lnf);
        vis.ph(R_PH2 + 3, i3);
        fpsi = c[R_PH2 + 1] * b.mf + c[R_PH2 + 2] - 3.0 * c[R_PH2 + 3] * i3;
    } else {
        const double d = c[R_PH3 + 6];
        const double c4 = c[R_PH3 + 4];
        const double t = c4 * b.iu2 / d;
        vis.ph(R_PH3 + 0, 1.0);
        vis.ph(R_PH3 + 1, b.mf);
        vis.ph(R_PH3 + 2, b.invf);
        vis.ph(R_PH3 + 3, b.f34);
        vis.ph(R_PH3 + 4, b.at);
        vis.ph(R_PH3 + 5, -t);
        vis.ph(R_PH3 + 6, -t * b.u);
        fpsi = c[R_PH3 + 1] * b.mf - c[R_PH3 + 2] * b.invf + 0.75 * c[R_PH3 + 3] * b.f34 + t * b.mf;
    }
    double fa;
    vis.am(R_LNA0, 1.0);
    if (b.areg == 1) {
        const double ia = 1.0 / b.ahat;
        double p = ia;
        double acc = 0.0;
        vis.am(R_AM1 + 0, p);
#pragma unroll
        for (int i = 1; i < 10; ++i) {
            p *= b.v;
            vis.am(R_AM1 + i, p);
            acc += c[R_AM1 + i] * p * (i * (1.0 / 3.0));
        }
        fa = acc;
    } else if (b.areg == 2) {
        const double ia = 1.0 / b.ahat;
        const double f = b.mf;
        double p = ia;
        double acc = 0.0;
        vis.am(R_AM2 + 0, p);
#pragma unroll
        for (int i = 1; i < 5; ++i) {
            p *= f;
            vis.am(R_AM2 + i, p);
            acc += c[R_AM2 + i] * p * i;
        }
        fa = acc;
    } else {
        const double x = b.x, den = b.den, g = c[R_AM3 + 2], r = c[R_AM3 + 3];
        const double tx = 2.0 * x / den;
        vis.am(R_AM3 + 0, 1.0 / c[R_AM3 + 0]);
        vis.am(R_AM3 + 1, tx + r);
        vis.am(R_AM3 + 2, -2.0 * g / den);
        vis.am(R_AM3 + 3, -x);
        fa = b.mf * (-tx - r);
    }
    vis.fd(fpsi, fa - 7.0 / 6.0);
}

// Chunk of bins [kb, ke) handled by wavefront `c` of `chunks` for one point.
__device__ __forceinline__ void chunk_range(double ms, const GridArgs& g, int c, int chunks, int64_t& kb,
                                            int64_t& ke) {
    int64_t klo, khi;
    active_range(ms, g, klo, khi);
    const int64_t len = khi - klo;
    int64_t per = (len + chunks - 1) / chunks;
    per = (per + 63) & ~static_cast<int64_t>(63);
    kb = klo + static_cast<int64_t>(c) * per;
    ke = kb + per;
    if (kb > khi) kb = khi;
    if (ke > khi) ke = khi;
}

// ---- deterministic wavefront reduction (fixed butterfly order) ---------------------
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

}  // namespace pd
