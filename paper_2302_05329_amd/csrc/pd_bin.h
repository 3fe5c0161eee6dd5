// Per-bin evaluation of the model from a coefficient record.
//
// Two things keep a bin cheap:
//  * source-independent per-bin factors are tabulated once per grid (per call):
//    cbrt f, 1/cbrt f, ln f, f^(3/4), 1/f, f^(-7/6), and the noise-weighted data
//    w f^(-7/6) d and weight w f^(-7/3) (w = 4 df / S_n).  With the per-point factors
//    stored in the record (cbrt(pi Ms), ln Ms, Ms^(3/4), ...), v = (pi Mf)^(1/3), ln Mf,
//    Mf^(3/4), 1/Mf and Mf^(-7/6) cost one multiply each; only sincos, atan and exp remain.
//  * the model regions are contiguous in k, so loops run over region segments with the
//    region fixed at compile time: no per-bin region branches and only that region's
//    accumulators live.
//
// The "basis visitor" exposes, for every record entry that influences a bin, the partial
// derivative of the phase Psi or of ln(amplitude) w.r.t. that entry.  It drives the
// gradient and mismatch-adjoint moments (sum_k weight_k * partial_k, contracted with the
// record tangents per point) and the per-bin tangents of the Fisher matrix.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "pd_math.h"
#include "pd_model.h"

namespace pd {

struct GridArgs {
    double f0, df, fmin, fref;
    int64_t nb;
};

// Per-bin tables (structure of arrays, each n_bins long).
enum : int { T_CB = 0, T_ICB, T_LF, T_F34, T_INF, T_F76, T_DWR, T_DWI, T_WW, T_N };

// One wave-uniform base pointer per table; bins are indexed with 32-bit offsets.
struct Tabs {
    const double* p[T_N];
    Tabs() = default;
    __device__ __forceinline__ Tabs(const double* __restrict__ t, int64_t nb) {
#pragma unroll
        for (int i = 0; i < T_N; ++i) p[i] = t + i * nb;
    }
    __device__ __forceinline__ double at(int which, int64_t k) const { return p[which][k]; }
    // 32-bit byte offset from a wave-uniform base: one shared offset register serves every table
    __device__ __forceinline__ double at(int which, unsigned k) const {
        return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(p[which]) + (k << 3));
    }
};

// The grid-table values one bin's evaluation reads, held in registers: a kernel that evaluates
// the same bin for many parameter points loads them once.
struct BinTabs {
    double cb, icb, lf, f34, inf;
    template <class KI>
    __device__ __forceinline__ void load(const Tabs& T, KI k) {
        cb = T.at(T_CB, k);
        icb = T.at(T_ICB, k);
        lf = T.at(T_LF, k);
        f34 = T.at(T_F34, k);
        inf = T.at(T_INF, k);
    }
    template <class KI>
    __device__ __forceinline__ double at(int which, KI) const {
        return which == T_CB ? cb : which == T_ICB ? icb : which == T_LF ? lf : which == T_F34 ? f34 : inf;
    }
};

// Frequency of bin k, rounded exactly as f0 + k*df (two roundings, no fused multiply-add).
__device__ __forceinline__ double bin_freq(const GridArgs& g, int64_t k) {
    return __dadd_rn(g.f0, __dmul_rn(static_cast<double>(k), g.df));
}
__device__ __forceinline__ double bin_freq(const GridArgs& g, unsigned k) {
    return __dadd_rn(g.f0, __dmul_rn(static_cast<double>(k), g.df));
}

__device__ __forceinline__ bool bin_active(const GridArgs& g, double f, double mf) {
    return (f >= g.fmin) && (mf <= kFCut);
}

// First k in [lo, hi] with pred(k) true, for a predicate monotone in k (false ... true),
// starting from an estimate and stepping to the exact bin.  Wave-uniform.
template <class Pred>
__device__ __forceinline__ int64_t first_true(Pred pred, int64_t est, int64_t lo, int64_t hi) {
    int64_t k = est < lo ? lo : (est > hi ? hi : est);
    while (k > lo && pred(k - 1)) --k;
    while (k < hi && !pred(k)) ++k;
    return k;
}

__device__ __forceinline__ int64_t clamp_est(double x, int64_t lo, int64_t hi) {
    if (!(x > static_cast<double>(lo))) return lo;
    if (x > static_cast<double>(hi)) return hi;
    return static_cast<int64_t>(x);
}

// Exact active range [ka, kz) of a source: f_k >= f_min and Ms f_k <= 0.2.
__device__ __forceinline__ void active_range(double ms, const GridArgs& g, int64_t& ka, int64_t& kz) {
    auto ge_min = [&](int64_t k) { return bin_freq(g, k) >= g.fmin; };
    auto above_cut = [&](int64_t k) { return ms * bin_freq(g, k) > kFCut; };
    ka = first_true(ge_min, clamp_est(ceil((g.fmin - g.f0) / g.df), 0, g.nb), 0, g.nb);
    kz = first_true(above_cut, clamp_est(floor((kFCut / ms - g.f0) / g.df), 0, g.nb), 0, g.nb);
    if (kz < ka) kz = ka;
}

// Wave-uniform copy of a value every lane already agrees on (bin indices fit in 32 bits).
__device__ __forceinline__ int uniform_i(int64_t x) { return __builtin_amdgcn_readfirstlane(static_cast<int>(x)); }

// Region segments of [kb, ke) (already inside the active range): segment i is
// [k[i], k[i+1]) (possibly empty) with phase region pr[i] and amplitude region ar[i].  Every
// index is a compile-time constant after unrolling, so the struct lives in registers.
struct Segs {
    int k[6];
    int pr[5], ar[5];
};

__device__ __forceinline__ void make_segments(const double* __restrict__ rec, const GridArgs& g, int64_t kb,
                                              int64_t ke, Segs& S) {
    const double ms = rec[R_MS];
    const double th[4] = {kFAmpJoin, kFPhaseJoin, rec[R_FP2], rec[R_FA2]};
    int64_t b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double t = th[i];
        auto ge = [&](int64_t k) { return ms * bin_freq(g, k) >= t; };
        b[i] = first_true(ge, clamp_est(ceil((t / ms - g.f0) / g.df), kb, ke), kb, ke);
    }
    // sort the four boundaries (tiny network)
#define PD_SW(i, j)                 \
    if (b[i] > b[j]) {              \
        const int64_t _t = b[i];    \
        b[i] = b[j];                \
        b[j] = _t;                  \
    }
    PD_SW(0, 1) PD_SW(2, 3) PD_SW(0, 2) PD_SW(1, 3) PD_SW(1, 2)
#undef PD_SW
    S.k[0] = static_cast<int>(kb);
#pragma unroll
    for (int i = 0; i < 4; ++i) S.k[i + 1] = static_cast<int>(b[i]);
    S.k[5] = static_cast<int>(ke);
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const double mf = ms * bin_freq(g, static_cast<int64_t>(S.k[i]));
        S.pr[i] = (mf < kFPhaseJoin) ? 1 : ((mf < rec[R_FP2]) ? 2 : 3);
        S.ar[i] = (mf < kFAmpJoin) ? 1 : ((mf < rec[R_FA2]) ? 2 : 3);
    }
}

// Segment tables are computed once per call (one thread per (point, chunk)) and read by every
// region launch: 16 ints per entry, k[6], pr[5], ar[5].
constexpr int kSegInts = 16;

__device__ __forceinline__ void store_segments(const Segs& S, int* __restrict__ dst) {
#pragma unroll
    for (int i = 0; i < 6; ++i) dst[i] = S.k[i];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        dst[6 + i] = S.pr[i];
        dst[11 + i] = S.ar[i];
    }
}

// Read by a whole wavefront from a wave-uniform address (scalar loads).
__device__ __forceinline__ void load_segments(const int* __restrict__ src, Segs& S) {
#pragma unroll
    for (int i = 0; i < 6; ++i) S.k[i] = src[i];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        S.pr[i] = src[6 + i];
        S.ar[i] = src[11 + i];
    }
}

// Record accessor for the merger-ringdown loops (fused likelihood, Fisher pass, mismatch column
// pass and adjoint, template generation of the overlap bank): the record plus products of its
// entries formed once per segment (FP64 products of two per-point constants would otherwise be
// recomputed in every bin, as there is no scalar FP64 arithmetic) and the arc tangent table.
// With the exponential recurrence, the merger-ringdown amplitude numerator R_AM3 is folded into
// the recurrence by the caller.  R: how the record is read (a pointer, or any type whose
// operator[] returns entry i).
template <class R = const double*>
struct RecMRDT {
    R p;
    const double2* __restrict__ atab;   // arc tangent table (c_j, atan c_j): an LDS copy or kAtanTab
    double q_id;   // R_PH3+5 * R_ID: u = Mf R_ID - q_id
    double g2;     // R_AM3+2 ^ 2
    double c4id;   // R_PH3+4 * R_ID
    double c3q;    // 3/4 R_PH3+3
    double m2g;    // -2 R_AM3+2
    __device__ __forceinline__ double operator[](int i) const { return p[i]; }
};
using RecMRD = RecMRDT<>;

template <class RC>
struct IsRecMRD {
    static constexpr bool value = false;
};
template <class R>
struct IsRecMRD<RecMRDT<R>> {
    static constexpr bool value = true;
};

// Wave-uniform copy of a double (both halves from the first active lane).
__device__ __forceinline__ double uniform_d(double x) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = __builtin_amdgcn_readfirstlane(static_cast<int>(static_cast<unsigned>(b)));
    const unsigned hi = __builtin_amdgcn_readfirstlane(static_cast<int>(static_cast<unsigned>(b >> 32)));
    return __builtin_bit_cast(double, (static_cast<unsigned long long>(hi) << 32) | lo);
}

template <class R>
__device__ __forceinline__ RecMRDT<R> rec_mrd(R c, const double2* __restrict__ atab) {
    RecMRDT<R> r;
    r.p = c;
    r.atab = atab;
    r.q_id = uniform_d(c[R_PH3 + 5] * c[R_ID]);
    r.g2 = uniform_d(c[R_AM3 + 2] * c[R_AM3 + 2]);
    r.c4id = uniform_d(c[R_PH3 + 4] * c[R_ID]);
    r.c3q = uniform_d(0.75 * c[R_PH3 + 3]);
    r.m2g = uniform_d(-2.0 * c[R_AM3 + 2]);
    return r;
}

// Everything one bin computes on the way to Ahat and Psi, kept for the visitors.
struct BinVals {
    double mf;
    double v, w, lv;         // v = (pi Mf)^(1/3), w = 1/v, ln v        (phase region 1)
    double lnf, invf;        // ln Mf, 1/Mf                              (phase regions 2, 3)
    double f34, u, at;       // Mf^(3/4), (Mf - q)/d, atan(u)            (phase region 3)
    double x, iden;          // Mf - f_RD, 1/(x^2 + g^2)                 (amplitude region 3)
    double iu2;              // 1/(1 + u^2)                              (phase region 3)
    double ahat;             // amplitude ratio
    double psi;              // phase
};

// HAVE_EX: the merger-ringdown amplitude exponential exp(-c3 (Mf - f_RD)) is supplied by the
// caller (a per-lane recurrence along a segment) instead of evaluated here.
// RC: the record (a pointer, or any type whose operator[] reads entry i); TB: the grid tables.
template <int PR, int AR, bool HAVE_EX = false, class RC, class TB, class KI>
__device__ __forceinline__ void eval_bin_t(RC c, const TB& T, KI k, double mf,
                                           BinVals& b, double ex = 0.0) {
    b.mf = mf;
    if (PR == 1 || AR == 1) {
        b.v = c[R_CS] * T.at(T_CB, k);
        b.w = c[R_ICS] * T.at(T_ICB, k);
    }
    if (PR == 1) {
        const double v = b.v, w = b.w;
        const double lv = fma(T.at(T_LF, k), sk(1.0 / 3.0), c[R_LCS]);
        b.lv = lv;
        const double w2 = w * w;
        const double neg = w * fma(w, fma(w, fma(w2, c[R_PH1 + 0], c[R_PH1 + 1]), c[R_PH1 + 2]), c[R_PH1 + 3]);
        double pos = fma(v, c[R_PH1 + 12], c[R_PH1 + 11]);
        pos = fma(v, pos, c[R_PH1 + 10]);
        pos = fma(v, pos, c[R_PH1 + 9]);
        pos = fma(v, pos, c[R_PH1 + 8]);
        pos = fma(v, pos, c[R_PH1 + 6]);
        pos = fma(v, pos, c[R_PH1 + 4]);
        b.psi = neg + pos + lv * fma(c[R_PH1 + 7], v, c[R_PH1 + 5]);
    } else if (PR == 2) {
        const double lnf = c[R_LMS] + T.at(T_LF, k);
        const double invf = c[R_IMS] * T.at(T_INF, k);
        b.lnf = lnf;
        b.invf = invf;
        b.psi = fma(c[R_PH2 + 3], invf * invf * invf, fma(c[R_PH2 + 2], lnf, c[R_PH2 + 1] * mf)) + c[R_PH2 + 0];
    } else {
        // merger-ringdown phase: atan(u) needs one division (after its argument reduction), the
        // phase derivative 1/(1 + u^2), and in amplitude region 3 the Lorentzian 1/(x^2 + g^2):
        // all three come from one reciprocal of their product
        constexpr bool D = IsRecMRD<RC>::value;
        const double invf = c[R_IMS] * T.at(T_INF, k);
        const double f34 = c[R_MS34] * T.at(T_F34, k);
        double u;
        if constexpr (D)
            u = fma(mf, c[R_ID], -c.q_id);
        else
            u = (mf - c[R_PH3 + 5]) * c[R_ID];
        // the merger-ringdown record form (RecMRD) carries an arc tangent table: the table
        // reduction (no branches, a shorter polynomial); a plain record keeps the two-level one
        using AP = std::conditional_t<D, AtanTabParts, AtanParts>;
        AP ap;
        if constexpr (D)
            ap = pd_atan_tab_reduce(u, c.atab);
        else
            ap = pd_atan_reduce(u);
        const double d1 = fma(u, u, 1.0);
        double d2 = 1.0, x = 0.0;
        if (AR == 3) {
            x = mf - c[R_AM3 + 1];
            if constexpr (D) {
                d2 = fma(x, x, c.g2);
            } else {
                const double g = c[R_AM3 + 2];
                d2 = fma(x, x, g * g);
            }
        }
        const double p12 = d1 * d2;
        const double r = pd_rcp(ap.den * p12);
        double at;
        if constexpr (D)
            at = pd_atan_tab_finish(ap, ap.num * (r * p12));
        else
            at = pd_atan_finish(ap, ap.num * (r * p12));
        const double rd = r * ap.den;
        b.iu2 = (AR == 3) ? rd * d2 : rd;
        b.invf = invf;
        b.f34 = f34;
        b.u = u;
        b.at = at;
        // the constant term last: every multiply-add then takes at most one record entry (a
        // scalar operand), so no entry is first copied to a vector register
        b.psi = fma(c[R_PH3 + 4], at, fma(c[R_PH3 + 3], f34, fma(c[R_PH3 + 2], invf, c[R_PH3 + 1] * mf))) +
                c[R_PH3 + 0];
        if (AR == 3) {
            const double iden = rd * d1;
            b.x = x;
            b.iden = iden;
            if constexpr (D && HAVE_EX)
                b.ahat = iden * ex;   // ex carries the numerator R_AM3
            else
                b.ahat = c[R_AM3 + 0] * iden * (HAVE_EX ? ex : pd_exp(-c[R_AM3 + 3] * x));
        }
    }
    if (AR == 1) {
        const double v = b.v;
        double a = c[R_AM1 + 9];
#pragma unroll
        for (int i = 8; i >= 0; --i) a = fma(a, v, c[R_AM1 + i]);
        b.ahat = a;
    } else if (AR == 2) {
        b.ahat = fma(mf, fma(mf, fma(mf, fma(mf, c[R_AM2 + 4], c[R_AM2 + 3]), c[R_AM2 + 2]), c[R_AM2 + 1]),
                     c[R_AM2 + 0]);
    } else if (PR != 3) {
        const double x = mf - c[R_AM3 + 1];
        const double g = c[R_AM3 + 2];
        const double iden = pd_rcp(fma(x, x, g * g));
        b.x = x;
        b.iden = iden;
        b.ahat = c[R_AM3 + 0] * iden * (HAVE_EX ? ex : pd_exp(-c[R_AM3 + 3] * x));
    }
}

// Per-lane geometric recurrence for the merger-ringdown amplitude exponential along a segment:
// a lane's bins are 64 apart, so exp(-c3 (Ms f_k - f_RD)) advances by the constant factor
// exp(-c3 Ms 64 df).  One exponential per lane and one per wave at the segment start, then one
// multiply per bin; the relative drift after n steps is at most about n ulp.
struct ExpRec {
    double e, r;
    __device__ __forceinline__ void init(const double* __restrict__ c, const GridArgs& g, unsigned k_first,
                                         double scale = 1.0) {
        const double c3 = c[R_AM3 + 3];
        e = scale * pd_exp(-c3 * (c[R_MS] * bin_freq(g, k_first) - c[R_AM3 + 1]));
        r = pd_exp(-c3 * (c[R_MS] * (64.0 * g.df)));
    }
    __device__ __forceinline__ double next() {
        const double v = e;
        e *= r;
        return v;
    }
};

// Runtime region dispatch for one-bin-per-thread kernels.
template <class RC, class TB>
__device__ __forceinline__ void eval_bin_rt(RC rec, const TB& T, int64_t k, double mf,
                                            BinVals& b) {
    const int pr = (mf < kFPhaseJoin) ? 1 : ((mf < rec[R_FP2]) ? 2 : 3);
    const int ar = (mf < kFAmpJoin) ? 1 : ((mf < rec[R_FA2]) ? 2 : 3);
    if (pr == 1) {
        if (ar == 1)
            eval_bin_t<1, 1>(rec, T, k, mf, b);
        else if (ar == 2)
            eval_bin_t<1, 2>(rec, T, k, mf, b);
        else
            eval_bin_t<1, 3>(rec, T, k, mf, b);
    } else if (pr == 2) {
        if (ar == 3)
            eval_bin_t<2, 3>(rec, T, k, mf, b);
        else
            eval_bin_t<2, 2>(rec, T, k, mf, b);
    } else {
        if (ar == 3)
            eval_bin_t<3, 3>(rec, T, k, mf, b);
        else
            eval_bin_t<3, 2>(rec, T, k, mf, b);
    }
}

// Record entries a (phase region, amplitude region) pair touches.
__host__ __device__ constexpr bool slot_touched(int pr, int ar, int s) {
    return s == R_MS || s == R_LNA0 || (pr == 1 && s >= R_PH1 && s < R_PH1 + 13) ||
           (pr == 2 && s >= R_PH2 && s < R_PH2 + 4) || (pr == 3 && s >= R_PH3 && s < R_PH3 + 7) ||
           (ar == 1 && s >= R_AM1 && s < R_AM1 + 10) || (ar == 2 && s >= R_AM2 && s < R_AM2 + 5) ||
           (ar == 3 && s >= R_AM3 && s < R_AM3 + 4);
}

// Record entries a phase-region pass can touch: those of every (phase region, amplitude region)
// pair that phase region meets (the inspiral meets amplitude regions 1-3, the others 2-3).
__host__ __device__ constexpr bool region_slot(int prg, int s) {
    return prg == 1 ? (slot_touched(1, 1, s) || slot_touched(1, 2, s) || slot_touched(1, 3, s))
                    : (slot_touched(prg, 2, s) || slot_touched(prg, 3, s));
}

// Bit s set for each record entry s the pass of phase region prg can touch.
__host__ __device__ constexpr unsigned long long region_slot_mask(int prg) {
    unsigned long long m = 0;
    for (int s = 0; s < REC_N; ++s)
        if (region_slot(prg, s)) m |= 1ull << s;
    return m;
}

// Width of phase region prg's compact partial row: (d|h), (h|h), then the region's entries in
// record order; and the position of entry s (0 <= s < 64) among them (-1: not kept).
// The masks are constants of the three regions, so both come down to a shift and a popcount.
constexpr unsigned long long kRegionSlotMask[3] = {region_slot_mask(1), region_slot_mask(2), region_slot_mask(3)};
__host__ __device__ constexpr int region_row_width(int prg) { return 2 + __builtin_popcountll(kRegionSlotMask[prg - 1]); }
__host__ __device__ inline int region_slot_pos(int prg, int s) {
    const unsigned long long m = prg == 1 ? kRegionSlotMask[0] : (prg == 2 ? kRegionSlotMask[1] : kRegionSlotMask[2]);
    return ((m >> s) & 1ull) ? __builtin_popcountll(m & ((1ull << s) - 1ull)) : -1;
}

// A visitor declares kFd = false when it only accumulates moments sum_k z_k b_k of the basis
// values: the moment of the explicit Mf-dependence is then a fixed combination of those moments
// (fd_from_moments), formed once after the bin loop, and the visit skips it per bin.  The
// merger-ringdown regions add two sums that are not basis moments (vis.ph_x: sum zi t Mf;
// vis.am_x: sum zr Mf (2 x / (x^2 + g^2) + c3)), and the phase entry R_PH3 + 6 is formed from
// them as well.
template <class V, class = void>
struct VisitsFd : std::true_type {};
template <class V>
struct VisitsFd<V, std::void_t<decltype(V::kFd)>> : std::bool_constant<V::kFd> {};

// Visit d Psi / d rec[s] (vis.ph), d ln A / d rec[s] (vis.am) and the explicit
// Mf-dependence: Mf dPsi/dMf and Mf d lnA/dMf (vis.fd), for one bin.
template <int PR, int AR, class V, class RC = const double*>
__device__ __forceinline__ void visit_bin_t(RC c, const BinVals& b, V& vis) {
    constexpr bool D = IsRecMRD<RC>::value;
    constexpr bool FD = VisitsFd<V>::value;
    double fpsi = 0.0;
    if (PR == 1) {
        const double v = b.v, w = b.w, lv = b.lv;
        const double w2 = w * w, w3 = w2 * w, w5 = w3 * w2;
        const double v2 = v * v, v3 = v2 * v, v4 = v3 * v, v5 = v4 * v, v6 = v5 * v;
        const double bs[13] = {w5, w3, w2, w, 1.0, lv, v, v * lv, v2, v3, v4, v5, v6};
        const int pw[13] = {-5, -3, -2, -1, 0, 0, 1, 1, 2, 3, 4, 5, 6};
        // Mf dPsi/dMf = (1/3) [c5 + c7 v + sum_j pw_j c_j b_j]: each term is (c_j b_j) times a small
        // integer, so no coefficient is multiplied by a constant in the bin loop
        double s3 = FD ? fma(c[R_PH1 + 7], v, c[R_PH1 + 5]) : 0.0;
#pragma unroll
        for (int j = 0; j < 13; ++j) {
            vis.ph(R_PH1 + j, bs[j]);
            if (FD && pw[j] != 0) {
                const double cb = c[R_PH1 + j] * bs[j];
                if (pw[j] == 1)
                    s3 += cb;
                else if (pw[j] == -1)
                    s3 -= cb;
                else
                    s3 = fma(static_cast<double>(pw[j]), cb, s3);
            }
        }
        if (FD) fpsi = s3 * sk(1.0 / 3.0);
    } else if (PR == 2) {
        const double i3 = b.invf * b.invf * b.invf;
        vis.ph(R_PH2 + 0, 1.0);
        vis.ph(R_PH2 + 1, b.mf);
        vis.ph(R_PH2 + 2, b.lnf);
        vis.ph(R_PH2 + 3, i3);
        if (FD) fpsi = fma(c[R_PH2 + 1], b.mf, fma(c[R_PH2 + 3] * i3, sk(-3.0), c[R_PH2 + 2]));
    } else if constexpr (D && !FD) {
        // t = R_PH3+4 R_ID / (1 + u^2) is a per-point constant times 1/(1 + u^2): the R_PH3 + 5
        // moment and the extra phase sum take 1/(1 + u^2) and are scaled once after the loop
        // (fd_from_moments)
        vis.ph(R_PH3 + 0, 1.0);
        vis.ph(R_PH3 + 1, b.mf);
        vis.ph(R_PH3 + 2, b.invf);
        vis.ph(R_PH3 + 3, b.f34);
        vis.ph(R_PH3 + 4, b.at);
        vis.ph(R_PH3 + 5, b.iu2);
        vis.ph_x(b.iu2 * b.mf);
    } else {
        double t;
        if constexpr (D)
            t = c.c4id * b.iu2;
        else
            t = c[R_PH3 + 4] * b.iu2 * c[R_ID];
        vis.ph(R_PH3 + 0, 1.0);
        vis.ph(R_PH3 + 1, b.mf);
        vis.ph(R_PH3 + 2, b.invf);
        vis.ph(R_PH3 + 3, b.f34);
        vis.ph(R_PH3 + 4, b.at);
        vis.ph(R_PH3 + 5, -t);
        if constexpr (FD) {
            vis.ph(R_PH3 + 6, -t * b.u);
            if constexpr (D)
                fpsi = fma(c[R_PH3 + 1], b.mf, fma(-c[R_PH3 + 2], b.invf, fma(c.c3q, b.f34, t * b.mf)));
            else
                fpsi = fma(c[R_PH3 + 1], b.mf,
                           fma(-c[R_PH3 + 2], b.invf, fma(c[R_PH3 + 3] * b.f34, sk(0.75), t * b.mf)));
        } else {
            vis.ph_x(t * b.mf);
        }
    }
    double fa = 0.0;
    vis.am(R_LNA0, 1.0);
    if (AR == 1) {
        const double ia = pd_rcp(b.ahat);
        double p = ia;
        double acc = 0.0;
        vis.am(R_AM1 + 0, p);
#pragma unroll
        for (int i = 1; i < 10; ++i) {
            p *= b.v;
            vis.am(R_AM1 + i, p);
            if (FD) acc = fma(static_cast<double>(i), c[R_AM1 + i] * p, acc);
        }
        if (FD) fa = acc * sk(1.0 / 3.0);
    } else if (AR == 2) {
        const double ia = pd_rcp(b.ahat);
        const double f = b.mf;
        double p = ia;
        double acc = 0.0;
        vis.am(R_AM2 + 0, p);
#pragma unroll
        for (int i = 1; i < 5; ++i) {
            p *= f;
            vis.am(R_AM2 + i, p);
            if (FD) acc = fma(static_cast<double>(i), c[R_AM2 + i] * p, acc);
        }
        fa = acc;
    } else if constexpr (D) {
        // a moment visitor's R_AM3 moment is R_IANUM times its ln A0 moment, formed after the
        // loop; a per-bin visitor gets the entry here
        if constexpr (FD) vis.am(R_AM3 + 0, c[R_IANUM]);
        const double x = b.x, r = c[R_AM3 + 3];
        const double txr = fma(x + x, b.iden, r);
        vis.am(R_AM3 + 1, txr);
        // -2 R_AM3+2 / (x^2 + g^2): without a moment visitor's after-loop scaling the per-point
        // factor is applied per bin
        vis.am(R_AM3 + 2, FD ? c.m2g * b.iden : b.iden);
        vis.am(R_AM3 + 3, -x);
        if constexpr (FD)
            fa = -b.mf * txr;
        else
            vis.am_x(b.mf * txr);
    } else {
        const double x = b.x, g = c[R_AM3 + 2], r = c[R_AM3 + 3];
        const double tx = 2.0 * x * b.iden;
        vis.am(R_AM3 + 0, c[R_IANUM]);
        vis.am(R_AM3 + 1, tx + r);
        vis.am(R_AM3 + 2, -2.0 * g * b.iden);
        vis.am(R_AM3 + 3, -x);
        if constexpr (FD)
            fa = -b.mf * (tx + r);
        else
            vis.am_x(b.mf * (tx + r));
    }
    if constexpr (FD) vis.fd(fpsi, fa - sk(7.0 / 6.0));
}

// After a bin loop whose visitor skipped the Mf-derivative (kFd = false): its moment
// mom[R_MS] = sum_k zi Mf dPsi/dMf + zr (Mf d lnA/dMf - 7/6) from the basis moments, following
// the same per-region expressions as visit_bin_t, and in phase region 3 the entry R_PH3 + 6
// (sum zi (-t u), u = Mf R_ID - R_PH3+5 R_ID) from stm = sum zi t Mf and the R_PH3 + 5 moment
// (sum zi (-t)).  sam = sum zr Mf (2 x iden + c3) in amplitude region 3.  Once per segment.
// With the merger-ringdown record (RecMRD) the visit accumulated 1/(1 + u^2) for the R_PH3 + 5
// moment and in stm, and 1/(x^2 + g^2) for the R_AM3 + 2 moment; MRD selects the scaling by the
// per-point factors here.
template <int PR, int AR, bool MRD, class RC>
__device__ __forceinline__ void fd_from_moments(RC c, double (&mom)[REC_N], double stm, double sam) {
    if constexpr (MRD && PR == 3) {
        const double c4id = c[R_PH3 + 4] * c[R_ID];
        mom[R_PH3 + 5] *= -c4id;
        stm *= c4id;
    }
    if constexpr (MRD && AR == 3) mom[R_AM3 + 2] *= -2.0 * c[R_AM3 + 2];
    double fp;
    if constexpr (PR == 1) {
        const int pw[13] = {-5, -3, -2, -1, 0, 0, 1, 1, 2, 3, 4, 5, 6};
        double s3 = fma(c[R_PH1 + 5], mom[R_PH1 + 4], c[R_PH1 + 7] * mom[R_PH1 + 6]);
#pragma unroll
        for (int j = 0; j < 13; ++j)
            if (pw[j] != 0) s3 = fma(static_cast<double>(pw[j]) * c[R_PH1 + j], mom[R_PH1 + j], s3);
        fp = s3 * (1.0 / 3.0);
    } else if constexpr (PR == 2) {
        fp = fma(c[R_PH2 + 1], mom[R_PH2 + 1], fma(-3.0 * c[R_PH2 + 3], mom[R_PH2 + 3], c[R_PH2 + 2] * mom[R_PH2 + 0]));
    } else {
        fp = fma(c[R_PH3 + 1], mom[R_PH3 + 1],
                 fma(-c[R_PH3 + 2], mom[R_PH3 + 2], fma(0.75 * c[R_PH3 + 3], mom[R_PH3 + 3], stm)));
        const double id = c[R_ID];
        mom[R_PH3 + 6] = fma(-id, stm, -(c[R_PH3 + 5] * id) * mom[R_PH3 + 5]);
    }
    double fa = 0.0;
    if constexpr (AR == 1) {
#pragma unroll
        for (int i = 1; i < 10; ++i) fa = fma(static_cast<double>(i) * c[R_AM1 + i], mom[R_AM1 + i], fa);
        fa *= 1.0 / 3.0;
    } else if constexpr (AR == 2) {
#pragma unroll
        for (int i = 1; i < 5; ++i) fa = fma(static_cast<double>(i) * c[R_AM2 + i], mom[R_AM2 + i], fa);
    } else {
        fa = -sam;
    }
    mom[R_MS] = fma(-7.0 / 6.0, mom[R_LNA0], fp + fa);
}

// Chunk `c` of `chunks` of the bins of phase region prg inside the active range: region 1 is
// [ka, b1), region 2 [b1, max(b1, b2)), region 3 [max(b1, b2), kz), where b1 and b2 are the first
// bins at or above the phase joins Mf = 0.018 and rec[R_FP2], found with the same test as the
// segment boundaries, so every segment of the chunk lies in region prg.  Splitting each region
// separately gives every region launch all of its waves.
// Chunks of a point's bins in phase region prg when a pass splits each point over `chunks` waves:
// the inspiral and intermediate regions are usually a small share of the bins, so they are split
// into a quarter as many (at least one); the merger-ringdown region uses all.  Partial-sum slots
// [point][chunk] keep the stride `chunks`; the reductions read the first region_chunks of them.
__host__ __device__ inline int region_chunks(int prg, int chunks) { return prg == 3 ? chunks : (chunks + 3) / 4; }

__device__ __forceinline__ void region_chunk_range(const double* __restrict__ rec, const GridArgs& g, int prg,
                                                   int c, int chunks, int64_t& kb, int64_t& ke) {
    const double ms = rec[R_MS];
    int64_t ka, kz;
    active_range(ms, g, ka, kz);
    auto bound = [&](double t) {
        auto ge = [&](int64_t k) { return ms * bin_freq(g, k) >= t; };
        return first_true(ge, clamp_est(ceil((t / ms - g.f0) / g.df), ka, kz), ka, kz);
    };
    const int64_t b1 = bound(kFPhaseJoin);
    const int64_t b2 = max(b1, bound(rec[R_FP2]));
    const int64_t rs = (prg == 1) ? ka : (prg == 2) ? b1 : b2;
    const int64_t re = (prg == 1) ? b1 : (prg == 2) ? b2 : kz;
    const int64_t len = re - rs;
    int64_t per = (len + chunks - 1) / chunks;
    per = (per + 63) & ~static_cast<int64_t>(63);
    kb = rs + static_cast<int64_t>(c) * per;
    ke = kb + per;
    if (kb > re) kb = re;
    if (ke > re) ke = re;
}

// ---- deterministic wavefront reduction (fixed butterfly order) ---------------------
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// ---- many-value wavefront reduction by recursive halving --------------------------------
// N per-lane values are summed over the 64 lanes in 6 exchange steps (offsets 32 .. 1): at each
// step a lane keeps one half of its current entries (the upper half if its lane bit is set),
// receives its partner's copy of that half and adds.  About N exchanges in total instead of
// 6 N for N separate butterflies, and still a fixed summation order.  Afterwards entry c
// (summed over all lanes) sits in lane halving_lane<N>(c); lane l holds entry halving_entry<N>(l)
// (>= N: nothing).
// Exchange across lane halves (OFF 32: lanes l and l + 32; OFF 16: rows of 16) with the gfx950
// lane-swap instructions: afterwards a holds [a_lo | b_lo] and b holds [a_hi | b_hi] by half, so
// a + b is the halving step with no select.
template <int OFF>
__device__ __forceinline__ void swap_halves(double& a, double& b) {
    const unsigned long long ua = __builtin_bit_cast(unsigned long long, a);
    const unsigned long long ub = __builtin_bit_cast(unsigned long long, b);
    const unsigned alo = static_cast<unsigned>(ua), ahi = static_cast<unsigned>(ua >> 32);
    const unsigned blo = static_cast<unsigned>(ub), bhi = static_cast<unsigned>(ub >> 32);
    unsigned rl0, rl1, rh0, rh1;
    if constexpr (OFF == 32) {
        const auto rl = __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
        const auto rh = __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
        rl0 = rl[0], rl1 = rl[1], rh0 = rh[0], rh1 = rh[1];
    } else {
        const auto rl = __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
        const auto rh = __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
        rl0 = rl[0], rl1 = rl[1], rh0 = rh[0], rh1 = rh[1];
    }
    a = __builtin_bit_cast(double, (static_cast<unsigned long long>(rh0) << 32) | rl0);
    b = __builtin_bit_cast(double, (static_cast<unsigned long long>(rh1) << 32) | rl1);
}

template <int N, int OFF>
struct Halve {
    static __device__ __forceinline__ double run(const double* v, int lane) {
        constexpr int H = (N + 1) / 2;
        double w[H];
        const bool up = (lane & OFF) != 0;
#pragma unroll
        for (int j = 0; j < H; ++j) {
            double a = v[j];
            double b = (H + j < N) ? v[H + j] : 0.0;
            if constexpr (OFF == 32 || OFF == 16) {
                swap_halves<OFF>(a, b);
                w[j] = a + b;
            } else {
                const double send = up ? a : b;
                const double keep = up ? b : a;
                w[j] = keep + __shfl_xor(send, OFF, 64);
            }
        }
        if constexpr (OFF == 1) {
            return w[0];
        } else {
            return Halve<H, OFF / 2>::run(w, lane);
        }
    }
};

template <int N>
__host__ __device__ constexpr int halving_lane(int c) {
    int lane = 0, n = N;
    for (int t = 0; t < 6; ++t) {
        const int h = (n + 1) / 2;
        if (c >= h) {
            c -= h;
            lane |= 32 >> t;
        }
        n = h;
    }
    return lane;
}

template <int N>
__host__ __device__ constexpr int halving_entry(int lane) {
    int hs[6] = {0, 0, 0, 0, 0, 0}, ns[6] = {0, 0, 0, 0, 0, 0};
    int n = N;
    for (int t = 0; t < 6; ++t) {
        ns[t] = n;
        hs[t] = (n + 1) / 2;
        n = hs[t];
    }
    // relative index within the range entering step t; it must stay inside that range
    int c = 0;
    for (int t = 5; t >= 0; --t) {
        if (lane & (32 >> t)) c += hs[t];
        if (c >= ns[t]) return N;
    }
    return c;
}

template <int N>
__device__ __forceinline__ double halving_reduce(const double (&v)[N], int lane) {
    static_assert(N >= 1 && N <= 64, "halving_reduce handles 1..64 entries");
    return Halve<N, 32>::run(v, lane);
}

// Record entries touched by a (phase, amplitude) region pair, in compact order:
// R_MS, R_LNA0, the phase block, the amplitude block.
__host__ __device__ constexpr int phase_block_len(int pr) { return pr == 1 ? 13 : (pr == 2 ? 4 : 7); }
__host__ __device__ constexpr int phase_block_start(int pr) { return pr == 1 ? R_PH1 : (pr == 2 ? R_PH2 : R_PH3); }
__host__ __device__ constexpr int amp_block_len(int ar) { return ar == 1 ? 10 : (ar == 2 ? 5 : 4); }
__host__ __device__ constexpr int amp_block_start(int ar) { return ar == 1 ? R_AM1 : (ar == 2 ? R_AM2 : R_AM3); }

template <int PR, int AR>
__host__ __device__ constexpr int touched_count() { return 2 + phase_block_len(PR) + amp_block_len(AR); }

template <int PR, int AR>
__host__ __device__ constexpr int touched_slot(int c) {
    return c == 0 ? R_MS
                  : (c == 1 ? R_LNA0
                            : (c < 2 + phase_block_len(PR) ? phase_block_start(PR) + c - 2
                                                            : amp_block_start(AR) + c - 2 - phase_block_len(PR)));
}

// Compact index of record entry s for the pair, or -1 if the pair does not touch it.
template <int PR, int AR>
__device__ __forceinline__ int touched_index(int s) {
    if (s == R_MS) return 0;
    if (s == R_LNA0) return 1;
    const int p0 = phase_block_start(PR), a0 = amp_block_start(AR);
    if (s >= p0 && s < p0 + phase_block_len(PR)) return 2 + s - p0;
    if (s >= a0 && s < a0 + amp_block_len(AR)) return 2 + phase_block_len(PR) + s - a0;
    return -1;
}

// Fold a segment's per-lane moments (entries the pair touches) into per-lane totals: lane s
// accumulates the wave sum of record entry s.
template <int PR, int AR>
__device__ __forceinline__ void flush_touched(const double (&mom)[REC_N], int lane, double& tot) {
    constexpr int N = touched_count<PR, AR>();
    double v[N];
#pragma unroll
    for (int c = 0; c < N; ++c) v[c] = mom[touched_slot<PR, AR>(c)];
    const double r = halving_reduce<N>(v, lane);
    const int c = touched_index<PR, AR>(lane);
    const double got = __shfl(r, halving_lane<N>(c < 0 ? 0 : c), 64);
    if (c >= 0) tot += got;
}

// Dispatch over the amplitude region for a fixed phase region.
template <int PR, class F>
__device__ __forceinline__ void dispatch_amp_region(int ar, F& f) {
    if (PR == 1) {
        if (ar == 1)
            f.template run<1, 1>();
        else if (ar == 2)
            f.template run<1, 2>();
        else
            f.template run<1, 3>();
    } else {
        if (ar == 3)
            f.template run<PR, 3>();
        else
            f.template run<PR, 2>();
    }
}

}  // namespace pd
