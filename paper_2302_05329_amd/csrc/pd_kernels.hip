// HIP kernels for gfx950: per-point setup, per-grid tables, strain output, fused
// likelihood (+gradient), Fisher matrices.
//
// Launch shapes
//   setup      one thread per point (value record, or record + 7 theta tangents), or one
//              thread per (point, fit parameter) for the 19 coefficient tangents.
//   tables     one thread per bin: source-independent factors of the grid, once per call.
//   waveform   one thread per bin, 256-bin blocks, point-major: writes complex128.
//   moments    one wavefront per (point, bin chunk).  The chunk is split into model-region
//              segments; each segment loop has its region fixed at compile time.  Lanes
//              take consecutive bins (coalesced table reads), accumulate per lane, and a
//              fixed-order butterfly reduces each segment's moments; lane s keeps slot s.
//   epilogue   one thread per point: sums the chunks in order, contracts moments with
//              record tangents.
// No atomics anywhere: results are bitwise reproducible run to run.
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/phenomd.h"
#include "pd_bin.h"
#include "pd_launch.h"
#include "pd_profile.h"

namespace pd {

// ==================================================================================
// setup
// ==================================================================================

__device__ __forceinline__ void load_row(const double* __restrict__ theta, int64_t i, double th[7]) {
#pragma unroll
    for (int j = 0; j < 7; ++j) th[j] = theta[i * 7 + j];
}

template <class T>
__device__ __forceinline__ void fit_params(const double* __restrict__ lam, const T& eta, const T& chi_pn,
                                           T out[kNumFit]) {
    T b[11];
    fit_basis(eta, chi_pn, b);
    for (int i = 0; i < kNumFit; ++i) {
        T acc = b[0] * lam[i * 11 + 0];
        for (int k = 1; k < 11; ++k) acc = acc + b[k] * lam[i * 11 + k];
        out[i] = acc;
    }
}

__device__ void tables_bin(const GridArgs& g, const double* __restrict__ data,
                           const double* __restrict__ inv_psd, double* __restrict__ tab, int64_t k, int part);

// The per-grid table job of a record setup launch (bt = 0: none).
struct TablesJob {
    GridArgs g;
    const double* data;
    const double* inv_psd;
    double* tab;
    unsigned bs, bt;   // setup blocks, table blocks per part (0: no tables)
};

// XF: theta is first computed from the sampler's coordinates (xform_point) and written out.
// Blocks at or above tj.bs fill the per-grid tables instead (tj.bt blocks per table part): the
// tables do not depend on the points, so they are built in the same launch as the records, on the
// CUs the records leave idle (one thread per point), without a second launch after them.
template <bool XF>
__global__ void __launch_bounds__(128) k_setup_value(double* __restrict__ theta, int64_t n, int param,
                                                     double f_ref, const double* __restrict__ lam,
                                                     double* __restrict__ recs, int32_t* __restrict__ status,
                                                     XForm xf, TablesJob tj) {
    if (blockIdx.x >= tj.bs) {
        const unsigned t = blockIdx.x - tj.bs;
        const int part = static_cast<int>(t / tj.bt);
        tables_bin(tj.g, tj.data, tj.inv_psd, tj.tab, static_cast<int64_t>(t % tj.bt) * blockDim.x + threadIdx.x,
                   part);
        return;
    }
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double th[7];
    if (XF) {
        xform_point(xf, i, th);
        for (int j = 0; j < 7; ++j) theta[i * 7 + j] = th[j];
    } else {
        load_row(theta, i, th);
    }
    double rec[REC_N];
    bool ok = domain_ok(th, param);
    if (ok) {
        const Source<double> s = source_map(th, param);
        double fit[kNumFit];
        fit_params(lam, s.eta, s.chi_pn, fit);
        ok = build_record(s, fit, f_ref, rec);
        for (int j = 0; j < REC_N; ++j) ok = ok && isfinite(rec[j]);
    }
    if (!ok) {
        for (int j = 0; j < REC_N; ++j) rec[j] = 0.0;
        rec[R_MS] = 1.0;
    }
    rec[R_VALID] = ok ? 1.0 : 0.0;
    double* out = recs + i * REC_N;
    for (int j = 0; j < REC_N; ++j) out[j] = rec[j];
    if (status) status[i] = ok ? 0 : -2;
}

// d rec / d theta[dir] for one of the four intrinsic entries (dir < 4), by forward mode with a
// single tangent; returns M_s.
__device__ __forceinline__ double intrinsic_tangent(const double* __restrict__ th_row, int param, double f_ref,
                                                    const double* __restrict__ lam, int dir, double tg[REC_N]) {
    using D = Dual<1>;
    D th[7];
    for (int j = 0; j < 7; ++j) th[j] = dconst<1>(th_row[j]);
    th[dir].d[0] = 1.0;
    const Source<D> s = source_map(th, param);
    D fit[kNumFit];
    fit_params(lam, s.eta, s.chi_pn, fit);
    D rec[REC_N];
    build_record(s, fit, f_ref, rec);
    for (int j = 0; j < REC_N; ++j) tg[j] = rec[j].d[0];
    return rec[R_MS].v;
}

// Record tangents along the 7 entries of theta.  The four intrinsic entries (masses or
// chirp mass and mass ratio, two spins) go through the setup in forward mode, one thread per
// (point, direction) with a single tangent (Dual<1>) so the live state stays small; the
// extrinsic ones enter the record in closed form: D (or ln D) only through ln A0, tc only
// through the Mf-linear phase coefficient (2 pi tc / Ms), phic only through the constant
// phase term (-2 phic).  Thread (point, 0) also writes the three extrinsic rows.
// ROWS 7: all seven rows (the Fisher kernels' layout); ROWS 4: the intrinsic rows only.  Thread
// (point, dir) does not read the record, so this can run while the records are being built.
template <int ROWS>
__global__ void __launch_bounds__(64) k_setup_theta_tangent(const double* __restrict__ theta, int64_t n,
                                                            int param, double f_ref,
                                                            const double* __restrict__ lam,
                                                            double* __restrict__ tans) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n * 4) return;
    const int64_t i = t >> 2;
    const int dir = static_cast<int>(t & 3);
    double* out = tans + i * ROWS * REC_N;
    if (ROWS == 7 && dir == 0)
        for (int j = 4 * REC_N; j < 7 * REC_N; ++j) out[j] = 0.0;
    double tg[REC_N];
    const double ms = intrinsic_tangent(theta + i * 7, param, f_ref, lam, dir, tg);
    for (int j = 0; j < REC_N; ++j) out[dir * REC_N + j] = tg[j];
    if (ROWS != 7 || dir != 0) return;
    out[4 * REC_N + R_LNA0] = (param == 1) ? -1.0 : -1.0 / theta[i * 7 + 4];
    const double dlin = 2.0 * kPi / ms;
    out[5 * REC_N + R_PH1 + 9] = dlin / kPi;
    out[5 * REC_N + R_PH2 + 1] = dlin;
    out[5 * REC_N + R_PH3 + 1] = dlin;
    out[6 * REC_N + R_PH1 + 4] = -2.0;
    out[6 * REC_N + R_PH2 + 0] = -2.0;
    out[6 * REC_N + R_PH3 + 0] = -2.0;
}

// Record tangents along the 19 fitted parameters: thread (point, l) seeds parameter l.
__global__ void __launch_bounds__(64) k_setup_fit_tangent(const double* __restrict__ theta, int64_t n, int param,
                                                          double f_ref, const double* __restrict__ lam,
                                                          const double* __restrict__ recs,
                                                          double* __restrict__ tans) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n * kNumFit) return;
    const int64_t i = t / kNumFit;
    const int l = static_cast<int>(t % kNumFit);
    double* out = tans + (i * kNumFit + l) * REC_N;
    if (recs[i * REC_N + R_VALID] == 0.0) {
        for (int j = 0; j < REC_N; ++j) out[j] = 0.0;
        return;
    }
    using D = Dual<1>;
    D th[7];
    for (int j = 0; j < 7; ++j) th[j] = dconst<1>(theta[i * 7 + j]);
    const Source<D> s = source_map(th, param);
    D fit[kNumFit];
    fit_params(lam, s.eta, s.chi_pn, fit);
    fit[l].d[0] = 1.0;
    D rec[REC_N];
    build_record(s, fit, f_ref, rec);
    for (int j = 0; j < REC_N; ++j) out[j] = rec[j].d[0];
}

// ==================================================================================
// per-grid tables
// ==================================================================================

// Bin k's part `part` of the per-grid tables: four parts per bin, one per transcendental (cbrt;
// log; f^(3/4); f^(-7/6) with the weighted data), each taken by its own range of blocks of the
// record setup launch: the table blocks are a few waves per SIMD, so their time is one thread's
// chain of calls, which this cuts to one call, and every wave runs a single part (no divergence).
__device__ void tables_bin(const GridArgs& g, const double* __restrict__ data,
                           const double* __restrict__ inv_psd, double* __restrict__ tab, int64_t k, int part) {
    if (k >= g.nb) return;
    const double f = bin_freq(g, k);
    const bool pos = f > 0.0;
    const int64_t nb = g.nb;
    if (part == 0) {
        double cb = 0.0, icb = 0.0, inf = 0.0;
        if (pos) {
            cb = cbrt(f);
            icb = 1.0 / cb;
            inf = 1.0 / f;
        }
        tab[T_CB * nb + k] = cb;
        tab[T_ICB * nb + k] = icb;
        tab[T_INF * nb + k] = inf;
    } else if (part == 1) {
        tab[T_LF * nb + k] = pos ? log(f) : 0.0;
    } else if (part == 2) {
        tab[T_F34 * nb + k] = pos ? pow(f, 0.75) : 0.0;
    } else {
        const double f76 = pos ? pow(f, -7.0 / 6.0) : 0.0;
        tab[T_F76 * nb + k] = f76;
        double dwr = 0.0, dwi = 0.0, ww = 0.0;
        if (inv_psd) {
            const double w = 4.0 * g.df * inv_psd[k];
            ww = w * f76 * f76;
            if (data) {
                const double2 d = reinterpret_cast<const double2*>(data)[k];
                dwr = w * f76 * d.x;
                dwi = w * f76 * d.y;
            }
        }
        tab[T_DWR * nb + k] = dwr;
        tab[T_DWI * nb + k] = dwi;
        tab[T_WW * nb + k] = ww;
    }
}


// ==================================================================================
// strain output
// ==================================================================================

// One block covers 256 * PT consecutive bins of one point; each thread writes PT bins strided by
// 256, so every store instruction of a wave is one contiguous 1 KB run.  Large batches take PT = 8
// (the per-point record loads and branch set-up shared by eight bins: 2.9 -> 4.0 TB/s of strain
// written at 10^4 points x 79361 bins; 4 and 16 measured 3.5 and 3.9 TB/s); small ones PT = 1,
// which keeps more blocks in flight.
template <int PT>
__global__ void __launch_bounds__(256) k_waveform(const double* __restrict__ recs, int64_t n, int64_t blocks_per_point,
                                                  GridArgs g, const double* __restrict__ tab, double* __restrict__ h) {
    constexpr int64_t kWfPerThread = PT;
    const int64_t b = blockIdx.x;
    const int64_t p = b / blocks_per_point;
    if (p >= n) return;
    const int64_t k0 = (b % blocks_per_point) * (256 * kWfPerThread) + threadIdx.x;
    const double* __restrict__ rec = recs + p * REC_N;
    const Tabs T(tab, g.nb);
    double2* __restrict__ hp = reinterpret_cast<double2*>(h) + p * g.nb;
    const bool valid = rec[R_VALID] != 0.0;
#pragma unroll 1
    for (int j = 0; j < kWfPerThread; ++j) {
        const int64_t k = k0 + j * 256;
        if (k >= g.nb) break;
        double2 out = make_double2(0.0, 0.0);
        if (!valid) {
            out = make_double2(__builtin_nan(""), __builtin_nan(""));
        } else {
            const double f = bin_freq(g, k);
            const double mf = rec[R_MS] * f;
            if (bin_active(g, f, mf)) {
                BinVals bv;
                eval_bin_rt(rec, T, k, mf, bv);
                const double A = rec[R_A0P] * T.at(T_F76, k) * bv.ahat;
                double s, c;
                pd_sincos(bv.psi, &s, &c);
                out = make_double2(A * c, -A * s);
            }
        }
        hp[k] = out;
    }
}

// ==================================================================================
// fused likelihood / gradient moments
// ==================================================================================

// Moments sum_k z_k b_k of the basis values; the Mf-derivative moment is formed after the loop
// (fd_from_moments) from them and the two extra sums x[0] (phase) and x[1] (amplitude).  The ln A0
// moment, sum zr = sum (px - a0p q), is formed after the loop from the segment's (d|h) and (h|h)
// sums, which the loop keeps anyway, so it is not accumulated per bin.
struct MomVis {
    static constexpr bool kFd = false;
    double* mom;
    double* x;
    double zr, zi;
    __device__ __forceinline__ void ph(int s, double b) { mom[s] = fma(zi, b, mom[s]); }
    __device__ __forceinline__ void am(int s, double b) {
        if (s != R_LNA0) mom[s] = fma(zr, b, mom[s]);
    }
    __device__ __forceinline__ void ph_x(double b) { x[0] = fma(zi, b, x[0]); }
    __device__ __forceinline__ void am_x(double b) { x[1] = fma(zr, b, x[1]); }
};

// One region segment of the likelihood loop.  MODE 0: (d|h), (h|h); MODE 1: + moments.  The
// moments are accumulated without the per-point amplitude factor a0p, which the caller applies
// once to the wave totals.
template <int MODE>
struct LnlSegment {
    const double* __restrict__ rec;
    Tabs T;
    GridArgs g;
    const double2* __restrict__ sct;   // (sin, cos) table in LDS
    // the wave's copy of the record in LDS, read by the code after each bin loop: the loop reloads
    // the record's uniform entries on its trips, and a loop-loaded value used after a loop whose
    // lanes leave at different trips is copied to vector registers on every trip; entries read
    // from LDS after the loop are never merged with the loop's loads
    const double* recl;
    int64_t k0, k1;
    int lane;
    double dh, hh, tot;

    template <int PR, int AR>
    __device__ __forceinline__ void run() {
        if constexpr (PR == 3)
            run_with<PR, AR>(rec_mrd(rec, sct + kSinCosN));
        else
            run_with<PR, AR>(rec);
    }

    template <int PR, int AR, class RC>
    __device__ __forceinline__ void run_with(RC c) {
        constexpr bool D = IsRecMRD<RC>::value;
        const double ms = rec[R_MS];
        const double a0p = rec[R_A0P];
        double mom[REC_N];
#pragma unroll
        for (int s = 0; s < REC_N; ++s) mom[s] = 0.0;
        double mx[2] = {0.0, 0.0};
        double dh_s = 0.0, hh_s = 0.0;   // this segment's (d|h) and (h|h) sums
        ExpRec er{};
        if (AR == 3) er.init(rec, g, static_cast<unsigned>(k0 + lane), D ? rec[R_AM3 + 0] : 1.0);
        for (unsigned k = static_cast<unsigned>(k0 + lane); k < static_cast<unsigned>(k1); k += 64u) {
            // merger-ringdown: every grid-table value of the bin is loaded here, before the
            // branches of the elementary functions, so all loads share one 32-bit offset from
            // scalar bases (the entries the region does not use are never loaded); the other
            // loops keep their loads at the uses (preloading the inspiral's six values spills)
            const double mf = ms * bin_freq(g, k);
            BinVals bv;
            double dwr, dwi, ww;
            if constexpr (PR == 3) {
                dwr = T.at(T_DWR, k);
                dwi = T.at(T_DWI, k);
                ww = T.at(T_WW, k);
                BinTabs bt;
                bt.load(T, k);
                eval_bin_t<PR, AR, AR == 3>(c, bt, k, mf, bv, (AR == 3) ? er.next() : 0.0);
            } else {
                eval_bin_t<PR, AR, AR == 3>(c, T, k, mf, bv, (AR == 3) ? er.next() : 0.0);
            }
            // px = Re(conj(d) h), py = Im(conj(d) h) with h = Ahat exp(-i Psi) (weights folded in);
            // the inspiral loop forms sin and cos first and loads the data after them (the fused
            // rotation, or the data loaded earlier, spills there)
            double px, py, hr = 0.0, hi = 0.0;
            if constexpr (PR == 2) {
                dwr = T.at(T_DWR, k);
                dwi = T.at(T_DWI, k);
                ww = T.at(T_WW, k);
            }
            if constexpr (PR != 1) {
                pd_rotate_data(bv.psi, bv.ahat, dwr, dwi, sct, px, py);
            } else {
                double sn, cs;
                pd_sincos(bv.psi, &sn, &cs, sct);
                hr = bv.ahat * cs;
                hi = -bv.ahat * sn;
                dwr = T.at(T_DWR, k);
                dwi = T.at(T_DWI, k);
                ww = T.at(T_WW, k);
                px = fma(dwr, hr, dwi * hi);
            }
            const double q = ww * bv.ahat * bv.ahat;
            dh_s += px;
            hh_s += q;
            if (MODE == 1) {
                if constexpr (PR == 1) py = fma(dwr, hi, -dwi * hr);
                MomVis vis{mom, mx, fma(-a0p, q, px), py};
                visit_bin_t<PR, AR>(c, bv, vis);
            }
        }
        dh += dh_s;
        hh += hh_s;
        if (MODE == 1) {
            mom[R_LNA0] = fma(-a0p, hh_s, dh_s);
            // (the inspiral loops read the record itself: its copy there measured more vector copies)
            fd_from_moments<PR, AR, D>(PR == 1 ? rec : recl, mom, mx[0], mx[1]);
            if (D && AR == 3) mom[R_AM3 + 0] = rec[R_IANUM] * mom[R_LNA0];
            flush_touched<PR, AR>(mom, lane, tot);
        }
    }
};

// Start of phase region prg's partial rows [n][chunks][width]: value passes 2 entries per row,
// gradient passes the compact row of region_row_width(prg) entries; the regions' blocks follow
// one another.
template <int MODE>
__host__ __device__ inline int64_t grad_group_offset(int prg, int64_t n, int chunks) {
    if (MODE == 0) return static_cast<int64_t>(prg - 1) * n * chunks * 2;
    int64_t off = 0;
    for (int r = 1; r < prg; ++r) off += n * chunks * region_row_width(r);
    return off;
}

// One wave's share of the fused pass: PRG is the phase region (1 inspiral, 2 intermediate,
// 3 merger-ringdown) whose segments it handles, `wave` its index among that region's waves.
template <int MODE, int PRG>
__device__ __forceinline__ void moments_wave(int64_t wave, const double* __restrict__ recs, int64_t n, int chunks,
                                             const GridArgs& g, const double* __restrict__ tab,
                                             const int* __restrict__ segs, const int* __restrict__ perm,
                                             double* __restrict__ partial_all, const double2* __restrict__ sct,
                                             double* recl) {
    // value passes keep (d|h), (h|h) per row; gradient passes a compact row of the region's entries
    constexpr int NS = (MODE == 0) ? 2 : region_row_width(PRG);
    double* __restrict__ partial = partial_all + grad_group_offset<MODE>(PRG, n, chunks);
    const int lane = threadIdx.x & 63;
    const int cr = region_chunks(PRG, chunks);
    // the wave's point and chunk are wave-uniform: kept in scalar registers, so the record pointer
    // (and every record entry read through it) stays scalar inside the bin loops
    const int64_t pi = uniform_i(wave / cr);
    const int c = uniform_i(wave - pi * cr);
    if (pi >= n) return;
    // waves visit the points in order of decreasing work (see k_order_scatter), or in index order
    const int64_t p = perm ? static_cast<int64_t>(__builtin_amdgcn_readfirstlane(perm[pi])) : pi;
    const double* __restrict__ rec = recs + p * REC_N;
    double* __restrict__ out = partial + (p * chunks + c) * NS;
    if (rec[R_VALID] == 0.0) {
        for (int s = lane; s < NS; s += 64) out[s] = 0.0;
        return;
    }
    if (MODE == 1 && lane < REC_N) recl[lane] = rec[lane];
    Segs S;
    load_segments(segs + ((PRG - 1) * n * chunks + p * chunks + c) * kSegInts, S);
    LnlSegment<MODE> seg{rec, Tabs(tab, g.nb), g, sct, recl, 0, 0, lane, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        if (uniform_i(S.k[i + 1]) > uniform_i(S.k[i]) && uniform_i(S.pr[i]) == PRG) {
            seg.k0 = uniform_i(S.k[i]);
            seg.k1 = uniform_i(S.k[i + 1]);
            dispatch_amp_region<PRG>(uniform_i(S.ar[i]), seg);
        }
    }
    const double a0p = rec[R_A0P];
    const double dv[2] = {seg.dh, seg.hh};
    const double r = halving_reduce<2>(dv, lane);
    if (lane == halving_lane<2>(0)) out[0] = r * a0p;
    if (lane == halving_lane<2>(1)) out[1] = r * (a0p * a0p);
    if (MODE == 1 && lane < REC_N) {
        const int pos = region_slot_pos(PRG, lane);
        if (pos >= 0) out[2 + pos] = seg.tot * a0p;
    }
}

// One launch per phase region (concurrent on three streams, or in sequence).
template <int MODE, int PRG>
__global__ void __launch_bounds__(256, 4) k_loglike_moments(const double* __restrict__ recs, int64_t n, int chunks,
                                                         GridArgs g, const double* __restrict__ tab,
                                                         const int* __restrict__ segs,
                                                         const int* __restrict__ perm,
                                                         double* __restrict__ partial_all) {
    __shared__ double2 sct[kSinCosN + kAtanN];   // (sin, cos) table, then the arc tangent table
    stage_sincos_table(sct);
    stage_atan_table(sct + kSinCosN);
    __syncthreads();
    const int64_t wave = __builtin_amdgcn_readfirstlane(static_cast<int>(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
    __shared__ double recl[4][REC_N];
    moments_wave<MODE, PRG>(wave, recs, n, chunks, g, tab, segs, perm, partial_all, sct, recl[threadIdx.x >> 6]);
}

// The three regions in one launch: blocks [0, nb3) take the merger-ringdown waves, the next nb2 the
// intermediate ones, the rest the inspiral ones (no stream fork and join; for small batches).
template <int MODE>
__global__ void __launch_bounds__(256, 4) k_loglike_moments_all(const double* __restrict__ recs, int64_t n,
                                                             int chunks, GridArgs g, const double* __restrict__ tab,
                                                             const int* __restrict__ segs,
                                                             const int* __restrict__ perm,
                                                             double* __restrict__ partial_all, unsigned nb3,
                                                             unsigned nb2) {
    __shared__ double2 sct[kSinCosN + kAtanN];   // (sin, cos) table, then the arc tangent table
    stage_sincos_table(sct);
    stage_atan_table(sct + kSinCosN);
    __shared__ double recl[4][REC_N];
    __syncthreads();
    const unsigned b = blockIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    if (b < nb3)
        moments_wave<MODE, 3>(static_cast<int64_t>(b) * 4 + w, recs, n, chunks, g, tab, segs, perm, partial_all, sct,
                              recl[w]);
    else if (b < nb3 + nb2)
        moments_wave<MODE, 2>(static_cast<int64_t>(b - nb3) * 4 + w, recs, n, chunks, g, tab, segs, perm,
                              partial_all, sct, recl[w]);
    else
        moments_wave<MODE, 1>(static_cast<int64_t>(b - nb3 - nb2) * 4 + w, recs, n, chunks, g, tab, segs, perm,
                              partial_all, sct, recl[w]);
}

// Value-only likelihood: one thread per point sums its (d|h), (h|h) partials over the region
// groups and chunks.
__global__ void __launch_bounds__(128) k_loglike_value_epilogue(const double* __restrict__ recs, int64_t n,
                                                                int chunks, const double* __restrict__ partial,
                                                                double* __restrict__ lnl) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= n) return;
    if (recs[p * REC_N + R_VALID] == 0.0) {
        lnl[p] = __builtin_nan("");
        return;
    }
    double dh = 0.0, hh = 0.0;
    for (int grp = 0; grp < 3; ++grp)
        for (int c = 0; c < region_chunks(grp + 1, chunks); ++c) {
            const double* src = partial + ((grp * n + p) * chunks + c) * 2;
            dh += src[0];
            hh += src[1];
        }
    lnl[p] = dh - 0.5 * hh;
}

// One wave per point: lane j (< 62) sums partial slot j over the three region groups and the
// point's chunks (a region's rows keep only the entries it touches; each row is contiguous), the four intrinsic
// directions are contracted lane-wise with the record tangents (computed concurrently by
// k_setup_theta_tangent<4>) and summed over the wave in a fixed order, and the three extrinsic
// entries use closed-form record tangents (D or ln D only through ln A0, tc only through the
// Mf-linear phase coefficient 2 pi tc / Ms, phic only through the constant phase term -2 phic).
__global__ void __launch_bounds__(256) k_loglike_grad_epilogue(const double* __restrict__ theta, int64_t n,
                                                               int param, const double* __restrict__ recs,
                                                               const double* __restrict__ tans, int chunks,
                                                               const double* __restrict__ partial,
                                                               double* __restrict__ lnl, double* __restrict__ grad,
                                                               PostTail tail, int has_tail) {
    constexpr int NS = kNSlot;
    static_assert(NS <= 64, "one lane per partial slot");
    const int lane = threadIdx.x & 63;
    const int64_t p = static_cast<int64_t>(blockIdx.x) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (p >= n) return;
    const double* __restrict__ rec = recs + p * REC_N;
    if (rec[R_VALID] == 0.0) {
        if (lane == 0) lnl[p] = __builtin_nan("");
        if (lane < 7) grad[p * 7 + lane] = __builtin_nan("");
        if (has_tail) {
            if (lane == 0) tail.logp[p] = -INFINITY;
            if (lane < 7) tail.grad[p * 7 + lane] = 0.0;
        }
        return;
    }
    double m = 0.0;     // lane 0: (d|h), lane 1: (h|h), lane 2 + j: moment j
    if (lane < NS) {
        for (int grp = 0; grp < 3; ++grp) {
            const int prg = grp + 1;
            // this lane's entry in the region's compact row (rows hold only the entries it touches)
            const int pos = (lane < 2) ? lane - 2 : region_slot_pos(prg, lane - 2);
            if (lane >= 2 && pos < 0) continue;
            const int col = 2 + pos;
            const int w = region_row_width(prg);
            const double* __restrict__ rows = partial + grad_group_offset<1>(prg, n, chunks);
            for (int c = 0; c < region_chunks(prg, chunks); ++c) m += rows[(p * chunks + c) * w + col];
        }
    }
    auto at = [&](int slot) {   // wave-uniform copy of one lane's sum
        const unsigned long long b = __builtin_bit_cast(unsigned long long, m);
        const unsigned lo = __builtin_amdgcn_readlane(static_cast<int>(static_cast<unsigned>(b)), slot);
        const unsigned hi = __builtin_amdgcn_readlane(static_cast<int>(static_cast<unsigned>(b >> 32)), slot);
        return __builtin_bit_cast(double, (static_cast<unsigned long long>(hi) << 32) | lo);
    };
    const double ms = rec[R_MS];
    // record entries the moments are contracted over: Ms (through ln Ms), ln A0 and the phase and
    // amplitude coefficients
    const int j = lane - 2;
    const bool used = j == R_MS || j == R_LNA0 || (j >= R_PH1 && j < R_VALID);
    const double wj = used ? ((j == R_MS) ? m / ms : m) : 0.0;
    double gd[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) gd[d] = used ? tans[(p * 4 + d) * REC_N + j] * wj : 0.0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int d = 0; d < 4; ++d) gd[d] += __shfl_xor(gd[d], off, 64);
    const double dlin = 2.0 * kPi / ms;
    double out = 0.0;
    if (lane < 4) out = (lane == 0) ? gd[0] : (lane == 1) ? gd[1] : (lane == 2) ? gd[2] : gd[3];
    if (lane == 4) out = ((param == 1) ? -1.0 : -1.0 / theta[p * 7 + 4]) * at(2 + R_LNA0);
    if (lane == 5) out = dlin * (at(2 + R_PH1 + 9) / kPi + at(2 + R_PH2 + 1) + at(2 + R_PH3 + 1));
    if (lane == 6) out = -2.0 * (at(2 + R_PH1 + 4) + at(2 + R_PH2 + 0) + at(2 + R_PH3 + 0));
    if (lane < 7) grad[p * 7 + lane] = out;
    const double lv = at(0) - 0.5 * at(1);
    if (lane == 0) lnl[p] = lv;
    if (has_tail) {
        const bool ok = isfinite(lv);
        double gx = 0.0;
        if (lane < 7) {
            gx = ok ? fma(out, tail.dtdx[p * 7 + lane], tail.dlj[p * 7 + lane]) : 0.0;
            tail.grad[p * 7 + lane] = gx;
        }
        if (lane == 0) tail.logp[p] = ok ? lv + tail.lj[p] : -INFINITY;
        if (tail.p) {
            double gk[7];
#pragma unroll
            for (int k = 0; k < 7; ++k) {
                const unsigned long long b = __builtin_bit_cast(unsigned long long, gx);
                const unsigned lo = __builtin_amdgcn_readlane(static_cast<int>(static_cast<unsigned>(b)), k);
                const unsigned hi = __builtin_amdgcn_readlane(static_cast<int>(static_cast<unsigned>(b >> 32)), k);
                gk[k] = __builtin_bit_cast(double, (static_cast<unsigned long long>(hi) << 32) | lo);
            }
            // lane j: p_j += weps sum_{k >= j} L[k][j] g_k (the metric's kick)
            if (lane < 7) {
                double acc = 0.0;
                if (tail.m.diag) {
                    acc = tail.m.L[lane][lane] * gk[lane];
                } else {
                    for (int k = lane; k < 7; ++k) acc = fma(tail.m.L[k][lane], gk[k], acc);
                }
                tail.p[p * 7 + lane] = fma(tail.weps, acc, tail.p[p * 7 + lane]);
            }
        }
    }
}

// ==================================================================================
// Fisher matrices
// ==================================================================================

// Per-bin derivatives of Psi and ln A along the four intrinsic directions (record tangents in
// LDS).  The extrinsic directions need no tangents: d ln A / d(D or ln D) is a per-point
// constant, d Psi / d tc = 2 pi f and d Psi / d phic = -2, so their Fisher entries come from
// weighted moments (see kFisherAcc).
constexpr int kFisherDirs = 4;
struct FisherVis {
    const double* T;   // [4][REC_N] tangents in LDS
    double ims;
    double dpsi[kFisherDirs], dlna[kFisherDirs];
    __device__ __forceinline__ void ph(int s, double b) {
#pragma unroll
        for (int q = 0; q < kFisherDirs; ++q) dpsi[q] = fma(T[q * REC_N + s], b, dpsi[q]);
    }
    __device__ __forceinline__ void am(int s, double b) {
#pragma unroll
        for (int q = 0; q < kFisherDirs; ++q) dlna[q] = fma(T[q * REC_N + s], b, dlna[q]);
    }
    __device__ __forceinline__ void fd(double fpsi, double fa) {
#pragma unroll
        for (int q = 0; q < kFisherDirs; ++q) {
            const double m = T[q * REC_N + R_MS] * ims;
            dpsi[q] = fma(m, fpsi, dpsi[q]);
            dlna[q] = fma(m, fa, dlna[q]);
        }
    }
};

// Per point and chunk: [0, 10) sum W (dlna_a dlna_b + dpsi_a dpsi_b), a <= b < 4;
// [10, 14) sum W dlna_a; [14, 18) sum W f dpsi_a; [18, 22) sum W dpsi_a; 22..24: sum W, W f, W f^2,
// with W = w |h|^2 and f the frequency in Hz.
constexpr int kFisherAcc = kFisherSlots;

struct FisherSegment {
    const double* __restrict__ rec;
    const double* Tl;
    const double2* __restrict__ atab;   // arc tangent table in LDS (merger-ringdown launch)
    Tabs T;
    GridArgs g;
    int64_t k0, k1;
    int lane;
    double F[kFisherAcc];

    // merger-ringdown segments use the record form with the table-reduced arc tangent
    template <int PR, int AR>
    __device__ __forceinline__ void run() {
        if constexpr (PR == 3)
            run_with<PR, AR>(rec_mrd(rec, atab));
        else
            run_with<PR, AR>(rec);
    }

    template <int PR, int AR, class RC>
    __device__ __forceinline__ void run_with(RC c) {
        constexpr bool D = IsRecMRD<RC>::value;
        const double ms = rec[R_MS];
        const double a0p = rec[R_A0P];
        ExpRec er{};
        // the merger-ringdown record form takes the amplitude numerator R_AM3 in the recurrence
        if (AR == 3) er.init(rec, g, static_cast<unsigned>(k0 + lane), D ? rec[R_AM3 + 0] : 1.0);
        for (unsigned k = static_cast<unsigned>(k0 + lane); k < static_cast<unsigned>(k1); k += 64u) {
            const double mf = ms * bin_freq(g, k);
            BinVals bv;
            eval_bin_t<PR, AR, AR == 3>(c, T, k, mf, bv, (AR == 3) ? er.next() : 0.0);
            const double W = (a0p * a0p) * T.at(T_WW, k) * bv.ahat * bv.ahat;
            FisherVis vis;
            // the tangents are re-read from LDS in every bin (broadcast reads): an opaque offset
            // keeps the compiler from hoisting 4 x REC_N of them into vector registers, which
            // would cut the occupancy to one or two waves per SIMD
            int toff = 0;
            asm volatile("" : "+s"(toff));
            vis.T = Tl + toff;
            vis.ims = rec[R_IMS];
#pragma unroll
            for (int q = 0; q < kFisherDirs; ++q) vis.dpsi[q] = vis.dlna[q] = 0.0;
            visit_bin_t<PR, AR>(c, bv, vis);
            int s = 0;
#pragma unroll
            for (int a = 0; a < kFisherDirs; ++a) {
                const double wa = W * vis.dlna[a], wp = W * vis.dpsi[a];
#pragma unroll
                for (int b = a; b < kFisherDirs; ++b) {
                    F[s] = fma(wa, vis.dlna[b], fma(wp, vis.dpsi[b], F[s]));
                    ++s;
                }
            }
            const double f = bin_freq(g, k);
            const double Wf = W * f;
#pragma unroll
            for (int a = 0; a < kFisherDirs; ++a) {
                F[10 + a] = fma(W, vis.dlna[a], F[10 + a]);
                F[14 + a] = fma(Wf, vis.dpsi[a], F[14 + a]);
                F[18 + a] = fma(W, vis.dpsi[a], F[18 + a]);
            }
            F[22] += W;
            F[23] += Wf;
            F[24] = fma(Wf, f, F[24]);
        }
    }
};

template <int PRG>
__global__ void __launch_bounds__(256, 3) k_fisher_partial(const double* __restrict__ recs,
                                                        const double* __restrict__ tans, int64_t n, int chunks,
                                                        GridArgs g, const double* __restrict__ tab,
                                                        const int* __restrict__ segs,
                                                        const int* __restrict__ perm,
                                                        double* __restrict__ partial_all) {
    double* __restrict__ partial = partial_all + static_cast<int64_t>(PRG - 1) * n * chunks * kFisherAcc;
    __shared__ double lds[4][kFisherDirs * REC_N];
    __shared__ double2 atl[PRG == 3 ? kAtanN : 1];
    if (PRG == 3) stage_atan_table(atl);
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    const int cr = region_chunks(PRG, chunks);
    const int64_t wave = __builtin_amdgcn_readfirstlane(static_cast<int>(blockIdx.x * 4 + wib));
    // wave-uniform point and chunk, kept in scalar registers (the record stays scalar in the loops)
    const int64_t pi = uniform_i(wave / cr);
    const int c = uniform_i(wave - pi * cr);
    const bool live = pi < n;
    // points in order of decreasing work, as in the likelihood passes
    const int64_t p = (live && perm) ? static_cast<int64_t>(__builtin_amdgcn_readfirstlane(perm[pi])) : pi;
    double* T = lds[wib];
    if (live) {
        for (int j = lane; j < kFisherDirs * REC_N; j += 64) T[j] = tans[p * 7 * REC_N + j];
    }
    __syncthreads();
    if (!live) return;
    const double* __restrict__ rec = recs + p * REC_N;
    double* __restrict__ out = partial + (p * chunks + c) * kFisherAcc;
    if (rec[R_VALID] == 0.0) {
        if (lane < kFisherAcc) out[lane] = 0.0;
        return;
    }
    Segs S;
    load_segments(segs + ((PRG - 1) * n * chunks + p * chunks + c) * kSegInts, S);
    FisherSegment seg;
    seg.rec = rec;
    seg.Tl = T;
    seg.atab = atl;
    seg.T = Tabs(tab, g.nb);
    seg.g = g;
    seg.lane = lane;
#pragma unroll
    for (int s = 0; s < kFisherAcc; ++s) seg.F[s] = 0.0;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        if (uniform_i(S.k[i + 1]) > uniform_i(S.k[i]) && uniform_i(S.pr[i]) == PRG) {
            seg.k0 = uniform_i(S.k[i]);
            seg.k1 = uniform_i(S.k[i + 1]);
            dispatch_amp_region<PRG>(uniform_i(S.ar[i]), seg);
        }
    }
    const double r = halving_reduce<kFisherAcc>(seg.F, lane);
    const int entry = halving_entry<kFisherAcc>(lane);
    if (entry < kFisherAcc) out[entry] = r;
}

__global__ void __launch_bounds__(128) k_fisher_epilogue(const double* __restrict__ theta, int param,
                                                         const double* __restrict__ recs, int64_t n, int chunks,
                                                         const double* __restrict__ partial,
                                                         double* __restrict__ F) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= n) return;
    double* out = F + p * 49;
    if (recs[p * REC_N + R_VALID] == 0.0) {
        for (int j = 0; j < 49; ++j) out[j] = __builtin_nan("");
        return;
    }
    double acc[kFisherAcc];
#pragma unroll
    for (int s = 0; s < kFisherAcc; ++s) acc[s] = 0.0;
    for (int grp = 0; grp < 3; ++grp)
        for (int c = 0; c < region_chunks(grp + 1, chunks); ++c)
#pragma unroll
            for (int s = 0; s < kFisherAcc; ++s) acc[s] += partial[((grp * n + p) * chunks + c) * kFisherAcc + s];
    // d ln A / d theta_4 (distance or its logarithm); d Psi / d tc = 2 pi f; d Psi / d phic = -2
    const double e4 = (param == 1) ? -1.0 : -1.0 / theta[p * 7 + 4];
    double M[7][7];
    int s = 0;
#pragma unroll
    for (int a = 0; a < kFisherDirs; ++a)
#pragma unroll
        for (int b = a; b < kFisherDirs; ++b) M[a][b] = acc[s++];
#pragma unroll
    for (int a = 0; a < kFisherDirs; ++a) {
        M[a][4] = e4 * acc[10 + a];
        M[a][5] = 2.0 * kPi * acc[14 + a];
        M[a][6] = -2.0 * acc[18 + a];
    }
    M[4][4] = e4 * e4 * acc[22];
    M[4][5] = 0.0;
    M[4][6] = 0.0;
    M[5][5] = 4.0 * kPi * kPi * acc[24];
    M[5][6] = -4.0 * kPi * acc[23];
    M[6][6] = 4.0 * acc[22];
#pragma unroll
    for (int a = 0; a < 7; ++a)
#pragma unroll
        for (int b = a; b < 7; ++b) {
            out[a * 7 + b] = M[a][b];
            out[b * 7 + a] = M[a][b];
        }
}

__global__ void k_transitions(const double* __restrict__ recs, int64_t n, double* __restrict__ out) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const double* rec = recs + p * REC_N;
    out[p * 4 + 0] = rec[R_MS];
    out[p * 4 + 1] = rec[R_FP2];
    out[p * 4 + 2] = rec[R_FA2];
    out[p * 4 + 3] = rec[R_VALID];
}

// ==================================================================================
// host-side launchers
// ==================================================================================

// Region segments of every (point, chunk), once per call.
// Segment tables [3 phase regions][n][chunks]: chunk c of region r covers the c-th piece of that
// region's own bins, so each region launch spreads its work over all of its waves.
__global__ void k_segments(const double* __restrict__ recs, int64_t n, int chunks, GridArgs g,
                           int* __restrict__ segs, int* __restrict__ order_counts) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    // the ordering counters (bucket sizes and fill cursors) start at zero for k_order_count
    if (order_counts && t < 2 * kOrderBuckets) order_counts[t] = 0;
    const int64_t per_region = n * chunks;
    if (t >= 3 * per_region) return;
    const int prg = static_cast<int>(t / per_region) + 1;
    const int64_t pc = t - (prg - 1) * per_region;
    const int64_t p = pc / chunks;
    const int c = static_cast<int>(pc - p * chunks);
    const double* __restrict__ rec = recs + p * REC_N;
    Segs S;
    if (rec[R_VALID] == 0.0) {
#pragma unroll
        for (int i = 0; i < 6; ++i) S.k[i] = 0;
#pragma unroll
        for (int i = 0; i < 5; ++i) S.pr[i] = S.ar[i] = 0;
    } else {
        // chunks past the region's own count are never read
        const int cr = region_chunks(prg, chunks);
        int64_t kb = 0, ke = 0;
        if (c < cr) region_chunk_range(rec, g, prg, c, cr, kb, ke);
        make_segments(rec, g, kb, ke, S);
    }
    store_segments(S, segs + t * kSegInts);
}

// ---- point ordering -------------------------------------------------------------------------
// Waves of one block share its resources until the slowest finishes, and per-point work varies
// several-fold with the total mass (the number of active bins).  A counting sort into 256 buckets
// of active-bin count, largest first, lets neighbouring waves carry similar work: at 65536 points x
// 16225 bins the fused pass went from 2.52 to 2.19 ms with pre-sorted input.  Each point's sums are
// independent of the order (it only changes which wave computes them), so results are unchanged;
// the order within a bucket is whatever the atomic cursors give.
__device__ __forceinline__ int work_bucket(const double* __restrict__ rec, const GridArgs& g) {
    if (rec[R_VALID] == 0.0) return kOrderBuckets - 1;
    const double lo = fmax(g.fmin, g.f0);
    const double hi = fmin(0.2 / rec[R_MS], g.f0 + static_cast<double>(g.nb - 1) * g.df);
    const double bins = (hi > lo) ? (hi - lo) / g.df : 0.0;
    const int b = static_cast<int>(fmin(bins * kOrderBuckets / static_cast<double>(g.nb), kOrderBuckets - 1.0));
    return kOrderBuckets - 1 - b;
}

// Each point's bucket is computed once, here, and stored: the scatter reads it back, so the two
// kernels cannot disagree on a bucket and the permutation is always a bijection of [0, n).
__global__ void __launch_bounds__(256) k_order_count(const double* __restrict__ recs, int64_t n, GridArgs g,
                                                     int* __restrict__ counts, unsigned char* __restrict__ bucket) {
    __shared__ int hist[kOrderBuckets];
    hist[threadIdx.x] = 0;
    __syncthreads();
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p < n) {
        const int b = work_bucket(recs + p * REC_N, g);
        bucket[p] = static_cast<unsigned char>(b);
        atomicAdd(&hist[b], 1);
    }
    __syncthreads();
    if (hist[threadIdx.x] > 0) atomicAdd(&counts[threadIdx.x], hist[threadIdx.x]);
}

__global__ void __launch_bounds__(256) k_order_scatter(const unsigned char* __restrict__ bucket, int64_t n,
                                                       const int* __restrict__ counts, int* __restrict__ fill,
                                                       int* __restrict__ perm) {
    __shared__ int base[kOrderBuckets], lcnt[kOrderBuckets], lbase[kOrderBuckets];
    base[threadIdx.x] = counts[threadIdx.x];
    lcnt[threadIdx.x] = 0;
    __syncthreads();
    // inclusive scan (Hillis-Steele), then shift to exclusive
    for (int d = 1; d < kOrderBuckets; d <<= 1) {
        const int v = (static_cast<int>(threadIdx.x) >= d) ? base[threadIdx.x - d] : 0;
        __syncthreads();
        base[threadIdx.x] += v;
        __syncthreads();
    }
    const int excl = base[threadIdx.x] - counts[threadIdx.x];
    __syncthreads();
    base[threadIdx.x] = excl;
    __syncthreads();
    // ranks within the block from LDS atomics; one global reservation per bucket present in the block
    // (per-point global atomics on a few crowded buckets serialised: 71 us at 65536 points)
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    int b = 0, r = 0;
    if (p < n) {
        b = bucket[p];
        r = atomicAdd(&lcnt[b], 1);
    }
    __syncthreads();
    if (lcnt[threadIdx.x] > 0) lbase[threadIdx.x] = atomicAdd(&fill[threadIdx.x], lcnt[threadIdx.x]);
    __syncthreads();
    if (p < n) perm[base[b] + lbase[b] + r] = static_cast<int>(p);
}

static inline unsigned blocks_for(int64_t threads, int per_block) {
    return static_cast<unsigned>((threads + per_block - 1) / per_block);
}

hipError_t launch_setup_value(const double* theta, int64_t n, int param, double f_ref, const double* lam,
                              double* recs, int32_t* status, hipStream_t s, const XForm* xf, const GridArgs* tg,
                              const double* data, const double* inv_psd, double* tab) {
    TablesJob tj{};
    tj.bs = blocks_for(n, 128);
    unsigned blocks = tj.bs;
    if (tg) {
        tj.g = *tg;
        tj.data = data;
        tj.inv_psd = inv_psd;
        tj.tab = tab;
        tj.bt = blocks_for(tg->nb, 128);
        blocks += 4 * tj.bt;
    }
    if (xf)
        hipLaunchKernelGGL(k_setup_value<true>, dim3(blocks), dim3(128), 0, s, const_cast<double*>(theta), n, param,
                           f_ref, lam, recs, status, *xf, tj);
    else
        hipLaunchKernelGGL(k_setup_value<false>, dim3(blocks), dim3(128), 0, s, const_cast<double*>(theta), n, param,
                           f_ref, lam, recs, status, XForm{}, tj);
    return hipGetLastError();
}

hipError_t launch_setup_theta_tangent(const double* theta, int64_t n, int param, double f_ref,
                                      const double* lam, int rows, double* tans, hipStream_t s) {
    if (rows == 4)
        hipLaunchKernelGGL(k_setup_theta_tangent<4>, dim3(blocks_for(4 * n, 64)), dim3(64), 0, s, theta, n, param,
                           f_ref, lam, tans);
    else
        hipLaunchKernelGGL(k_setup_theta_tangent<7>, dim3(blocks_for(4 * n, 64)), dim3(64), 0, s, theta, n, param,
                           f_ref, lam, tans);
    return hipGetLastError();
}

hipError_t launch_setup_fit_tangent(const double* theta, int64_t n, int param, double f_ref, const double* lam,
                                    const double* recs, double* tans, hipStream_t s) {
    hipLaunchKernelGGL(k_setup_fit_tangent, dim3(blocks_for(n * kNumFit, 64)), dim3(64), 0, s, theta, n, param,
                       f_ref, lam, recs, tans);
    return hipGetLastError();
}

hipError_t launch_transitions(const double* recs, int64_t n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_transitions, dim3(blocks_for(n, 128)), dim3(128), 0, s, recs, n, out);
    return hipGetLastError();
}

hipError_t launch_waveform(const double* recs, int64_t n, const GridArgs& g, const double* tab, int precision,
                           double* h, hipStream_t s) {
    const bool wide = n * g.nb >= (int64_t(1) << 24);
    const int64_t per_block = wide ? 8 * 256 : 256;
    const int64_t bpp = (g.nb + per_block - 1) / per_block;
    ProfRange pr(PD_K_WAVEFORM, s);
    if (wide)
        hipLaunchKernelGGL(k_waveform<8>, dim3(static_cast<unsigned>(bpp * n)), dim3(256), 0, s, recs, n, bpp, g, tab, h);
    else
        hipLaunchKernelGGL(k_waveform<1>, dim3(static_cast<unsigned>(bpp * n)), dim3(256), 0, s, recs, n, bpp, g, tab, h);
    (void)precision;
    return hipGetLastError();
}

// Two side streams (default priority) per host thread and device for the region launches.
RegionStreams* region_streams() {
    thread_local std::vector<RegionStreams> pool;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    for (auto& e : pool)
        if (e.dev == dev) return e.ok ? &e : nullptr;
    RegionStreams e;
    e.dev = dev;
    e.ok = hipStreamCreateWithFlags(&e.s[0], hipStreamNonBlocking) == hipSuccess &&
           hipStreamCreateWithFlags(&e.s[1], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&e.fork, hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&e.join[0], hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&e.join[1], hipEventDisableTiming) == hipSuccess;
    if (!e.ok) (void)hipGetLastError();
    pool.push_back(e);
    return pool.back().ok ? &pool.back() : nullptr;
}

// Segments of every (region, point, chunk), then, for batches of at least kOrderMinPoints points,
// the work ordering (order: [0, 256) bucket sizes, [256, 512) fill cursors, then the permutation
// [n]).  Returns the permutation, or nullptr for index order: below that size the two extra
// launches cost more than the ordering gains (4096 chains x 8033 bins, one HMC leapfrog step).
constexpr int64_t kOrderMinPoints = 16384;

static int* launch_order(const double* recs, int64_t n, int chunks, const GridArgs& g, int* segs, int* order,
                         hipStream_t s) {
    const int64_t waves = n * chunks;
    const bool ordered = n >= kOrderMinPoints;
    int* counts = ordered ? order : nullptr;
    // the grid also covers the 512 counters it clears when 3 x waves is smaller
    const int64_t seg_threads = 3 * waves > 2 * kOrderBuckets ? 3 * waves : 2 * kOrderBuckets;
    hipLaunchKernelGGL(k_segments, dim3(blocks_for(seg_threads, 128)), dim3(128), 0, s, recs, n, chunks, g, segs,
                       counts);
    if (!ordered) return nullptr;
    int* perm = order + 2 * kOrderBuckets;
    unsigned char* bucket = reinterpret_cast<unsigned char*>(perm + n);
    hipLaunchKernelGGL(k_order_count, dim3(blocks_for(n, 256)), dim3(256), 0, s, recs, n, g, counts, bucket);
    hipLaunchKernelGGL(k_order_scatter, dim3(blocks_for(n, 256)), dim3(256), 0, s, bucket, n, counts,
                       counts + kOrderBuckets, perm);
    return perm;
}

// Below this many points the three region passes run as one launch (the fork and join of the
// region streams cost more than the separate register budgets gain at sampler batch sizes).
constexpr int64_t kMergedMaxPoints = 16384;

template <int MODE>
static void launch_region_moments(const double* recs, int64_t n, int chunks, const GridArgs& g,
                                  const double* tab, const int* segs, const int* perm, double* partial,
                                  hipStream_t s, bool concurrent) {
    if (n < kMergedMaxPoints) {
        const unsigned nb3 = blocks_for(n * region_chunks(3, chunks), 4);
        const unsigned nb12 = blocks_for(n * region_chunks(1, chunks), 4);
        hipLaunchKernelGGL((k_loglike_moments_all<MODE>), dim3(nb3 + 2 * nb12), dim3(256), 0, s, recs, n, chunks, g,
                           tab, segs, perm, partial, nb3, nb12);
        return;
    }
    launch_regions(s, [&](int region, hipStream_t rs) {
        const dim3 grid(blocks_for(n * region_chunks(region, chunks), 4));
        if (region == 3)
            hipLaunchKernelGGL((k_loglike_moments<MODE, 3>), grid, dim3(256), 0, rs, recs, n, chunks, g, tab,
                               segs, perm, partial);
        else if (region == 2)
            hipLaunchKernelGGL((k_loglike_moments<MODE, 2>), grid, dim3(256), 0, rs, recs, n, chunks, g, tab,
                               segs, perm, partial);
        else
            hipLaunchKernelGGL((k_loglike_moments<MODE, 1>), grid, dim3(256), 0, rs, recs, n, chunks, g, tab,
                               segs, perm, partial);
    }, concurrent);
}

hipError_t launch_loglike(const double* theta, int param, const double* recs, const double* tans, int64_t n,
                          int chunks, const GridArgs& g, const double* tab, int* segs, int* order, double* partial,
                          double* lnl, double* grad, hipEvent_t before_epilogue, hipStream_t s, bool concurrent,
                          const PostTail* tail) {
    int* perm = launch_order(recs, n, chunks, g, segs, order, s);
    if (grad) {
        {
            ProfRange pr(PD_K_LOGLIKE_GRAD, s);
            launch_region_moments<1>(recs, n, chunks, g, tab, segs, perm, partial, s, concurrent);
        }
        if (before_epilogue) {
            const hipError_t e = hipStreamWaitEvent(s, before_epilogue, 0);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k_loglike_grad_epilogue, dim3(blocks_for(n, 4)), dim3(256), 0, s, theta, n, param, recs,
                           tans, chunks, partial, lnl, grad, tail ? *tail : PostTail{}, tail ? 1 : 0);
    } else {
        {
            ProfRange pr(PD_K_LOGLIKE, s);
            launch_region_moments<0>(recs, n, chunks, g, tab, segs, perm, partial, s, concurrent);
        }
        hipLaunchKernelGGL(k_loglike_value_epilogue, dim3(blocks_for(n, 128)), dim3(128), 0, s, recs, n, chunks,
                           partial, lnl);
    }
    return hipGetLastError();
}

hipError_t launch_fisher(const double* theta, int param, const double* recs, const double* tans, int64_t n,
                         int chunks, const GridArgs& g, const double* tab, int* segs, int* order, double* partial,
                         double* F, hipStream_t s) {
    int* perm = launch_order(recs, n, chunks, g, segs, order, s);
    {
        // sequential: run concurrently, the three launches (three waves per SIMD each, LDS-resident
        // tangents) measured 1.7x slower
        ProfRange pr(PD_K_FISHER, s);
        const dim3 grid3(blocks_for(n * region_chunks(3, chunks), 4));
        const dim3 grid12(blocks_for(n * region_chunks(1, chunks), 4));
        hipLaunchKernelGGL(k_fisher_partial<3>, grid3, dim3(256), 0, s, recs, tans, n, chunks, g, tab, segs, perm,
                           partial);
        hipLaunchKernelGGL(k_fisher_partial<2>, grid12, dim3(256), 0, s, recs, tans, n, chunks, g, tab, segs, perm,
                           partial);
        hipLaunchKernelGGL(k_fisher_partial<1>, grid12, dim3(256), 0, s, recs, tans, n, chunks, g, tab, segs, perm,
                           partial);
    }
    hipLaunchKernelGGL(k_fisher_epilogue, dim3(blocks_for(n, 128)), dim3(128), 0, s, theta, param, recs, n, chunks,
                       partial, F);
    return hipGetLastError();
}

__global__ void k_elementary(int fn, const double* __restrict__ x, int64_t n, double* __restrict__ out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = x[i];
    double r;
    if (fn == PD_FN_SIN || fn == PD_FN_COS) {
        double sn, cs;
        pd_sincos(v, &sn, &cs);
        r = (fn == PD_FN_SIN) ? sn : cs;
    } else if (fn == PD_FN_ATAN) {
        r = pd_atan(v);
    } else if (fn == PD_FN_ATAN_TABLE) {
        const AtanTabParts ap = pd_atan_tab_reduce(v);
        r = pd_atan_tab_finish(ap, pd_div(ap.num, ap.den));
    } else if (fn == PD_FN_EXP) {
        r = pd_exp(v);
    } else {
        r = pd_rcp(v);
    }
    out[i] = r;
}

hipError_t launch_elementary(int fn, const double* x, int64_t n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_elementary, dim3(blocks_for(n, 256)), dim3(256), 0, s, fn, x, n, out);
    return hipGetLastError();
}

}  // namespace pd
