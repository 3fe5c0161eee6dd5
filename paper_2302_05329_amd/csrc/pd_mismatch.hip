// Mismatch against fixed targets and its adjoint over the 209 fit coefficients
// (paper Sec. 3.1: Eq. 5, averaged over targets in Eq. 7; the maximum
// over the coalescence time is taken with a Fourier transform, Sec. 2).
//
// Pipeline per target (N = 65536 = 256 x 256):
//   1. overlap input   x_k = w_k conj(h_k) t_k (model recomputed per bin), partial
//                      sums of (h|h) and (t|t)                         one thread / bin
//   2. column pass     256-point inverse DFTs over k2 of x[k1 + 256 k2] in LDS
//                      (radix-2 Stockham), twiddle exp(2 pi i j2 k1 / N), store
//                      transposed                                      8 columns / block
//   3. row pass        256-point inverse DFTs over k1, |z|^2 and arg-max fused; the
//                      overlap series itself is never written           8 rows / block
//   4. finalize        lag j*, |z_j*|, mismatch                         one thread / target
//   5. adjoint         moments of the mismatch adjoint per bin (model recomputed, no
//                      per-bin storage)                                 one wave / (target, chunk)
//   6. chain rule      record tangents along the 19 fitted parameters -> d M / d Lambda,
//                      times the 11 fit-basis values -> d M / d lambda, summed over
//                      targets in a fixed order
#include <hip/hip_runtime.h>

#include "../../include/phenomd.h"
#include "pd_launch.h"
#include "pd_mismatch.h"
#include "pd_profile.h"

namespace pd {

namespace {

constexpr int kCols = 8;   // columns (or rows) per FFT block; 2 x 32 KiB LDS ping-pong

struct MMScratch {
    double2* X;       // [nt][N]
    double2* Y;       // [nt][256][256] (transposed after the column pass)
    double* ab;       // [nt][N/256][2]
    double* mx;       // [nt][256/kCols][4]  (|z|^2, index, zr, zi)
    double* scal;     // [nt][kSlotMM]
    double* mom;      // [nt][chunks][kNSlot]
    double* dlam;     // [nt][19]
    double* mred;     // [nt][REC_N]
    int chunks;
};

constexpr size_t kAl = 256;
inline size_t al(size_t x) { return (x + kAl - 1) / kAl * kAl; }

MMScratch carve(void* base, int64_t nt, int64_t nb) {
    MMScratch m;
    char* p = static_cast<char*>(base);
    size_t off = 0;
    const size_t n = static_cast<size_t>(nt);
    m.chunks = chunks_for(nt, nb);
    m.X = reinterpret_cast<double2*>(p + off);
    off = al(off + n * kFFTN * sizeof(double2));
    m.Y = reinterpret_cast<double2*>(p + off);
    off = al(off + n * kFFTN * sizeof(double2));
    m.ab = reinterpret_cast<double*>(p + off);
    off = al(off + n * (kFFTN / 256) * 2 * sizeof(double));
    m.mx = reinterpret_cast<double*>(p + off);
    off = al(off + n * (kFFTR / kCols) * 4 * sizeof(double));
    m.scal = reinterpret_cast<double*>(p + off);
    off = al(off + n * kSlotMM * sizeof(double));
    m.mom = reinterpret_cast<double*>(p + off);
    off = al(off + 3 * n * m.chunks * kNSlot * sizeof(double));
    m.dlam = reinterpret_cast<double*>(p + off);
    off = al(off + n * kNumFit * sizeof(double));
    m.mred = reinterpret_cast<double*>(p + off);
    off = al(off + n * REC_N * sizeof(double));
    return m;
}

size_t carve_size(int64_t nt, int64_t nb) {
    const size_t n = static_cast<size_t>(nt);
    const int chunks = chunks_for(nt, nb);
    size_t off = 0;
    off = al(off + n * kFFTN * sizeof(double2));
    off = al(off + n * kFFTN * sizeof(double2));
    off = al(off + n * (kFFTN / 256) * 2 * sizeof(double));
    off = al(off + n * (kFFTR / kCols) * 4 * sizeof(double));
    off = al(off + n * kSlotMM * sizeof(double));
    off = al(off + 3 * n * chunks * kNSlot * sizeof(double));
    off = al(off + n * kNumFit * sizeof(double));
    off = al(off + n * REC_N * sizeof(double));
    return off;
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// exp(2 pi i num / den) for an exact rational argument
__device__ __forceinline__ double2 expi_ratio(int64_t num, int64_t den) {
    double s, c;
    sincospi(2.0 * static_cast<double>(num) / static_cast<double>(den), &s, &c);
    return make_double2(c, s);
}

// ---- 1. overlap input -----------------------------------------------------------------
__global__ void __launch_bounds__(256) k_mm_input(const double* __restrict__ recs, int64_t nt, GridArgs g,
                                                  const double* __restrict__ tab,
                                                  const double* __restrict__ targets,
                                                  const double* __restrict__ inv_psd, double2* __restrict__ X,
                                                  double* __restrict__ ab) {
    __shared__ double red[2][4];
    const int64_t blocks = kFFTN / 256;
    const int64_t p = blockIdx.x / blocks;
    const int64_t kb = (blockIdx.x % blocks) * 256;
    const int64_t k = kb + threadIdx.x;
    const double* __restrict__ rec = recs + p * REC_N;
    const Tabs T(tab, g.nb);
    const double2 t = reinterpret_cast<const double2*>(targets)[p * kFFTN + k];
    const double w = 4.0 * g.df * inv_psd[k];
    double2 h = make_double2(0.0, 0.0);
    if (rec[R_VALID] != 0.0) {
        const double f = bin_freq(g, k);
        const double mf = rec[R_MS] * f;
        if (bin_active(g, f, mf)) {
            BinVals bv;
            eval_bin_rt(rec, T, k, mf, bv);
            const double A = rec[R_A0P] * T.at(T_F76, k) * bv.ahat;
            double sn, cs;
            pd_sincos(bv.psi, &sn, &cs);
            h = make_double2(A * cs, -A * sn);
        }
    }
    // x = w conj(h) t
    X[p * kFFTN + k] = make_double2(w * (h.x * t.x + h.y * t.y), w * (h.x * t.y - h.y * t.x));
    const double a = wave_sum(w * (h.x * h.x + h.y * h.y));
    const double b = wave_sum(w * (t.x * t.x + t.y * t.y));
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][wid] = a;
        red[1][wid] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double* o = ab + (p * blocks + (blockIdx.x % blocks)) * 2;
        o[0] = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
        o[1] = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
    }
}

// ---- LDS radix-2 Stockham inverse DFT of length 256 on kCols columns -----------------
// buf/tmp: [kCols][256]; 32 threads per column, 4 butterflies each per stage.
// Returns the buffer that holds the result (always `buf` after 8 stages).
__device__ __forceinline__ void lds_idft256(double2 (*buf)[kFFTR], double2 (*tmp)[kFFTR],
                                            const double2* __restrict__ tw) {
    const int col = threadIdx.x >> 5;
    const int r = threadIdx.x & 31;
    double2(*x)[kFFTR] = buf;
    double2(*y)[kFFTR] = tmp;
    int n = kFFTR, s = 1;
#pragma unroll
    for (int stage = 0; stage < 8; ++stage) {
        const int m = n >> 1;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int b = r + 32 * i;        // butterfly index in [0, 128)
            const int q = b % s;
            const int pp = b / s;
            const double2 a = x[col][q + s * pp];
            const double2 c = x[col][q + s * (pp + m)];
            const double2 w = tw[pp * (kFFTR / n)];    // exp(2 pi i pp / n)
            y[col][q + s * (2 * pp)] = make_double2(a.x + c.x, a.y + c.y);
            y[col][q + s * (2 * pp + 1)] = cmul(make_double2(a.x - c.x, a.y - c.y), w);
        }
        __syncthreads();
        double2(*t)[kFFTR] = x;
        x = y;
        y = t;
        n = m;
        s <<= 1;
    }
}

__device__ __forceinline__ void fill_twiddles(double2* tw) {
    const int j = threadIdx.x;   // blockDim = 256
    double sn, cs;
    sincospi(2.0 * j / 256.0, &sn, &cs);
    tw[j] = make_double2(cs, sn);
}

// ---- 2. column pass ------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_mm_fft_cols(const double2* __restrict__ X, double2* __restrict__ Y) {
    __shared__ double2 buf[kCols][kFFTR];
    __shared__ double2 tmp[kCols][kFFTR];
    __shared__ double2 tw[kFFTR];
    const int groups = kFFTR / kCols;
    const int64_t p = blockIdx.x / groups;
    const int gcol = (blockIdx.x % groups) * kCols;
    fill_twiddles(tw);
    const double2* __restrict__ src = X + p * kFFTN;
#pragma unroll
    for (int i = 0; i < kCols; ++i) {
        const int idx = threadIdx.x + 256 * i;
        const int c = idx % kCols, k2 = idx / kCols;
        buf[c][k2] = src[(gcol + c) + kFFTR * k2];
    }
    __syncthreads();
    lds_idft256(buf, tmp, tw);
    double2* __restrict__ dst = Y + p * kFFTN;
#pragma unroll
    for (int i = 0; i < kCols; ++i) {
        const int idx = threadIdx.x + 256 * i;
        const int c = idx % kCols, j2 = idx / kCols;
        const int k1 = gcol + c;
        const double2 v = cmul(buf[c][j2], expi_ratio(static_cast<int64_t>(j2) * k1, kFFTN));
        dst[static_cast<int64_t>(j2) * kFFTR + k1] = v;
    }
}

// ---- 3. row pass with fused arg-max of |z|^2 ------------------------------------------
__device__ __forceinline__ bool better(double v, int i, double bv, int bi) {
    return (v > bv) || (v == bv && i < bi);
}

__global__ void __launch_bounds__(256) k_mm_fft_rows_max(const double2* __restrict__ Y, double* __restrict__ mx) {
    __shared__ double2 buf[kCols][kFFTR];
    __shared__ double2 tmp[kCols][kFFTR];
    __shared__ double2 tw[kFFTR];
    __shared__ double rv[256];
    __shared__ int ri[256];
    const int groups = kFFTR / kCols;
    const int64_t p = blockIdx.x / groups;
    const int grow = (blockIdx.x % groups) * kCols;
    fill_twiddles(tw);
    const double2* __restrict__ src = Y + p * kFFTN;
#pragma unroll
    for (int i = 0; i < kCols; ++i) {
        const int idx = threadIdx.x + 256 * i;
        const int rrow = idx / kFFTR, k1 = idx % kFFTR;
        buf[rrow][k1] = src[static_cast<int64_t>(grow + rrow) * kFFTR + k1];
    }
    __syncthreads();
    lds_idft256(buf, tmp, tw);
    double best = -1.0;
    int bidx = 0x7fffffff;
#pragma unroll
    for (int i = 0; i < kCols; ++i) {
        const int idx = threadIdx.x + 256 * i;
        const int rrow = idx / kFFTR, j1 = idx % kFFTR;
        const double2 z = buf[rrow][j1];
        const double a2 = z.x * z.x + z.y * z.y;
        const int j = (grow + rrow) + kFFTR * j1;
        if (better(a2, j, best, bidx)) {
            best = a2;
            bidx = j;
        }
    }
    rv[threadIdx.x] = best;
    ri[threadIdx.x] = bidx;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            const double ov = rv[threadIdx.x + off];
            const int oi = ri[threadIdx.x + off];
            if (better(ov, oi, rv[threadIdx.x], ri[threadIdx.x])) {
                rv[threadIdx.x] = ov;
                ri[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int j = ri[0];
        const int j2 = j % kFFTR - grow, j1 = j / kFFTR;
        const double2 z = buf[j2][j1];
        double* o = mx + (p * groups + (blockIdx.x % groups)) * 4;
        o[0] = rv[0];
        o[1] = static_cast<double>(j);
        o[2] = z.x;
        o[3] = z.y;
    }
}

// ---- 4. finalize ---------------------------------------------------------------------
__global__ void k_mm_finalize(const double* __restrict__ recs, int64_t nt, const double* __restrict__ ab,
                              const double* __restrict__ mx, double* __restrict__ scal,
                              double* __restrict__ mismatch, int32_t* __restrict__ lag) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= nt) return;
    double* sc = scal + p * kSlotMM;
    if (recs[p * REC_N + R_VALID] == 0.0) {
        for (int i = 0; i < kSlotMM; ++i) sc[i] = 0.0;
        mismatch[p] = __builtin_nan("");
        if (lag) lag[p] = -1;
        return;
    }
    const int blocks = kFFTN / 256;
    double A = 0.0, B = 0.0;
    for (int b = 0; b < blocks; ++b) {
        A += ab[(p * blocks + b) * 2 + 0];
        B += ab[(p * blocks + b) * 2 + 1];
    }
    const int groups = kFFTR / kCols;
    double best = -1.0;
    int bi = 0x7fffffff;
    double zr = 0.0, zi = 0.0;
    for (int gi = 0; gi < groups; ++gi) {
        const double* o = mx + (p * groups + gi) * 4;
        const int j = static_cast<int>(o[1]);
        if (better(o[0], j, best, bi)) {
            best = o[0];
            bi = j;
            zr = o[2];
            zi = o[3];
        }
    }
    const double az = sqrt(best);
    const double mm = 1.0 - az / sqrt(A * B);
    sc[0] = A;
    sc[1] = B;
    sc[2] = az;
    sc[3] = zr;
    sc[4] = zi;
    sc[5] = static_cast<double>(bi);
    sc[6] = mm;
    sc[7] = 0.0;
    mismatch[p] = mm;
    if (lag) lag[p] = bi;
}

// ---- 5. adjoint moments ------------------------------------------------------------------
struct MMVis {
    double* mom;
    double zr, zi;
    __device__ __forceinline__ void ph(int s, double b) { mom[s] = fma(zi, b, mom[s]); }
    __device__ __forceinline__ void am(int s, double b) { mom[s] = fma(zr, b, mom[s]); }
    __device__ __forceinline__ void fd(double fpsi, double fa) { mom[R_MS] = fma(zi, fpsi, fma(zr, fa, mom[R_MS])); }
};

struct AdjSegment {
    const double* __restrict__ rec;
    Tabs T;
    GridArgs g;
    const double2* __restrict__ tgt;
    const double* __restrict__ inv_psd;
    double ur, ui, inv_sab, cfa;
    int64_t j;
    int64_t k0, k1;
    int lane;
    double tot;

    template <int PR, int AR>
    __device__ __forceinline__ void run() {
        const double ms = rec[R_MS];
        const double a0p = rec[R_A0P];
        const double w4 = 4.0 * g.df;
        double mom[REC_N];
#pragma unroll
        for (int s = 0; s < REC_N; ++s) mom[s] = 0.0;
        ExpRec er{};
        if (AR == 3) er.init(rec, g, static_cast<unsigned>(k0 + lane));
        for (unsigned k = static_cast<unsigned>(k0 + lane); k < static_cast<unsigned>(k1); k += 64u) {
            const double mf = ms * bin_freq(g, k);
            BinVals bv;
            eval_bin_t<PR, AR, AR == 3>(rec, T, k, mf, bv, (AR == 3) ? er.next() : 0.0);
            const double Aamp = a0p * T.at(T_F76, k) * bv.ahat;
            double sn, cs;
            pd_sincos(bv.psi, &sn, &cs);
            const double hr = Aamp * cs, hi = -Aamp * sn;
            const double w = w4 * inv_psd[k];
            const double2 t = tgt[k];
            const double2 e = expi_ratio((k * j) % kFFTN, kFFTN);
            const double2 x = cmul(make_double2(w * t.x, w * t.y), e);
            // G = conj(u) x
            const double gr = ur * x.x + ui * x.y, gi = ur * x.y - ui * x.x;
            // R = -G / sqrt(AB) + |z| w h / (A^(3/2) B^(1/2))
            const double rr = -gr * inv_sab + cfa * w * hr;
            const double ri = -gi * inv_sab + cfa * w * hi;
            // conj(h) R: weight of d ln A is Re, weight of d Psi is -Im
            const double cr = hr * rr + hi * ri, ci = hr * ri - hi * rr;
            MMVis vis{mom, cr, -ci};
            visit_bin_t<PR, AR>(rec, bv, vis);
        }
        flush_touched<PR, AR>(mom, lane, tot);
    }
};

template <int PRG>
__global__ void __launch_bounds__(256) k_mm_adjoint(const double* __restrict__ recs, int64_t nt, int chunks,
                                                    GridArgs g, const double* __restrict__ tab,
                                                    const double* __restrict__ targets,
                                                    const double* __restrict__ inv_psd,
                                                    const double* __restrict__ scal, double* __restrict__ part_all) {
    double* __restrict__ part = part_all + static_cast<int64_t>(PRG - 1) * nt * chunks * kNSlot;
    const int lane = threadIdx.x & 63;
    const int64_t wave = __builtin_amdgcn_readfirstlane(static_cast<int>(blockIdx.x * 4 + (threadIdx.x >> 6)));
    const int64_t p = wave / chunks;
    const int c = static_cast<int>(wave - p * chunks);
    if (p >= nt) return;
    const double* __restrict__ rec = recs + p * REC_N;
    double* __restrict__ out = part + (p * chunks + c) * kNSlot;
    if (rec[R_VALID] == 0.0) {
        for (int s = lane; s < kNSlot; s += 64) out[s] = 0.0;
        return;
    }
    const double* sc = scal + p * kSlotMM;
    const double A = sc[0], B = sc[1], az = sc[2];
    AdjSegment seg;
    seg.rec = rec;
    seg.T = Tabs(tab, g.nb);
    seg.g = g;
    seg.tgt = reinterpret_cast<const double2*>(targets) + p * kFFTN;
    seg.inv_psd = inv_psd;
    // unit phase u = z / |z|; G_k = conj(u) x_k with x_k = w t_k exp(2 pi i k j / N)
    seg.ur = sc[3] / az;
    seg.ui = sc[4] / az;
    seg.inv_sab = 1.0 / sqrt(A * B);
    seg.cfa = az / (A * sqrt(A * B));   // |z| / (A^(3/2) B^(1/2))
    seg.j = static_cast<int64_t>(sc[5]);
    seg.lane = lane;
    seg.tot = 0.0;
    int64_t kb, ke;
    region_chunk_range(rec, g, PRG, c, chunks, kb, ke);
    Segs S;
    make_segments(rec, g, kb, ke, S);
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        if (uniform_i(S.k[i + 1]) > uniform_i(S.k[i]) && uniform_i(S.pr[i]) == PRG) {
            seg.k0 = uniform_i(S.k[i]);
            seg.k1 = uniform_i(S.k[i + 1]);
            dispatch_amp_region<PRG>(uniform_i(S.ar[i]), seg);
        }
    }
    if (lane == 0) {
        out[0] = 0.0;
        out[1] = 0.0;
    }
    if (lane < REC_N) out[2 + lane] = seg.tot;
}

// ---- 6. chain rule to the fit parameters and to the 209 coefficients ------------------------
// (a) one wave per target: lane s sums slot s over the three region groups and the chunks
__global__ void __launch_bounds__(64) k_mm_reduce(const double* __restrict__ recs, int64_t nt, int chunks,
                                                  const double* __restrict__ part, double* __restrict__ mred) {
    const int64_t p = blockIdx.x;
    const int s = threadIdx.x;
    if (p >= nt || s >= REC_N) return;
    double m = 0.0;
    for (int grp = 0; grp < 3; ++grp)
        for (int c = 0; c < chunks; ++c) m += part[((grp * nt + p) * chunks + c) * kNSlot + 2 + s];
    const double* rec = recs + p * REC_N;
    if (s == R_MS) m /= rec[R_MS];
    const bool used = (s == R_MS || s == R_LNA0 || (s >= R_PH1 && s < R_VALID));
    mred[p * REC_N + s] = (used && rec[R_VALID] != 0.0) ? m : 0.0;
}

// (b) one thread per (target, fitted parameter): dM/dLambda_l = tangent_l . moments
__global__ void k_mm_contract(const double* __restrict__ tans, int64_t nt, const double* __restrict__ mred,
                              double* __restrict__ dlam) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= nt * kNumFit) return;
    const int64_t p = t / kNumFit;
    const double* tn = tans + t * REC_N;
    const double* m = mred + p * REC_N;
    double acc = 0.0;
    for (int s = 0; s < REC_N; ++s) acc = fma(tn[s], m[s], acc);
    dlam[t] = acc;
}

// (c) one block per coefficient: sum over targets of dM/dLambda_l * B_b(eta, chi_PN)
__global__ void __launch_bounds__(256) k_mm_lambda_sum(const double* __restrict__ recs, int64_t nt,
                                                       const double* __restrict__ dlam, double* __restrict__ out) {
    __shared__ double red[256];
    const int m = blockIdx.x;
    const int l = m / 11, b = m % 11;
    double acc = 0.0;
    for (int64_t p = threadIdx.x; p < nt; p += 256) {
        const double* rec = recs + p * REC_N;
        if (rec[R_VALID] == 0.0) continue;
        double basis[11];
        fit_basis(rec[R_ETA], rec[R_CHIPN], basis);
        acc = fma(dlam[p * kNumFit + l], basis[b], acc);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[m] = red[0];
}

}  // namespace

size_t mismatch_scratch_bytes(int64_t nt, int64_t nb) { return carve_size(nt, nb); }

hipError_t launch_mismatch(const double* recs, const double* fit_tans, int64_t nt, const GridArgs& g,
                           const double* tab, const double* targets, const double* inv_psd, void* scratch, double* mismatch,
                           double* dsum_dlambda, int32_t* lag, hipStream_t s) {
    MMScratch m = carve(scratch, nt, g.nb);
    const unsigned bin_blocks = static_cast<unsigned>(nt * (kFFTN / 256));
    {
        ProfRange pr(PD_K_MISMATCH_INPUT, s);
        hipLaunchKernelGGL(k_mm_input, dim3(bin_blocks), dim3(256), 0, s, recs, nt, g, tab, targets, inv_psd, m.X,
                           m.ab);
    }
    const unsigned fft_blocks = static_cast<unsigned>(nt * (kFFTR / kCols));
    {
        ProfRange pr(PD_K_MISMATCH_FFT, s);
        hipLaunchKernelGGL(k_mm_fft_cols, dim3(fft_blocks), dim3(256), 0, s, m.X, m.Y);
        hipLaunchKernelGGL(k_mm_fft_rows_max, dim3(fft_blocks), dim3(256), 0, s, m.Y, m.mx);
    }
    hipLaunchKernelGGL(k_mm_finalize, dim3(static_cast<unsigned>((nt + 127) / 128)), dim3(128), 0, s, recs, nt,
                       m.ab, m.mx, m.scal, mismatch, lag);
    if (dsum_dlambda) {
        const int64_t waves = nt * m.chunks;
        {
            ProfRange pr(PD_K_MISMATCH_ADJ, s);
            const dim3 grid(static_cast<unsigned>((waves + 3) / 4));
            launch_regions(s, [&](int region, hipStream_t rs) {
                if (region == 3)
                    hipLaunchKernelGGL(k_mm_adjoint<3>, grid, dim3(256), 0, rs, recs, nt, m.chunks, g, tab, targets,
                                       inv_psd, m.scal, m.mom);
                else if (region == 2)
                    hipLaunchKernelGGL(k_mm_adjoint<2>, grid, dim3(256), 0, rs, recs, nt, m.chunks, g, tab, targets,
                                       inv_psd, m.scal, m.mom);
                else
                    hipLaunchKernelGGL(k_mm_adjoint<1>, grid, dim3(256), 0, rs, recs, nt, m.chunks, g, tab, targets,
                                       inv_psd, m.scal, m.mom);
            });
        }
        hipLaunchKernelGGL(k_mm_reduce, dim3(static_cast<unsigned>(nt)), dim3(64), 0, s, recs, nt, m.chunks, m.mom,
                           m.mred);
        hipLaunchKernelGGL(k_mm_contract, dim3(static_cast<unsigned>((nt * kNumFit + 127) / 128)), dim3(128), 0,
                           s, fit_tans, nt, m.mred, m.dlam);
        hipLaunchKernelGGL(k_mm_lambda_sum, dim3(kNumLambda), dim3(256), 0, s, recs, nt, m.dlam, dsum_dlambda);
    }
    return hipGetLastError();
}

// One gradient-descent step on the coefficients (Sec. 3.1, Eq. 6 with the mean loss of Eq. 7):
// lambda -= scale * dsum, scale = alpha / n_targets.
__global__ void k_lambda_update(double* __restrict__ lam, const double* __restrict__ dsum, double scale) {
    const int i = threadIdx.x;
    if (i < kNumLambda) lam[i] = fma(-scale, dsum[i], lam[i]);
}

hipError_t launch_lambda_update(double* lam, const double* dsum, double scale, hipStream_t s) {
    hipLaunchKernelGGL(k_lambda_update, dim3(1), dim3(256), 0, s, lam, dsum, scale);
    return hipGetLastError();
}

}  // namespace pd
