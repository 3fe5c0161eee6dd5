// Template-bank overlaps on the FP64 matrix cores: for N_t templates h_t (generated from
// their parameters) and N_s data streams d_s on one grid,
//   O[t][s] = sum_k w_k conj(h_t,k) d_s,k,     w_k = 4 df / S_n(f_k),
// so Re O[t][s] = (h_t | d_s) of Eq. 1 and |O| is the phase-maximised overlap.  Together with
// (h_t | h_t) this gives ln L for every (template, stream) pair.
//
// As a real GEMM over the bins:  [Re O | Im O] = [a_r | a_i] * [[D_r, D_i], [D_i, -D_r]]
// with a = h / (A0 f^-7/6) (the per-template part of the strain) and D = w f^-7/6 d (the
// per-bin part, prepared once per call).  The template operand is never stored: each block
// generates its 32 templates x 64 bins into LDS chunk by chunk and contracts them at once
// with v_mfma_f64_16x16x4f64 (lane layout checked on gfx950: with A[i][k] from lane
// (i + 16 k) and B[k][j] from lane (j + 16 k), register r of lane l holds C[l/16 + 4 r][l%16]).
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/phenomd.h"
#include "pd_bin.h"
#include "pd_launch.h"
#include "pd_profile.h"

namespace pd {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kKC = 64;              // bins per chunk
constexpr int kKR = 2 * kKC;         // real contraction length per chunk
constexpr int kTT = 32;              // templates per block
constexpr int kRTT = kTT / 16;       // row tiles of the block's output
constexpr int kRPW = kTT / 4;        // template rows each of the 4 waves generates
static_assert(kTT == 32 || kTT == 64, "block tiling covers 32 or 64 templates");

// B' [chunk][128][2 nsp]: rows k < 64 carry (D_r | D_i) of bin chunk*64 + k, rows 64 + k carry
// (D_i | -D_r); columns s and nsp + s belong to stream s; zero beyond n_bins and ns.
__global__ void k_ov_prep(GridArgs g, const double* __restrict__ data, int64_t ns, int nsp,
                          const double* __restrict__ tab, const double* __restrict__ inv_psd,
                          double* __restrict__ bp, int64_t n_chunks) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t cols = 2 * nsp;
    const int64_t total = n_chunks * kKR * cols;
    if (idx >= total) return;
    const int64_t col = idx % cols;
    const int64_t row = (idx / cols) % kKR;
    const int64_t ch = idx / (cols * kKR);
    const int64_t k = ch * kKC + (row % kKC);
    const bool im_row = row >= kKC;
    const int64_t s = col % nsp;
    const bool im_col = col >= nsp;
    double v = 0.0;
    if (k < g.nb && s < ns) {
        const double wf = 4.0 * g.df * inv_psd[k] * tab[T_F76 * g.nb + k];
        const double2 d = reinterpret_cast<const double2*>(data)[s * g.nb + k];
        const double dr = wf * d.x, di = wf * d.y;
        v = im_row ? (im_col ? -dr : di) : (im_col ? di : dr);
    }
    bp[idx] = v;
}

// A record spread over the wave: lane e holds entry e (lanes past the record hold zero), and
// entry i is read with two lane reads into scalar registers.  Loaded one template ahead of its
// use, so the per-template coefficients never stall the generation on memory.
struct LaneRec {
    double v;
    __device__ __forceinline__ double operator[](int i) const {
        const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
        const unsigned lo = __builtin_amdgcn_readlane(static_cast<int>(static_cast<unsigned>(b)), i);
        const unsigned hi = __builtin_amdgcn_readlane(static_cast<int>(static_cast<unsigned>(b >> 32)), i);
        return __builtin_bit_cast(double, (static_cast<unsigned long long>(hi) << 32) | lo);
    }
};

// Region pair (phase region, amplitude region) of frequency Mf, coded 4 pr + ar; the amplitude
// join (Mf = 0.014) lies below the phase join (0.018), so pr >= 2 implies ar >= 2.
template <class RC>
__device__ __forceinline__ int region_pair(const RC& rec, double mf) {
    const int pr = (mf < kFPhaseJoin) ? 1 : ((mf < rec[R_FP2]) ? 2 : 3);
    const int ar = (mf < kFAmpJoin) ? 1 : ((mf < rec[R_FA2]) ? 2 : 3);
    return 4 * pr + ar;
}

__device__ __forceinline__ void store_a(double* __restrict__ arow, int kk, int sw, bool on, double amp, double psi) {
    double sn, cs;
    pd_sincos(psi, &sn, &cs);
    arow[kk ^ sw] = on ? amp * cs : 0.0;
    arow[(kKC + kk) ^ sw] = on ? -amp * sn : 0.0;
}

// One bin of one template whose active bins in this chunk all lie in region pair (PR, AR); an
// inactive bin goes through the same formulas and is stored as zero.
template <int PR, int AR, class RC>
__device__ __forceinline__ void gen_bin(const RC& rec, const BinTabs& bt, int64_t k, double mf,
                                        bool on, double* __restrict__ arow, int kk, int sw) {
    BinVals bv;
    eval_bin_t<PR, AR>(rec, bt, k, mf, bv);
    store_a(arow, kk, sw, on, rec[R_A0P] * bv.ahat, bv.psi);
}

// Tiles of the block's output: kRTT row tiles (16 templates each) x CT column tiles (16 real
// columns each).  Wave w owns RT row tiles x CB column tiles: every row tile and CT/4 column tiles
// when CT >= 4 (each wave then fetches a quarter of the data operand), otherwise RT rows of one
// column; waves whose column would lie past CT take no part in the contraction.
template <int CT>
struct OvTiling {
    static constexpr int RT = CT >= 4 ? kRTT : (kRTT * CT >= 4 ? kRTT * CT / 4 : 1);
    static constexpr int CB = CT >= 4 ? CT / 4 : 1;
    __device__ static int row0(int w) { return CT >= 4 ? 0 : (w * RT) % kRTT; }
    __device__ static int col0(int w) { return CT >= 4 ? w * CB : (w * RT) / kRTT; }
    __device__ static bool active(int w) { return col0(w) < CT; }
};

template <int CT>
__global__ void __launch_bounds__(256, 4) k_ov_gemm(const double* __restrict__ recs, int64_t nt, GridArgs g,
                                                 const double* __restrict__ tab, const double* __restrict__ bp,
                                                 int nsp, int64_t ns, double* __restrict__ out,
                                                 double* __restrict__ hh) {
    using TL = OvTiling<CT>;
    constexpr int RT = TL::RT, CB = TL::CB;
    // kTT template rows x 128 real k (32 KB: with four waves per SIMD, four blocks share a CU's
    // LDS); element (r, kk) sits at column kk ^ (4 (r % 16)), so the
    // MFMA reads (16 rows x 4 consecutive kk) and the generation writes (one row, 64 kk) both
    // touch 64 distinct columns
    __shared__ double As[kTT][kKR];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform: records via the scalar cache
    const int64_t tb = static_cast<int64_t>(blockIdx.x) * kTT;
    const Tabs T(tab, g.nb);

    // active bin range [ka, kz) of each of the block's templates (empty for padding rows and
    // invalid points), then the block's range: their union
    __shared__ __attribute__((aligned(8))) int Kr[kTT][2];
    if (threadIdx.x < kTT) {
        const int64_t t = tb + threadIdx.x;
        int64_t ka = 0, kz = 0;
        if (t < nt && recs[t * REC_N + R_VALID] != 0.0) active_range(recs[t * REC_N + R_MS], g, ka, kz);
        Kr[threadIdx.x][0] = static_cast<int>(ka);
        Kr[threadIdx.x][1] = static_cast<int>(kz);
    }
    __syncthreads();
    int klo = static_cast<int>(g.nb), khi = 0;
    for (int j = 0; j < kTT; ++j) {
        const int ka = Kr[j][0], kz = Kr[j][1];
        if (kz > ka) {
            klo = min(klo, ka);
            khi = max(khi, kz);
        }
    }
    klo = __builtin_amdgcn_readfirstlane(klo);
    khi = __builtin_amdgcn_readfirstlane(khi);
    const int c0 = klo / kKC;
    const int c1 = (khi > klo) ? (khi + kKC - 1) / kKC : c0;

    const int rt0 = TL::row0(w), cb0 = TL::col0(w);
    const bool mma_wave = TL::active(w);
    const bool hh_wave = mma_wave && (cb0 == 0);     // the waves holding column tile 0 also sum (h|h)
    d4 acc[CB][RT];
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
        for (int r = 0; r < RT; ++r) acc[c][r] = d4{0.0, 0.0, 0.0, 0.0};
    double hsum[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) hsum[r] = 0.0;

    const int ia = lane & 15, ka4 = lane >> 4;     // MFMA operand coordinates of this lane
    const int64_t bstride = 2 * nsp;
    for (int ch = c0; ch < c1; ++ch) {
        // generate a = h / (A0 f^-7/6): wave w fills rows kRPW w .. kRPW w + kRPW - 1 (lane = bin); the
        // bin's table values are loaded once for all of them
        {
            const int64_t kch = static_cast<int64_t>(ch) * kKC;
            const int64_t k = kch + lane;
            const int64_t kc = (k < g.nb) ? k : g.nb - 1;
            const double f = bin_freq(g, kc);
            BinTabs bt;
            bt.load(T, kc);
            // the next row's record and active range are fetched while this row is evaluated
            const int64_t t0 = tb + kRPW * w;
            // merger-ringdown template bins: the record form with the table-reduced arc tangent
            // (table in constant memory)
            const double2* __restrict__ atab = reinterpret_cast<const double2*>(kAtanTab);
            auto rec_fetch = [&](int j) -> double {
                const int64_t t = t0 + j;
                return (t < nt && lane < REC_N) ? recs[t * REC_N + lane] : 0.0;
            };
            double rec_next = rec_fetch(0);
            int2 kr_next = *reinterpret_cast<const int2*>(&Kr[kRPW * w][0]);
#pragma unroll 1
            for (int j = 0; j < kRPW; ++j) {
                const int row = kRPW * w + j;
                const LaneRec rec{rec_next};
                const int ka = __builtin_amdgcn_readfirstlane(kr_next.x);
                const int kz = __builtin_amdgcn_readfirstlane(kr_next.y);
                rec_next = rec_fetch(min(j + 1, kRPW - 1));
                kr_next = *reinterpret_cast<const int2*>(&Kr[kRPW * w + min(j + 1, kRPW - 1)][0]);
                const int lo = max(static_cast<int>(kch), ka), hi = min(static_cast<int>(kch) + kKC, kz);
                double* __restrict__ arow = &As[row][0];
                const int sw = 4 * (row & 15);
                const bool on = k >= lo && k < hi;
                // region pair of the row's active bins in this chunk: one pair for all of them lets the
                // wave run the evaluation instantiated for it; -1 if it changes, -2 if none is active
                int code = -2;
                if (hi > lo) {
                    const double ms = rec[R_MS];
                    const int c_lo = region_pair(rec, ms * bin_freq(g, static_cast<int64_t>(lo)));
                    const int c_hi = region_pair(rec, ms * bin_freq(g, static_cast<int64_t>(hi - 1)));
                    code = (c_lo == c_hi) ? c_lo : -1;
                }
                code = __builtin_amdgcn_readfirstlane(code);
                if (code == -2) {
                    arow[lane ^ sw] = 0.0;
                    arow[(kKC + lane) ^ sw] = 0.0;
                    continue;
                }
                const double mf = rec[R_MS] * f;
                switch (code) {
                    case 4 * 1 + 1: gen_bin<1, 1>(rec, bt, kc, mf, on, arow, lane, sw); break;
                    case 4 * 1 + 2: gen_bin<1, 2>(rec, bt, kc, mf, on, arow, lane, sw); break;
                    case 4 * 1 + 3: gen_bin<1, 3>(rec, bt, kc, mf, on, arow, lane, sw); break;
                    case 4 * 2 + 2: gen_bin<2, 2>(rec, bt, kc, mf, on, arow, lane, sw); break;
                    case 4 * 2 + 3: gen_bin<2, 3>(rec, bt, kc, mf, on, arow, lane, sw); break;
                    case 4 * 3 + 2: gen_bin<3, 2>(rec_mrd(rec, atab), bt, kc, mf, on, arow, lane, sw); break;
                    case 4 * 3 + 3: gen_bin<3, 3>(rec_mrd(rec, atab), bt, kc, mf, on, arow, lane, sw); break;
                    default: {
                        double amp = 0.0, psi = 0.0;
                        if (on) {
                            BinVals bv;
                            eval_bin_rt(rec, bt, kc, mf, bv);
                            amp = rec[R_A0P] * bv.ahat;
                            psi = bv.psi;
                        }
                        store_a(arow, lane, sw, on, amp, psi);
                    }
                }
            }
        }
        __syncthreads();
        // contract: each k-step reads RT operand values from LDS and CB from the data operand;
        // data values are fetched two k-steps ahead of their use
        if (mma_wave) {
        const double* __restrict__ bch = bp + static_cast<int64_t>(ch) * kKR * bstride + 16 * cb0 + ia;
        const double* __restrict__ wwc = T.p[T_WW] + static_cast<int64_t>(ch) * kKC;
        const int64_t kmax = g.nb - static_cast<int64_t>(ch) * kKC;    // bins of this chunk inside the grid
        double b0[2][CB], b1[2][CB];
        auto fetch = [&](double (&dst)[2][CB], int sg) {
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int c = 0; c < CB; ++c) dst[u][c] = bch[(8 * sg + 4 * u + ka4) * bstride + 16 * c];
        };
        auto step = [&](const double (&src)[2][CB], int sg) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int kk = 8 * sg + 4 * u + ka4;
                const int kb = kk & (kKC - 1);
                const double ww = (hh_wave && kb < kmax) ? wwc[kb] : 0.0;
#pragma unroll
                for (int r = 0; r < RT; ++r) {
                    const double a = As[16 * (rt0 + r) + ia][kk ^ (4 * ia)];
                    hsum[r] = fma(ww * a, a, hsum[r]);
#pragma unroll
                    for (int c = 0; c < CB; ++c)
                        acc[c][r] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, src[u][c], acc[c][r], 0, 0, 0);
                }
            }
        };
        fetch(b0, 0);
#pragma unroll 1
        for (int sg = 0; sg < kKR / 8; sg += 2) {
            fetch(b1, sg + 1);
            step(b0, sg);
            if (sg + 2 < kKR / 8) fetch(b0, sg + 2);
            step(b1, sg + 1);
        }
        }
        __syncthreads();
    }
    if (!mma_wave) return;

    // (h|h): the four lanes holding row ia of a row tile (ka4 = 0..3) together saw all its bins
    // twice (real and imaginary part)
    if (hh_wave) {
#pragma unroll
        for (int r = 0; r < RT; ++r) {
            double v = hsum[r];
            v += __shfl_xor(v, 16, 64);
            v += __shfl_xor(v, 32, 64);
            const int64_t t = tb + 16 * (rt0 + r) + ia;
            if (ka4 == 0 && hh && t < nt) hh[t] = (recs[t * REC_N + R_VALID] != 0.0) ? v : __builtin_nan("");
        }
    }
#pragma unroll
    for (int c = 0; c < CB; ++c) {
        const int col = 16 * (cb0 + c) + ia;
        const bool im = col >= nsp;
        const int64_t s = im ? col - nsp : col;
#pragma unroll
        for (int r = 0; r < RT; ++r) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t t = tb + 16 * (rt0 + r) + ka4 + 4 * q;
                if (t < nt && s < ns) {
                    const bool ok = recs[t * REC_N + R_VALID] != 0.0;
                    out[(t * ns + s) * 2 + (im ? 1 : 0)] = ok ? acc[c][r][q] : __builtin_nan("");
                }
            }
        }
    }
}

inline unsigned nblk(int64_t threads, int per) { return static_cast<unsigned>((threads + per - 1) / per); }

}  // namespace

int64_t overlap_chunks(int64_t nb) { return (nb + kKC - 1) / kKC; }

// Streams padded to 8, 16, 32 or 64 (8 x the kernel's column-tile count).
int overlap_padded_streams(int64_t ns) { return ns <= 8 ? 8 : ns <= 16 ? 16 : ns <= 32 ? 32 : 64; }

size_t overlap_bprime_bytes(int64_t nb, int64_t ns) {
    const int64_t nsp = overlap_padded_streams(ns);
    return static_cast<size_t>(overlap_chunks(nb)) * kKR * 2 * nsp * sizeof(double);
}

hipError_t launch_overlap(const double* recs, int64_t nt, const GridArgs& g, const double* tab,
                          const double* data, int64_t ns, const double* inv_psd, double* bp, double* out,
                          double* hh, hipStream_t s) {
    const int nsp = overlap_padded_streams(ns);
    const int64_t n_chunks = overlap_chunks(g.nb);
    const int64_t total = n_chunks * kKR * 2 * nsp;
    hipLaunchKernelGGL(k_ov_prep, dim3(nblk(total, 256)), dim3(256), 0, s, g, data, ns, nsp, tab, inv_psd, bp,
                       n_chunks);
    {
        // column tiles of 16 real columns: 2 nsp / 16 = nsp / 8 of them
        ProfRange pr(PD_K_OVERLAP, s);
        const dim3 grid(nblk(nt, kTT)), block(256);
        if (nsp <= 8)
            hipLaunchKernelGGL(k_ov_gemm<1>, grid, block, 0, s, recs, nt, g, tab, bp, nsp, ns, out, hh);
        else if (nsp <= 16)
            hipLaunchKernelGGL(k_ov_gemm<2>, grid, block, 0, s, recs, nt, g, tab, bp, nsp, ns, out, hh);
        else if (nsp <= 32)
            hipLaunchKernelGGL(k_ov_gemm<4>, grid, block, 0, s, recs, nt, g, tab, bp, nsp, ns, out, hh);
        else
            hipLaunchKernelGGL(k_ov_gemm<8>, grid, block, 0, s, recs, nt, g, tab, bp, nsp, ns, out, hh);
    }
    return hipGetLastError();
}

}  // namespace pd
