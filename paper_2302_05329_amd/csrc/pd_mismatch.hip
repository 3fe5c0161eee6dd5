// Mismatch against fixed targets and its adjoint over the 209 fit coefficients
// (paper Sec. 3.1: Eq. 5, averaged over targets in Eq. 7; the maximum
// over the coalescence time is taken with a Fourier transform, Sec. 2).
//
// Pipeline per target (N = N1 x N2 bins, a power of two from 2^6 to 2^16 = 256 x 256):
//   0. twiddles        exp(2 pi i m / N) = hi[m >> 8] lo[m & 255] tables      one block / call
//   1. column pass     the overlap input x_k = w_k conj(h_k) t_k (model recomputed per bin, never
//                      stored) for the bins k1 + N1 k2 of a group of columns k1, partial sums of
//                      (h|h) and (t|t), N2-point inverse DFTs over k2 in LDS (radix-4
//                      Stockham, one buffer), twiddle exp(2 pi i j2 k1 / N), store transposed
//                                                                      2048 / N2 columns / block
//   2. row pass        N1-point inverse DFTs over k1, |z|^2 and arg-max fused (lag
//                      j = j2 + N2 j1); the overlap series itself is never written
//                                                                      1024 / N1 rows / block
//   3. finalize        lag j*, |z_j*|, mismatch                         one thread / target
//   4. adjoint         moments of the mismatch adjoint per bin (model recomputed, no
//                      per-bin storage)                                 one wave / (target, chunk)
//   5. chain rule      record tangents along the 19 fitted parameters -> d M / d Lambda,
//                      times the 11 fit-basis values -> d M / d lambda, summed over
//                      targets in a fixed order
#include <hip/hip_runtime.h>

#include "../../include/phenomd.h"
#include "pd_launch.h"
#include "pd_mismatch.h"
#include "pd_profile.h"

namespace pd {

namespace {

// Four-step plan of one overlap length.
struct FFTPlan {
    int64_t n;          // N
    int n1, n2;         // columns (row length) and column length
    int cb, rb;         // columns per column-pass block, rows per row-pass block
    int gc, gr;         // column groups and row groups per target
};

// complex points per block (one LDS buffer, plus padding): the column pass evaluates the model
// for its points, so it keeps fewer, larger blocks; the row pass only loads and transforms, and
// more, smaller blocks per compute unit overlap its loads with other blocks' transforms
constexpr int kColPts = 2048;
constexpr int kRowPts = 1024;
constexpr int kTw = 256;        // entries of each twiddle table

inline FFTPlan make_plan(int64_t n) {
    FFTPlan f;
    f.n = n;
    int lg = 0;
    while ((int64_t(1) << lg) < n) ++lg;
    f.n1 = 1 << ((lg + 1) / 2);
    f.n2 = 1 << (lg / 2);
    f.cb = kColPts / f.n2 < f.n1 ? kColPts / f.n2 : f.n1;
    f.rb = kRowPts / f.n1 < f.n2 ? kRowPts / f.n1 : f.n2;
    f.gc = f.n1 / f.cb;
    f.gr = f.n2 / f.rb;
    return f;
}

struct MMScratch {
    double2* Y;       // [nt][N2][N1] (transposed after the column pass)
    double2* tw;      // [2][kTw]: lo[i] = exp(2 pi i i / N), hi[i] = exp(2 pi i 256 i / N)
    double* ab;       // [nt][gc][2]
    double* mx;       // [nt][gr][4]  (|z|^2, index, zr, zi)
    double* scal;     // [nt][kSlotMM]
    double* mom;      // [nt][chunks][kNSlot]
    double* dlam;     // [nt][19]
    double* mred;     // [nt][REC_N]
    int chunks;
};

constexpr size_t kAl = 256;
inline size_t al(size_t x) { return (x + kAl - 1) / kAl * kAl; }

// Carves the scratch (base may be null: then only the size is computed).
size_t carve_into(void* base, int64_t nt, int64_t nb, MMScratch* m) {
    const FFTPlan f = make_plan(nb);
    char* p = static_cast<char*>(base);
    size_t off = 0;
    const size_t n = static_cast<size_t>(nt);
    auto take = [&](size_t bytes) {
        char* q = p ? p + off : nullptr;
        off = al(off + bytes);
        return q;
    };
    MMScratch t;
    t.chunks = chunks_for(nt, nb);
    t.Y = reinterpret_cast<double2*>(take(n * f.n * sizeof(double2)));
    t.tw = reinterpret_cast<double2*>(take(2 * kTw * sizeof(double2)));
    t.ab = reinterpret_cast<double*>(take(n * f.gc * 2 * sizeof(double)));
    t.mx = reinterpret_cast<double*>(take(n * f.gr * 4 * sizeof(double)));
    t.scal = reinterpret_cast<double*>(take(n * kSlotMM * sizeof(double)));
    t.mom = reinterpret_cast<double*>(take(3 * n * t.chunks * kNSlot * sizeof(double)));
    t.dlam = reinterpret_cast<double*>(take(n * kNumFit * sizeof(double)));
    t.mred = reinterpret_cast<double*>(take(n * REC_N * sizeof(double)));
    if (m) *m = t;
    return off;
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// ---- 0. twiddle tables ------------------------------------------------------------------
// exp(2 pi i m / N) for 0 <= m < N (N a power of two, N <= 2^16) as hi[m >> 8] * lo[m & 255]
// with lo[i] = exp(2 pi i i / N) and hi[i] = exp(2 pi i 256 i / N), each from sincospi of an exact
// argument; the product is within about two units in the last place.
__global__ void k_mm_twiddles(int64_t n, double2* __restrict__ tw) {
    const int i = threadIdx.x;
    double s, c;
    sincospi(2.0 * static_cast<double>(i) / static_cast<double>(n), &s, &c);
    tw[i] = make_double2(c, s);
    sincospi(2.0 * static_cast<double>(256 * i) / static_cast<double>(n), &s, &c);
    tw[kTw + i] = make_double2(c, s);
}

__device__ __forceinline__ double2 twiddle(const double2* __restrict__ tw, unsigned m) {
    return cmul(tw[kTw + (m >> 8)], tw[m & 255u]);
}

// ---- LDS radix-4 Stockham inverse DFT of length LEN on `cols` columns ----------------------
// Column c of `buf` starts at c * (LEN + 1) (one point of padding spreads the columns over the
// banks; cols * LEN <= PTS, the block's tile, so the buffer holds PTS + PTS / LEN points).  Stages
// of radix 4 (X_j = sum_k a_k i^(jk) for the inverse transform), then one of radix 2 when
// log2(LEN) is odd; tw[j] = exp(2 pi i j / LEN).  A stage loads the inputs of each thread's
// butterflies into registers, the block synchronises, the outputs are written in place, the block
// synchronises.  Two ends can skip the buffer: with SRC the first stage reads its inputs through
// src(col, index) (from global memory, say), and with SINK the last stage hands each output to
// sink(col, index, value) instead of writing it back (and needs no synchronisation).  COLFAST
// gives the last stage's butterflies to threads column-fastest, so that consecutive threads take
// the same output index of consecutive columns (coalesced stores of a transposed layout).
// Without SINK the result is in natural order in `buf`.
template <int LEN, int PTS, bool SRC, bool SINK, bool COLFAST, class Src, class Sink>
__device__ __forceinline__ void lds_idft_io(double2* buf, int cols, const double2* __restrict__ tw, Src&& src,
                                            Sink&& sink) {
    constexpr int kLog2 = __builtin_ctz(LEN);
    constexpr int kR4 = kLog2 / 2;
    constexpr bool kOdd = (kLog2 & 1) != 0;
    constexpr int kLd = LEN + 1;
    constexpr int kPer4 = (PTS / 4 + 255) / 256;   // radix-4 butterflies per thread (at most)
    const int nb4 = cols * (LEN / 4);
#pragma unroll
    for (int st = 0; st < kR4; ++st) {
        const bool from_src = SRC && st == 0;
        const bool to_sink = SINK && !kOdd && st == kR4 - 1;
        const bool colfast = COLFAST && !kOdd && st == kR4 - 1;
        const int n = LEN >> (2 * st), s = 1 << (2 * st), m = n >> 2;
        double2 a[kPer4][4];
        int cl[kPer4], bb[kPer4];
#pragma unroll
        for (int r = 0; r < kPer4; ++r) {
            const int idx = threadIdx.x + 256 * r;
            cl[r] = colfast ? idx % cols : idx / (LEN / 4);
            bb[r] = colfast ? idx / cols : idx % (LEN / 4);
            if (idx < nb4) {
                const int q = bb[r] & (s - 1), pp = bb[r] >> (2 * st);
                const int i0 = q + s * pp;
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    a[r][t] = from_src ? src(cl[r], i0 + t * s * m) : buf[cl[r] * kLd + i0 + t * s * m];
            }
        }
        // every read of this stage is done before any thread overwrites its inputs
        if (!from_src && !to_sink) __syncthreads();
#pragma unroll
        for (int r = 0; r < kPer4; ++r) {
            const int idx = threadIdx.x + 256 * r;
            if (idx < nb4) {
                const int q = bb[r] & (s - 1), pp = bb[r] >> (2 * st);
                const double2 b0 = make_double2(a[r][0].x + a[r][2].x, a[r][0].y + a[r][2].y);
                const double2 b1 = make_double2(a[r][0].x - a[r][2].x, a[r][0].y - a[r][2].y);
                const double2 b2 = make_double2(a[r][1].x + a[r][3].x, a[r][1].y + a[r][3].y);
                // i (a1 - a3)
                const double2 b3 = make_double2(a[r][3].y - a[r][1].y, a[r][1].x - a[r][3].x);
                const int ts = pp * (LEN / n);
                const int o = q + s * 4 * pp;
                const double2 y0 = make_double2(b0.x + b2.x, b0.y + b2.y);
                const double2 y1 = cmul(make_double2(b1.x + b3.x, b1.y + b3.y), tw[ts]);
                const double2 y2 = cmul(make_double2(b0.x - b2.x, b0.y - b2.y), tw[2 * ts]);
                const double2 y3 = cmul(make_double2(b1.x - b3.x, b1.y - b3.y), tw[3 * ts]);
                if (to_sink) {
                    sink(cl[r], o, y0);
                    sink(cl[r], o + s, y1);
                    sink(cl[r], o + 2 * s, y2);
                    sink(cl[r], o + 3 * s, y3);
                } else {
                    double2* yc = buf + cl[r] * kLd + o;
                    yc[0] = y0;
                    yc[s] = y1;
                    yc[2 * s] = y2;
                    yc[3 * s] = y3;
                }
            }
        }
        if (!to_sink) __syncthreads();
    }
    if constexpr (kOdd) {
        // last stage: n = 2, s = LEN / 2, twiddle 1
        constexpr int s = LEN / 2;
        constexpr int kPer2 = (PTS / 2 + 255) / 256;
        const int nb2 = cols * (LEN / 2);
        double2 a[kPer2][2];
        int cl[kPer2], qq[kPer2];
#pragma unroll
        for (int r = 0; r < kPer2; ++r) {
            const int idx = threadIdx.x + 256 * r;
            cl[r] = COLFAST ? idx % cols : idx / (LEN / 2);
            qq[r] = COLFAST ? idx / cols : idx % (LEN / 2);
            if (idx < nb2) {
                a[r][0] = buf[cl[r] * kLd + qq[r]];
                a[r][1] = buf[cl[r] * kLd + qq[r] + s];
            }
        }
        if (!SINK) __syncthreads();
#pragma unroll
        for (int r = 0; r < kPer2; ++r) {
            const int idx = threadIdx.x + 256 * r;
            if (idx < nb2) {
                const double2 y0 = make_double2(a[r][0].x + a[r][1].x, a[r][0].y + a[r][1].y);
                const double2 y1 = make_double2(a[r][0].x - a[r][1].x, a[r][0].y - a[r][1].y);
                if (SINK) {
                    sink(cl[r], qq[r], y0);
                    sink(cl[r], qq[r] + s, y1);
                } else {
                    buf[cl[r] * kLd + qq[r]] = y0;
                    buf[cl[r] * kLd + qq[r] + s] = y1;
                }
            }
        }
        if (!SINK) __syncthreads();
    }
}

template <int LEN>
__device__ __forceinline__ void fill_twiddles(double2* tw) {
    for (int j = threadIdx.x; j < LEN; j += 256) {
        double sn, cs;
        sincospi(2.0 * j / static_cast<double>(LEN), &sn, &cs);
        tw[j] = make_double2(cs, sn);
    }
}

// ---- 1. column pass with the overlap input -------------------------------------------------
// LEN = N2: block (target p, column group) computes x_k for the bins k = k1 + N1 k2 of the columns
// k1 = gcol .. gcol + cols - 1 and transforms each column over k2.
template <int LEN>
__global__ void __launch_bounds__(256) k_mm_cols(const double* __restrict__ recs, GridArgs g,
                                                 const double* __restrict__ tab, const double* __restrict__ targets,
                                                 const double* __restrict__ inv_psd,
                                                 const double2* __restrict__ twg, double2* __restrict__ Y,
                                                 double* __restrict__ ab, int n1, int cols) {
    constexpr int kLd = LEN + 1;
    __shared__ double2 buf[kColPts + kColPts / LEN];
    __shared__ double2 tw[LEN];
    __shared__ double red[2][4];
    const int64_t N = g.nb;
    const int groups = n1 / cols;
    const int64_t p = blockIdx.x / groups;
    const int gcol = (blockIdx.x % groups) * cols;
    fill_twiddles<LEN>(tw);
    const double* __restrict__ rec = recs + p * REC_N;
    const bool valid = rec[R_VALID] != 0.0;
    const Tabs T(tab, g.nb);
    const double2* __restrict__ tg = reinterpret_cast<const double2*>(targets) + p * N;
    // the merger-ringdown record form: table-reduced arc tangent (table in constant memory)
    const RecMRD rm = rec_mrd(rec, reinterpret_cast<const double2*>(kAtanTab));
    const double2* __restrict__ sct = reinterpret_cast<const double2*>(kSinCosTab);
    double a = 0.0, b = 0.0;
    for (int idx = threadIdx.x; idx < cols * LEN; idx += 256) {
        const int c = idx % cols, k2 = idx / cols;
        const int64_t k = gcol + c + static_cast<int64_t>(n1) * k2;
        const double2 t = tg[k];
        const double w = 4.0 * g.df * inv_psd[k];
        // x = w conj(h) t with h = A exp(-i Psi): conj(h) t = A t exp(i Psi), formed from the
        // sin/cos table angle directly (its real part is px and its imaginary part -py)
        double xr = 0.0, xi = 0.0, hh = 0.0;
        if (valid) {
            const double f = bin_freq(g, k);
            const double mf = rec[R_MS] * f;
            if (bin_active(g, f, mf)) {
                BinVals bv;
                eval_bin_rt(rm, T, k, mf, bv);
                const double A = rec[R_A0P] * T.at(T_F76, k) * bv.ahat;
                double px, py;
                pd_rotate_data(bv.psi, A, t.x, t.y, sct, px, py);
                xr = px;
                xi = -py;
                hh = A * A;
            }
        }
        buf[c * kLd + k2] = make_double2(w * xr, w * xi);
        a = fma(w, hh, a);
        b = fma(w, t.x * t.x + t.y * t.y, b);
    }
    a = wave_sum(a);
    b = wave_sum(b);
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][wid] = a;
        red[1][wid] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double* o = ab + (p * groups + (blockIdx.x % groups)) * 2;
        o[0] = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
        o[1] = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
    }
    // the last stage's outputs go straight to the transposed store, times exp(2 pi i j2 k1 / N)
    double2* __restrict__ dst = Y + p * N;
    const unsigned mask = static_cast<unsigned>(N - 1);
    lds_idft_io<LEN, kColPts, false, true, true>(
        buf, cols, tw, [](int, int) { return make_double2(0.0, 0.0); },
        [&](int c, int j2, double2 v) {
            const int k1 = gcol + c;
            dst[static_cast<int64_t>(j2) * n1 + k1] = cmul(v, twiddle(twg, (static_cast<unsigned>(j2) * k1) & mask));
        });
}

// ---- 2. row pass with fused arg-max of |z|^2 ------------------------------------------
__device__ __forceinline__ bool better(double v, int i, double bv, int bi) {
    return (v > bv) || (v == bv && i < bi);
}

// LEN = N1: block (target p, row group) transforms rows grow .. grow + rows - 1 (rows of the
// transposed array are indexed by j2); the lag of output j1 of row j2 is j = j2 + N2 j1.
template <int LEN>
__global__ void __launch_bounds__(256) k_mm_rows_max(const double2* __restrict__ Y, double* __restrict__ mx,
                                                     int n2, int rows) {
    __shared__ double2 buf[kRowPts + kRowPts / LEN];
    __shared__ double2 tw[LEN];
    __shared__ double rv[4];
    __shared__ int ri[4];
    __shared__ double2 rz[4];
    const int64_t N = static_cast<int64_t>(n2) * LEN;
    const int groups = n2 / rows;
    const int64_t p = blockIdx.x / groups;
    const int grow = (blockIdx.x % groups) * rows;
    fill_twiddles<LEN>(tw);
    const double2* __restrict__ src = Y + p * N + static_cast<int64_t>(grow) * LEN;
    __syncthreads();   // twiddles
    // the first stage reads the rows from global memory; the last stage's outputs feed the
    // arg-max of |z|^2 (ties to the smaller lag) in registers
    double best = -1.0;
    int bidx = 0x7fffffff;
    double2 bz = make_double2(0.0, 0.0);
    lds_idft_io<LEN, kRowPts, true, true, false>(
        buf, rows, tw, [&](int rrow, int k1) { return src[rrow * LEN + k1]; },
        [&](int rrow, int j1, double2 z) {
            const double a2 = z.x * z.x + z.y * z.y;
            const int j = (grow + rrow) + n2 * j1;
            if (better(a2, j, best, bidx)) {
                best = a2;
                bidx = j;
                bz = z;
            }
        });
    // arg-max over the wave by lane exchanges, then over the block's four waves
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bidx, off, 64);
        const double ozx = __shfl_xor(bz.x, off, 64);
        const double ozy = __shfl_xor(bz.y, off, 64);
        if (better(ov, oi, best, bidx)) {
            best = ov;
            bidx = oi;
            bz = make_double2(ozx, ozy);
        }
    }
    if ((threadIdx.x & 63) == 0) {
        rv[threadIdx.x >> 6] = best;
        ri[threadIdx.x >> 6] = bidx;
        rz[threadIdx.x >> 6] = bz;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w)
            if (better(rv[w], ri[w], rv[0], ri[0])) {
                rv[0] = rv[w];
                ri[0] = ri[w];
                rz[0] = rz[w];
            }
        // no comparable |z|^2 (all NaN): report lag 0 with a NaN modulus
        const bool none = ri[0] == 0x7fffffff;
        const int j = none ? grow : ri[0];
        const double2 z = none ? make_double2(__builtin_nan(""), __builtin_nan("")) : rz[0];
        double* o = mx + (p * groups + (blockIdx.x % groups)) * 4;
        o[0] = none ? __builtin_nan("") : rv[0];
        o[1] = static_cast<double>(j);
        o[2] = z.x;
        o[3] = z.y;
    }
}

// ---- 4. finalize ---------------------------------------------------------------------
__global__ void k_mm_finalize(const double* __restrict__ recs, int64_t nt, const double* __restrict__ ab,
                              const double* __restrict__ mx, double* __restrict__ scal,
                              double* __restrict__ mismatch, int32_t* __restrict__ lag, int blocks, int groups) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= nt) return;
    double* sc = scal + p * kSlotMM;
    if (recs[p * REC_N + R_VALID] == 0.0) {
        for (int i = 0; i < kSlotMM; ++i) sc[i] = 0.0;
        mismatch[p] = __builtin_nan("");
        if (lag) lag[p] = -1;
        return;
    }
    double A = 0.0, B = 0.0;
    for (int b = 0; b < blocks; ++b) {
        A += ab[(p * blocks + b) * 2 + 0];
        B += ab[(p * blocks + b) * 2 + 1];
    }
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
    if (bi == 0x7fffffff) {   // every |z|^2 NaN: NaN mismatch at lag 0
        bi = 0;
        best = __builtin_nan("");
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
// Moments sum_k z_k b_k of the basis values; the Mf-derivative moment is formed after the loop
// (fd_from_moments) from them and the two extra sums x[0] (phase) and x[1] (amplitude).
struct MMVis {
    static constexpr bool kFd = false;
    double* mom;
    double* x;
    double zr, zi;
    __device__ __forceinline__ void ph(int s, double b) { mom[s] = fma(zi, b, mom[s]); }
    __device__ __forceinline__ void am(int s, double b) { mom[s] = fma(zr, b, mom[s]); }
    __device__ __forceinline__ void ph_x(double b) { x[0] = fma(zi, b, x[0]); }
    __device__ __forceinline__ void am_x(double b) { x[1] = fma(zr, b, x[1]); }
};

struct AdjSegment {
    const double* __restrict__ rec;
    Tabs T;
    GridArgs g;
    const double2* __restrict__ tgt;
    const double* __restrict__ inv_psd;
    const double2* __restrict__ tw;    // twiddle tables in LDS
    const double2* __restrict__ sct;   // (sin, cos) table in LDS
    // the wave's copy of the record in LDS, read after each bin loop (loop-loaded uniform entries
    // used after a loop with a divergent exit are copied to vector registers on every trip)
    const double* recl;
    double ur, ui, inv_sab, cfa;
    int64_t j;
    int64_t k0, k1;
    int lane;
    double tot;

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
        const double w4 = 4.0 * g.df;
        double mom[REC_N];
#pragma unroll
        for (int s = 0; s < REC_N; ++s) mom[s] = 0.0;
        double mx[2] = {0.0, 0.0};
        ExpRec er{};
        if (AR == 3) er.init(rec, g, static_cast<unsigned>(k0 + lane), D ? rec[R_AM3 + 0] : 1.0);
        for (unsigned k = static_cast<unsigned>(k0 + lane); k < static_cast<unsigned>(k1); k += 64u) {
            const double mf = ms * bin_freq(g, k);
            BinVals bv;
            double f76, ipsd;
            double2 t;
            if constexpr (PR == 3) {
                // merger-ringdown: every per-bin load issued before the elementary functions'
                // branches, sharing one 32-bit offset from scalar bases
                f76 = T.at(T_F76, k);
                ipsd = inv_psd[k];
                t = tgt[k];
                BinTabs bt;
                bt.load(T, k);
                eval_bin_t<PR, AR, AR == 3>(c, bt, k, mf, bv, (AR == 3) ? er.next() : 0.0);
            } else {
                eval_bin_t<PR, AR, AR == 3>(c, T, k, mf, bv, (AR == 3) ? er.next() : 0.0);
                f76 = T.at(T_F76, k);
                ipsd = inv_psd[k];
                t = tgt[k];
            }
            const double Aamp = a0p * f76 * bv.ahat;
            const double w = w4 * ipsd;
            const double2 e = twiddle(tw, (k * static_cast<unsigned>(j)) & static_cast<unsigned>(g.nb - 1));
            const double2 x = cmul(make_double2(w * t.x, w * t.y), e);
            // G = conj(u) x
            const double gr = ur * x.x + ui * x.y, gi = ur * x.y - ui * x.x;
            // R = -G / sqrt(AB) + |z| w h / (A^(3/2) B^(1/2)), h = Aamp exp(-i Psi); the weights are
            // conj(h) R: Re (of d ln A) = -inv_sab Re(conj(h) G) + cfa w Aamp^2, and -Im (of d Psi)
            // = inv_sab Im(conj(h) G), with conj(h) G = Aamp G exp(i Psi) formed from the table
            // angle directly: its real part is px and its imaginary part -py
            double px, py;
            pd_rotate_data(bv.psi, Aamp, gr, gi, sct, px, py);
            const double cr = fma(-inv_sab, px, (cfa * w) * (Aamp * Aamp));
            MMVis vis{mom, mx, cr, -inv_sab * py};
            visit_bin_t<PR, AR>(c, bv, vis);
        }
        // (the inspiral loops read the record itself: its copy there measured more vector copies)
        fd_from_moments<PR, AR, D>(PR == 1 ? rec : recl, mom, mx[0], mx[1]);
        if (D && AR == 3) mom[R_AM3 + 0] = rec[R_IANUM] * mom[R_LNA0];
        flush_touched<PR, AR>(mom, lane, tot);
    }
};

template <int PRG>
__global__ void __launch_bounds__(256) k_mm_adjoint(const double* __restrict__ recs, int64_t nt, int chunks,
                                                    GridArgs g, const double* __restrict__ tab,
                                                    const double* __restrict__ targets,
                                                    const double* __restrict__ inv_psd,
                                                    const double2* __restrict__ tw,
                                                    const double* __restrict__ scal, double* __restrict__ part_all) {
    // the (sin, cos) and twiddle tables every bin reads, staged in LDS by the whole block first
    __shared__ double2 sct[kSinCosN + kAtanN];   // (sin, cos) table, then the arc tangent table
    __shared__ double2 twl[2 * kTw];
    __shared__ double recl[4][REC_N];
    stage_sincos_table(sct);
    stage_atan_table(sct + kSinCosN);
    for (int i = threadIdx.x; i < 2 * kTw; i += blockDim.x) twl[i] = tw[i];
    __syncthreads();
    double* __restrict__ part = part_all + static_cast<int64_t>(PRG - 1) * nt * chunks * kNSlot;
    const int lane = threadIdx.x & 63;
    const int cr = region_chunks(PRG, chunks);
    const int64_t wave = __builtin_amdgcn_readfirstlane(static_cast<int>(blockIdx.x * 4 + (threadIdx.x >> 6)));
    // wave-uniform point and chunk, kept in scalar registers (the record stays scalar in the loops)
    const int64_t p = uniform_i(wave / cr);
    const int c = uniform_i(wave - p * cr);
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
    seg.tgt = reinterpret_cast<const double2*>(targets) + p * g.nb;
    seg.inv_psd = inv_psd;
    seg.tw = twl;
    seg.sct = sct;
    if (lane < REC_N) recl[threadIdx.x >> 6][lane] = rec[lane];
    seg.recl = recl[threadIdx.x >> 6];
    // unit phase u = z / |z|; G_k = conj(u) x_k with x_k = w t_k exp(2 pi i k j / N)
    seg.ur = sc[3] / az;
    seg.ui = sc[4] / az;
    seg.inv_sab = 1.0 / sqrt(A * B);
    seg.cfa = az / (A * sqrt(A * B));   // |z| / (A^(3/2) B^(1/2))
    seg.j = static_cast<int64_t>(sc[5]);
    seg.lane = lane;
    seg.tot = 0.0;
    int64_t kb, ke;
    region_chunk_range(rec, g, PRG, c, cr, kb, ke);
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
        for (int c = 0; c < region_chunks(grp + 1, chunks); ++c) m += part[((grp * nt + p) * chunks + c) * kNSlot + 2 + s];
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

size_t mismatch_scratch_bytes(int64_t nt, int64_t nb) { return carve_into(nullptr, nt, nb, nullptr); }

template <int LEN>
static void launch_cols(unsigned blocks, const double* recs, const GridArgs& g, const double* tab,
                        const double* targets, const double* inv_psd, const double2* tw, double2* Y, double* ab,
                        int n1, int cols, hipStream_t s) {
    hipLaunchKernelGGL(k_mm_cols<LEN>, dim3(blocks), dim3(256), 0, s, recs, g, tab, targets, inv_psd, tw, Y, ab, n1,
                       cols);
}
template <int LEN>
static void launch_rows(unsigned blocks, const double2* Y, double* mx, int n2, int rows, hipStream_t s) {
    hipLaunchKernelGGL(k_mm_rows_max<LEN>, dim3(blocks), dim3(256), 0, s, Y, mx, n2, rows);
}

hipError_t launch_mismatch(const double* recs, const double* fit_tans, int64_t nt, const GridArgs& g,
                           const double* tab, const double* targets, const double* inv_psd, void* scratch, double* mismatch,
                           double* dsum_dlambda, int32_t* lag, hipStream_t s) {
    MMScratch m;
    carve_into(scratch, nt, g.nb, &m);
    const FFTPlan f = make_plan(g.nb);
    const unsigned col_blocks = static_cast<unsigned>(nt * f.gc);
    const unsigned row_blocks = static_cast<unsigned>(nt * f.gr);
    hipLaunchKernelGGL(k_mm_twiddles, dim3(1), dim3(kTw), 0, s, g.nb, m.tw);
    {
        ProfRange pr(PD_K_MISMATCH_INPUT, s);
        switch (f.n2) {
            case 8: launch_cols<8>(col_blocks, recs, g, tab, targets, inv_psd, m.tw, m.Y, m.ab, f.n1, f.cb, s); break;
            case 16: launch_cols<16>(col_blocks, recs, g, tab, targets, inv_psd, m.tw, m.Y, m.ab, f.n1, f.cb, s); break;
            case 32: launch_cols<32>(col_blocks, recs, g, tab, targets, inv_psd, m.tw, m.Y, m.ab, f.n1, f.cb, s); break;
            case 64: launch_cols<64>(col_blocks, recs, g, tab, targets, inv_psd, m.tw, m.Y, m.ab, f.n1, f.cb, s); break;
            case 128: launch_cols<128>(col_blocks, recs, g, tab, targets, inv_psd, m.tw, m.Y, m.ab, f.n1, f.cb, s); break;
            default: launch_cols<256>(col_blocks, recs, g, tab, targets, inv_psd, m.tw, m.Y, m.ab, f.n1, f.cb, s); break;
        }
    }
    {
        ProfRange pr(PD_K_MISMATCH_FFT, s);
        switch (f.n1) {
            case 8: launch_rows<8>(row_blocks, m.Y, m.mx, f.n2, f.rb, s); break;
            case 16: launch_rows<16>(row_blocks, m.Y, m.mx, f.n2, f.rb, s); break;
            case 32: launch_rows<32>(row_blocks, m.Y, m.mx, f.n2, f.rb, s); break;
            case 64: launch_rows<64>(row_blocks, m.Y, m.mx, f.n2, f.rb, s); break;
            case 128: launch_rows<128>(row_blocks, m.Y, m.mx, f.n2, f.rb, s); break;
            default: launch_rows<256>(row_blocks, m.Y, m.mx, f.n2, f.rb, s); break;
        }
    }
    hipLaunchKernelGGL(k_mm_finalize, dim3(static_cast<unsigned>((nt + 127) / 128)), dim3(128), 0, s, recs, nt,
                       m.ab, m.mx, m.scal, mismatch, lag, f.gc, f.gr);
    if (dsum_dlambda) {
        {
            ProfRange pr(PD_K_MISMATCH_ADJ, s);
            launch_regions(s, [&](int region, hipStream_t rs) {
                const dim3 grid(static_cast<unsigned>((nt * region_chunks(region, m.chunks) + 3) / 4));
                if (region == 3)
                    hipLaunchKernelGGL(k_mm_adjoint<3>, grid, dim3(256), 0, rs, recs, nt, m.chunks, g, tab, targets,
                                       inv_psd, m.tw, m.scal, m.mom);
                else if (region == 2)
                    hipLaunchKernelGGL(k_mm_adjoint<2>, grid, dim3(256), 0, rs, recs, nt, m.chunks, g, tab, targets,
                                       inv_psd, m.tw, m.scal, m.mom);
                else
                    hipLaunchKernelGGL(k_mm_adjoint<1>, grid, dim3(256), 0, rs, recs, nt, m.chunks, g, tab, targets,
                                       inv_psd, m.tw, m.scal, m.mom);
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
// lambda_i -= scale * P_i * dsum_i, scale = alpha / n_targets, P_i = precond[i] (1 without one).
__global__ void k_lambda_update(double* __restrict__ lam, const double* __restrict__ dsum,
                                const double* __restrict__ precond, double scale) {
    const int i = threadIdx.x;
    if (i < kNumLambda) {
        const double step = precond ? scale * precond[i] : scale;
        lam[i] = fma(-step, dsum[i], lam[i]);
    }
}

hipError_t launch_lambda_update(double* lam, const double* dsum, const double* precond, double scale,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_lambda_update, dim3(1), dim3(256), 0, s, lam, dsum, precond, scale);
    return hipGetLastError();
}

}  // namespace pd
