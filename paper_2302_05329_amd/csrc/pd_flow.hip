// RealNVP normalising flow on the GPU: the learned independence proposal for the
// sampler (the follow-up the paper announces at the end of Sec. 3.3: normalising flows
// + GPU + gradient-based sampler).
//
// Architecture (fixed): 7-D, a fixed standardisation y = (x - mu) * isd, then 8 affine
// coupling layers (Dinh et al. 2017).  Layer l conditions on dims {0,1,2} (l even) or
// {3,...,6} (l odd) and transforms the others:
//   in = m * y;  h1 = tanh(W1^T in + b1);  h2 = tanh(W2^T h1 + b2);  o = W3^T h2 + b3
//   s = 2 tanh(o[0:7] / 2) (1 - m),  t = o[7:14] (1 - m)
//   forward (data -> latent):  y' = m y + (1 - m) (y exp(s) + t),  log det += sum s
//   inverse:                   y  = m y' + (1 - m) (y' - t) exp(-s)
// log q(x) = sum_d [-z_d^2/2 - log(2 pi)/2] + sum_l sum s_l + sum_d log isd_d.
//
// Parameter layout (float32): per layer W1[7][128], b1[128], W2[128][128], b2[128],
// W3[128][14], b3[14] (19342 floats), 8 layers, then mu[7], isd[7].
//
// Kernels: one block of 1024 threads per tile of samples, all 8 layers fused, activations
// in LDS, weights read through the caches.  Training saves each layer's input, hidden
// activations and outputs; the backward kernel writes one row of weight-gradient partial
// sums per tile, reduced in a fixed order (no atomics).
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/phenomd.h"
#include "pd_launch.h"

namespace pd {

namespace {

constexpr int kD = 7;
constexpr int kH = 128;
constexpr int kO = 14;
constexpr int kLayers = 8;
constexpr int kLayerP = kD * kH + kH + kH * kH + kH + kH * kO + kO;   // 19342
constexpr int kP = kLayers * kLayerP + 2 * kD;                         // + mu, isd
constexpr int kOffW1 = 0, kOffB1 = kD * kH, kOffW2 = kOffB1 + kH, kOffB2 = kOffW2 + kH * kH,
              kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + kH * kO;
constexpr int kOffStd = kLayers * kLayerP;
constexpr float kSC = 2.0f;                 // bound of the log-scale
constexpr int kSave = 8 + kH + kH + 16;     // per sample per layer: y_in, h1, h2, o
constexpr int kTF = 16;                     // samples per tile, forward / inverse
constexpr int kTB = 32;                     // samples per tile, backward
constexpr int kNTF = 1024;                  // threads per block of the FP32 kernels
static_assert((kTF * kH) % kNTF == 0 && (kTB * kH) % kNTF == 0, "whole samples per thread");
constexpr float kHalfLog2Pi = 0.91893853320467274178f;

__device__ __forceinline__ bool cond_dim(int layer, int d) { return (layer & 1) ? (d >= 3) : (d < 3); }

// Fused 8-layer pass over one tile.  INV: latent -> data.  SAVE: keep activations.
template <bool INV, bool SAVE>
__global__ void __launch_bounds__(kNTF) k_flow(const float* __restrict__ P, const double* __restrict__ in, int64_t n,
                                              double* __restrict__ out, double* __restrict__ logq,
                                              float* __restrict__ saved) {
    __shared__ float y[kTF][8];
    __shared__ float h1[kTF][kH];
    __shared__ float h2[kTF][kH];
    __shared__ float o[kTF][16];
    __shared__ float sv[kTF][8];
    const int t = threadIdx.x;
    const int64_t s0 = static_cast<int64_t>(blockIdx.x) * kTF;
    const float* mu = P + kOffStd;
    const float* isd = mu + kD;
    if (t < kTF * 8) {
        const int s = t / 8, d = t % 8;
        float v = 0.0f;
        if (d < kD && s0 + s < n) {
            const float xv = static_cast<float>(in[(s0 + s) * kD + d]);
            v = INV ? xv : (xv - mu[d]) * isd[d];
        }
        y[s][d] = v;
        sv[s][d] = 0.0f;
    }
    __syncthreads();
    for (int step = 0; step < kLayers; ++step) {
        const int layer = INV ? (kLayers - 1 - step) : step;
        const float* W1 = P + layer * kLayerP + kOffW1;
        const float* B1 = P + layer * kLayerP + kOffB1;
        const float* W2 = P + layer * kLayerP + kOffW2;
        const float* B2 = P + layer * kLayerP + kOffB2;
        const float* W3 = P + layer * kLayerP + kOffW3;
        const float* B3 = P + layer * kLayerP + kOffB3;
        if (SAVE && t < kTF * 8) {
            const int s = t / 8, d = t % 8;
            if (s0 + s < n) saved[((s0 + s) * kLayers + layer) * kSave + d] = y[s][d];
        }
        // hidden layer 1
        for (int idx = t; idx < kTF * kH; idx += kNTF) {
            const int s = idx / kH, j = idx % kH;
            float a = B1[j];
#pragma unroll
            for (int d = 0; d < kD; ++d)
                if (cond_dim(layer, d)) a = fmaf(W1[d * kH + j], y[s][d], a);
            h1[s][j] = tanhf(a);
        }
        __syncthreads();
        // hidden layer 2: thread -> column j, kSF samples
        {
            constexpr int kSF = kTF * kH / kNTF;
            const int j = t % kH, sg = (t / kH) * kSF;
            float acc[kSF];
#pragma unroll
            for (int r = 0; r < kSF; ++r) acc[r] = B2[j];
            for (int k = 0; k < kH; ++k) {
                const float w = W2[k * kH + j];
#pragma unroll
                for (int r = 0; r < kSF; ++r) acc[r] = fmaf(w, h1[sg + r][k], acc[r]);
            }
#pragma unroll
            for (int r = 0; r < kSF; ++r) h2[sg + r][j] = tanhf(acc[r]);
        }
        __syncthreads();
        // output layer
        if (t < kTF * kO) {
            const int s = t / kO, c = t % kO;
            float a = B3[c];
            for (int k = 0; k < kH; ++k) a = fmaf(W3[k * kO + c], h2[s][k], a);
            o[s][c] = a;
        }
        __syncthreads();
        if (SAVE) {
            for (int idx = t; idx < kTF * (2 * kH + 16); idx += kNTF) {
                const int s = idx / (2 * kH + 16), r = idx % (2 * kH + 16);
                if (s0 + s >= n) continue;
                float v;
                if (r < kH)
                    v = h1[s][r];
                else if (r < 2 * kH)
                    v = h2[s][r - kH];
                else
                    v = (r - 2 * kH < kO) ? o[s][r - 2 * kH] : 0.0f;
                saved[((s0 + s) * kLayers + layer) * kSave + 8 + r] = v;
            }
        }
        // coupling update
        if (t < kTF * kD) {
            const int s = t / kD, d = t % kD;
            if (!cond_dim(layer, d)) {
                const float svv = kSC * tanhf(o[s][d] / kSC);
                const float tt = o[s][kD + d];
                y[s][d] = INV ? (y[s][d] - tt) * expf(-svv) : fmaf(y[s][d], expf(svv), tt);
                sv[s][d] += svv;
            }
        }
        __syncthreads();
    }
    if (t < kTF) {
        const int s = t;
        if (s0 + s < n) {
            double lq = 0.0;
            for (int d = 0; d < kD; ++d) {
                const double z = INV ? static_cast<double>(in[(s0 + s) * kD + d]) : static_cast<double>(y[s][d]);
                lq += -0.5 * z * z - static_cast<double>(kHalfLog2Pi) + static_cast<double>(sv[s][d]) +
                      log(static_cast<double>(isd[d]));
            }
            logq[s0 + s] = lq;
        }
    }
    if (t < kTF * kD) {
        const int s = t / kD, d = t % kD;
        if (s0 + s < n && out) {
            out[(s0 + s) * kD + d] =
                INV ? static_cast<double>(y[s][d] / isd[d] + mu[d]) : static_cast<double>(y[s][d]);
        }
    }
}

// Backward pass of loss = -mean(log q) over one tile of kTB samples; writes this tile's
// weight-gradient partial sums partial[tile][P].
__global__ void __launch_bounds__(kNTF) k_flow_backward(const float* __restrict__ P, int64_t n,
                                                       const double* __restrict__ z, const float* __restrict__ saved,
                                                       float* __restrict__ partial) {
    __shared__ float yin[kTB][8];
    __shared__ float h1[kTB][kH];
    __shared__ float h2[kTB][kH];
    __shared__ float go[kTB][16];
    __shared__ float gh[kTB][kH];
    __shared__ float gy[kTB][8];
    const int t = threadIdx.x;
    const int64_t s0 = static_cast<int64_t>(blockIdx.x) * kTB;
    float* gp = partial + static_cast<int64_t>(blockIdx.x) * kP;
    const float invB = 1.0f / static_cast<float>(n);
    if (t < kTB * 8) {
        const int s = t / 8, d = t % 8;
        gy[s][d] = (d < kD && s0 + s < n) ? static_cast<float>(z[(s0 + s) * kD + d]) * invB : 0.0f;
    }
    for (int i = t; i < 2 * kD; i += kNTF) gp[kOffStd + i] = 0.0f;
    __syncthreads();
    for (int layer = kLayers - 1; layer >= 0; --layer) {
        const float* W1 = P + layer * kLayerP + kOffW1;
        const float* W2 = P + layer * kLayerP + kOffW2;
        const float* W3 = P + layer * kLayerP + kOffW3;
        float* G = gp + layer * kLayerP;
        // load the saved activations of this layer
        for (int idx = t; idx < kTB * kSave; idx += kNTF) {
            const int s = idx / kSave, r = idx % kSave;
            const float v = (s0 + s < n) ? saved[((s0 + s) * kLayers + layer) * kSave + r] : 0.0f;
            if (r < 8)
                yin[s][r] = v;
            else if (r < 8 + kH)
                h1[s][r - 8] = v;
            else if (r < 8 + 2 * kH)
                h2[s][r - 8 - kH] = v;
            else
                go[s][r - 8 - 2 * kH] = v;   // o for now
        }
        __syncthreads();
        // coupling backward: go <- d loss / d o, gy <- direct part of d loss / d y_in
        if (t < kTB * kD) {
            const int s = t / kD, d = t % kD;
            const bool live = s0 + s < n;
            if (!cond_dim(layer, d)) {
                const float svv = kSC * tanhf(go[s][d] / kSC);
                const float e = expf(svv);
                const float gyo = gy[s][d];
                const float gs = live ? fmaf(gyo * yin[s][d], e, -invB) : 0.0f;
                const float q = svv / kSC;
                go[s][d] = gs * (1.0f - q * q);
                go[s][kD + d] = gyo;
                gy[s][d] = gyo * e;
            } else {
                go[s][d] = 0.0f;
                go[s][kD + d] = 0.0f;
            }
        }
        __syncthreads();
        // output layer: gW3, gb3, gh2 = W3 go
        for (int idx = t; idx < kH * kO + kO; idx += kNTF) {
            float a = 0.0f;
            if (idx < kH * kO) {
                const int k = idx / kO, c = idx % kO;
                for (int s = 0; s < kTB; ++s) a = fmaf(h2[s][k], go[s][c], a);
                G[kOffW3 + idx] = a;
            } else {
                const int c = idx - kH * kO;
                for (int s = 0; s < kTB; ++s) a += go[s][c];
                G[kOffB3 + c] = a;
            }
        }
        for (int idx = t; idx < kTB * kH; idx += kNTF) {
            const int s = idx / kH, k = idx % kH;
            float a = 0.0f;
#pragma unroll
            for (int c = 0; c < kO; ++c) a = fmaf(W3[k * kO + c], go[s][c], a);
            gh[s][k] = a * (1.0f - h2[s][k] * h2[s][k]);   // d loss / d a2
        }
        __syncthreads();
        // hidden layer 2: gW2[k][j] = sum_s h1[s][k] ga2[s][j], gb2, then gh1 = W2 ga2
        for (int idx = t; idx < kH * kH; idx += kNTF) {
            const int k = idx / kH, j = idx % kH;
            float a = 0.0f;
            for (int s = 0; s < kTB; ++s) a = fmaf(h1[s][k], gh[s][j], a);
            G[kOffW2 + idx] = a;
        }
        if (t < kH) {
            float a = 0.0f;
            for (int s = 0; s < kTB; ++s) a += gh[s][t];
            G[kOffB2 + t] = a;
        }
        // gh1 into h2's storage (h2 no longer needed): thread -> row k, kSB samples
        {
            constexpr int kSB = kTB * kH / kNTF;
            const int k = t % kH, sg = (t / kH) * kSB;
            float acc[kSB];
#pragma unroll
            for (int r = 0; r < kSB; ++r) acc[r] = 0.0f;
            for (int j = 0; j < kH; ++j) {
                const float w = W2[k * kH + j];
#pragma unroll
                for (int r = 0; r < kSB; ++r) acc[r] = fmaf(w, gh[sg + r][j], acc[r]);
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < kSB; ++r) h2[sg + r][k] = acc[r] * (1.0f - h1[sg + r][k] * h1[sg + r][k]);
        }
        __syncthreads();
        // hidden layer 1 (ga1 in h2): gW1[d][j] = sum_s in[s][d] ga1[s][j], gb1, gin = W1 ga1
        for (int idx = t; idx < kD * kH + kH; idx += kNTF) {
            float a = 0.0f;
            if (idx < kD * kH) {
                const int d = idx / kH, j = idx % kH;
                if (cond_dim(layer, d))
                    for (int s = 0; s < kTB; ++s) a = fmaf(yin[s][d], h2[s][j], a);
                G[kOffW1 + idx] = a;
            } else {
                const int j = idx - kD * kH;
                for (int s = 0; s < kTB; ++s) a += h2[s][j];
                G[kOffB1 + j] = a;
            }
        }
        if (t < kTB * kD) {
            const int s = t / kD, d = t % kD;
            if (cond_dim(layer, d)) {
                float a = 0.0f;
                for (int j = 0; j < kH; ++j) a = fmaf(W1[d * kH + j], h2[s][j], a);
                gy[s][d] += a;
            }
        }
        __syncthreads();
    }
}

// ---- BF16 matrix-core variant -------------------------------------------------------
// The 128 x 128 hidden layer and the 128 -> 14 output layer (and in training the gradient
// GEMMs of both) run on v_mfma_f32_16x16x32_bf16: operands rounded to bfloat16, products
// accumulated in FP32.  The 7 -> 128 input layer, the couplings and the log-determinants stay
// in FP32.  Lane layout (checked on gfx950 with an in-bounds probe): lane l supplies
// A[l%16][8 (l/16) + e] and B[8 (l/16) + e][l%16], e = 0..7, and receives C[4 (l/16) + r][l%16],
// r = 0..3.  A fixed flow in this mode is still an exact bijection with log|det J| = sum s:
// within a layer s and t depend only on the unchanged dims, so rounding them changes the map,
// not its triangular structure.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kTM = 32;   // samples per block in the matrix-core kernels
constexpr int kNT = 1024;  // threads per block in the matrix-core kernels (16 waves share a tile)
constexpr int kNW = kNT / 64;

// One 16 x 16 output tile C[mt][nt] += A[16 mt.., 0..K) B[0..K, 16 nt..] with A(i, k) and
// B(k, j) supplied as FP32 and rounded to bfloat16.  K is a multiple of 32.
template <int K, class FA, class FB>
__device__ __forceinline__ f4 mfma_tile(FA a_at, FB b_at, int mt, int nt, int lane) {
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    const int i = 16 * mt + (lane & 15), j = 16 * nt + (lane & 15), kq = 8 * (lane >> 4);
#pragma unroll
    for (int ks = 0; ks < K / 32; ++ks) {
        bf8 a, b;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            a[e] = static_cast<__bf16>(a_at(i, 32 * ks + kq + e));
            b[e] = static_cast<__bf16>(b_at(32 * ks + kq + e, j));
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
    return acc;
}

// Row of output element r of this lane in a tile, and its column.
__device__ __forceinline__ int tile_row(int mt, int lane, int r) { return 16 * mt + 4 * (lane >> 4) + r; }
__device__ __forceinline__ int tile_col(int nt, int lane) { return 16 * nt + (lane & 15); }

template <bool INV, bool SAVE>
__global__ void __launch_bounds__(kNT) k_flow_mf(const float* __restrict__ P, const double* __restrict__ in, int64_t n,
                                                 double* __restrict__ out, double* __restrict__ logq,
                                                 float* __restrict__ saved) {
    __shared__ float y[kTM][8];
    __shared__ float h1[kTM][kH + 1];
    __shared__ float h2[kTM][kH + 1];
    __shared__ float o[kTM][16];
    __shared__ float sv[kTM][8];
    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6;
    const int64_t s0 = static_cast<int64_t>(blockIdx.x) * kTM;
    const float* mu = P + kOffStd;
    const float* isd = mu + kD;
    if (t < kTM * 8) {
        const int s = t / 8, d = t % 8;
        float v = 0.0f;
        if (d < kD && s0 + s < n) {
            const float xv = static_cast<float>(in[(s0 + s) * kD + d]);
            v = INV ? xv : (xv - mu[d]) * isd[d];
        }
        y[s][d] = v;
        sv[s][d] = 0.0f;
    }
    __syncthreads();
    for (int step = 0; step < kLayers; ++step) {
        const int layer = INV ? (kLayers - 1 - step) : step;
        const float* W1 = P + layer * kLayerP + kOffW1;
        const float* B1 = P + layer * kLayerP + kOffB1;
        const float* W2 = P + layer * kLayerP + kOffW2;
        const float* B2 = P + layer * kLayerP + kOffB2;
        const float* W3 = P + layer * kLayerP + kOffW3;
        const float* B3 = P + layer * kLayerP + kOffB3;
        if (SAVE && t < kTM * 8) {
            const int s = t / 8, d = t % 8;
            if (s0 + s < n) saved[((s0 + s) * kLayers + layer) * kSave + d] = y[s][d];
        }
        // input layer (FP32)
        for (int idx = t; idx < kTM * kH; idx += kNT) {
            const int s = idx / kH, j = idx % kH;
            float a = B1[j];
#pragma unroll
            for (int d = 0; d < kD; ++d)
                if (cond_dim(layer, d)) a = fmaf(W1[d * kH + j], y[s][d], a);
            h1[s][j] = tanhf(a);
        }
        __syncthreads();
        // hidden layer on the matrix cores: 2 x 8 tiles, 4 per wave
        for (int tt = w; tt < 16; tt += kNW) {
            const int mt = tt >> 3, nt = tt & 7;
            const f4 acc = mfma_tile<kH>([&](int i, int k) { return h1[i][k]; },
                                         [&](int k, int j) { return W2[k * kH + j]; }, mt, nt, lane);
            const int j = tile_col(nt, lane);
#pragma unroll
            for (int r = 0; r < 4; ++r) h2[tile_row(mt, lane, r)][j] = tanhf(acc[r] + B2[j]);
        }
        __syncthreads();
        // output layer on the matrix cores: 2 x 1 tiles (columns 14, 15 are zero padding)
        if (w < 2) {
            const f4 acc = mfma_tile<kH>([&](int i, int k) { return h2[i][k]; },
                                         [&](int k, int c) { return c < kO ? W3[k * kO + c] : 0.0f; }, w, 0, lane);
            const int c = tile_col(0, lane);
#pragma unroll
            for (int r = 0; r < 4; ++r) o[tile_row(w, lane, r)][c] = (c < kO) ? acc[r] + B3[c] : 0.0f;
        }
        __syncthreads();
        if (SAVE) {
            for (int idx = t; idx < kTM * (2 * kH + 16); idx += kNT) {
                const int s = idx / (2 * kH + 16), r = idx % (2 * kH + 16);
                if (s0 + s >= n) continue;
                const float v = (r < kH) ? h1[s][r] : ((r < 2 * kH) ? h2[s][r - kH] : o[s][r - 2 * kH]);
                saved[((s0 + s) * kLayers + layer) * kSave + 8 + r] = v;
            }
        }
        // coupling update
        if (t < kTM * kD) {
            const int s = t / kD, d = t % kD;
            if (!cond_dim(layer, d)) {
                const float svv = kSC * tanhf(o[s][d] / kSC);
                const float tt = o[s][kD + d];
                y[s][d] = INV ? (y[s][d] - tt) * expf(-svv) : fmaf(y[s][d], expf(svv), tt);
                sv[s][d] += svv;
            }
        }
        __syncthreads();
    }
    if (t < kTM) {
        const int s = t;
        if (s0 + s < n) {
            double lq = 0.0;
            for (int d = 0; d < kD; ++d) {
                const double z = INV ? static_cast<double>(in[(s0 + s) * kD + d]) : static_cast<double>(y[s][d]);
                lq += -0.5 * z * z - static_cast<double>(kHalfLog2Pi) + static_cast<double>(sv[s][d]) +
                      log(static_cast<double>(isd[d]));
            }
            logq[s0 + s] = lq;
        }
    }
    if (t < kTM * kD) {
        const int s = t / kD, d = t % kD;
        if (s0 + s < n && out) {
            out[(s0 + s) * kD + d] =
                INV ? static_cast<double>(y[s][d] / isd[d] + mu[d]) : static_cast<double>(y[s][d]);
        }
    }
}

// Backward pass of loss = -mean(log q) over one tile of kTM samples with the GEMMs of the
// hidden and output layers on the matrix cores; writes the tile's weight-gradient row.
__global__ void __launch_bounds__(kNT) k_flow_backward_mf(const float* __restrict__ P, int64_t n,
                                                          const double* __restrict__ z,
                                                          const float* __restrict__ saved,
                                                          float* __restrict__ partial) {
    __shared__ float yin[kTM][8];
    __shared__ float h1[kTM][kH + 1];
    __shared__ float h2[kTM][kH + 1];
    __shared__ float go[kTM][16];
    __shared__ float gh[kTM][kH + 1];
    __shared__ float gy[kTM][8];
    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6;
    const int64_t s0 = static_cast<int64_t>(blockIdx.x) * kTM;
    float* gp = partial + static_cast<int64_t>(blockIdx.x) * kP;
    const float invB = 1.0f / static_cast<float>(n);
    if (t < kTM * 8) {
        const int s = t / 8, d = t % 8;
        gy[s][d] = (d < kD && s0 + s < n) ? static_cast<float>(z[(s0 + s) * kD + d]) * invB : 0.0f;
    }
    for (int i = t; i < 2 * kD; i += kNT) gp[kOffStd + i] = 0.0f;
    __syncthreads();
    for (int layer = kLayers - 1; layer >= 0; --layer) {
        const float* W1 = P + layer * kLayerP + kOffW1;
        const float* W2 = P + layer * kLayerP + kOffW2;
        const float* W3 = P + layer * kLayerP + kOffW3;
        float* G = gp + layer * kLayerP;
        for (int idx = t; idx < kTM * kSave; idx += kNT) {
            const int s = idx / kSave, r = idx % kSave;
            const float v = (s0 + s < n) ? saved[((s0 + s) * kLayers + layer) * kSave + r] : 0.0f;
            if (r < 8)
                yin[s][r] = v;
            else if (r < 8 + kH)
                h1[s][r - 8] = v;
            else if (r < 8 + 2 * kH)
                h2[s][r - 8 - kH] = v;
            else
                go[s][r - 8 - 2 * kH] = v;   // o for now
        }
        __syncthreads();
        // coupling backward: go <- d loss / d o, gy <- direct part of d loss / d y_in
        if (t < kTM * kD) {
            const int s = t / kD, d = t % kD;
            const bool live = s0 + s < n;
            if (!cond_dim(layer, d)) {
                const float svv = kSC * tanhf(go[s][d] / kSC);
                const float e = expf(svv);
                const float gyo = gy[s][d];
                const float gs = live ? fmaf(gyo * yin[s][d], e, -invB) : 0.0f;
                const float q = svv / kSC;
                go[s][d] = gs * (1.0f - q * q);
                go[s][kD + d] = gyo;
                gy[s][d] = gyo * e;
            } else {
                go[s][d] = 0.0f;
                go[s][kD + d] = 0.0f;
            }
        }
        if (t < kTM) {
            go[t][14] = 0.0f;
            go[t][15] = 0.0f;
        }
        __syncthreads();
        // output layer: gW3 = H2^T go (8 x 1 tiles, K = 32 samples), gb3, and
        // gh2 = go W3^T (2 x 8 tiles, K = 16 padded to 32)
        for (int tt = w; tt < 8; tt += kNW) {
            const f4 acc = mfma_tile<kTM>([&](int k, int s) { return h2[s][k]; },
                                          [&](int s, int c) { return go[s][c]; }, tt, 0, lane);
            const int c = tile_col(0, lane);
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (c < kO) G[kOffW3 + tile_row(tt, lane, r) * kO + c] = acc[r];
        }
        if (t < kO) {
            float a = 0.0f;
            for (int s = 0; s < kTM; ++s) a += go[s][t];
            G[kOffB3 + t] = a;
        }
        for (int tt = w; tt < 16; tt += kNW) {
            const int mt = tt >> 3, nt = tt & 7;
            const f4 acc = mfma_tile<32>([&](int s, int c) { return c < 16 ? go[s][c] : 0.0f; },
                                         [&](int c, int j) { return c < kO ? W3[j * kO + c] : 0.0f; }, mt, nt, lane);
            const int j = tile_col(nt, lane);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int s = tile_row(mt, lane, r);
                gh[s][j] = acc[r] * (1.0f - h2[s][j] * h2[s][j]);   // d loss / d a2
            }
        }
        __syncthreads();
        // hidden layer: gW2 = H1^T ga2 (8 x 8 tiles, K = 32 samples), gb2
        for (int tt = w; tt < 64; tt += kNW) {
            const int mt = tt >> 3, nt = tt & 7;
            const f4 acc = mfma_tile<kTM>([&](int k, int s) { return h1[s][k]; },
                                          [&](int s, int j) { return gh[s][j]; }, mt, nt, lane);
            const int j = tile_col(nt, lane);
#pragma unroll
            for (int r = 0; r < 4; ++r) G[kOffW2 + tile_row(mt, lane, r) * kH + j] = acc[r];
        }
        if (t < kH) {
            float a = 0.0f;
            for (int s = 0; s < kTM; ++s) a += gh[s][t];
            G[kOffB2 + t] = a;
        }
        // gh1 = ga2 W2^T (2 x 8 tiles, K = 128), into h2's storage (h2 is no longer needed)
        for (int tt = w; tt < 16; tt += kNW) {
            const int mt = tt >> 3, nt = tt & 7;
            const f4 acc = mfma_tile<kH>([&](int s, int j) { return gh[s][j]; },
                                         [&](int j, int k) { return W2[k * kH + j]; }, mt, nt, lane);
            const int k = tile_col(nt, lane);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int s = tile_row(mt, lane, r);
                h2[s][k] = acc[r] * (1.0f - h1[s][k] * h1[s][k]);   // d loss / d a1
            }
        }
        __syncthreads();
        // input layer (FP32): gW1, gb1, and the part of gy through the conditioning dims
        for (int idx = t; idx < kD * kH + kH; idx += kNT) {
            float a = 0.0f;
            if (idx < kD * kH) {
                const int d = idx / kH, j = idx % kH;
                if (cond_dim(layer, d))
                    for (int s = 0; s < kTM; ++s) a = fmaf(yin[s][d], h2[s][j], a);
                G[kOffW1 + idx] = a;
            } else {
                const int j = idx - kD * kH;
                for (int s = 0; s < kTM; ++s) a += h2[s][j];
                G[kOffB1 + j] = a;
            }
        }
        if (t < kTM * kD) {
            const int s = t / kD, d = t % kD;
            if (cond_dim(layer, d)) {
                float a = 0.0f;
                for (int j = 0; j < kH; ++j) a = fmaf(W1[d * kH + j], h2[s][j], a);
                gy[s][d] += a;
            }
        }
        __syncthreads();
    }
}

// Sum of the tiles' gradient rows in a fixed order: eight interleaved running sums (tile i goes
// to sum i mod 8, so eight loads are in flight per thread), then those eight in order.
__global__ void k_grad_reduce(const float* __restrict__ partial, int tiles, float* __restrict__ grad) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= kP) return;
    float a[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    int i = 0;
    for (; i + 8 <= tiles; i += 8) {
#pragma unroll
        for (int r = 0; r < 8; ++r) a[r] += partial[static_cast<int64_t>(i + r) * kP + p];
    }
    for (int r = 0; i < tiles; ++i, ++r) a[r] += partial[static_cast<int64_t>(i) * kP + p];
    grad[p] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

__global__ void k_loss(const double* __restrict__ logq, int64_t n, double* __restrict__ loss) {
    __shared__ double red[256];
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) a += logq[i];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = -red[0] / static_cast<double>(n);
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t count, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = fmaf(b1, m[i], (1.0f - b1) * gi);
    const float vi = fmaf(b2, v[i], (1.0f - b2) * gi * gi);
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

constexpr size_t kAl = 256;
inline size_t al(size_t x) { return (x + kAl - 1) / kAl * kAl; }

}  // namespace

int64_t flow_param_count() { return kP; }

size_t flow_ws_bytes(int64_t n) {
    const size_t N = static_cast<size_t>(n);
    const size_t tiles = (N + kTB - 1) / kTB;
    size_t off = 0;
    off = al(off + N * kLayers * kSave * sizeof(float));   // saved activations
    off = al(off + N * kD * sizeof(double));               // z
    off = al(off + N * sizeof(double));                    // log q
    off = al(off + tiles * kP * sizeof(float));            // gradient partials
    return off;
}

int flow_forward(const float* params, const double* x, int64_t n, double* z, double* logq, int mode, hipStream_t s) {
    if (mode == PD_FLOW_BF16) {
        hipLaunchKernelGGL((k_flow_mf<false, false>), dim3(static_cast<unsigned>((n + kTM - 1) / kTM)), dim3(kNT), 0, s,
                           params, x, n, z, logq, nullptr);
    } else {
        hipLaunchKernelGGL((k_flow<false, false>), dim3(static_cast<unsigned>((n + kTF - 1) / kTF)), dim3(kNTF), 0, s,
                           params, x, n, z, logq, nullptr);
    }
    return hipGetLastError() == hipSuccess ? PD_OK : PD_EHIP;
}

int flow_sample(const float* params, const double* z, int64_t n, double* x, double* logq, int mode, hipStream_t s) {
    if (mode == PD_FLOW_BF16) {
        hipLaunchKernelGGL((k_flow_mf<true, false>), dim3(static_cast<unsigned>((n + kTM - 1) / kTM)), dim3(kNT), 0, s,
                           params, z, n, x, logq, nullptr);
    } else {
        hipLaunchKernelGGL((k_flow<true, false>), dim3(static_cast<unsigned>((n + kTF - 1) / kTF)), dim3(kNTF), 0, s,
                           params, z, n, x, logq, nullptr);
    }
    return hipGetLastError() == hipSuccess ? PD_OK : PD_EHIP;
}

int flow_loss_grad(const float* params, const double* x, int64_t n, float* grad, double* loss, void* ws, int mode,
                   hipStream_t s) {
    const size_t N = static_cast<size_t>(n);
    char* base = static_cast<char*>(ws);
    size_t off = 0;
    float* saved = reinterpret_cast<float*>(base + off);
    off = al(off + N * kLayers * kSave * sizeof(float));
    double* z = reinterpret_cast<double*>(base + off);
    off = al(off + N * kD * sizeof(double));
    double* lq = reinterpret_cast<double*>(base + off);
    off = al(off + N * sizeof(double));
    float* partial = reinterpret_cast<float*>(base + off);
    const unsigned fblocks = static_cast<unsigned>((n + kTF - 1) / kTF);
    const int tiles = static_cast<int>((n + kTB - 1) / kTB);
    static_assert(kTM == kTB, "both backward kernels write one gradient row per 32-sample tile");
    if (mode == PD_FLOW_BF16) {
        hipLaunchKernelGGL((k_flow_mf<false, true>), dim3(static_cast<unsigned>((n + kTM - 1) / kTM)), dim3(kNT), 0, s,
                           params, x, n, z, lq, saved);
        hipLaunchKernelGGL(k_flow_backward_mf, dim3(tiles), dim3(kNT), 0, s, params, n, z, saved, partial);
    } else {
        hipLaunchKernelGGL((k_flow<false, true>), dim3(fblocks), dim3(kNTF), 0, s, params, x, n, z, lq, saved);
        hipLaunchKernelGGL(k_flow_backward, dim3(tiles), dim3(kNTF), 0, s, params, n, z, saved, partial);
    }
    hipLaunchKernelGGL(k_grad_reduce, dim3((kP + 255) / 256), dim3(256), 0, s, partial, tiles, grad);
    if (loss) hipLaunchKernelGGL(k_loss, dim3(1), dim3(256), 0, s, lq, n, loss);
    return hipGetLastError() == hipSuccess ? PD_OK : PD_EHIP;
}

int adam_step(float* params, const float* grad, float* m, float* v, int64_t count, double lr, double b1, double b2,
              double eps, int64_t t, hipStream_t s) {
    const float c1 = static_cast<float>(1.0 - std::pow(b1, static_cast<double>(t)));
    const float c2 = static_cast<float>(1.0 - std::pow(b2, static_cast<double>(t)));
    hipLaunchKernelGGL(k_adam, dim3(static_cast<unsigned>((count + 255) / 256)), dim3(256), 0, s, params, grad, m, v,
                       count, static_cast<float>(lr), static_cast<float>(b1), static_cast<float>(b2),
                       static_cast<float>(eps), c1, c2);
    return hipGetLastError() == hipSuccess ? PD_OK : PD_EHIP;
}

}  // namespace pd
