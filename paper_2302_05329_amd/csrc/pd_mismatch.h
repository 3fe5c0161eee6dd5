// Internal interface of the mismatch pipeline (Sec. 3.1): overlap series by FFT, maximum
// over lag and phase, adjoint of the mismatch w.r.t. the 209 fit coefficients.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "pd_bin.h"

namespace pd {

// Overlap lengths: N = 2^n bins, kFFTMinLog2 <= n <= kFFTMaxLog2, computed as an N1 x N2 four-step
// FFT with N1 = 2^ceil(n/2) columns of length N2 = 2^floor(n/2) (at most 256 x 256).
constexpr int kFFTMinLog2 = 6;
constexpr int kFFTMaxLog2 = 16;
constexpr int kSlotMM = 8;         // per-target scalars: A, B, |z|, zr, zi, lag, mismatch, pad

size_t mismatch_scratch_bytes(int64_t nt, int64_t nb);

hipError_t launch_mismatch(const double* recs, const double* fit_tans, int64_t nt, const GridArgs& g,
                           const double* tab, const double* targets, const double* inv_psd, void* scratch, double* mismatch,
                           double* dsum_dlambda, int32_t* lag, hipStream_t s);

hipError_t launch_lambda_update(double* lam, const double* dsum, const double* precond, double scale,
                                hipStream_t s);

}  // namespace pd
