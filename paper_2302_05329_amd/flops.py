"""Algorithmic FP64 work of the per-bin kernels, for roofline accounting.

A unit is one (point, active bin).  Its cost depends on the model region the bin falls
in (phase: inspiral / intermediate / merger-ringdown; amplitude likewise), so the work of
a batch is summed from per-point bin counts in each region.

Counting convention (stated once, used everywhere):
  * +, -, *, / and sqrt: 1 flop each; a fused multiply-add: 2 flops.
  * elementary functions are charged the flops of an FP64-accurate software evaluation
    (argument reduction + minimax polynomial by Horner's rule + reconstruction):
      exp 26, log 26, cbrt 26, atan 40, sin+cos of one argument 40.
  * comparisons, index arithmetic, loads and stores: 0.
The per-region figures below are those counts applied to the formulas the kernels
evaluate (the minimal form: each basis function value computed once).
"""
import numpy as np

T_EXP, T_LOG, T_CBRT, T_ATAN, T_SINCOS = 26, 26, 26, 40, 40

# value path ----------------------------------------------------------------------------
COMMON_VALUE = 2 + 1 + 2 + T_SINCOS + 2           # f_k, Mf, A = A0 pf Ahat, sincos, h
PHASE_VALUE = {
    1: 1 + T_CBRT + 1 + T_LOG + 1 + 8 + 12 + 3 + 2 + 4,        # v, 1/v, ln v, Horner x2, log terms, Mf^-7/6
    2: T_LOG + 1 + 2 + 6 + 1 + T_EXP,                            # ln f, 1/f, f^-3, 4 terms, exp(-7/6 ln f)
    3: 1 + 2 + 1 + 2 + T_ATAN + 3 + 8 + T_LOG + 1 + T_EXP,       # 1/f, f^3/4, u, atan, 1/(1+u^2), 5 terms
}
AMP_VALUE = {1: 18, 2: 8, 3: 7 + T_EXP}
LNL_EPILOGUE = 1 + 5 + 5                                          # w_k, (d|h), (h|h)
# gradient moments -----------------------------------------------------------------------
GRAD_COMMON = 2 + 8 + 1 + 5                                       # d - h, zr, zi, lnA0 moment, Mf moment
PHASE_GRAD = {1: 63, 2: 13, 3: 25}
AMP_GRAD = {1: 48, 2: 23, 3: 16}
# Fisher: per-bin tangents along the 4 intrinsic directions (the extrinsic ones are closed
# form: d ln A / d ln D constant, d Psi / d tc = 2 pi f, d Psi / d phic = -2), 10 intrinsic
# products and 15 weighted moments for the mixed and extrinsic entries ---------------------
FISHER_COMMON = 3 + 1 + 4 * 5 + 10 * 4 + 12 * 2 + 4               # W, W f, explicit-Mf terms, products, moments
PHASE_FISHER = {1: 8 + 4 * 26 + 26, 2: 4 * 8 + 5, 3: 2 + 4 * 14 + 8}
AMP_FISHER = {1: 1 + 9 + 4 * 20 + 18, 2: 1 + 4 + 4 * 10 + 8, 3: 5 + 4 * 8 + 2}
# mismatch adjoint: per-bin weights from the overlap (twiddle, R_k) + moments --------------
MM_ADJ_COMMON = 1 + T_SINCOS + 6 + 4 + 8 + 4 + GRAD_COMMON - 10


def per_bin_flops(mode, preg, areg):
    v = COMMON_VALUE + PHASE_VALUE[preg] + AMP_VALUE[areg]
    if mode == "waveform":
        return v
    if mode == "loglike":
        return v + LNL_EPILOGUE
    if mode == "loglike_grad":
        return v + LNL_EPILOGUE + GRAD_COMMON + PHASE_GRAD[preg] + AMP_GRAD[areg]
    if mode == "fisher":
        return v + FISHER_COMMON + PHASE_FISHER[preg] + AMP_FISHER[areg]
    if mode == "mismatch_adjoint":
        return v + MM_ADJ_COMMON + PHASE_GRAD[preg] + AMP_GRAD[areg]
    raise ValueError(mode)


def region_counts(trans, grid):
    """Active-bin counts per (phase region, amplitude region) for each point.

    trans: [n, 4] array of (Ms, Mf_phase_join2, Mf_amp_join2, valid);
    grid: (f0, df, n_bins, f_min, f_ref).  Returns dict {(preg, areg): counts[n]}.
    """
    f0, df, nb, fmin, _ = grid
    ms = trans[:, 0]
    valid = trans[:, 3] > 0

    def n_below(mf_edge):
        """number of bins k in [k_lo, nb) with Ms f_k < mf_edge"""
        k = np.ceil((mf_edge / ms - f0) / df)
        return np.clip(k, 0, nb)

    klo = np.clip(np.ceil((fmin - f0) / df), 0, nb)
    khi = np.clip(np.floor((0.2 / ms - f0) / df) + 1, 0, nb)
    edges_p = [0.018 * np.ones_like(ms), trans[:, 1]]
    edges_a = [0.014 * np.ones_like(ms), trans[:, 2]]

    def clamp(x):
        return np.clip(x, klo, np.maximum(klo, khi))

    pe = [klo, clamp(n_below(edges_p[0])), clamp(n_below(edges_p[1])), np.maximum(klo, khi)]
    ae = [klo, clamp(n_below(edges_a[0])), clamp(n_below(edges_a[1])), np.maximum(klo, khi)]
    out = {}
    for pr in (1, 2, 3):
        for ar in (1, 2, 3):
            lo = np.maximum(pe[pr - 1], ae[ar - 1])
            hi = np.minimum(pe[pr], ae[ar])
            out[(pr, ar)] = np.where(valid, np.maximum(hi - lo, 0), 0)
    return out


def batch_flops(mode, trans, grid):
    """(total algorithmic FP64 flops, active units) of one call over the batch."""
    counts = region_counts(np.asarray(trans), grid)
    total = 0.0
    units = 0.0
    for (pr, ar), c in counts.items():
        total += float(np.sum(c)) * per_bin_flops(mode, pr, ar)
        units += float(np.sum(c))
    return total, units
