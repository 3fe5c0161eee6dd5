"""Sampler diagnostics: autocorrelation and effective sample size (paper Sec. 3.3, Fig. 6).

The paper reports ESS from arviz; this is an own implementation of the same estimator
family: rank-normalised split chains (Vehtari et al. 2021), autocorrelation by FFT,
Geyer's initial monotone sequence to truncate the sum of autocorrelations.
"""
import numpy as np
from scipy.special import ndtri
from scipy.stats import rankdata


def autocorr(x):
    """Normalised autocorrelation of a 1-D series at lags 0..n-1 (FFT, biased estimator)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    x = x - x.mean()
    m = 1 << int(np.ceil(np.log2(2 * n)))
    f = np.fft.rfft(x, m)
    ac = np.fft.irfft(f * np.conj(f), m)[:n]
    return ac / ac[0] if ac[0] > 0 else np.zeros(n)


def _ess_raw(chains):
    """ESS of draws [n_chains, n_draws] (no rank normalisation)."""
    chains = np.asarray(chains, dtype=np.float64)
    m, n = chains.shape
    if n < 4:
        return float(m * n)
    means = chains.mean(axis=1)
    var_within = chains.var(axis=1, ddof=1)
    w = var_within.mean()
    b_over_n = means.var(ddof=1) if m > 1 else 0.0
    var_plus = (n - 1) / n * w + b_over_n
    if var_plus <= 0:
        return float(m * n)
    acov = np.stack([autocorr(c) * v for c, v in zip(chains, chains.var(axis=1))])
    rho = 1.0 - (w - acov.mean(axis=0)) / var_plus
    rho[0] = 1.0
    # Geyer: sum of adjacent pairs while positive, forced monotone
    tau = -1.0
    prev = np.inf
    t = 0
    while t + 1 < n:
        pair = rho[t] + rho[t + 1]
        if pair <= 0:
            break
        pair = min(pair, prev)
        tau += 2.0 * pair
        prev = pair
        t += 2
    tau = max(tau, 1.0 / np.log10(max(m * n, 10)))
    return float(m * n / tau)


def ess(chains):
    """Bulk ESS of draws [n_chains, n_draws]: split chains, rank-normalise, Geyer truncation."""
    chains = np.asarray(chains, dtype=np.float64)
    m, n = chains.shape
    half = n // 2
    split = np.concatenate([chains[:, :half], chains[:, half:2 * half]], axis=0)
    r = rankdata(split, method="average").reshape(split.shape)
    z = ndtri((r - 0.375) / (split.size + 0.25))
    return _ess_raw(z)
