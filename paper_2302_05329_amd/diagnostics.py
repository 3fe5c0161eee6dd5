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


# ---- Pareto-smoothed importance weights ---------------------------------------------------------
# Vehtari, Simpson, Gelman, Yao and Gabry (2024), "Pareto smoothed importance sampling": the largest
# M = min(S / 5, 3 sqrt(S)) of S importance ratios are replaced by the expected order statistics of
# a generalised Pareto distribution fitted to their excess over the next-largest ratio, which bounds
# the variance the few largest ratios cause; the fitted shape k-hat is the reliability diagnostic
# (below 0.7 the self-normalised estimate is trustworthy, below 0.5 the raw one already has finite
# variance).  The shape and scale come from the profile-likelihood grid estimator of Zhang and
# Stephens (2009), written here for the distribution F(y) = 1 - (1 + xi y / sigma)^(-1 / xi).

def gpd_fit(y):
    """(xi, sigma) of a generalised Pareto fit to the excesses y > 0: with theta = xi / sigma, the
    likelihood for fixed theta is maximised at xi(theta) = mean log(1 + theta y), giving the profile
    log-likelihood n (log(theta / xi) - xi - 1); theta is its likelihood-weighted mean over the
    Zhang-Stephens grid, then xi is shrunk towards 0.5 by a weak prior worth 10 observations."""
    y = np.sort(np.asarray(y, dtype=np.float64))
    n = y.size
    m = 30 + int(np.sqrt(n))
    yq = y[max(int(n / 4 + 0.5) - 1, 0)]
    j = np.arange(1, m + 1, dtype=np.float64)
    theta = -1.0 / y[-1] + (np.sqrt(m / (j - 0.5)) - 1.0) / (3.0 * yq)
    xi = np.log1p(theta[:, None] * y[None, :]).mean(axis=1)
    prof = n * (np.log(theta / xi) - xi - 1.0)
    w = np.exp(prof - prof.max())
    w /= w.sum()
    th = float(np.sum(theta * w))
    xi_hat = float(np.log1p(th * y).mean())
    sigma = xi_hat / th
    xi_hat = (n * xi_hat + 10 * 0.5) / (n + 10)
    return xi_hat, sigma


def gpd_quantile(p, xi, sigma):
    """Inverse CDF of the generalised Pareto distribution."""
    p = np.asarray(p, dtype=np.float64)
    if abs(xi) < 1e-12:
        return -sigma * np.log1p(-p)
    return sigma * np.expm1(-xi * np.log1p(-p)) / xi


def psis(log_w):
    """Pareto-smoothed log weights and the shape diagnostic k-hat for log importance ratios log_w
    (any additive constant); non-finite entries get weight zero."""
    lw = np.asarray(log_w, dtype=np.float64).copy()
    ok = np.isfinite(lw)
    s = int(ok.sum())
    m = int(np.ceil(min(0.2 * s, 3.0 * np.sqrt(s))))
    if m < 5:
        return lw, float("nan")
    top = lw[ok].max()
    order = np.argsort(np.where(ok, lw, -np.inf))
    tail = order[-m:]
    cut = lw[order[-m - 1]]
    w_tail = np.exp(lw[tail] - top)
    u = np.exp(cut - top)
    xi, sigma = gpd_fit(w_tail - u)
    if np.isfinite(xi) and sigma > 0:
        smooth = u + gpd_quantile((np.arange(1, m + 1) - 0.5) / m, xi, sigma)
        lw[tail] = np.log(np.minimum(smooth, 1.0)) + top
    lw[~ok] = -np.inf
    return lw, xi
