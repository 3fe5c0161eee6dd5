"""Pins of the sampler oracle and of the ESS estimator (CPU only)."""
import math

import numpy as np
import pytest

from oracle import sampler_oracle as S
from paper_2302_05329_amd import diagnostics as D


MU = np.array([0.3, -1.0, 2.0, 0.0, 0.5, -0.2, 1.1])
SIG = np.array([0.5, 1.0, 2.0, 0.1, 1.5, 0.7, 0.3])
ISIG2 = 1.0 / SIG**2


def gauss(x):
    return S.logp_gauss(x, MU, ISIG2)


def test_leapfrog_is_reversible():
    rng = np.random.default_rng(1)
    x0 = MU + SIG * rng.standard_normal(7)
    p0 = rng.standard_normal(7)
    mass = SIG**-2
    lp, g = gauss(x0)
    x1, p1, _, g1 = S.leapfrog(gauss, x0, p0, g, 20, 0.05, mass)
    x2, p2, _, _ = S.leapfrog(gauss, x1, -p1, g1, 20, 0.05, mass)
    assert np.max(np.abs(x2 - x0)) < 1e-12
    assert np.max(np.abs(p2 + p0)) < 1e-12


def test_energy_error_is_second_order():
    rng = np.random.default_rng(2)
    x0 = MU + SIG * rng.standard_normal(7)
    xi = rng.standard_normal(7)
    mass = np.ones(7)
    lp, g = gauss(x0)
    dhs = []
    for eps in (0.02, 0.01, 0.005):
        n = int(round(0.4 / eps))
        dhs.append(abs(S.hmc_step(gauss, x0, lp, g, xi, 0.999, n, eps, mass)[4]))
    r1, r2 = dhs[0] / dhs[1], dhs[1] / dhs[2]
    assert 3.5 < r1 < 4.5 and 3.5 < r2 < 4.5, dhs


def test_log_jacobian_against_finite_differences():
    lo = np.array([20.0, 0.125, -0.9, -0.9, 500.0, -0.1, -0.5 * np.pi])
    hi = np.array([40.0, 1.0, 0.9, 0.9, 7000.0, 0.1, 0.5 * np.pi])
    rng = np.random.default_rng(3)
    for _ in range(5):
        x = rng.normal(0, 1.5, 7)
        th, d, lj, dl = S.transform(x, lo, hi)
        for j in range(7):
            h = 1e-6
            xp, xm = x.copy(), x.copy()
            xp[j] += h
            xm[j] -= h
            fd = (S.transform(xp, lo, hi)[0][j] - S.transform(xm, lo, hi)[0][j]) / (2 * h)
            assert abs(fd - d[j]) < 1e-8 * max(1.0, abs(d[j]))
            fdl = (S.transform(xp, lo, hi)[2] - S.transform(xm, lo, hi)[2]) / (2 * h)
            assert abs(fdl - dl[j]) < 1e-7
        assert abs(lj - np.sum(np.log(d))) < 1e-12


def test_hmc_recovers_gaussian_target():
    rng = np.random.default_rng(4)
    n_chains, n_steps = 400, 60
    mass = ISIG2.copy()
    xs = MU + 3 * SIG * rng.standard_normal((n_chains, 7))
    lps, gs = zip(*[gauss(x) for x in xs])
    lps, gs = list(lps), list(gs)
    samples = []
    acc = 0
    for t in range(n_steps):
        for c in range(n_chains):
            xs[c], lps[c], gs[c], a, _ = S.hmc_step(gauss, xs[c], lps[c], gs[c], rng.standard_normal(7),
                                                   rng.uniform(), 8, 0.2, mass)
            acc += a == 1
        if t >= 20:
            samples.append(xs.copy())
    s = np.concatenate(samples)
    assert acc / (n_chains * n_steps) > 0.6
    # standard errors: draws are nearly independent for this tuning; allow 5 sigma
    se = SIG / np.sqrt(n_chains * 10)
    assert np.all(np.abs(s.mean(axis=0) - MU) < 5 * se)
    assert np.all(np.abs(s.std(axis=0) / SIG - 1) < 0.05)


def test_independence_mh_exactness_on_gaussian():
    """An independence proposal q = N(0, 2^2) for a N(0, 1) target keeps the target moments."""
    rng = np.random.default_rng(5)
    n = 20000
    x = rng.standard_normal(n) * 3.0
    lp = -0.5 * x**2
    lq = -0.5 * (x / 2.0) ** 2 - math.log(2.0)
    for _ in range(30):
        xp = 2.0 * rng.standard_normal(n)
        lpp = -0.5 * xp**2
        lqp = -0.5 * (xp / 2.0) ** 2 - math.log(2.0)
        u = rng.uniform(size=n)
        la = (lpp - lp) + (lq - lqp)
        acc = np.log(u) < la
        x = np.where(acc, xp, x)
        lp = np.where(acc, lpp, lp)
        lq = np.where(acc, lqp, lq)
    assert abs(x.mean()) < 0.05 and abs(x.std() - 1.0) < 0.03
    # the scalar oracle agrees with the vectorised rule above
    out = S.independence_mh(np.zeros(7), -1.0, -2.0, np.ones(7), -0.5, -3.0, 0.3)
    assert out[3] == 1


def test_rwmh_stationary_acceptance_matches_closed_form():
    """Random walk on a normal target N(mu, sig^2) with steps N(0, (s sig)^2), started in
    stationarity: the expected acceptance rate is (2/pi) arctan(2/s) (the one-dimensional
    result of Gelman, Roberts and Gilks 1996).  Only coordinate 0 moves (zero step elsewhere)."""
    rng = np.random.default_rng(8)
    mu = np.array([0.7, -0.3, 0.0, 1.0, 2.0, -1.0, 0.5])
    sig = np.array([1.3, 1.0, 0.5, 2.0, 1.0, 0.7, 1.0])
    isig2 = 1.0 / sig**2

    def lpf(x):
        return S.logp_gauss(x, mu, isig2)[0]

    n = 60000
    for s in (1.0, 2.4):
        scale = np.zeros(7)
        scale[0] = s * sig[0]
        x = mu + sig * rng.standard_normal((n, 7))
        xi = rng.standard_normal((n, 7))
        u = rng.uniform(size=n)
        acc = 0
        for i in range(n):
            xn, _, a = S.rwmh_step(lpf, x[i], lpf(x[i]), xi[i], u[i], scale)
            acc += a
            assert np.array_equal(xn[1:], x[i][1:])
        expect = 2.0 / math.pi * math.atan(2.0 / s)
        assert abs(acc / n - expect) < 0.01, (s, acc / n, expect)


def test_rwmh_keeps_gaussian_target():
    """From stationarity, 30 random-walk steps keep a 7-D normal target's mean and spread."""
    rng = np.random.default_rng(9)
    mu = np.array([0.3, -1.0, 2.0, 0.0, 0.5, -0.2, 1.1])
    sig = np.array([0.5, 1.0, 2.0, 0.1, 1.5, 0.7, 0.3])
    isig2 = 1.0 / sig**2

    def lpf(x):
        return S.logp_gauss(x, mu, isig2)[0]

    n = 2000
    x = mu + sig * rng.standard_normal((n, 7))
    lp = np.array([lpf(r) for r in x])
    for _ in range(30):
        xi = rng.standard_normal((n, 7))
        u = rng.uniform(size=n)
        for i in range(n):
            x[i], lp[i], _ = S.rwmh_step(lpf, x[i], lp[i], xi[i], u[i], 0.8 * sig)
    se = sig / math.sqrt(n)
    assert np.all(np.abs(x.mean(axis=0) - mu) < 5 * se)
    assert np.all(np.abs(x.std(axis=0) / sig - 1) < 0.08)


def test_rwmh_special_cases():
    def lpf(x):
        return S.logp_gauss(x, np.zeros(7), np.ones(7))[0]

    x = np.linspace(-1, 1, 7)
    # a zero step proposes the current point: log pi(x') - log pi(x) = 0 > log u always
    xn, lpn, a = S.rwmh_step(lpf, x, lpf(x), np.ones(7), 0.999, np.zeros(7))
    assert a == 1 and np.array_equal(xn, x) and lpn == lpf(x)
    # a proposal outside the support (log pi = -inf) is rejected, even for a tiny u
    xn, lpn, a = S.rwmh_step(lambda y: -np.inf, x, -1.0, np.ones(7), 1e-300, np.ones(7))
    assert a == 0 and np.array_equal(xn, x) and lpn == -1.0
    # a chain outside the support takes any finite proposal, even for u close to 1
    xn, lpn, a = S.rwmh_step(lpf, x, -np.inf, np.ones(7), 1 - 1e-16, np.full(7, 50.0))
    assert a == 1 and np.allclose(xn, x + 50.0)


def test_ess_of_ar1_matches_closed_form():
    """AR(1) with coefficient rho: ESS = N (1 - rho) / (1 + rho)."""
    rng = np.random.default_rng(6)
    for rho in (0.0, 0.5, 0.9):
        m, n = 8, 20000
        e = rng.standard_normal((m, n))
        x = np.zeros((m, n))
        x[:, 0] = e[:, 0] / math.sqrt(1 - rho**2)
        for t in range(1, n):
            x[:, t] = rho * x[:, t - 1] + e[:, t]
        expect = m * n * (1 - rho) / (1 + rho)
        got = D.ess(x)
        assert abs(got / expect - 1) < 0.12, (rho, got, expect)


def test_autocorr_of_white_noise():
    rng = np.random.default_rng(7)
    ac = D.autocorr(rng.standard_normal(100000))
    assert ac[0] == pytest.approx(1.0)
    assert np.max(np.abs(ac[1:50])) < 0.02


def test_ensemble_autocorr_of_ar1():
    """The lag autocorrelation reported for the HMC/random-walk comparison, on stationary AR(1)
    chains: rho^lag for the six non-periodic features (the phase enters through cos 2 phic and
    sin 2 phic, which are not AR(1))."""
    from paper_2302_05329_amd import rwmh_baseline as RB
    rng = np.random.default_rng(10)
    m, n, rho = 64, 4000, 0.9
    x = np.zeros((m, n, 7))
    x[:, 0] = rng.standard_normal((m, 7))
    for t in range(1, n):
        x[:, t] = rho * x[:, t - 1] + math.sqrt(1 - rho**2) * rng.standard_normal((m, 7))
    ac = RB.mean_autocorr(x)
    for k, lag in enumerate(RB.LAGS):
        assert np.all(np.abs(ac[k][:6] - rho**lag) < 0.02), (lag, ac[k])


def test_network_posterior_with_one_optimal_site_is_the_single_detector_posterior(lam0):
    """One site at the geocentre with the source overhead, face-on, F+ = 1 (fixed orientation):
    the network posterior and its gradient are the single-detector ones."""
    from paper_2302_05329_amd import workloads as W
    det = ((0.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0))
    grid = W.Grid(20.0, 0.25, 1001, 20.0, 20.0)
    g = grid.as_tuple()
    psd = W.psd_aligo_zdhp_fit(grid.freqs())
    data = W.complex_noise(psd, grid.df, 3)
    lo = np.array([10.0, 0.2, -0.9, -0.9, 100.0, -0.1, -1.6])
    hi = np.array([40.0, 1.0, 0.9, 0.9, 900.0, 0.1, 1.6])
    a = 0.8
    orient = (0.0, math.pi / 2 - a, a, math.pi / 2)
    x = np.array([0.1, -0.2, 0.3, 0.0, 0.5, -0.1, 0.2])
    lp1, g1 = S.logp_gw(x, lam0, g, data, 1 / psd, lo, hi)
    lpn, gn = S.logp_gw_network(x, lam0, g, [det], data[None], (1 / psd)[None], lo, hi, 0.0, orient)
    assert lpn == pytest.approx(lp1, rel=1e-12)
    assert np.allclose(gn, g1, rtol=1e-9, atol=1e-9 * np.max(np.abs(g1)))


# ---------------------------------------------------------------------------------
# HMC with a dense metric
# ---------------------------------------------------------------------------------
def _corr_gauss(seed=3):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((7, 7))
    cov = A @ A.T / 7.0 + 0.05 * np.eye(7)
    mu = rng.standard_normal(7)
    prec = np.linalg.inv(cov)

    def lpf(x):
        r = np.asarray(x) - mu
        return -0.5 * float(r @ prec @ r), -(prec @ r)
    return mu, cov, lpf


def test_dense_hmc_with_diagonal_metric_is_the_diagonal_step():
    """L = diag(1/sqrt(m)) reproduces the diagonal-mass transition."""
    mu, cov, lpf = _corr_gauss()
    rng = np.random.default_rng(4)
    mass = rng.uniform(0.5, 3.0, 7)
    x = mu + rng.standard_normal(7)
    lp, g = lpf(x)
    xi = rng.standard_normal(7)
    a = S.hmc_step(lpf, x, lp, g, xi, 0.3, 7, 0.05, mass)
    b = S.hmc_step_dense(lpf, x, lp, g, xi, 0.3, 7, 0.05, np.diag(1.0 / np.sqrt(mass)))
    assert a[3] == b[3]
    assert np.max(np.abs(a[0] - b[0])) <= 1e-13 and abs(a[4] - b[4]) <= 1e-12


def test_dense_leapfrog_is_reversible_and_second_order():
    mu, cov, lpf = _corr_gauss()
    L = np.linalg.cholesky(cov)
    minv = L @ L.T
    rng = np.random.default_rng(5)
    x0 = mu + L @ rng.standard_normal(7)
    p0 = np.linalg.solve(L.T, rng.standard_normal(7))
    lp0, g0 = lpf(x0)
    x1, p1, lp1, g1 = S.leapfrog_dense(lpf, x0, p0, g0, 12, 0.1, minv)
    x2, p2, _, _ = S.leapfrog_dense(lpf, x1, -p1, g1, 12, 0.1, minv)
    assert np.max(np.abs(x2 - x0)) <= 1e-12 and np.max(np.abs(-p2 - p0)) <= 1e-12
    errs = []
    for eps in (0.2, 0.1, 0.05):
        n = int(round(1.2 / eps))
        x1, p1, lp1, _ = S.leapfrog_dense(lpf, x0, p0, g0, n, eps, minv)
        errs.append(abs((-lp1 + 0.5 * p1 @ minv @ p1) - (-lp0 + 0.5 * p0 @ minv @ p0)))
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0


def test_dense_hmc_with_exact_metric_solves_a_correlated_gaussian():
    """With M^-1 equal to the target covariance the dynamics is a rotation in whitened
    coordinates: a trajectory of length pi/2 moves to an independent draw (eps -> 0 limit), so
    chains recover the mean and covariance of a strongly correlated target quickly."""
    mu, cov, lpf = _corr_gauss()
    L = np.linalg.cholesky(cov)
    rng = np.random.default_rng(6)
    n_chain, steps = 200, 60
    xs = mu + (L @ rng.standard_normal((7, n_chain))).T
    draws = []
    for t in range(steps):
        for c in range(n_chain):
            lp, g = lpf(xs[c])
            xs[c], _, _, _, _ = S.hmc_step_dense(lpf, xs[c], lp, g, rng.standard_normal(7), rng.uniform(), 8,
                                                 math.pi / 16, L)
        if t >= 10:
            draws.append(xs.copy())
    d = np.concatenate(draws)
    se = np.sqrt(np.diag(cov) / len(d)) * 3.0    # draws are nearly independent
    assert np.all(np.abs(d.mean(axis=0) - mu) <= 6.0 * se)
    assert np.max(np.abs(np.cov(d.T) - cov)) <= 0.08 * np.max(np.abs(cov))


def test_psis_shape_matches_the_gaussian_tail_index():
    """Target N(0, 1), proposal N(0, s^2) with s < 1: the ratio w = p / q satisfies
    P(w > t) ~ t^(-1 / (1 - s^2)), so the generalised Pareto shape of its tail is k = 1 - s^2; with
    s > 1 the ratio is bounded (k <= 0)."""
    rng = np.random.default_rng(41)
    for s2, lo, hi in ((0.25, 0.62, 0.88), (0.5, 0.38, 0.62)):
        x = rng.normal(0.0, math.sqrt(s2), 200000)
        lw = -0.5 * x * x + 0.5 * x * x / s2
        _, k = D.psis(lw)
        assert lo < k < hi, (s2, k)
    x = rng.normal(0.0, 2.0, 200000)
    _, k = D.psis(-0.5 * x * x + 0.5 * x * x / 4.0)
    assert k < 0.2, k


def test_psis_self_normalised_moments_are_consistent():
    """Moments of N(1, 1) from a N(0, 1.5^2) proposal with smoothed weights: within a few standard
    errors of the exact ones; smoothing leaves light-tailed weights almost unchanged."""
    rng = np.random.default_rng(43)
    x = rng.normal(0.0, 1.5, 400000)
    lw = -0.5 * (x - 1.0) ** 2 + 0.5 * (x / 1.5) ** 2
    lws, k = D.psis(lw)
    w = np.exp(lws - lws.max())
    w /= w.sum()
    m = float(w @ x)
    v = float(w @ (x - m) ** 2)
    assert abs(m - 1.0) < 0.01 and abs(v - 1.0) < 0.02, (m, v, k)
    w0 = np.exp(lw - lw.max())
    w0 /= w0.sum()
    assert abs(float(w0 @ x) - m) < 1e-3


def test_gpd_fit_recovers_known_parameters():
    """Exceedances drawn from a generalised Pareto distribution by inversion: the fitted shape and
    scale are close to the generating ones (the prior pulls the shape towards 0.5 by 10 / (n + 10))."""
    rng = np.random.default_rng(44)
    for xi, sig in ((0.3, 2.0), (0.7, 0.5), (-0.2, 1.0)):
        y = D.gpd_quantile(rng.random(20000), xi, sig)
        xh, sh = D.gpd_fit(y)
        assert abs(xh - xi) < 0.05 and abs(sh / sig - 1.0) < 0.06, (xi, sig, xh, sh)
