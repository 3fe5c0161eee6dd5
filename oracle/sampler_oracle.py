"""Plain numpy samplers: the CPU oracle of the GPU sampler kernels.

TEST INFRASTRUCTURE ONLY: used by the tests (and nothing in the product path).

Sec. 3.3 of the paper samples the 7-parameter posterior with Hamiltonian Monte Carlo
(leapfrog, hand-tuned diagonal mass matrix, Metropolis accept).  Here:
  * coordinates: theta_i = lo_i + (hi_i - lo_i) sigmoid(x_i) for all seven parameters
    (Mc, q, chi1, chi2, D, tc, phic) under uniform priors; phic enters the strain as
    exp(2 i phic), so an interval of length pi is one whole period of the likelihood;
    log pi(x) = lnL(theta(x)) + log|d theta / d x|;
  * HMC (Neal 2011): p = sqrt(m) xi, H = -log pi(x) + p^2/(2m) summed, leapfrog with a half
    kick at each end, accept if log u < -(H_end - H_start); non-finite or |dH| > 1000 is
    rejected as divergent;
  * HMC with a dense metric: momenta p ~ N(0, M) with inverse mass matrix M^-1 = L L^T for a
    lower-triangular L, drawn as p = L^-T xi (a triangular solve), H = -log pi + p^T M^-1 p / 2,
    the drift x += eps M^-1 p (Neal 2011, Sec. 5.4.1: a mass matrix is a linear change of
    coordinates);
  * the two-detector posterior of the paper's injection: the network likelihood of
    network_oracle with (iota, psi, ra, dec) held fixed;
  * random-walk Metropolis-Hastings, the baseline Sec. 3.3 compares HMC with (Metropolis et al.
    1953): a Gaussian step x' = x + s xi, accepted with probability min(1, pi(x') / pi(x));
  * independence Metropolis-Hastings with a proposal density q:
    accept x' with probability min(1, pi(x') q(x) / (pi(x) q(x'))).
Pinned by tests/test_sampler_oracle.py (reversibility, O(eps^2) energy error, the log-Jacobian
against finite differences, recovery of a Gaussian target's moments, the closed-form stationary
acceptance rate of the random walk on a normal target).
"""
import math

import numpy as np

from . import network_oracle as N
from . import phenomd_oracle as O


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def transform(x, lo, hi):
    """x [7] -> (theta [7], dtheta/dx [7], log|dtheta/dx|, d log|dtheta/dx| / dx [7])."""
    x = np.asarray(x, dtype=np.float64)
    theta = x.copy()
    d = np.ones(7)
    dl = np.zeros(7)
    lj = 0.0
    for j in range(7):
        s = sigmoid(x[j])
        w = hi[j] - lo[j]
        theta[j] = lo[j] + w * s
        d[j] = w * s * (1.0 - s)
        lj += math.log(d[j])
        dl[j] = 1.0 - 2.0 * s
    return theta, d, lj, dl


def logp_gw(x, lam, grid, data, inv_psd, lo, hi, want_grad=True):
    theta, d, lj, dl = transform(x, lo, hi)
    if not O.domain_ok(theta, O.PARAM_MC_Q):
        return -np.inf, np.zeros(7)
    lnl = O.loglike(theta, O.PARAM_MC_Q, lam, grid, data, inv_psd)
    if not want_grad:
        return lnl + lj, None
    g = O.loglike_grad(theta, O.PARAM_MC_Q, lam, grid, data, inv_psd)
    return lnl + lj, g * d + dl


def logp_gw_network(x, lam, grid, dets, data, inv_psd, lo, hi, gmst, orient, want_grad=True):
    """The same posterior with the network likelihood over `dets`, the orientation and sky
    position held at `orient` = (iota, psi, ra, dec)."""
    theta, d, lj, dl = transform(x, lo, hi)
    if not O.domain_ok(theta, O.PARAM_MC_Q):
        return -np.inf, np.zeros(7)
    th11 = np.concatenate([theta, np.asarray(orient, dtype=np.float64)])
    lnl = N.loglike(th11, O.PARAM_MC_Q, lam, grid, dets, data, inv_psd, gmst)
    if not want_grad:
        return lnl + lj, None
    g = N.loglike_grad(th11, O.PARAM_MC_Q, lam, grid, dets, data, inv_psd, gmst)[:7]
    return lnl + lj, g * d + dl


def logp_gauss(x, mu, isig2):
    r = np.asarray(x) - mu
    return -0.5 * float(np.sum(r * r * isig2)), -r * isig2


def leapfrog(logp_fn, x, p, grad, n_steps, eps, mass):
    """n_steps leapfrog steps from (x, p) with gradient grad at x; returns (x, p, logp, grad)."""
    x = np.array(x, dtype=np.float64)
    p = np.array(p, dtype=np.float64) + 0.5 * eps * grad
    lp = None
    for step in range(n_steps):
        x = x + eps * p / mass
        lp, grad = logp_fn(x)
        w = eps if step + 1 < n_steps else 0.5 * eps
        p = p + w * grad
    return x, p, lp, grad


def hmc_step(logp_fn, x, lp, grad, xi, u, n_steps, eps, mass):
    """One HMC transition; returns (x, logp, grad, accepted (1/0/-1), dH)."""
    mass = np.asarray(mass, dtype=np.float64)
    p0 = np.sqrt(mass) * xi
    h0 = -lp + 0.5 * float(np.sum(p0 * p0 / mass))
    x1, p1, lp1, g1 = leapfrog(logp_fn, x, p0, grad, n_steps, eps, mass)
    h1 = -lp1 + 0.5 * float(np.sum(p1 * p1 / mass))
    dh = h1 - h0
    if not np.isfinite(dh) or abs(dh) > 1000.0:
        return x, lp, grad, -1, dh
    if math.log(u) < -dh:
        return x1, lp1, g1, 1, dh
    return x, lp, grad, 0, dh


def leapfrog_dense(logp_fn, x, p, grad, n_steps, eps, minv):
    """Leapfrog with inverse mass matrix minv [7][7]; returns (x, p, logp, grad)."""
    x = np.array(x, dtype=np.float64)
    p = np.array(p, dtype=np.float64) + 0.5 * eps * grad
    lp = None
    for step in range(n_steps):
        x = x + eps * (minv @ p)
        lp, grad = logp_fn(x)
        w = eps if step + 1 < n_steps else 0.5 * eps
        p = p + w * grad
    return x, p, lp, grad


def hmc_step_dense(logp_fn, x, lp, grad, xi, u, n_steps, eps, chol):
    """One HMC transition with inverse mass matrix L L^T (chol = L, lower triangular) and the
    momentum p = L^-T xi; returns (x, logp, grad, accepted (1/0/-1), dH)."""
    L = np.tril(np.asarray(chol, dtype=np.float64))
    minv = L @ L.T
    p0 = np.linalg.solve(L.T, np.asarray(xi, dtype=np.float64))
    h0 = -lp + 0.5 * float(p0 @ minv @ p0)
    x1, p1, lp1, g1 = leapfrog_dense(logp_fn, x, p0, grad, n_steps, eps, minv)
    h1 = -lp1 + 0.5 * float(p1 @ minv @ p1)
    dh = h1 - h0
    if not np.isfinite(dh) or abs(dh) > 1000.0:
        return x, lp, grad, -1, dh
    if math.log(u) < -dh:
        return x1, lp1, g1, 1, dh
    return x, lp, grad, 0, dh


def rwmh_step(logp_fn, x, lp, xi, u, scale):
    """One random-walk MH transition with step x' = x + scale * xi; returns (x, logp, accepted).
    logp_fn returns log pi at a point (a non-finite value rejects the proposal; a current
    state with non-finite log pi takes any finite proposal)."""
    xp = np.asarray(x, dtype=np.float64) + np.asarray(scale, dtype=np.float64) * np.asarray(xi, dtype=np.float64)
    lpp = logp_fn(xp)
    if np.isfinite(lpp) and (math.log(u) < lpp - lp or not np.isfinite(lp)):
        return xp, lpp, 1
    return np.array(x, dtype=np.float64), lp, 0


def rwmh_step_dense(logp_fn, x, lp, xi, u, chol):
    """Random-walk MH with a correlated Gaussian step x' = x + L xi (L = chol, lower
    triangular); returns (x, logp, accepted)."""
    L = np.tril(np.asarray(chol, dtype=np.float64))
    xp = np.asarray(x, dtype=np.float64) + L @ np.asarray(xi, dtype=np.float64)
    lpp = logp_fn(xp)
    if np.isfinite(lpp) and (math.log(u) < lpp - lp or not np.isfinite(lp)):
        return xp, lpp, 1
    return np.array(x, dtype=np.float64), lp, 0


def independence_mh(x, lp, lq, xp, lpp, lqp, u):
    """One independence-MH accept step; returns (x, logp, logq, accepted)."""
    la = (lpp - lp) + (lq - lqp)
    if np.isfinite(lpp) and np.isfinite(lqp) and (math.log(u) < la or not np.isfinite(lp)):
        return np.array(xp), lpp, lqp, 1
    return np.array(x), lp, lq, 0
