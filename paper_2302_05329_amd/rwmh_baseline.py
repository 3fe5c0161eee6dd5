"""HMC against the random-walk Metropolis-Hastings baseline on one injection (Sec. 3.3, Fig. 6):
autocorrelation as a function of lag and effective sample size per parameter.

The paper runs HMC for 2e5 steps and the random walk for 7.5 times as many (1.5e6), both
hand-tuned, and finds the HMC effective sample size 2-7 times larger per parameter.  Here both
samplers start from the same warmed-up states of the learned-proposal workload (4096 chains,
8033 bins, diagonal preconditioning for both) and the random walk takes the same 7.5-fold step
count.  Its Gaussian steps are the warm-up spread of each coordinate times one factor, tuned on
the ensemble towards the acceptance rate 0.234 (the optimal-scaling result of Roberts, Gelman and
Gilks 1997) before production.

The chains start in stationarity, so the autocorrelation at lag l is estimated from products of
lagged draws standardised with the ensemble mean and variance.  On this posterior both samplers
move diffusively along its narrow correlated ridge: over the run the autocorrelation stays close
to one and falls linearly with the lag, rho(l) ~ 1 - l / tau, which gives the integrated
autocorrelation time tau ~ l / (1 - rho(l)) (an estimate valid while l << tau) and from it the
effective samples per step 1 / tau.  The bulk ESS of so short a run would only count the chains.

Every transition runs in the HIP library; this module draws random numbers on the device,
schedules the calls and copies chain states to the host for the diagnostics.
"""
import math
import time

import numpy as np
import torch

from . import diagnostics, sampling
from . import learned_proposal as LP

LAGS = (1, 2, 5, 10, 20, 50, 100, 200)
TAU_LAG = 100
PAPER_STEPS = (2e5, 1.5e6)


def _run(sampler, gen, steps, record):
    """`steps` transitions of an HMC or RWMH ensemble; returns (draws [record, steps, 7] in theta of
    the first `record` chains, seconds, acceptance)."""
    acc = 0.0
    states = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        xi, u = LP._rand(gen, sampler.n)
        acc += (sampler.step(xi, u) == 1).double().mean()
        states.append(sampler.x[:record].clone())
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    draws = np.stack([sampler.post.to_theta(s.cpu().numpy()) for s in states], axis=1)
    return draws, sec, float(acc) / steps


def tune_scale(post, x, sd, gen, steps=200, target=0.234):
    """Random-walk step factor f (steps f * sd) adapted on the ensemble towards `target`
    acceptance; the chains' states after tuning are discarded."""
    f = 2.38 / math.sqrt(7.0)
    rw = sampling.RWMH(post, x, f * sd)
    for _ in range(steps):
        xi, u = LP._rand(gen, rw.n)
        acc = float((rw.step(xi, u) == 1).double().mean())
        f *= math.exp(acc - target)
        rw.scale = type(rw.scale)(*(f * sd).tolist())
    return f


def mean_autocorr(draws, lags=LAGS):
    """Autocorrelation at `lags` per parameter, [len(lags)][7]: products of lagged draws averaged
    over chains and time, standardised with the mean and variance of all draws (the chains are
    stationary from the start, so one ensemble mean serves every chain)."""
    z = (draws - draws.mean(axis=(0, 1))) / draws.std(axis=(0, 1))
    out = np.full((len(lags), draws.shape[2]), np.nan)
    for k, lag in enumerate(lags):
        if lag < draws.shape[1]:
            out[k] = np.mean(z[:, :-lag] * z[:, lag:], axis=(0, 1))
    return out


def compare(lam, n_chains=4096, warm=300, steps=500, rw_factor=7.5, n_leapfrog=10, record=512, seed=1005,
            n_bins=None, log=None):
    pb = LP.gw_problem(lam, n_bins=n_bins)
    post = pb["post"]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    rng = np.random.default_rng(seed)
    x0, mass0 = LP.fisher_ball(pb, n_chains, rng)
    hmc, eps, mass = LP.warmup(post, x0, gen, steps=warm, n_leapfrog=n_leapfrog, mass0=mass0, log=log)
    x_start = hmc.x.clone()
    sd = x_start.std(dim=0).cpu().numpy()
    f = tune_scale(post, x_start, sd, gen)
    if log:
        log(f"random-walk step factor {f:.4g} x warm-up spread")
    da, ta, acc_a = _run(sampling.HMC(post, x_start, eps, n_leapfrog, mass), gen, steps, record)
    rw_steps = int(round(rw_factor * steps))
    db, tb, acc_b = _run(sampling.RWMH(post, x_start, f * sd), gen, rw_steps, record)
    ac_a, ac_b = mean_autocorr(da), mean_autocorr(db)
    k = LAGS.index(TAU_LAG)
    tau_a = TAU_LAG / (1.0 - ac_a[k])
    tau_b = TAU_LAG / (1.0 - ac_b[k])
    sa, sb = ta / steps, tb / rw_steps
    return dict(
        n_chains=n_chains, chains_in_diagnostics=da.shape[0], n_bins=pb["grid"].n_bins, n_leapfrog=n_leapfrog,
        hmc=dict(steps=steps, seconds=ta, s_per_step=sa, acceptance=acc_a, eps=eps, autocorr=ac_a.tolist(),
                 tau_steps=tau_a.tolist(), ess_per_s=(n_chains / tau_a / sa).tolist()),
        rwmh=dict(steps=rw_steps, seconds=tb, s_per_step=sb, acceptance=acc_b, step_factor=f, autocorr=ac_b.tolist(),
                  tau_steps=tau_b.tolist(), ess_per_s=(n_chains / tau_b / sb).tolist()),
        # effective samples of HMC over those of the random walk at the paper's step counts, and at equal time
        ess_ratio_paper_steps=((PAPER_STEPS[0] / tau_a) / (PAPER_STEPS[1] / tau_b)).tolist(),
        ess_ratio_equal_time=((sb * tau_b) / (sa * tau_a)).tolist(),
        lags=list(LAGS), tau_lag=TAU_LAG, names=list(LP.NAMES))
