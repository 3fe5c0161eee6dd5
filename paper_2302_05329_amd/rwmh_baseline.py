"""HMC against the random-walk Metropolis-Hastings baseline on one injection (Sec. 3.3, Fig. 6):
autocorrelation as a function of lag and effective sample size per parameter.

The paper runs HMC for 2e5 steps and the random walk for 7.5 times as many (1.5e6), both
hand-tuned, and finds the HMC effective sample size 2-7 times larger per parameter.  Here both
samplers start from the same warmed-up states of the learned-proposal workload (4096 chains,
8033 bins) with the same preconditioning: HMC's dense metric is the chains' covariance after
warm-up, and the random walk's Gaussian steps have that covariance times one factor, tuned on the
ensemble towards the acceptance rate 0.234 (the optimal-scaling result of Roberts, Gelman and
Gilks 1997).

Both move diffusively on this posterior, so each one's autocorrelation time (a property of one
chain) is measured on a long run of a subset of the chains, many autocorrelation times long, from
the bulk ESS of within-chain autocorrelation (rank-normalised split chains, Geyer truncation);
the times per transition are measured on all 4096 chains.  The effective samples at the paper's
step counts and at equal time follow from these.  ESS and autocorrelation are taken over the
summary features (phic through cos 2 phic and sin 2 phic).  The autocorrelation at a few lags
(ensemble-standardised, after burn-in) gives the shape of Fig. 6.

Every transition runs in the HIP library; this module draws random numbers on the device,
schedules the calls and copies chain states to the host for the diagnostics.
"""
import math
import time

import numpy as np
import torch

from . import diagnostics, sampling
from . import learned_proposal as LP

LAGS = (1, 2, 4, 8, 16, 32, 64, 128)   # in stored draws
PAPER_STEPS = (2e5, 1.5e6)


def _run(sampler, gen, steps, record, thin=1):
    """`steps` transitions of an HMC or RWMH ensemble; returns (draws [record, steps / thin, 7] in
    theta of the first `record` chains, every `thin`-th state, seconds, acceptance)."""
    acc = 0.0
    states = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(steps):
        xi, u = LP._rand(gen, sampler.n)
        acc += (sampler.step(xi, u) == 1).double().mean()
        if (t + 1) % thin == 0:
            states.append(sampler.x[:record].clone())
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    draws = np.stack([sampler.post.to_theta(s.cpu().numpy()) for s in states], axis=1)
    return draws, sec, float(acc) / steps


def tune_scale(post, x, chol, gen, steps=200, target=0.234):
    """Random-walk step factor f (steps f L xi, L the metric's Cholesky factor) adapted on the
    ensemble towards `target` acceptance; the chains' states after tuning are discarded."""
    f = 2.38 / math.sqrt(7.0)
    rw = sampling.RWMH(post, x, chol=f * chol)
    for _ in range(steps):
        xi, u = LP._rand(gen, rw.n)
        acc = float((rw.step(xi, u) == 1).double().mean())
        f *= math.exp(acc - target)
        rw.set_step(chol=f * chol)
    return f


def mean_autocorr(draws, lags=LAGS):
    """Autocorrelation at `lags` (in stored draws) per summary feature, [len(lags)][8]: products
    of lagged features averaged over chains and time, standardised with the mean and variance of
    all draws (the chains are stationary after burn-in, so one ensemble mean serves every chain)."""
    f = LP.features(draws)
    z = (f - f.mean(axis=(0, 1))) / f.std(axis=(0, 1))
    out = np.full((len(lags), z.shape[2]), np.nan)
    for k, lag in enumerate(lags):
        if lag < draws.shape[1]:
            out[k] = np.mean(z[:, :-lag] * z[:, lag:], axis=(0, 1))
    return out


def tuned_hmc(post, x_start, chol, eps0, gen, n_leapfrog, n_run, burn, steps, thin, log=None):
    """HMC with longer trajectories (n_leapfrog steps, the step size re-tuned towards acceptance
    0.7 on the ensemble): autocorrelation times from a long run of the first n_run chains, and the
    time per transition of the full ensemble.  Returns (tau [8], seconds per transition,
    acceptance, eps)."""
    h = sampling.HMC(post, x_start.clone(), eps0, n_leapfrog, chol=chol)
    eps = eps0
    for _ in range(100):
        xi, u = LP._rand(gen, h.n)
        acc = float((h.step(xi, u) == 1).double().mean())
        eps *= math.exp(0.5 * (acc - 0.7))
        h.eps = eps
    t_step = LP.time_per_step(sampling.HMC(post, h.x.clone(), eps, n_leapfrog, chol=chol), gen, 5)
    r = sampling.HMC(post, h.x[:n_run].clone(), eps, n_leapfrog, chol=chol)
    _run(r, gen, burn, n_run, burn)
    d, _, acc = _run(r, gen, steps, n_run, thin)
    tau = n_run * steps / LP.ess_per_param(d)
    if log:
        log(f"HMC with {n_leapfrog} leapfrog steps: eps {eps:.3g}, tau {np.round(tau, 1)} transitions")
    return tau, t_step, acc, eps


def compare(lam, n_chains=4096, warm=600, n_leapfrog=10, n_rw=256, rw_burn=20000, rw_steps=200000, rw_thin=100,
            n_hmc=512, hmc_burn=4000, hmc_steps=20000, hmc_thin=10, hmc=None, long_leapfrog=100, long_run=512,
            long_burn=1000, long_steps=5000, long_thin=5, seed=1005, n_bins=None, log=None):
    """HMC against the random walk.  `hmc`, if given, is the "hmc" entry of
    learned_proposal.compare on the same workload (its autocorrelation times and time per
    transition); otherwise HMC's long run is made here.  Each long run discards its first
    `*_burn` transitions.  The paper hand-tunes the trajectory length; HMC with `long_leapfrog`
    leapfrog steps per transition (long_leapfrog=0 skips it) is compared too, at the paper's
    step counts and at equal time."""
    pb = LP.gw_problem(lam, n_bins=n_bins)
    post = pb["post"]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    rng = np.random.default_rng(seed)
    x0, cov0 = LP.fisher_ball(pb, n_chains, rng)
    hmc_w, eps, chol = LP.warmup(post, x0, gen, steps=warm, n_leapfrog=n_leapfrog, cov0=cov0, target_acc=0.65,
                                 log=log)
    x_start = hmc_w.x.clone()
    ac_a = None
    if hmc is None:
        t_hmc = LP.time_per_step(sampling.HMC(post, x_start, eps, n_leapfrog, chol=chol), gen, 20)
        ha = sampling.HMC(post, x_start[:n_hmc].clone(), eps, n_leapfrog, chol=chol)
        _run(ha, gen, hmc_burn, n_hmc, hmc_burn)
        da, _, acc_a = _run(ha, gen, hmc_steps, n_hmc, hmc_thin)
        tau_a = n_hmc * hmc_steps / LP.ess_per_param(da)
        ac_a = mean_autocorr(da)
        del da
    else:
        t_hmc = hmc["ms_per_step"] * 1e-3
        tau_a = np.asarray(hmc["tau_steps"])
        acc_a = hmc["acceptance"]
    long = None
    if long_leapfrog:
        tau_l, t_l, acc_l, eps_l = tuned_hmc(post, x_start, chol, eps, gen, long_leapfrog, long_run, long_burn,
                                             long_steps, long_thin, log=log)
        long = (tau_l, t_l, acc_l, eps_l)
    f = tune_scale(post, x_start, chol, gen)
    if log:
        log(f"random-walk step factor {f:.4g} x the metric")
    t_rw = LP.time_per_step(sampling.RWMH(post, x_start, chol=f * chol), gen, 100)
    rw = sampling.RWMH(post, x_start[:n_rw].clone(), chol=f * chol)
    _run(rw, gen, rw_burn, n_rw, rw_burn)
    db, tb, acc_b = _run(rw, gen, rw_steps, n_rw, rw_thin)
    ess_b = LP.ess_per_param(db)
    tau_b = n_rw * rw_steps / ess_b
    ac_b = mean_autocorr(db)
    del db
    out_long = None
    if long is not None:
        tau_l, t_l, acc_l, eps_l = long
        out_long = dict(n_leapfrog=long_leapfrog, eps=eps_l, acceptance=acc_l, s_per_step=t_l,
                        tau_steps=tau_l.tolist(), run=dict(chains=long_run, burn_in_steps=long_burn, steps=long_steps,
                                                           steps_over_tau=float(long_steps / tau_l.max())),
                        ess_per_s=(n_chains / tau_l / t_l).tolist(),
                        ess_ratio_paper_steps=((PAPER_STEPS[0] / tau_l) / (PAPER_STEPS[1] / tau_b)).tolist(),
                        ess_ratio_equal_time=((t_rw * tau_b) / (t_l * tau_l)).tolist())
    return dict(
        hmc_long=out_long,
        n_chains=n_chains, n_bins=pb["grid"].n_bins, n_leapfrog=n_leapfrog,
        hmc=dict(s_per_step=t_hmc, acceptance=acc_a, eps=eps, tau_steps=tau_a.tolist(),
                 ess_per_s=(n_chains / tau_a / t_hmc).tolist(),
                 autocorr=None if ac_a is None else ac_a.tolist()),
        rwmh=dict(chains=n_rw, burn_in_steps=rw_burn, steps=rw_steps, seconds=tb, s_per_step=t_rw, acceptance=acc_b,
                  step_factor=f, autocorr=ac_b.tolist(), ess=ess_b.tolist(), tau_steps=tau_b.tolist(),
                  ess_per_s=(n_chains / tau_b / t_rw).tolist(), steps_over_tau=float(rw_steps / tau_b.max())),
        # effective samples of HMC over those of the random walk at the paper's step counts, and at equal time
        ess_ratio_paper_steps=((PAPER_STEPS[0] / tau_a) / (PAPER_STEPS[1] / tau_b)).tolist(),
        ess_ratio_equal_time=((t_rw * tau_b) / (t_hmc * tau_a)).tolist(),
        lags_rwmh_steps=[lag * rw_thin for lag in LAGS], features=list(LP.FEATURES),
        metric="dense (ensemble covariance), shared by both samplers")
