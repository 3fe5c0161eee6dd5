"""Learned-proposal sampling of one injection (Sec. 3.3 and its closing remark): plain HMC
against HMC interleaved with flow-proposal independence MH, compared by effective samples per
second, with the posterior moments of both samplers checked against a long plain-HMC reference
run (plain HMC is the judge).

Both samplers use HMC with a dense metric: the inverse mass matrix is the chains' covariance in the
unconstrained coordinates, adapted during warm-up (the paper's HMC has a hand-tuned mass matrix).
On this posterior, a curved ridge in chirp mass, mass ratio and spins, no linear metric whitens
the target: the step size stays small and plain HMC moves diffusively, with autocorrelation times
of several hundred transitions.  The autocorrelation time is a property of one chain, so plain
HMC's is measured on a long run of a subset of the chains (the reference run, many times its
autocorrelation time), and its effective samples per second on the full ensemble follow as
n_chains / tau / (time per transition of the full ensemble).  Effective sample sizes are the bulk
ESS from within-chain autocorrelation (rank-normalised split chains, Geyer truncation).

Every transition, log-density, flow pass and training step runs in the HIP library; this
module only draws random numbers (torch generator on the device), schedules the calls and
copies chain states to the host for the ESS estimate.
"""
import math
import time

import numpy as np
import torch

from . import api, diagnostics, flow, sampling
from . import workloads as W

NAMES = ("Mc", "q", "chi1", "chi2", "D", "tc", "phic")


def gw_problem(lam, snr=20.0, n_bins=None):
    """The injection, data and priors of the learned-proposal workload, built on the GPU:
    the distance is set so that the optimal SNR sqrt((h|h)) is `snr` exactly."""
    cfg = W.config5()
    grid = cfg["grid"] if n_bins is None else W.Grid(cfg["grid"].f0, cfg["grid"].df, n_bins, cfg["grid"].f_min,
                                                     cfg["grid"].f_ref)
    psd = W.psd_aligo_zdhp_fit(grid.freqs())
    inv_psd = torch.as_tensor(1.0 / psd, device="cuda")
    inj = cfg["inj_unit_distance"].copy()
    zero = torch.zeros(grid.n_bins, dtype=torch.complex128, device="cuda")
    lnl, _, _ = api.loglike_and_grad(inj[None], api.PARAM_M1M2, grid, lam, zero, inv_psd, want_grad=False)
    hh_unit = -2.0 * float(lnl[0])
    inj[4] = math.sqrt(hh_unit) / snr
    h, _ = api.waveform_eval(inj[None], api.PARAM_M1M2, grid, lam)
    noise = torch.as_tensor(W.complex_noise(psd, grid.df, 1005), device="cuda")
    data = noise + h[0]
    theta = W.to_param(inj[None], api.PARAM_MC_Q)[0]
    lo = np.array([20.0, 0.125, -0.9, -0.9, 0.2 * inj[4], -0.1, -0.5 * math.pi])
    hi = np.array([40.0, 1.0, 0.9, 0.9, 3.0 * inj[4], 0.1, 0.5 * math.pi])
    post = sampling.Posterior(0, grid=grid, lam=lam, data=data, inv_psd=inv_psd, lo=lo, hi=hi)
    return dict(post=post, theta_inj=theta, grid=grid, lo=lo, hi=hi, d_inj=inj[4], inv_psd=inv_psd, lam=lam)


def gw_network_problem(lam, snr=20.0, dets=("H1", "L1"), orient=None, gmst=1.234, n_bins=None):
    """The paper's two-detector version of the injection (Sec. 3.3): the same source seen by the
    LIGO sites with inclination, polarisation and sky position fixed (each pi/3, as in the paper),
    the distance set for network SNR `snr`, independent noise per site.  Built on the GPU."""
    cfg = W.config5()
    grid = cfg["grid"] if n_bins is None else W.Grid(cfg["grid"].f0, cfg["grid"].df, n_bins, cfg["grid"].f_min,
                                                     cfg["grid"].f_ref)
    orient = np.full(4, math.pi / 3) if orient is None else np.asarray(orient, dtype=np.float64)
    geo = [W.DETECTORS[d] for d in dets]
    psd = W.psd_aligo_zdhp_fit(grid.freqs())
    inv_psd = torch.as_tensor(np.stack([1.0 / psd] * len(dets)), device="cuda")
    inj = cfg["inj_unit_distance"].copy()
    th11 = np.concatenate([inj, orient])[None]
    zero = torch.zeros((len(dets), grid.n_bins), dtype=torch.complex128, device="cuda")
    lnl, _, _ = api.network_loglike_and_grad(th11, api.PARAM_M1M2, grid, lam, geo, gmst, zero, inv_psd,
                                             want_grad=False)
    inj[4] = math.sqrt(-2.0 * float(lnl[0])) / snr
    th11 = np.concatenate([inj, orient])[None]
    # each site's noise-free strain is the model at the site's effective parameters
    # (the network call with zero data gives -(h|h)/2 only, so the strains are built per site)
    data = []
    for k, det in enumerate(geo):
        h = api.network_strain(th11, api.PARAM_M1M2, grid, lam, det, gmst)
        data.append(torch.as_tensor(W.complex_noise(psd, grid.df, 1105 + k), device="cuda") + h[0])
    data = torch.stack(data)
    theta = W.to_param(inj[None], api.PARAM_MC_Q)[0]
    lo = np.array([20.0, 0.125, -0.9, -0.9, 0.2 * inj[4], -0.1, -0.5 * math.pi])
    hi = np.array([40.0, 1.0, 0.9, 0.9, 3.0 * inj[4], 0.1, 0.5 * math.pi])
    post = sampling.Posterior(api.PD_TARGET_GW_NETWORK, grid=grid, lam=lam, data=data, inv_psd=inv_psd, lo=lo, hi=hi,
                              detectors=geo, gmst=gmst, orient=orient)
    return dict(post=post, theta_inj=theta, grid=grid, lo=lo, hi=hi, d_inj=inj[4], inv_psd=inv_psd, lam=lam,
                geometry=geo, gmst=gmst, orient=orient)


def fisher_ball(pb, n, rng, prior_precision=0.3):
    """Starting states: x ~ N(x_inj, (J F J + c I)^-1) in the unconstrained coordinates, with F
    the library's Fisher matrix at the injection, J = d theta / d x, and c a weak precision that
    keeps the ball inside the prior along directions the data do not constrain.  Returns the
    states and the ball's covariance (a first metric)."""
    post = pb["post"]
    th0 = pb["theta_inj"]
    if "geometry" in pb:
        # the sampled 7 parameters' block of the network Fisher matrix (orientation fixed)
        F, st = api.network_fisher(np.r_[th0, pb["orient"]][None], api.PARAM_MC_Q, pb["grid"], pb["lam"],
                                   pb["geometry"], pb["gmst"], pb["inv_psd"])
        F = F[0, :7, :7].cpu().numpy()
    else:
        F, st = api.fisher(th0[None], api.PARAM_MC_Q, pb["grid"], pb["lam"], pb["inv_psd"])
        F = F[0].cpu().numpy()
    s = (th0 - pb["lo"]) / (pb["hi"] - pb["lo"])
    J = (pb["hi"] - pb["lo"]) * s * (1.0 - s)
    Fx = J[:, None] * F * J[None, :] + prior_precision * np.eye(7)
    cov = np.linalg.inv(Fx)
    cov = 0.5 * (cov + cov.T)
    chol = np.linalg.cholesky(cov)
    x = post.to_x(th0) + rng.standard_normal((n, 7)) @ chol.T
    return x, cov


def _rand(gen, n):
    xi = torch.randn((n, 7), dtype=torch.float64, device="cuda", generator=gen)
    u = torch.rand(n, dtype=torch.float64, device="cuda", generator=gen)
    return xi, u


def ensemble_chol(x, jitter=1e-10):
    """Cholesky factor of the chains' covariance [7][7] (host), with a relative jitter on the
    diagonal."""
    c = np.cov(x.cpu().numpy().T)
    c = 0.5 * (c + c.T) + jitter * np.diag(np.diag(c))
    return np.linalg.cholesky(c)


# A chain whose log-density is this far below the ensemble median sits where the posterior has
# no mass (for 7 Gaussian coordinates -log p - min is chi2_7 / 2, which exceeds 25 with
# probability ~1e-8): during warm-up it is restarted from another chain's state.
STRAGGLER_DROP = 25.0


def reseed_stragglers(x, logp, gen, drop=STRAGGLER_DROP):
    """Copies of randomly chosen chains replace those with logp < median - drop (or NaN).
    Returns (new x, number replaced).  Warm-up only: this is not a Markov transition."""
    lp = logp.double()
    med = torch.nanmedian(lp)
    bad = ~(lp >= med - drop)
    nbad = int(bad.sum())
    if nbad == 0:
        return x, 0
    good = torch.nonzero(~bad).flatten()
    pick = good[torch.randint(len(good), (nbad,), device=x.device, generator=gen)]
    x = x.clone()
    x[bad] = x[pick]
    return x, nbad


def warmup(post, x0, gen, steps=300, n_leapfrog=10, eps0=0.5, target_acc=0.8, cov0=None, log=None):
    """Ensemble warm-up with a dense metric: chains start around x0; every 50 steps chains stuck
    where the posterior has no mass are restarted from other chains (reseed_stragglers), the
    inverse mass matrix is set to the covariance across chains (its Cholesky factor is the
    metric), and the shared step size follows the acceptance rate towards target_acc.  Returns the
    HMC object (chains at the end), eps and the metric's Cholesky factor."""
    x0 = torch.as_tensor(x0, device="cuda")
    chol = np.linalg.cholesky(cov0) if cov0 is not None else ensemble_chol(x0)
    eps = eps0
    hmc = sampling.HMC(post, x0, eps, n_leapfrog, chol=chol)
    for t in range(steps):
        xi, u = _rand(gen, hmc.n)
        acc = float((hmc.step(xi, u) == 1).double().mean())
        eps *= math.exp(0.5 * (acc - target_acc))
        hmc.eps = eps
        if (t + 1) % 50 == 0 and t + 1 < steps:
            x, nbad = reseed_stragglers(hmc.x, hmc.logp, gen)
            chol = ensemble_chol(x)
            hmc = sampling.HMC(post, x, eps, n_leapfrog, chol=chol)
            if log:
                log(f"warmup {t + 1}: acc {acc:.2f} eps {eps:.3g} restarted {nbad}")
    return hmc, eps, chol


def _record(post, hmc_x, out):
    out.append(post.to_theta(hmc_x.cpu().numpy()))


def run_hmc(hmc, gen, steps, thin=1):
    """Plain HMC: returns (draws [chains, steps / thin, 7] in theta, every `thin`-th state, seconds,
    acceptance)."""
    draws = []
    acc = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    states = []
    for t in range(steps):
        xi, u = _rand(gen, hmc.n)
        acc += (hmc.step(xi, u) == 1).double().mean()
        if (t + 1) % thin == 0:
            states.append(hmc.x.clone())
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    for s in states:
        _record(hmc.post, s, draws)
    return np.stack(draws, axis=1), sec, float(acc) / steps


def run_flow_hmc(hmc, fl, gen, steps, thin=1):
    """HMC step then flow-proposal MH step, `steps` times: (draws, seconds, HMC acc, MH acc)."""
    fh = flow.FlowHMC(hmc, fl)
    draws = []
    acc_h = 0.0
    acc_m = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    states = []
    for t in range(steps):
        xi, u = _rand(gen, hmc.n)
        acc_h += (fh.hmc_step(xi, u) == 1).double().mean()
        z, u2 = _rand(gen, hmc.n)
        acc_m += (fh.mh_step(z, u2) == 1).double().mean()
        if (t + 1) % thin == 0:
            states.append(hmc.x.clone())
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    for s in states:
        _record(hmc.post, s, draws)
    return np.stack(draws, axis=1), sec, float(acc_h) / steps, float(acc_m) / steps


def train_flow(samples_x, gen, steps=1500, batch=4096, lr=1e-3, seed=1005, fl=None, mode="bf16"):
    """Fit a flow to unconstrained chain states [m, 7] (device), starting from `fl` if given
    (its standardisation is kept) or from a fresh identity flow standardised on the samples;
    returns (flow, seconds, losses)."""
    if fl is None:
        mu, sd = flow.standardisation(samples_x)
        fl = flow.Flow(W.flow_init_params(seed, mu=mu, sd=sd), mode=mode)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = fl.fit(samples_x, steps, batch, lr, gen, log_every=max(1, steps // 10))
    torch.cuda.synchronize()
    return fl, time.perf_counter() - t0, losses


def flow_burn_in(hmc, gen, rounds=4, per_round=50, first_steps=1500, later_steps=500, log=None, mode="bf16",
                 keep=None):
    """Training phase: alternate `per_round` transitions (HMC, plus flow MH once a flow exists)
    with refitting the flow on the states of the last two rounds.  With `keep` given, its chains are
    the ones advanced (`hmc` is then unused).  Returns (flow, seconds)."""
    if keep is not None:
        hmc = keep
    fl = None
    pool = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(rounds):
        fh = flow.FlowHMC(hmc, fl) if fl is not None else None
        states = []
        acc_m = 0.0
        for _ in range(per_round):
            xi, u = _rand(gen, hmc.n)
            hmc.step(xi, u)
            if fh is not None:
                fh.lq = None
                z, u2 = _rand(gen, hmc.n)
                acc_m += (fh.mh_step(z, u2) == 1).double().mean()
            states.append(hmc.x.clone())
        pool = pool[-1:] + [torch.cat(states)]
        fl, _, losses = train_flow(torch.cat(pool), gen, steps=first_steps if fl is None else later_steps, fl=fl,
                                   mode=mode)
        if log:
            log(f"burn-in round {r}: flow MH acceptance {float(acc_m) / per_round:.3f}, "
                f"loss {losses[0]:.3f} -> {losses[-1]:.3f}")
    torch.cuda.synchronize()
    return fl, time.perf_counter() - t0


FEATURES = ("Mc", "q", "chi1", "chi2", "D", "tc", "cos2phic", "sin2phic")


def features(draws):
    """Draws [chains, steps, 7] in theta -> [chains, steps, 8]: the six non-periodic parameters,
    then cos 2 phic and sin 2 phic (the phase enters the strain as 2 phic, so it is periodic with
    period pi and is summarised by these two)."""
    ph = 2.0 * draws[:, :, 6]
    return np.concatenate([draws[:, :, :6], np.cos(ph)[:, :, None], np.sin(ph)[:, :, None]], axis=2)


def ess_per_param(draws):
    """Bulk ESS of each summary feature of draws [chains, steps, 7] (within-chain
    autocorrelation of all chains; rank-normalised split chains, Geyer truncation)."""
    f = features(draws)
    return np.array([diagnostics.ess(f[:, :, j]) for j in range(f.shape[2])])


def min_ess(draws):
    """Minimum over the summary features of the bulk ESS of draws [chains, steps, 7]."""
    return float(np.min(ess_per_param(draws)))


def _moments(draws):
    f = features(draws)
    d = f.reshape(-1, f.shape[2])
    return d.mean(axis=0), d.std(axis=0)


def time_per_step(sampler, gen, steps):
    """Seconds per transition of an HMC or random-walk ensemble (after one untimed step)."""
    xi, u = _rand(gen, sampler.n)
    sampler.step(xi, u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        xi, u = _rand(gen, sampler.n)
        sampler.step(xi, u)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def importance_check(post, fl, gen, center, n_draws=1 << 20, batch=32768, mix=(0.4, 0.4, 0.2), nu=3.0, scale=1.5,
                     seed=0):
    """Self-normalised importance sampling of the posterior with a defensive mixture proposal
    g = m_f q + m_k K + m_t t: q the trained flow; K a Gaussian kernel mixture centred on the states
    `center` [n, 7] (kernel covariance h^2 C, C their covariance, h = (4 / (d + 2))^(1 / (d + 4))
    n^(-1 / (d + 4)) with d = 7, the normal-reference bandwidth); t a multivariate Student-t (nu
    degrees of freedom) with their mean and `scale` times C.  x ~ g, weights pi(x) / g(x),
    Pareto-smoothed (diagnostics.psis) and normalised to sum one.  K covers the region the chains visit at its own local width (the flow can
    under-weight parts of it, e.g. near the spin prior edges where the likelihood flattens), and t
    keeps the weights bounded where the posterior's tails in the unconstrained coordinates are
    heavier than Gaussian (the logit Jacobian decays only exponentially).  Returns the weighted mean
    and standard deviation of each summary feature, their Monte Carlo standard errors (delta
    method, sqrt(sum w^2 (f - mean)^2) for a mean), Kish's effective sample size 1 / sum w^2 (smoothed
    and raw), the Pareto shape k_hat (reliable below 0.7) and the largest raw normalised weight.  The estimate is consistent for any proposal whose support covers pi
    and involves no Markov chain, so it checks the flow-MH chains' equilibrium independently of
    their accept/reject bookkeeping."""
    from scipy.special import gammaln
    c = np.asarray(center.cpu().numpy() if torch.is_tensor(center) else center, dtype=np.float64)
    nc = c.shape[0]
    mu = c.mean(axis=0)
    cov_l = np.linalg.cholesky(np.cov(c.T))
    lt_ = cov_l * scale
    lt_inv = np.linalg.inv(lt_)
    lt_norm = (gammaln((nu + 7) / 2) - gammaln(nu / 2) - 3.5 * math.log(nu * math.pi)
               - float(np.sum(np.log(np.diag(lt_)))))
    h = (4.0 / 9.0) ** (1.0 / 11.0) * nc ** (-1.0 / 11.0)
    lk = cov_l * h
    lk_inv = torch.as_tensor(np.linalg.inv(lk), device="cuda")
    ck = torch.as_tensor(c, device="cuda") @ lk_inv.T
    ck2 = (ck * ck).sum(dim=1)
    lk_norm = -math.log(nc) - 3.5 * math.log(2.0 * math.pi) - float(np.sum(np.log(np.diag(lk))))
    lmix = np.log(np.asarray(mix, dtype=np.float64))
    rng = np.random.default_rng(seed)
    lws, fs = [], []
    ws = sampling.Workspace()
    for _ in range(n_draws // batch):
        comp = rng.choice(3, size=batch, p=np.asarray(mix) / np.sum(mix))
        z = torch.randn((batch, 7), dtype=torch.float64, device="cuda", generator=gen)
        xf, _ = fl.sample(z)
        zk = rng.standard_normal((batch, 7))
        xk = c[rng.integers(0, nc, batch)] + zk @ lk.T
        zt = rng.standard_normal((batch, 7))
        xt = mu + (zt @ lt_.T) / np.sqrt(rng.chisquare(nu, batch) / nu)[:, None]
        xo = np.where((comp == 1)[:, None], xk, xt)
        x = torch.where(torch.as_tensor(comp == 0, device="cuda")[:, None], xf,
                        torch.as_tensor(xo, device="cuda")).contiguous()
        _, lqf = fl.forward(x, want_z=False)
        # kernel mixture density, in chunks of 4096 draws against all centres
        lkd = []
        for i0 in range(0, batch, 4096):
            y = x[i0:i0 + 4096] @ lk_inv.T
            d2 = ((y * y).sum(dim=1)[:, None] + ck2[None, :] - 2.0 * (y @ ck.T)).clamp_min(0.0)
            lkd.append(torch.logsumexp(-0.5 * d2, dim=1))
        lkd = torch.cat(lkd).cpu().numpy() + lk_norm
        xh = x.cpu().numpy()
        d = (xh - mu) @ lt_inv.T
        ltd = lt_norm - (nu + 7) / 2 * np.log1p(np.sum(d * d, axis=1) / nu)
        lg = np.logaddexp(np.logaddexp(lmix[0] + lqf.cpu().numpy(), lmix[1] + lkd), lmix[2] + ltd)
        lp, _ = sampling.logp(post, x, want_grad=False, ws=ws)
        lws.append(lp.cpu().numpy() - lg)
        fs.append(features(post.to_theta(xh)[:, None, :])[:, 0, :])
    lw = np.concatenate(lws)
    f = np.concatenate(fs)
    lw = np.where(np.isfinite(lw), lw, -np.inf)
    w_raw = np.exp(lw - lw.max())
    w_raw /= w_raw.sum()
    # Pareto-smoothed weights (diagnostics.psis): k_hat < 0.7 marks a reliable estimate
    lws, k_hat = diagnostics.psis(lw)
    w = np.exp(lws - lws.max())
    w /= w.sum()
    mean = w @ f
    var = w @ (f - mean) ** 2
    se_mean = np.sqrt((w ** 2) @ (f - mean) ** 2)
    return dict(draws=int(len(w)), mean=mean, std=np.sqrt(var), se_mean=se_mean, kish_ess=float(1.0 / np.sum(w ** 2)),
                kish_ess_raw=float(1.0 / np.sum(w_raw ** 2)), k_hat=float(k_hat), max_weight=float(w_raw.max()),
                proposal=(f"{mix[0]:g} flow + {mix[1]:g} Gaussian kernels on {nc} chain states (bandwidth {h:.3f} x "
                          f"their covariance) + {mix[2]:g} Student-t (nu {nu:g}, {scale:g} x their covariance)"))


def stationarity_check(post, x_flow, eps0, chol, gen, n_run=512, n_leapfrog=100, steps=3000, thin=5, log=None):
    """Plain HMC (dense metric, `n_leapfrog` steps per transition, step size re-tuned towards
    acceptance 0.7) started from the first `n_run` flow-MH end states.  HMC leaves the posterior
    invariant, so if those states are posterior draws the ensemble's moments stay where they are;
    a flow-MH bias would show as a drift towards the posterior.  Returns the moments of the whole
    run and of its two halves, the ESS and autocorrelation times."""
    h = sampling.HMC(post, x_flow[:n_run].clone(), eps0, n_leapfrog, chol=chol)
    eps = eps0
    for _ in range(60):
        xi, u = _rand(gen, h.n)
        acc = float((h.step(xi, u) == 1).double().mean())
        eps *= math.exp(0.5 * (acc - 0.7))
        h.eps = eps
    d, sec, acc = run_hmc(h, gen, steps, thin)
    m, s = _moments(d)
    half = d.shape[1] // 2
    m1, _ = _moments(d[:, :half])
    m2, _ = _moments(d[:, half:])
    ess = ess_per_param(d)
    if log:
        log(f"stationarity: plain HMC ({n_leapfrog} leapfrog steps) from flow-MH states, {n_run} x {steps}, "
            f"{sec:.1f} s")
    return dict(mean=m, std=s, mean1=m1, mean2=m2, ess=ess, tau=n_run * steps / ess, acceptance=acc, eps=eps)


def compare(lam, n_chains=4096, warm=600, n_ref=512, ref_burn=4000, ref_steps=20000, ref_thin=10, flow_steps=600,
            n_leapfrog=10, rounds=6, per_round=50, seed=1005, n_bins=None, log=None, flow_mode="bf16",
            two_site=False, stat_chains=512, stat_leapfrog=100, stat_steps=3000):
    """The full comparison; returns a dict of rates, acceptance, autocorrelation times and the
    agreement of the flow sampler's moments with the plain-HMC reference run.

    Chains start in a Fisher-scaled ball around the injection and are warmed up by HMC (dense
    metric and step size adapted, stragglers restarted).  Plain HMC: the first `n_ref` warmed-up
    chains run `ref_burn` further transitions (discarded), then `ref_steps` transitions with their
    own random numbers (draws kept every `ref_thin`); this run is the reference for the moments and
    gives HMC's autocorrelation times, and HMC's time per transition is measured on all
    `n_chains`, so its ESS per second is n_chains / tau / (seconds per transition).  Learned
    proposal: a training phase refits the flow on the chains' states while flow MH helps them mix,
    then production on all chains with the metric and the flow frozen (exact MCMC), many of its
    own autocorrelation times long.  ESS and moments are taken over the summary features."""
    pb = gw_network_problem(lam, n_bins=n_bins) if two_site else gw_problem(lam, n_bins=n_bins)
    post = pb["post"]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    rng = np.random.default_rng(seed)
    th0 = pb["theta_inj"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x0, cov0 = fisher_ball(pb, n_chains, rng)
    hmc, eps, chol = warmup(post, x0, gen, steps=warm, n_leapfrog=n_leapfrog, cov0=cov0, target_acc=0.65, log=log)
    t_warm = time.perf_counter() - t0
    x_warm = hmc.x.clone()
    # plain HMC: time per transition of the full ensemble, then the long reference run
    t_hmc = time_per_step(sampling.HMC(post, x_warm, eps, n_leapfrog, chol=chol), gen, 20)
    gen_ref = torch.Generator(device="cuda")
    gen_ref.manual_seed(seed + 7919)
    ref = sampling.HMC(post, x_warm[:n_ref].clone(), eps, n_leapfrog, chol=chol)
    _, t_burn, _ = run_hmc(ref, gen_ref, ref_burn, ref_burn)
    dr, tr, acc_r = run_hmc(ref, gen_ref, ref_steps, ref_thin)
    ess_r = ess_per_param(dr)
    mr, sr = _moments(dr)
    # the reference's drift: second-half minus first-half moments, in reference sigmas
    h = dr.shape[1] // 2
    m1, s1 = _moments(dr[:, :h])
    m2, s2 = _moments(dr[:, h:])
    del dr
    tau_r = n_ref * ref_steps / ess_r
    if log:
        log(f"reference: {n_ref} chains x ({ref_burn} + {ref_steps}) HMC steps, tau {np.round(tau_r, 1)} steps")
    ess_per_s_hmc = n_chains / tau_r / t_hmc
    fl, t_train = flow_burn_in(None, gen, rounds=rounds, per_round=per_round, log=log, mode=flow_mode, keep=hmc)
    x_start = hmc.x.clone()
    prod = sampling.HMC(post, x_start, eps, n_leapfrog, chol=chol)
    db, tb, acc_bh, acc_bm = run_flow_hmc(prod, fl, gen, flow_steps)
    ess_b = ess_per_param(db)
    mb, sb = _moments(db)
    del db
    tau_b = n_chains * flow_steps / ess_b
    isr = importance_check(post, fl, gen, x_start, seed=seed)
    # flow-MH mean minus importance-sampling mean, in combined Monte Carlo standard errors
    z_is = (mb - isr["mean"]) / np.sqrt(sb ** 2 / ess_b + isr["se_mean"] ** 2)
    st = stationarity_check(post, prod.x, eps, chol, gen, n_run=stat_chains, n_leapfrog=stat_leapfrog,
                            steps=stat_steps, log=log)
    return dict(
        n_chains=n_chains, warm=warm, n_ref=n_ref, ref_burn=ref_burn, ref_steps=ref_steps, ref_thin=ref_thin,
        flow_steps=flow_steps, n_leapfrog=n_leapfrog, eps=eps, n_bins=pb["grid"].n_bins, flow_mode=flow_mode,
        warmup_seconds=t_warm, metric="dense (ensemble covariance)", features=list(FEATURES),
        hmc=dict(tau_steps=tau_r.tolist(), ms_per_step=1e3 * t_hmc, ess_per_s_per_param=ess_per_s_hmc.tolist(),
                 ess_per_s=float(ess_per_s_hmc.min()), acceptance=acc_r),
        flow_hmc=dict(ess=float(ess_b.min()), ess_per_param=ess_b.tolist(), tau_steps=tau_b.tolist(), seconds=tb,
                      ms_per_step=1e3 * tb / flow_steps, ess_per_s=float(ess_b.min()) / tb,
                      ess_per_s_incl_training=float(ess_b.min()) / (tb + t_train), acceptance_hmc=acc_bh,
                      acceptance_flow=acc_bm, training_phase_seconds=t_train,
                      steps_over_tau=float(flow_steps / tau_b.max())),
        reference=dict(chains=n_ref, burn_in_steps=ref_burn, steps=ref_steps, seconds=tr + t_burn, acceptance=acc_r,
                       ess=float(ess_r.min()), ess_per_param=ess_r.tolist(), tau_steps=tau_r.tolist(),
                       steps_over_tau=float(ref_steps / tau_r.max()), mean=mr.tolist(), std=sr.tolist(),
                       drift_mean_sigma=((m2 - m1) / sr).tolist(), drift_std_rel=((s2 - s1) / sr).tolist()),
        # agreement of the learned-proposal sampler with the reference, in units of the reference sigma
        mean_diff_sigma_flow=(np.abs(mb - mr) / sr).tolist(), std_diff_sigma_flow=(np.abs(sb - sr) / sr).tolist(),
        mean_flow=mb.tolist(), std_flow=sb.tolist(), theta_inj=th0.tolist(),
        stationarity=dict(chains=stat_chains, n_leapfrog=stat_leapfrog, steps=stat_steps, eps=st["eps"],
                          acceptance=st["acceptance"], tau_steps=st["tau"].tolist(),
                          mean_diff_sigma=((st["mean"] - mb) / sb).tolist(),
                          std_diff_rel=((st["std"] - sb) / sb).tolist(),
                          drift_mean_sigma=((st["mean2"] - st["mean1"]) / sb).tolist(),
                          se_sigma=(1.0 / np.sqrt(st["ess"])).tolist(),
                          # relative standard error of the difference of the two standard deviations
                          # (a Gaussian marginal's sample std has relative variance 1 / (2 ESS))
                          se_std_rel=np.sqrt(0.5 / st["ess"] + 0.5 / ess_b).tolist()),
        importance=dict(draws=isr["draws"], kish_ess=isr["kish_ess"], kish_ess_raw=isr["kish_ess_raw"],
                        k_hat=isr["k_hat"], max_weight=isr["max_weight"],
                        proposal=isr["proposal"],
                        mean=isr["mean"].tolist(), std=isr["std"].tolist(), se_mean=isr["se_mean"].tolist(),
                        z_mean_flow_minus_is=z_is.tolist(),
                        mean_diff_sigma_flow=(np.abs(mb - isr["mean"]) / isr["std"]).tolist(),
                        std_diff_sigma_flow=(np.abs(sb - isr["std"]) / isr["std"]).tolist()))
