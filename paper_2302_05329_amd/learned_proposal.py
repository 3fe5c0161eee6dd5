"""Learned-proposal sampling of one injection (Sec. 3.3 and its closing remark): plain HMC
against HMC interleaved with flow-proposal independence MH, compared by effective samples per
second, with the posterior moments of the two samplers checked against each other.

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
    states and the inverse of the ball's marginal variances (a first mass matrix)."""
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
    return x, 1.0 / np.diag(cov)


def _rand(gen, n):
    xi = torch.randn((n, 7), dtype=torch.float64, device="cuda", generator=gen)
    u = torch.rand(n, dtype=torch.float64, device="cuda", generator=gen)
    return xi, u


def warmup(post, x0, gen, steps=300, n_leapfrog=10, eps0=0.05, target_acc=0.75, mass0=None, log=None):
    """Ensemble warm-up: chains start around x0; every 50 steps the diagonal mass matrix is set
    to the inverse variance across chains, and the shared step size follows the acceptance rate
    towards target_acc.  Returns the HMC object (chains at the end), eps, mass."""
    x0 = torch.as_tensor(x0, device="cuda")
    mass = np.ones(7) if mass0 is None else np.asarray(mass0, dtype=np.float64)
    eps = eps0
    hmc = sampling.HMC(post, x0, eps, n_leapfrog, mass)
    for t in range(steps):
        xi, u = _rand(gen, hmc.n)
        acc = float((hmc.step(xi, u) == 1).double().mean())
        eps *= math.exp(0.5 * (acc - target_acc))
        hmc.eps = eps
        if (t + 1) % 50 == 0 and t + 1 < steps:
            var = hmc.x.var(dim=0).cpu().numpy()
            mass = 1.0 / np.maximum(var, 1e-12)
            x, lp, g = hmc.x, hmc.logp, hmc.grad
            hmc = sampling.HMC(post, x, eps, n_leapfrog, mass)
            if log:
                log(f"warmup {t + 1}: acc {acc:.2f} eps {eps:.3g}")
    return hmc, eps, mass


def _record(post, hmc_x, out):
    out.append(post.to_theta(hmc_x.cpu().numpy()))


def run_hmc(hmc, gen, steps):
    """Plain HMC: returns (draws [chains, steps, 7] in theta, seconds, acceptance)."""
    draws = []
    acc = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    states = []
    for _ in range(steps):
        xi, u = _rand(gen, hmc.n)
        acc += (hmc.step(xi, u) == 1).double().mean()
        states.append(hmc.x.clone())
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    for s in states:
        _record(hmc.post, s, draws)
    return np.stack(draws, axis=1), sec, float(acc) / steps


def run_flow_hmc(hmc, fl, gen, steps):
    """HMC step then flow-proposal MH step, `steps` times: (draws, seconds, HMC acc, MH acc)."""
    fh = flow.FlowHMC(hmc, fl)
    draws = []
    acc_h = 0.0
    acc_m = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    states = []
    for _ in range(steps):
        xi, u = _rand(gen, hmc.n)
        acc_h += (fh.hmc_step(xi, u) == 1).double().mean()
        z, u2 = _rand(gen, hmc.n)
        acc_m += (fh.mh_step(z, u2) == 1).double().mean()
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


def flow_burn_in(hmc, gen, rounds=4, per_round=50, first_steps=1500, later_steps=500, log=None, mode="bf16"):
    """Training phase: alternate `per_round` transitions (HMC, plus flow MH once a flow exists)
    with refitting the flow on the states of the last two rounds.  Returns (flow, seconds)."""
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


def min_ess(draws):
    """Minimum over the 7 parameters of the bulk ESS of draws [chains, steps, 7]."""
    return min(diagnostics.ess(draws[:, :, j]) for j in range(draws.shape[2]))


def compare(lam, n_chains=4096, warm=300, steps=300, n_leapfrog=10, rounds=6, per_round=50, seed=1005,
            n_bins=None, log=None, flow_mode="bf16", two_site=False):
    """The full comparison; returns a dict of rates, acceptance and moment agreement.

    Chains start in a Fisher-scaled ball around the injection and are warmed up by HMC (mass
    matrix and step size adapted); a training phase then refits the flow on the chains' states while
    flow MH helps them mix.  Production starts both samplers from the same states at the end
    of that phase, with the flow frozen, so both are exact MCMC from the same start."""
    pb = gw_network_problem(lam, n_bins=n_bins) if two_site else gw_problem(lam, n_bins=n_bins)
    post = pb["post"]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    rng = np.random.default_rng(seed)
    th0 = pb["theta_inj"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x0, mass0 = fisher_ball(pb, n_chains, rng)
    hmc, eps, mass = warmup(post, x0, gen, steps=warm, n_leapfrog=n_leapfrog, mass0=mass0, log=log)
    fl, t_train = flow_burn_in(hmc, gen, rounds=rounds, per_round=per_round, log=log, mode=flow_mode)
    t_warm = time.perf_counter() - t0 - t_train
    x_start = hmc.x.clone()
    hmc_a = sampling.HMC(post, x_start, eps, n_leapfrog, mass)
    da, ta, acc_a = run_hmc(hmc_a, gen, steps)
    hmc_b = sampling.HMC(post, x_start, eps, n_leapfrog, mass)
    db, tb, acc_bh, acc_bm = run_flow_hmc(hmc_b, fl, gen, steps)
    ess_a, ess_b = min_ess(da), min_ess(db)
    ma, sa = da.reshape(-1, 7).mean(axis=0), da.reshape(-1, 7).std(axis=0)
    mb, sb = db.reshape(-1, 7).mean(axis=0), db.reshape(-1, 7).std(axis=0)
    return dict(
        n_chains=n_chains, steps=steps, n_leapfrog=n_leapfrog, eps=eps, n_bins=pb["grid"].n_bins, flow_mode=flow_mode,
        warmup_seconds=t_warm,
        hmc=dict(ess=ess_a, seconds=ta, ess_per_s=ess_a / ta, acceptance=acc_a),
        flow_hmc=dict(ess=ess_b, seconds=tb, ess_per_s=ess_b / tb, ess_per_s_incl_training=ess_b / (tb + t_train),
                      acceptance_hmc=acc_bh, acceptance_flow=acc_bm, training_phase_seconds=t_train),
        mean_diff_sigma=(np.abs(ma - mb) / sa).tolist(), std_diff_sigma=(np.abs(sa - sb) / sa).tolist(),
        theta_inj=th0.tolist(), mean=ma.tolist(), std=sa.tolist())


def two_site_hmc(lam, n_chains=4096, warm=300, steps=300, n_leapfrog=10, seed=1105, log=None):
    """HMC on the paper's two-detector posterior (H1 and L1, orientation and sky position fixed):
    warm-up as for the one-detector workload, then `steps` transitions from the warmed-up states.
    Returns time per transition, acceptance, the bulk ESS (chain-count floor for runs this short)
    and the autocorrelation-time estimate of ESS per second (tau ~ l / (1 - rho(l)), l = 100)."""
    from . import rwmh_baseline as RB
    pb = gw_network_problem(lam)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    rng = np.random.default_rng(seed)
    x0, mass0 = fisher_ball(pb, n_chains, rng)
    hmc, eps, mass = warmup(pb["post"], x0, gen, steps=warm, n_leapfrog=n_leapfrog, mass0=mass0, log=log)
    run = sampling.HMC(pb["post"], hmc.x.clone(), eps, n_leapfrog, mass)
    draws, sec, acc = RB._run(run, gen, steps, 512)
    ac = RB.mean_autocorr(draws)
    tau = RB.TAU_LAG / (1.0 - ac[RB.LAGS.index(RB.TAU_LAG)])
    return dict(n_chains=n_chains, steps=steps, n_leapfrog=n_leapfrog, eps=eps, ms_per_step=1e3 * sec / steps,
                acceptance=acc, min_bulk_ess_512=min_ess(draws), tau_steps=tau.tolist(),
                min_ess_per_s_tau=float(np.min(n_chains / tau / (sec / steps))), snr=20.0,
                n_bins=pb["grid"].n_bins, sites=2)
