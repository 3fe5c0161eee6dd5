"""GPU samplers against the numpy sampler oracle, and exactness on a Gaussian target."""
import math
import sys

import numpy as np
import pytest

from error_model import lnl_tolerance, network_lnl_tolerance
from oracle import phenomd_oracle as O
from oracle import sampler_oracle as S
from paper_2302_05329_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _c5_problem(lam, n_bins=8033):
    """The learned-proposal workload's injection (SNR 20 in one face-on detector) and priors,
    built with the oracle waveform."""
    cfg = W.config5()
    grid = W.Grid(20.0, 0.125, n_bins)
    g = grid.as_tuple()
    inj = cfg["inj_unit_distance"].copy()
    psd = W.psd_aligo_zdhp_fit(grid.freqs())
    h1 = O.waveform(inj, O.PARAM_M1M2, lam, g)
    snr1 = math.sqrt(O.inner(h1, h1, 1 / psd, g[1]))
    inj[4] = snr1 / 20.0
    data = W.complex_noise(psd, grid.df, 1005) + O.waveform(inj, O.PARAM_M1M2, lam, g)
    mc_q = W.to_param(inj[None, :], O.PARAM_MC_Q)[0]
    lo = np.array([20.0, 0.125, -0.9, -0.9, 0.2 * inj[4], -0.1, -0.5 * math.pi])
    hi = np.array([40.0, 1.0, 0.9, 0.9, 3.0 * inj[4], 0.1, 0.5 * math.pi])
    return dict(grid=grid, data=data, inv_psd=1 / psd, lo=lo, hi=hi, theta_inj=mc_q)


def _lp_tol(pb, lam, x, ref_lp):
    """log posterior = ln L(theta(x)) + log-Jacobian: the likelihood's rounding bound at theta(x)
    plus a few ulp of the sum."""
    th = S.transform(x, pb["lo"], pb["hi"])[0]
    return (lnl_tolerance(th, O.PARAM_MC_Q, lam, pb["grid"].as_tuple(), pb["data"], pb["inv_psd"])
            + 8.0 * np.spacing(abs(ref_lp) + 100.0))


def test_posterior_logp_parity_gw(gpu, lam0):
    import torch
    from paper_2302_05329_amd import sampling
    pb = _c5_problem(lam0)
    post = sampling.Posterior(0, grid=pb["grid"], lam=lam0, data=pb["data"], inv_psd=pb["inv_psd"], lo=pb["lo"],
                              hi=pb["hi"])
    rng = np.random.default_rng(11)
    x0 = post.to_x(pb["theta_inj"])
    xs = x0 + 0.05 * rng.standard_normal((12, 7))
    _say("posterior logp GW n=12")
    lp, g = sampling.logp(post, xs)
    torch.cuda.synchronize()
    lp, g = lp.cpu().numpy(), g.cpu().numpy()
    gr = pb["grid"].as_tuple()
    for i, x in enumerate(xs):
        ref_lp, ref_g = S.logp_gw(x, lam0, gr, pb["data"], pb["inv_psd"], pb["lo"], pb["hi"])
        assert abs(lp[i] - ref_lp) <= _lp_tol(pb, lam0, x, ref_lp), (lp[i], ref_lp)
        th, d, _, _ = S.transform(x, pb["lo"], pb["hi"])
        F = O.fisher(th, O.PARAM_MC_Q, lam0, gr, pb["inv_psd"])
        h = O.waveform(th, O.PARAM_MC_Q, lam0, gr)
        r = pb["data"] - h
        scale = np.sqrt(O.inner(r, r, pb["inv_psd"], gr[1]) * np.diag(F)) * d + 1.0
        assert np.all(np.abs(g[i] - ref_g) <= 1e-10 * scale), (g[i], ref_g)


def test_hmc_step_parity_gw(gpu, lam0):
    import torch
    from paper_2302_05329_amd import sampling
    pb = _c5_problem(lam0, n_bins=4001)
    post = sampling.Posterior(0, grid=pb["grid"], lam=lam0, data=pb["data"], inv_psd=pb["inv_psd"], lo=pb["lo"],
                              hi=pb["hi"])
    rng = np.random.default_rng(12)
    x0 = post.to_x(pb["theta_inj"]) + 0.02 * rng.standard_normal((6, 7))
    mass = np.array([400.0, 50.0, 20.0, 20.0, 10.0, 4e3, 4.0])
    eps, L = 0.02, 4
    xi = rng.standard_normal((6, 7))
    u = rng.uniform(size=6)
    _say("hmc step GW n=6 L=4")
    hmc = sampling.HMC(post, x0, eps, L, mass)
    acc = hmc.step(torch.as_tensor(xi, device="cuda"), torch.as_tensor(u, device="cuda"))
    torch.cuda.synchronize()
    xg, lpg, dhg, accg = hmc.x.cpu().numpy(), hmc.logp.cpu().numpy(), hmc.dh.cpu().numpy(), acc.cpu().numpy()
    gr = pb["grid"].as_tuple()

    def lpf(x):
        return S.logp_gw(x, lam0, gr, pb["data"], pb["inv_psd"], pb["lo"], pb["hi"])

    for i in range(6):
        lp0, g0 = lpf(x0[i])
        xr, lpr, _, ar, dhr = S.hmc_step(lpf, x0[i], lp0, g0, xi[i], u[i], L, eps, mass)
        assert abs(dhg[i] - dhr) <= 1e-8 * max(1.0, abs(dhr)), (dhg[i], dhr)
        if abs(-dhr - math.log(u[i])) > 1e-6:
            assert accg[i] == ar
            assert np.max(np.abs(xg[i] - xr)) <= 1e-9 * (1 + np.max(np.abs(xr)))


def test_posterior_and_hmc_full_c5_sampled(gpu, lam0):
    """The learned-proposal workload at its full size (4096 chains x 8033 bins, the chunked
    small-batch launch configuration) in one call: log posterior and gradient of sampled chains, and
    one HMC transition of 10 leapfrog steps, against the oracle."""
    import torch
    from paper_2302_05329_amd import sampling
    pb = _c5_problem(lam0)
    post = sampling.Posterior(0, grid=pb["grid"], lam=lam0, data=pb["data"], inv_psd=pb["inv_psd"], lo=pb["lo"],
                              hi=pb["hi"])
    n = 4096
    rng = np.random.default_rng(13)
    x0 = post.to_x(pb["theta_inj"]) + 0.02 * rng.standard_normal((n, 7))
    mass = np.array([400.0, 50.0, 20.0, 20.0, 10.0, 4e3, 4.0])
    eps, L = 0.02, 10
    xi = rng.standard_normal((n, 7))
    u = rng.uniform(size=n)
    _say(f"posterior logp + HMC step GW n={n} nb={pb['grid'].n_bins} L={L}")
    lp, g = sampling.logp(post, x0)
    hmc = sampling.HMC(post, x0, eps, L, mass)
    acc = hmc.step(torch.as_tensor(xi, device="cuda"), torch.as_tensor(u, device="cuda"))
    torch.cuda.synchronize()
    lp, g = lp.cpu().numpy(), g.cpu().numpy()
    xg, dhg, accg = hmc.x.cpu().numpy(), hmc.dh.cpu().numpy(), acc.cpu().numpy()
    gr = pb["grid"].as_tuple()

    def lpf(x):
        return S.logp_gw(x, lam0, gr, pb["data"], pb["inv_psd"], pb["lo"], pb["hi"])

    rows = sorted({0, n - 1} | set(int(i) for i in rng.choice(n, 2, replace=False)))
    for i in rows:
        ref_lp, ref_g = lpf(x0[i])
        assert abs(lp[i] - ref_lp) <= _lp_tol(pb, lam0, x0[i], ref_lp), (i, lp[i], ref_lp)
        th, d, _, _ = S.transform(x0[i], pb["lo"], pb["hi"])
        F = O.fisher(th, O.PARAM_MC_Q, lam0, gr, pb["inv_psd"])
        r = pb["data"] - O.waveform(th, O.PARAM_MC_Q, lam0, gr)
        scale = np.sqrt(O.inner(r, r, pb["inv_psd"], gr[1]) * np.diag(F)) * d + 1.0
        assert np.all(np.abs(g[i] - ref_g) <= 1e-10 * scale), (i, g[i], ref_g)
    for i in rows[:2]:
        lp0, g0 = lpf(x0[i])
        xr, _, _, ar, dhr = S.hmc_step(lpf, x0[i], lp0, g0, xi[i], u[i], L, eps, mass)
        assert abs(dhg[i] - dhr) <= 1e-8 * max(1.0, abs(dhr)), (i, dhg[i], dhr)
        if abs(-dhr - math.log(u[i])) > 1e-6:
            assert accg[i] == ar
            assert np.max(np.abs(xg[i] - xr)) <= 1e-9 * (1 + np.max(np.abs(xr)))


def _rwmh_parity(pb, lam0, n, rows, seed):
    import torch
    from paper_2302_05329_amd import sampling
    post = sampling.Posterior(0, grid=pb["grid"], lam=lam0, data=pb["data"], inv_psd=pb["inv_psd"], lo=pb["lo"],
                              hi=pb["hi"])
    rng = np.random.default_rng(seed)
    x0 = post.to_x(pb["theta_inj"]) + 0.02 * rng.standard_normal((n, 7))
    scale = np.array([0.02, 0.05, 0.1, 0.1, 0.05, 0.01, 0.2])
    xi = rng.standard_normal((n, 7))
    u = rng.uniform(size=n)
    _say(f"random-walk MH step GW n={n} nb={pb['grid'].n_bins}")
    rw = sampling.RWMH(post, x0, scale)
    lp0 = rw.logp.cpu().numpy()
    acc = rw.step(torch.as_tensor(xi, device="cuda"), torch.as_tensor(u, device="cuda"))
    torch.cuda.synchronize()
    xg, lpg, accg = rw.x.cpu().numpy(), rw.logp.cpu().numpy(), acc.cpu().numpy()
    gr = pb["grid"].as_tuple()

    def lpf(x):
        return S.logp_gw(x, lam0, gr, pb["data"], pb["inv_psd"], pb["lo"], pb["hi"], want_grad=False)[0]

    checked = 0
    for i in rows:
        ref0 = lpf(x0[i])
        assert abs(lp0[i] - ref0) <= _lp_tol(pb, lam0, x0[i], ref0), (i, lp0[i], ref0)
        xr, lpr, ar = S.rwmh_step(lpf, x0[i], ref0, xi[i], u[i], scale)
        lpp = lpf(x0[i] + scale * xi[i])
        if abs(lpp - ref0 - math.log(u[i])) > 1e-6:
            assert accg[i] == ar, (i, accg[i], ar)
            assert np.max(np.abs(xg[i] - xr)) <= 1e-14 * (1 + np.max(np.abs(xr))), (i, xg[i], xr)
            assert abs(lpg[i] - lpr) <= _lp_tol(pb, lam0, xr, lpr), (i, lpg[i], lpr)
            checked += 1
    assert checked >= len(rows) - 1
    return accg


def test_rwmh_step_parity_gw(gpu, lam0):
    pb = _c5_problem(lam0, n_bins=4001)
    acc = _rwmh_parity(pb, lam0, 24, range(24), 15)
    assert 0 < acc.sum() < 24


def test_rwmh_full_c5_sampled(gpu, lam0):
    """One random-walk transition of the learned-proposal workload at its full size (4096 chains x
    8033 bins) against the oracle on sampled chains."""
    pb = _c5_problem(lam0)
    rng = np.random.default_rng(16)
    rows = sorted({0, 4095} | set(int(i) for i in rng.choice(4096, 3, replace=False)))
    _rwmh_parity(pb, lam0, 4096, rows, 16)


def test_rwmh_on_gaussian_target_gpu(gpu):
    """Closed-form stationary acceptance (2/pi) arctan(2/s) of a one-coordinate walk, the target's
    moments kept over 30 steps, and a zero step accepting every chain."""
    import torch
    from paper_2302_05329_amd import sampling
    mu = np.array([0.3, -1.0, 2.0, 0.0, 0.5, -0.2, 1.1])
    sig = np.array([0.5, 1.0, 2.0, 0.1, 1.5, 0.7, 0.3])
    post = sampling.Posterior(1, mu=mu, isig2=1 / sig**2)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(17)
    mu_t = torch.as_tensor(mu, device="cuda")
    sig_t = torch.as_tensor(sig, device="cuda")
    n = 1 << 18
    _say(f"random-walk MH gaussian n={n}")
    for s in (1.0, 2.4):
        x0 = mu_t + sig_t * torch.randn((n, 7), dtype=torch.float64, device="cuda", generator=gen)
        scale = np.zeros(7)
        scale[0] = s * sig[0]
        rw = sampling.RWMH(post, x0, scale)
        xi = torch.randn((n, 7), dtype=torch.float64, device="cuda", generator=gen)
        u = torch.rand(n, dtype=torch.float64, device="cuda", generator=gen)
        rate = float((rw.step(xi, u) == 1).double().mean())
        expect = 2.0 / math.pi * math.atan(2.0 / s)
        assert abs(rate - expect) < 0.005, (s, rate, expect)
        assert torch.equal(rw.x[:, 1:], x0[:, 1:])
    n = 8192
    x0 = mu_t + sig_t * torch.randn((n, 7), dtype=torch.float64, device="cuda", generator=gen)
    rw = sampling.RWMH(post, x0, 0.8 * sig)
    for _ in range(30):
        rw.step(torch.randn((n, 7), dtype=torch.float64, device="cuda", generator=gen),
                torch.rand(n, dtype=torch.float64, device="cuda", generator=gen))
    x = rw.x.cpu().numpy()
    assert np.all(np.abs(x.mean(axis=0) - mu) < 5 * sig / math.sqrt(n))
    assert np.all(np.abs(x.std(axis=0) / sig - 1) < 0.05)
    u = torch.full((n,), 0.999, dtype=torch.float64, device="cuda")
    a = rw.step(torch.randn((n, 7), dtype=torch.float64, device="cuda", generator=gen), u)
    assert int((a == 1).sum()) < n  # a non-zero step rejects some chains at u = 0.999
    rw.scale = type(rw.scale)(*([0.0] * 7))
    x1 = rw.x.clone()
    a = rw.step(torch.randn((n, 7), dtype=torch.float64, device="cuda", generator=gen), u)
    assert int((a == 1).sum()) == n and torch.equal(rw.x, x1)


def _two_site_problem(lam, n_bins, seed=1105):
    """The two-detector injection (H1, L1; iota = psi = ra = dec = pi/3), built with the oracle."""
    from oracle import network_oracle as N
    cfg = W.config5()
    grid = W.Grid(20.0, 0.125, n_bins)
    g = grid.as_tuple()
    dets = [W.DETECTORS["H1"], W.DETECTORS["L1"]]
    orient = np.full(4, math.pi / 3)
    gmst = 1.234
    psd = W.psd_aligo_zdhp_fit(grid.freqs())
    inj = cfg["inj_unit_distance"].copy()
    inj[4] = 500.0
    data = np.stack([W.complex_noise(psd, grid.df, seed + k) + N.strain(np.r_[inj, orient], O.PARAM_M1M2, lam, g, d,
                                                                          gmst) for k, d in enumerate(dets)])
    mc_q = W.to_param(inj[None, :], O.PARAM_MC_Q)[0]
    lo = np.array([20.0, 0.125, -0.9, -0.9, 100.0, -0.1, -0.5 * math.pi])
    hi = np.array([40.0, 1.0, 0.9, 0.9, 1500.0, 0.1, 0.5 * math.pi])
    return dict(grid=grid, data=data, inv_psd=np.stack([1 / psd] * 2), lo=lo, hi=hi, theta_inj=mc_q, dets=dets,
                orient=orient, gmst=gmst)


def _two_site_post(pb, lam):
    from paper_2302_05329_amd import sampling
    return sampling.Posterior(2, grid=pb["grid"], lam=lam, data=pb["data"], inv_psd=pb["inv_psd"], lo=pb["lo"],
                              hi=pb["hi"], detectors=pb["dets"], gmst=pb["gmst"], orient=pb["orient"])


def _two_site_lpf(pb, lam):
    gr = pb["grid"].as_tuple()

    def lpf(x):
        return S.logp_gw_network(x, lam, gr, pb["dets"], pb["data"], pb["inv_psd"], pb["lo"], pb["hi"], pb["gmst"],
                                 pb["orient"])
    return lpf


def _two_site_grad_scale(pb, lam, x):
    """Per coordinate, the Cauchy-Schwarz bound sqrt(sum_d (r_d|r_d) F_pp) on the likelihood term of
    the gradient (F the network Fisher matrix), times d theta / d x, plus 1."""
    from oracle import network_oracle as N
    gr = pb["grid"].as_tuple()
    th, d, _, _ = S.transform(x, pb["lo"], pb["hi"])
    th11 = np.r_[th, pb["orient"]]
    F = N.fisher(th11, O.PARAM_MC_Q, lam, gr, pb["dets"], pb["inv_psd"], pb["gmst"])
    rr = 0.0
    for k, det in enumerate(pb["dets"]):
        r = pb["data"][k] - N.strain(th11, O.PARAM_MC_Q, lam, gr, det, pb["gmst"])
        rr += O.inner(r, r, pb["inv_psd"][k], gr[1])
    return np.sqrt(rr * np.diag(F)[:7]) * d + 1.0


def _two_site_lp_tol(pb, lam, x, ref_lp):
    th = S.transform(x, pb["lo"], pb["hi"])[0]
    th11 = np.r_[th, pb["orient"]]
    return (network_lnl_tolerance(th11, O.PARAM_MC_Q, lam, pb["grid"].as_tuple(), pb["dets"], pb["data"],
                                  pb["inv_psd"], pb["gmst"]) + 8.0 * np.spacing(abs(ref_lp) + 100.0))


def test_two_site_posterior_and_hmc_parity(gpu, lam0):
    """The two-detector posterior (network likelihood, fixed orientation) and one HMC transition
    against the oracle."""
    import torch
    from paper_2302_05329_amd import sampling
    pb = _two_site_problem(lam0, 4001)
    post = _two_site_post(pb, lam0)
    rng = np.random.default_rng(18)
    x0 = post.to_x(pb["theta_inj"]) + 0.02 * rng.standard_normal((6, 7))
    _say("two-site posterior logp + HMC step n=6 nb=4001")
    lp, g = sampling.logp(post, x0)
    mass = np.array([400.0, 50.0, 20.0, 20.0, 10.0, 4e3, 4.0])
    eps, L = 0.02, 4
    xi = rng.standard_normal((6, 7))
    u = rng.uniform(size=6)
    hmc = sampling.HMC(post, x0, eps, L, mass)
    acc = hmc.step(torch.as_tensor(xi, device="cuda"), torch.as_tensor(u, device="cuda"))
    torch.cuda.synchronize()
    lp, g = lp.cpu().numpy(), g.cpu().numpy()
    xg, dhg, accg = hmc.x.cpu().numpy(), hmc.dh.cpu().numpy(), acc.cpu().numpy()
    lpf = _two_site_lpf(pb, lam0)
    for i in range(6):
        ref_lp, ref_g = lpf(x0[i])
        assert abs(lp[i] - ref_lp) <= _two_site_lp_tol(pb, lam0, x0[i], ref_lp), (i, lp[i], ref_lp)
        assert np.all(np.abs(g[i] - ref_g) <= 1e-10 * _two_site_grad_scale(pb, lam0, x0[i])), (i, g[i], ref_g)
    for i in range(2):
        lp0, g0 = lpf(x0[i])
        xr, _, _, ar, dhr = S.hmc_step(lpf, x0[i], lp0, g0, xi[i], u[i], L, eps, mass)
        assert abs(dhg[i] - dhr) <= 1e-8 * max(1.0, abs(dhr)), (i, dhg[i], dhr)
        if abs(-dhr - math.log(u[i])) > 1e-6:
            assert accg[i] == ar
            assert np.max(np.abs(xg[i] - xr)) <= 1e-9 * (1 + np.max(np.abs(xr)))


def test_two_site_posterior_full_c5_sampled(gpu, lam0):
    """The two-detector posterior at the learned-proposal workload's size (4096 chains x 8033 bins x
    2 sites, one call) on sampled chains against the oracle."""
    import torch
    from paper_2302_05329_amd import sampling
    pb = _two_site_problem(lam0, 8033)
    post = _two_site_post(pb, lam0)
    n = 4096
    rng = np.random.default_rng(19)
    x0 = post.to_x(pb["theta_inj"]) + 0.02 * rng.standard_normal((n, 7))
    _say(f"two-site posterior logp n={n} nb=8033")
    lp, g = sampling.logp(post, x0)
    torch.cuda.synchronize()
    lp, g = lp.cpu().numpy(), g.cpu().numpy()
    lpf = _two_site_lpf(pb, lam0)
    for i in sorted({0, n - 1} | set(int(k) for k in rng.choice(n, 2, replace=False))):
        ref_lp, ref_g = lpf(x0[i])
        assert abs(lp[i] - ref_lp) <= _two_site_lp_tol(pb, lam0, x0[i], ref_lp), (i, lp[i], ref_lp)
        assert np.all(np.abs(g[i] - ref_g) <= 1e-10 * _two_site_grad_scale(pb, lam0, x0[i])), (i, g[i], ref_g)


def test_hmc_recovers_gaussian_target_on_gpu(gpu):
    import torch
    from paper_2302_05329_amd import sampling
    mu = np.array([0.3, -1.0, 2.0, 0.0, 0.5, -0.2, 1.1])
    sig = np.array([0.5, 1.0, 2.0, 0.1, 1.5, 0.7, 0.3])
    post = sampling.Posterior(1, mu=mu, isig2=1 / sig**2)
    n = 4096
    rng = np.random.default_rng(13)
    x0 = mu + 3 * sig * rng.standard_normal((n, 7))
    hmc = sampling.HMC(post, x0, 0.2, 8, 1 / sig**2)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(13)
    draws = []
    acc = 0
    _say("hmc gaussian n=4096 steps=40")
    for t in range(40):
        xi = torch.randn((n, 7), dtype=torch.float64, device="cuda", generator=gen)
        u = torch.rand(n, dtype=torch.float64, device="cuda", generator=gen)
        a = hmc.step(xi, u)
        acc += int((a == 1).sum())
        if t >= 10:
            draws.append(hmc.x.cpu().numpy())
    s = np.concatenate(draws)
    assert acc / (40 * n) > 0.6
    se = sig / np.sqrt(n * 5)
    assert np.all(np.abs(s.mean(axis=0) - mu) < 5 * se)
    assert np.all(np.abs(s.std(axis=0) / sig - 1) < 0.03)


def test_independence_mh_matches_rule(gpu):
    import torch
    from paper_2302_05329_amd import sampling
    rng = np.random.default_rng(14)
    n = 1000
    x = rng.standard_normal((n, 7))
    lp = rng.normal(-5, 2, n)
    lq = rng.normal(-5, 2, n)
    xp = rng.standard_normal((n, 7))
    lpp = rng.normal(-5, 2, n)
    lqp = rng.normal(-5, 2, n)
    lpp[:10] = -np.inf
    u = rng.uniform(size=n)
    g = rng.standard_normal((n, 7))
    gp = rng.standard_normal((n, 7))
    t = [torch.as_tensor(a, device="cuda").contiguous() for a in (x, lp, lq, xp, lpp, lqp, u, g, gp)]
    _say("independence MH n=1000")
    acc = sampling.independence_mh(*t[:7], grad=t[7], grad_p=t[8]).cpu().numpy()
    xs, lps, lqs, gs = (t[i].cpu().numpy() for i in (0, 1, 2, 7))
    for i in range(n):
        xr, lpr, lqr, ar = S.independence_mh(x[i], lp[i], lq[i], xp[i], lpp[i], lqp[i], u[i])
        assert acc[i] == ar
        assert np.array_equal(xs[i], xr) and lps[i] == lpr and lqs[i] == lqr
        assert np.array_equal(gs[i], gp[i] if ar else g[i])


def test_dense_hmc_step_parity_gw(gpu, lam0):
    """One dense-metric HMC transition on the gravitational-wave posterior against the oracle's
    momentum-space formulation (p = L^-T xi, drift eps L L^T p)."""
    import torch
    from paper_2302_05329_amd import sampling
    pb = _c5_problem(lam0, n_bins=4001)
    post = sampling.Posterior(0, grid=pb["grid"], lam=lam0, data=pb["data"], inv_psd=pb["inv_psd"], lo=pb["lo"],
                              hi=pb["hi"])
    rng = np.random.default_rng(22)
    x0 = post.to_x(pb["theta_inj"]) + 0.02 * rng.standard_normal((6, 7))
    A = rng.standard_normal((7, 7)) * 0.01
    cov = A @ A.T + np.diag([2e-3, 1e-2, 5e-2, 5e-2, 1e-1, 2e-4, 2e-1])
    chol = np.linalg.cholesky(cov)
    eps, L = 0.1, 4
    xi = rng.standard_normal((6, 7))
    u = rng.uniform(size=6)
    _say("dense-metric hmc step GW n=6 L=4")
    hmc = sampling.HMC(post, x0, eps, L, chol=chol)
    acc = hmc.step(torch.as_tensor(xi, device="cuda"), torch.as_tensor(u, device="cuda"))
    torch.cuda.synchronize()
    xg, dhg, accg = hmc.x.cpu().numpy(), hmc.dh.cpu().numpy(), acc.cpu().numpy()
    gr = pb["grid"].as_tuple()

    def lpf(x):
        return S.logp_gw(x, lam0, gr, pb["data"], pb["inv_psd"], pb["lo"], pb["hi"])

    for i in range(6):
        lp0, g0 = lpf(x0[i])
        xr, lpr, _, ar, dhr = S.hmc_step_dense(lpf, x0[i], lp0, g0, xi[i], u[i], L, eps, chol)
        assert abs(dhg[i] - dhr) <= 1e-8 * max(1.0, abs(dhr)), (dhg[i], dhr)
        if abs(-dhr - math.log(u[i])) > 1e-6:
            assert accg[i] == ar
            assert np.max(np.abs(xg[i] - xr)) <= 1e-9 * (1 + np.max(np.abs(xr)))


def test_dense_hmc_recovers_gaussian_target_on_gpu(gpu):
    """Any metric leaves the target invariant: a deliberately skewed dense metric on the Gaussian
    test target still recovers its moments."""
    import torch
    from paper_2302_05329_amd import sampling
    mu = np.array([0.3, -1.0, 2.0, 0.0, 0.5, -0.2, 1.1])
    sig = np.array([0.5, 1.0, 2.0, 0.1, 1.5, 0.7, 0.3])
    post = sampling.Posterior(1, mu=mu, isig2=1 / sig**2)
    rng = np.random.default_rng(23)
    A = np.tril(rng.standard_normal((7, 7)) * 0.3)
    chol = np.diag(sig) + A - np.diag(np.diag(A))
    n = 4096
    gen = torch.Generator(device="cuda")
    gen.manual_seed(24)
    x0 = mu + sig * rng.standard_normal((n, 7))
    _say(f"dense-metric hmc on a Gaussian target n={n}")
    hmc = sampling.HMC(post, x0, 0.25, 6, chol=chol)
    draws = []
    for t in range(80):
        xi = torch.randn((n, 7), dtype=torch.float64, device="cuda", generator=gen)
        u = torch.rand(n, dtype=torch.float64, device="cuda", generator=gen)
        hmc.step(xi, u)
        if t >= 20:
            draws.append(hmc.x.cpu().numpy())
    d = np.concatenate(draws)
    assert np.all(np.abs(d.mean(axis=0) - mu) <= 0.02 * sig)
    assert np.all(np.abs(d.std(axis=0) / sig - 1.0) <= 0.02)


def test_dense_rwmh_step_parity_gw(gpu, lam0):
    """Correlated random-walk steps x + L xi on the gravitational-wave posterior against the oracle."""
    import torch
    from paper_2302_05329_amd import sampling
    pb = _c5_problem(lam0, n_bins=4001)
    post = sampling.Posterior(0, grid=pb["grid"], lam=lam0, data=pb["data"], inv_psd=pb["inv_psd"], lo=pb["lo"],
                              hi=pb["hi"])
    rng = np.random.default_rng(25)
    n = 16
    x0 = post.to_x(pb["theta_inj"]) + 0.02 * rng.standard_normal((n, 7))
    A = rng.standard_normal((7, 7)) * 0.005
    chol = np.linalg.cholesky(A @ A.T + np.diag([1e-4, 4e-4, 2e-3, 2e-3, 4e-3, 1e-5, 1e-2]))
    xi = rng.standard_normal((n, 7))
    u = rng.uniform(size=n)
    _say(f"dense random-walk MH step GW n={n}")
    rw = sampling.RWMH(post, x0, chol=chol)
    lp0 = rw.logp.cpu().numpy()
    acc = rw.step(torch.as_tensor(xi, device="cuda"), torch.as_tensor(u, device="cuda"))
    torch.cuda.synchronize()
    xg, accg = rw.x.cpu().numpy(), acc.cpu().numpy()
    gr = pb["grid"].as_tuple()

    def lpf(x):
        return S.logp_gw(x, lam0, gr, pb["data"], pb["inv_psd"], pb["lo"], pb["hi"], want_grad=False)[0]

    checked = 0
    for i in range(n):
        ref0 = lpf(x0[i])
        assert abs(lp0[i] - ref0) <= _lp_tol(pb, lam0, x0[i], ref0)
        xr, lpr, ar = S.rwmh_step_dense(lpf, x0[i], ref0, xi[i], u[i], chol)
        lpp = lpf(x0[i] + np.tril(chol) @ xi[i])
        if abs(lpp - ref0 - math.log(u[i])) > 1e-6:
            assert accg[i] == ar, (i, accg[i], ar)
            assert np.max(np.abs(xg[i] - xr)) <= 1e-14 * (1 + np.max(np.abs(xr)))
            checked += 1
    assert checked >= n - 1 and 0 < accg.sum() < n
