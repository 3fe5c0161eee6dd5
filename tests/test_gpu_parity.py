"""GPU (HIP, gfx950) against the CPU oracle on identical seeded inputs.

Tolerances (FP64 mode):
  strain       max_k |dh_k| / max_k |h_k| <= 1e-10 per point
  ln L         |d lnL| <= the per-point rounding bound of tests/error_model.py: 1e-10 plus the
               FP64 rounding of the phase summands (ulp scale) and of the amplitude, weighted
               by w_k |d_k| |h_k| and summed over bins
  gradient     |d g_p| <= 1e-10 * sqrt((d-h|d-h) F_pp)  (Cauchy-Schwarz bound of |g_p|)
  Fisher       |d F_pq| <= 1e-10 * sqrt(F_pp F_qq)
  mismatch     |d M| <= 1e-12; lag identical unless the top two |z_j| are within 1e-12;
               gradient normwise max|d g| <= 1e-8 * max|g|
"""
import math
import sys

import numpy as np
import pytest

from error_model import lnl_tolerance
from oracle import phenomd_oracle as O
from paper_2302_05329_amd import workloads as W

pytestmark = pytest.mark.gpu

P = O.PARAM_M1M2


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _strain_err(hg, hr):
    return np.max(np.abs(hg - hr)) / np.max(np.abs(hr))


def test_waveform_parity_config1(gpu, lam0):
    import torch
    cfg = W.config1(n=1024)
    g = cfg["grid"].as_tuple()
    _say(f"waveform_eval C1 n=1024 nb={g[2]}")
    h, st = gpu.api.waveform_eval(cfg["theta"], P, cfg["grid"], lam0)
    torch.cuda.synchronize()
    h = h.cpu().numpy()
    assert np.all(st.cpu().numpy() == 0)
    idx = np.linspace(0, 1023, 40).astype(int)
    for i in idx:
        ref = O.waveform(cfg["theta"][i], P, lam0, g)
        assert _strain_err(h[i], ref) <= 1e-10, i
        big = np.abs(ref) > 1e-6 * np.max(np.abs(ref))
        assert np.max(np.abs(h[i][big] - ref[big]) / np.abs(ref[big])) <= 1e-10, i
        assert np.all(h[i][ref == 0] == 0)


@pytest.mark.parametrize("param", [O.PARAM_MC_ETA, O.PARAM_LNMC_ETA_LND, O.PARAM_MC_Q])
def test_waveform_parity_parameterisations(gpu, lam0, param):
    import torch
    rows = W.draw_sources(12, 77, d_range=(100, 2000), tc_range=(-0.1, 0.1), phic_random=True)
    th = W.to_param(rows, param)
    grid = W.Grid(20.0, 0.125, 16225)
    _say(f"waveform_eval param={param} n=12 nb=16225")
    h, st = gpu.api.waveform_eval(th, param, grid, lam0)
    torch.cuda.synchronize()
    h = h.cpu().numpy()
    for i in range(len(th)):
        ref = O.waveform(th[i], param, lam0, grid.as_tuple())
        assert _strain_err(h[i], ref) <= 1e-10, i


def test_loglike_and_grad_parity_config2_grid(gpu, lam0):
    import torch
    cfg = W.config2(n=24)
    g = cfg["grid"].as_tuple()
    data, ip = cfg["data"], cfg["inv_psd"]
    # add a loud injection so that the likelihood surface has structure
    data = data + O.waveform(cfg["theta"][0] * np.array([1.002, 0.998, 1, 1, 1, 1, 1]), P, lam0, g)
    _say(f"loglike_and_grad C2-grid n=24 nb={g[2]}")
    lnl, grad, st = gpu.api.loglike_and_grad(cfg["theta"], P, cfg["grid"], lam0, data, ip)
    lnl0, _, _ = gpu.api.loglike_and_grad(cfg["theta"], P, cfg["grid"], lam0, data, ip, want_grad=False)
    torch.cuda.synchronize()
    lnl, grad, lnl0 = lnl.cpu().numpy(), grad.cpu().numpy(), lnl0.cpu().numpy()
    for i in range(len(cfg["theta"])):
        th = cfg["theta"][i]
        h = O.waveform(th, P, lam0, g)
        hh = O.inner(h, h, ip, g[1])
        ref = O.loglike(th, P, lam0, g, data, ip)
        tol = lnl_tolerance(th, P, lam0, g, data, ip)
        _say(f"lnL i={i}: |d| = {abs(lnl[i] - ref):.2e} (value only {abs(lnl0[i] - ref):.2e}), bound {tol:.2e}, "
             f"(h|h) = {hh:.3e}")
        assert abs(lnl[i] - ref) <= tol, (i, lnl[i], ref)
        assert abs(lnl0[i] - ref) <= tol, (i, lnl0[i], ref)
        gref = O.loglike_grad(th, P, lam0, g, data, ip)
        F = O.fisher(th, P, lam0, g, ip)
        r = data - h
        scale = np.sqrt(O.inner(r, r, ip, g[1]) * np.diag(F))
        assert np.all(np.abs(grad[i] - gref) <= 1e-10 * scale), (i, grad[i], gref, scale)


def test_loglike_and_grad_full_c2_sampled(gpu, lam0):
    """The full batched-throughput workload in the benchmark's launch configuration (65536
    points x 16225 bins, one call): sampled points against the oracle one by one -- the
    lightest and heaviest systems, the largest and smallest |lnL|, and random ones."""
    import torch
    cfg = W.config2()
    g = cfg["grid"].as_tuple()
    data, ip = cfg["data"], cfg["inv_psd"]
    th_all = cfg["theta"]
    _say(f"loglike_and_grad full C2 n={len(th_all)} nb={g[2]}")
    lnl, grad, st = gpu.api.loglike_and_grad(th_all, P, cfg["grid"], lam0, data, ip)
    torch.cuda.synchronize()
    lnl, grad, st = lnl.cpu().numpy(), grad.cpu().numpy(), st.cpu().numpy()
    assert np.all(st == 0) and np.all(np.isfinite(lnl)) and np.all(np.isfinite(grad))
    mt = th_all[:, 0] + th_all[:, 1]
    rng = np.random.default_rng(2)
    pick = {int(np.argmin(mt)), int(np.argmax(mt)), int(np.argmax(np.abs(lnl))), int(np.argmin(np.abs(lnl)))}
    pick |= set(int(i) for i in rng.choice(len(th_all), 6, replace=False))
    for i in sorted(pick):
        th = th_all[i]
        h = O.waveform(th, P, lam0, g)
        hh = O.inner(h, h, ip, g[1])
        ref = O.loglike(th, P, lam0, g, data, ip)
        tol = lnl_tolerance(th, P, lam0, g, data, ip)
        _say(f"lnL i={i}: |d| = {abs(lnl[i] - ref):.2e}, bound {tol:.2e}, (h|h) = {hh:.3e}")
        assert abs(lnl[i] - ref) <= tol, (i, lnl[i], ref)
        gref = O.loglike_grad(th, P, lam0, g, data, ip)
        F = O.fisher(th, P, lam0, g, ip)
        r = data - h
        scale = np.sqrt(O.inner(r, r, ip, g[1]) * np.diag(F))
        assert np.all(np.abs(grad[i] - gref) <= 1e-10 * scale), (i, grad[i], gref, scale)


@pytest.mark.parametrize("param", [O.PARAM_LNMC_ETA_LND, O.PARAM_MC_Q, O.PARAM_MC_ETA])
def test_fisher_parity_config3_grid(gpu, lam0, param):
    import torch
    cfg = W.config3(n=10)
    g = cfg["grid"].as_tuple()
    th = W.to_param(cfg["theta"], param)
    _say(f"fisher C3-grid param={param} n=10 nb={g[2]}")
    F, st = gpu.api.fisher(th, param, cfg["grid"], lam0, cfg["inv_psd"])
    torch.cuda.synchronize()
    F = F.cpu().numpy()
    for i in range(len(th)):
        ref = O.fisher(th[i], param, lam0, g, cfg["inv_psd"])
        scale = np.sqrt(np.outer(np.diag(ref), np.diag(ref)))
        assert np.all(np.abs(F[i] - ref) <= 1e-10 * scale), (i, np.max(np.abs(F[i] - ref) / scale))
        assert np.array_equal(F[i], F[i].T)


def test_mismatch_grad_parity_config4_shape(gpu, lam0):
    import torch
    cfg = W.config4(n=4)
    g = cfg["grid"].as_tuple()
    th = cfg["theta"]
    w = cfg["inv_psd"]
    targets = np.stack([O.waveform(t, P, cfg["lam_star"], g) for t in th])
    _say(f"mismatch_grad C4-shape nt=4 nb={g[2]}")
    mm, dl, lag = gpu.api.mismatch_grad(th, P, cfg["grid"], lam0, targets, w)
    torch.cuda.synchronize()
    mm, dl, lag = mm.cpu().numpy(), dl.cpu().numpy(), lag.cpu().numpy()
    gsum = np.zeros(209)
    for i in range(len(th)):
        m_ref, j_ref, gap, gref = O.mismatch_grad_lambda(th[i], P, lam0, g, targets[i], 4 * g[1] * w)
        assert gap > 1e-12, "ambiguous lag in the fixture"
        assert lag[i] == j_ref
        assert abs(mm[i] - m_ref) <= 1e-12, (mm[i], m_ref)
        gsum += gref
    assert np.max(np.abs(dl - gsum)) <= 1e-8 * np.max(np.abs(gsum)), np.max(np.abs(dl - gsum)) / np.max(np.abs(gsum))


def test_domain_errors_give_nan_and_status(gpu, lam0):
    import torch
    rows = W.draw_sources(6, 5)
    rows[1, 0] = -3.0                      # negative mass
    rows[2, 4] = 0.0                       # D = 0
    rows[3, 2] = 1.5                       # |chi| > 1
    rows[4, 5] = np.nan                    # non-finite
    grid = W.Grid(20.0, 0.25, 4017)
    _say("domain errors waveform/loglike n=6")
    h, st = gpu.api.waveform_eval(rows, P, grid, lam0)
    psd = W.psd_aligo_zdhp_fit(grid.freqs())
    data = W.complex_noise(psd, grid.df, 3)
    lnl, grad, st2 = gpu.api.loglike_and_grad(rows, P, grid, lam0, data, 1 / psd)
    torch.cuda.synchronize()
    st = st.cpu().numpy()
    assert list(st) == [0, -2, -2, -2, -2, 0]
    assert np.array_equal(st, st2.cpu().numpy())
    h = h.cpu().numpy()
    for i in (1, 2, 3, 4):
        assert np.all(np.isnan(h[i]))
        assert np.isnan(lnl[i].item()) and np.all(np.isnan(grad[i].cpu().numpy()))
    for i in (0, 5):
        ref = O.waveform(rows[i], P, lam0, grid.as_tuple())
        assert _strain_err(h[i], ref) <= 1e-10


def test_eta_quarter_mc_eta_is_domain_ok(gpu, lam0):
    import torch
    th = np.array([[20.0, 0.25, 0.1, -0.2, 500.0, 0.0, 0.0]])
    grid = W.Grid(20.0, 0.25, 4017)
    _say("eta = 1/4 in (Mc, eta)")
    h, st = gpu.api.waveform_eval(th, O.PARAM_MC_ETA, grid, lam0)
    torch.cuda.synchronize()
    assert st.item() == 0
    ref = O.waveform(th[0], O.PARAM_MC_ETA, lam0, grid.as_tuple())
    assert _strain_err(h[0].cpu().numpy(), ref) <= 1e-10


def test_empty_and_short_active_ranges(gpu, lam0):
    """A source whose cutoff lies below the grid gives zero strain, lnL = 0, grad = 0; a source
    with a handful of active bins matches the oracle."""
    import torch
    rows = np.array([[3000.0, 2500.0, 0.1, 0.2, 500.0, 0.0, 0.0],     # f_cut ~ 7 Hz < 20 Hz
                     [1100.0, 900.0, 0.1, 0.2, 500.0, 0.0, 0.0],      # f_cut ~ 20.3 Hz
                     [30.0, 20.0, 0.1, 0.2, 500.0, 0.0, 0.0]])
    grid = W.Grid(20.0, 0.125, 8033)
    psd = W.psd_aligo_zdhp_fit(grid.freqs())
    data = W.complex_noise(psd, grid.df, 9)
    _say("short active ranges n=3")
    h, st = gpu.api.waveform_eval(rows, P, grid, lam0)
    lnl, grad, _ = gpu.api.loglike_and_grad(rows, P, grid, lam0, data, 1 / psd)
    torch.cuda.synchronize()
    h = h.cpu().numpy()
    assert np.all(h[0] == 0) and lnl[0].item() == 0.0 and np.all(grad[0].cpu().numpy() == 0.0)
    for i in (1, 2):
        ref = O.waveform(rows[i], P, lam0, grid.as_tuple())
        assert np.count_nonzero(ref) == np.count_nonzero(h[i])
        assert _strain_err(h[i], ref) <= 1e-10
        lref = O.loglike(rows[i], P, lam0, grid.as_tuple(), data, 1 / psd)
        assert abs(lnl[i].item() - lref) <= 1e-10 * max(1.0, abs(lref))


def test_batch_errors_raise_without_launch(gpu, lam0):
    import ctypes
    from paper_2302_05329_amd import _lib as L
    g = L.make_grid(20.0, 0.25, 100, 20.0, 20.0)
    rc = L.lib().pd_waveform_eval(None, 1, 3, ctypes.byref(g), None, 0, None, None, None, 0, None)
    assert rc == L.PD_EINVAL
    assert b"NULL" in L.lib().pd_last_error()
    bad = L.make_grid(20.0, -1.0, 100, 20.0, 20.0)
    with pytest.raises(L.PdError):
        gpu.api.waveform_eval(np.array([[30.0, 20.0, 0, 0, 400, 0, 0]]), P, bad, lam0)
    with pytest.raises(ValueError):
        gpu.api.waveform_eval(np.zeros((2, 6)), P, W.Grid(20, 0.25, 100), lam0)


def test_mixed_precision_is_unsupported_and_launches_nothing(gpu, lam0):
    """PD_MIXED is reserved: every entry point that takes a precision returns PD_EUNSUPPORTED and
    leaves its outputs untouched."""
    import ctypes
    import torch
    from paper_2302_05329_amd import _lib as L
    from paper_2302_05329_amd.api import _ptr
    cfg = W.config2(n=64)
    g = cfg["grid"]
    gr = L.make_grid(*g.as_tuple())
    th = torch.as_tensor(cfg["theta"], device="cuda")
    lam = torch.as_tensor(lam0, device="cuda")
    d = torch.as_tensor(np.stack([cfg["data"].real, cfg["data"].imag], -1), device="cuda").contiguous()
    ip = torch.as_tensor(cfg["inv_psd"], device="cuda")
    lnl = torch.full((64,), 7.0, dtype=torch.float64, device="cuda")
    grad = torch.full((64, 7), 7.0, dtype=torch.float64, device="cuda")
    h = torch.full((64, g.n_bins, 2), 7.0, dtype=torch.float64, device="cuda")
    nb = L.lib().pd_workspace_bytes(L.PD_OP_LOGLIKE_GRAD, 64, g.n_bins)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    lib = L.lib()
    rcs = [lib.pd_loglike_and_grad(_ptr(th), 64, P, ctypes.byref(gr), _ptr(lam), _ptr(d), _ptr(ip), L.PD_MIXED,
                                   _ptr(lnl), _ptr(grad), None, _ptr(ws), nb, None),
           lib.pd_loglike_and_grad_noalloc(_ptr(th), 64, P, ctypes.byref(gr), _ptr(lam), _ptr(d), _ptr(ip),
                                           L.PD_MIXED, _ptr(lnl), _ptr(grad), None, None)]
    nbw = L.lib().pd_workspace_bytes(L.PD_OP_WAVEFORM, 64, g.n_bins)
    wsw = torch.empty(nbw, dtype=torch.uint8, device="cuda")
    rcs.append(lib.pd_waveform_eval(_ptr(th), 64, P, ctypes.byref(gr), _ptr(lam), L.PD_MIXED, _ptr(h), None,
                                    _ptr(wsw), nbw, None))
    torch.cuda.synchronize()
    assert rcs == [L.PD_EUNSUPPORTED] * 3, rcs
    assert b"PD_MIXED" in lib.pd_last_error()
    assert bool(torch.all(lnl == 7.0)) and bool(torch.all(grad == 7.0)) and bool(torch.all(h == 7.0))


def test_results_are_bitwise_reproducible(gpu, lam0):
    import torch
    cfg = W.config2(n=256)
    _say("determinism loglike_and_grad n=256")
    a = gpu.api.loglike_and_grad(cfg["theta"], P, cfg["grid"], lam0, cfg["data"], cfg["inv_psd"])
    b = gpu.api.loglike_and_grad(cfg["theta"], P, cfg["grid"], lam0, cfg["data"], cfg["inv_psd"])
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_fisher_full_c3_sampled(gpu, lam0):
    """The full Fisher workload (16384 sources, 16065 bins, (ln Mc, eta, chi1, chi2, ln D, tc,
    phic)) in one call: sampled matrices against the oracle, all symmetric and finite."""
    import torch
    cfg = W.config3()
    g = cfg["grid"].as_tuple()
    th = W.to_param(cfg["theta"], O.PARAM_LNMC_ETA_LND)
    _say(f"fisher full C3 n={len(th)} nb={g[2]}")
    F, st = gpu.api.fisher(th, O.PARAM_LNMC_ETA_LND, cfg["grid"], lam0, cfg["inv_psd"])
    torch.cuda.synchronize()
    F, st = F.cpu().numpy(), st.cpu().numpy()
    assert np.all(st == 0) and np.all(np.isfinite(F))
    assert np.array_equal(F, np.swapaxes(F, 1, 2))
    rng = np.random.default_rng(4)
    for i in sorted({0, len(th) - 1} | set(int(x) for x in rng.choice(len(th), 3, replace=False))):
        ref = O.fisher(th[i], O.PARAM_LNMC_ETA_LND, lam0, g, cfg["inv_psd"])
        scale = np.sqrt(np.outer(np.diag(ref), np.diag(ref)))
        assert np.all(np.abs(F[i] - ref) <= 1e-10 * scale), (i, np.max(np.abs(F[i] - ref) / scale))


def test_mismatch_full_c4(gpu, lam0):
    """The full mismatch workload (512 targets x 2^16 bins) in one call.  At the targets' own
    coefficients lambda* the mismatches and the summed gradient vanish (a property that holds at
    any size); at lambda0 sampled mismatches and lags match the oracle."""
    import torch
    cfg = W.config4()
    g = cfg["grid"].as_tuple()
    th = cfg["theta"]
    w = cfg["inv_psd"]
    lam_star = cfg["lam_star"]
    targets, _ = gpu.api.waveform_eval(th, P, cfg["grid"], lam_star)
    _say(f"mismatch full C4 nt={len(th)} nb={g[2]}")
    mm0, dl0, lag0 = gpu.api.mismatch_grad(th, P, cfg["grid"], lam0, targets, w)
    mms, dls, _ = gpu.api.mismatch_grad(th, P, cfg["grid"], lam_star, targets, w)
    torch.cuda.synchronize()
    mm0, dl0, lag0 = mm0.cpu().numpy(), dl0.cpu().numpy(), lag0.cpu().numpy()
    mms, dls = mms.cpu().numpy(), dls.cpu().numpy()
    assert np.all(np.isfinite(mm0)) and np.all(mm0 > 0)
    assert np.max(np.abs(mms)) <= 1e-12
    assert np.max(np.abs(dls * lam_star)) <= 1e-6 * np.max(np.abs(dl0 * lam0))
    tg = targets.cpu().numpy()
    rng = np.random.default_rng(5)
    for i in sorted({0, len(th) - 1} | set(int(x) for x in rng.choice(len(th), 2, replace=False))):
        # the oracle works on its own target strain, which the library's matches to 1e-10
        tg_ref = O.waveform(th[i], P, lam_star, g)
        assert _strain_err(tg[i], tg_ref) <= 1e-10, i
        m_ref, j_ref, gap = O.mismatch(th[i], P, lam0, g, tg_ref, 4 * g[1] * w)
        if gap > 1e-12:
            assert lag0[i] == j_ref
        assert abs(mm0[i] - m_ref) <= 1e-12, (i, mm0[i], m_ref)


def test_fit_lambda_step_parity_config4_shape(gpu, lam0):
    """One coefficient-descent step (Sec. 3.1, Eqs. 6-7) against the oracle: mismatches, summed
    gradient and the updated coefficients; a zero step leaves the coefficients bit-identical."""
    import torch
    from paper_2302_05329_amd import api
    cfg = W.config4(n=2)
    g = cfg["grid"].as_tuple()
    th, w = cfg["theta"], cfg["inv_psd"]
    targets = np.stack([O.waveform(t, P, cfg["lam_star"], g) for t in th])
    _say(f"fit_lambda_step C4-shape nt=2 nb={g[2]}")
    fit0 = api.LambdaFit(th, P, cfg["grid"], lam0, targets, w, 0.0)
    fit0.step()
    alpha = 3e-3
    fit = api.LambdaFit(th, P, cfg["grid"], lam0, targets, w, alpha)
    fit.step()
    torch.cuda.synchronize()
    assert np.array_equal(fit0.lam.cpu().numpy(), lam0)
    lam1, mm, dl = fit.lam.cpu().numpy(), fit.mismatch.cpu().numpy(), fit.dsum.cpu().numpy()
    lam_ref, mm_ref, g_ref = O.fit_lambda_step(th, P, lam0, g, targets, 4 * g[1] * w, alpha)
    assert np.max(np.abs(mm - mm_ref)) <= 1e-12, (mm, mm_ref)
    scale = np.max(np.abs(g_ref))
    assert np.max(np.abs(dl - g_ref)) <= 1e-8 * scale
    step_tol = alpha / len(th) * 1e-8 * scale + 4 * np.spacing(np.abs(lam0))
    assert np.all(np.abs(lam1 - lam_ref) <= step_tol), np.max(np.abs(lam1 - lam_ref) / step_tol)


def test_fit_lambda_descent_full_c4(gpu, lam0):
    """The descent loop at the full mismatch workload (512 targets x 2^16 bins, one library call per
    step with no host synchronisation): with a step that lowers the mean mismatch by 1% to first
    order, 20 steps lower it monotonically, each step by between a half of that first-order
    prediction and (allowing for rounding and higher orders) 1.05 times it."""
    import torch
    from paper_2302_05329_amd import api
    cfg = W.config4()
    th, w = cfg["theta"], cfg["inv_psd"]
    targets, _ = api.waveform_eval(th, P, cfg["grid"], cfg["lam_star"])
    probe = api.LambdaFit(th, P, cfg["grid"], lam0, targets, w, 0.0)
    probe.step()
    loss0 = float(probe.mismatch.mean())
    grad = probe.dsum.cpu().numpy() / len(th)
    alpha = 0.01 * loss0 / float(grad @ grad)
    _say(f"fit_lambda descent C4 nt={len(th)} 20 steps alpha={alpha:.3g}")
    fit = api.LambdaFit(th, P, cfg["grid"], lam0, targets, w, alpha)
    losses, pred = [], []
    for _ in range(20):
        fit.step()
        losses.append(fit.mismatch.mean())
        pred.append(alpha * (fit.dsum / len(th)).square().sum())
    torch.cuda.synchronize()
    losses = np.array([float(x) for x in losses])
    pred = np.array([float(x) for x in pred])
    assert losses[0] == pytest.approx(loss0, rel=1e-12)
    drop = losses[:-1] - losses[1:]
    assert np.all(drop > 0.5 * pred[:-1]) and np.all(drop <= 1.05 * pred[:-1]), (drop / pred[:-1])


def test_fit_lambda_relative_step_parity(gpu, lam0):
    """One preconditioned step (Eq. 6 in u = lam / lam0 - 1, i.e. the factor lam0^2 on each
    coefficient's step) against the oracle's summed gradient."""
    import torch
    from paper_2302_05329_amd import api
    cfg = W.config4(n=2, n_fft=1 << 12)
    g = cfg["grid"].as_tuple()
    th, w = cfg["theta"], cfg["inv_psd"]
    targets = np.stack([O.waveform(t, P, cfg["lam_star"], g) for t in th])
    _say("fit_lambda_step relative coordinates nt=2 nb=2^12")
    alpha = 2e-3
    fit = api.LambdaFit(th, P, cfg["grid"], lam0, targets, w, alpha, relative=True)
    fit.step()
    torch.cuda.synchronize()
    lam1 = fit.lam.cpu().numpy()
    _, _, g_ref = O.fit_lambda_step(th, P, lam0, g, targets, 4 * g[1] * w, 0.0)
    l0 = lam0.reshape(-1)
    lam_ref = l0 - alpha / len(th) * l0 ** 2 * g_ref
    scale = np.max(np.abs(l0 ** 2 * g_ref))
    tol = alpha / len(th) * 1e-8 * scale + 4 * np.spacing(np.abs(l0))
    assert np.all(np.abs(lam1 - lam_ref) <= tol), np.max(np.abs(lam1 - lam_ref) / tol)


def test_fit_lambda_descent_relative_full_c4(gpu, lam0):
    """Eq. 6 in u = lam / lam0 - 1 at the full workload (512 targets x 2^16 bins) with alpha = 1 /
    (largest Hessian eigenvalue in u, by power iteration): 300 steps lower the mean mismatch at
    every step and end below 0.5 of the start."""
    import torch
    from paper_2302_05329_amd import api
    cfg = W.config4()
    th, w = cfg["theta"], cfg["inv_psd"]
    targets, _ = api.waveform_eval(th, P, cfg["grid"], cfg["lam_star"])
    fit = api.LambdaFit(th, P, cfg["grid"], lam0, targets, w, 0.0, relative=True)
    lmax = fit.max_curvature()
    assert lmax > 0
    fit.alpha = 1.0 / lmax
    _say(f"fit_lambda descent in u, C4 nt={len(th)}: 300 steps alpha={fit.alpha:.3g}")
    losses = []
    for _ in range(301):
        fit.step()
        losses.append(fit.mismatch.mean())
    torch.cuda.synchronize()
    losses = np.array([float(x) for x in losses])
    _say(f"loss {losses[0]:.4e} -> {losses[-1]:.4e} ({losses[0] / losses[-1]:.2f}x)")
    assert np.all(np.diff(losses) < 0), np.nonzero(np.diff(losses) >= 0)
    assert losses[-1] < 0.5 * losses[0]


def test_autograd_wrappers(gpu, lam0):
    """LogLike returns ln L and, through torch.autograd, the weighted gradient of the same fused call;
    Mismatch returns the mismatches and, for an equally weighted loss, the adjoint gradient over the
    coefficients recomputed in its backward."""
    import torch
    from paper_2302_05329_amd import api
    cfg = W.config2(n=16)
    th = torch.as_tensor(cfg["theta"], device="cuda").requires_grad_(True)
    _say("autograd LogLike n=16 nb=16225")
    lnl = api.LogLike.apply(th, P, cfg["grid"], lam0, cfg["data"], cfg["inv_psd"])
    wts = torch.linspace(0.5, 2.0, 16, dtype=torch.float64, device="cuda")
    (lnl * wts).sum().backward()
    ref_l, ref_g, _ = api.loglike_and_grad(cfg["theta"], P, cfg["grid"], lam0, cfg["data"], cfg["inv_psd"])
    torch.cuda.synchronize()
    assert torch.equal(lnl.detach(), ref_l)
    assert torch.equal(th.grad, wts[:, None] * ref_g)
    c4 = W.config4(n=4)
    targets = np.stack([O.waveform(t, P, c4["lam_star"], c4["grid"].as_tuple()) for t in c4["theta"]])
    lam = torch.as_tensor(lam0, device="cuda").requires_grad_(True)
    _say("autograd Mismatch nt=4 nb=65536")
    mm = api.Mismatch.apply(lam, c4["theta"], P, c4["grid"], targets, c4["inv_psd"])
    mm.mean().backward()
    ref_m, ref_d, _ = api.mismatch_grad(c4["theta"], P, c4["grid"], lam0, targets, c4["inv_psd"])
    torch.cuda.synchronize()
    assert torch.equal(mm.detach(), ref_m)
    assert torch.allclose(lam.grad, ref_d / 4, rtol=1e-14, atol=0)
    lam.grad = None
    mm = api.Mismatch.apply(lam, c4["theta"], P, c4["grid"], targets, c4["inv_psd"])
    with pytest.raises(NotImplementedError):
        (mm * torch.arange(4, dtype=torch.float64, device="cuda")).sum().backward()


def test_work_ordering_every_point(gpu, lam0):
    """Batches of >= 16384 points are visited through a work-sorted permutation; every point of a
    ragged batch of 16411 (with invalid rows) must get the result it gets in index-order
    sub-batches (< 16384 points, no permutation): value, gradient and Fisher matrix.  The
    sub-batches cut the bins into more chunks, so sums are regrouped: equal to rounding."""
    import torch
    from paper_2302_05329_amd import api
    n = 16411
    rows = W.draw_sources(n, 4242, d_range=(100, 2000), tc_range=(-0.1, 0.1), phic_random=True)
    bad = [3, 9000, 16410]
    rows[bad[0], 0] = -1.0
    rows[bad[1], 3] = 2.0
    rows[bad[2], 1] = 0.0
    grid = W.Grid(20.0, 0.125, 16225)
    psd = W.psd_aligo_zdhp_fit(grid.freqs())
    data = W.complex_noise(psd, grid.df, 4243)
    lam = torch.as_tensor(lam0, device="cuda")
    th = torch.as_tensor(rows, device="cuda")
    d = torch.view_as_real(torch.as_tensor(data, device="cuda")).contiguous()
    ip = torch.as_tensor(1.0 / psd, device="cuda")
    cuts = [(0, 8000), (8000, 16000), (16000, n)]
    _say(f"work ordering n={n} nb={grid.n_bins}: lnL value, lnL + gradient, Fisher")
    for want_grad in (False, True):
        ws1, ws2 = api.Workspace(), api.Workspace()
        lnl, grad, st = api.loglike_and_grad(th, P, grid, lam, d, ip, want_grad=want_grad, ws=ws1)
        parts = [api.loglike_and_grad(th[a:b].contiguous(), P, grid, lam, d, ip, want_grad=want_grad, ws=ws2)
                 for a, b in cuts]
        torch.cuda.synchronize()
        lnl, st = lnl.cpu().numpy(), st.cpu().numpy()
        lnl_r = np.concatenate([p[0].cpu().numpy() for p in parts])
        st_r = np.concatenate([p[2].cpu().numpy() for p in parts])
        assert np.array_equal(st, st_r) and sorted(np.nonzero(st)[0].tolist()) == bad
        ok = st == 0
        assert np.all(np.isnan(lnl[~ok]))
        assert np.all(np.abs(lnl[ok] - lnl_r[ok]) <= 1e-12 * np.maximum(1.0, np.abs(lnl_r[ok])))
        if want_grad:
            grad = grad.cpu().numpy()
            grad_r = np.concatenate([p[1].cpu().numpy() for p in parts])
            assert np.all(np.isnan(grad[~ok]))
            dg = np.max(np.abs(grad[ok] - grad_r[ok]), axis=1) / np.max(np.abs(grad_r[ok]), axis=1)
            assert np.all(dg <= 1e-11), float(dg.max())
    ws1, ws2 = api.Workspace(), api.Workspace()
    F, st = api.fisher(th, P, grid, lam, ip, ws=ws1)
    parts = [api.fisher(th[a:b].contiguous(), P, grid, lam, ip, ws=ws2) for a, b in cuts]
    torch.cuda.synchronize()
    F, st = F.cpu().numpy(), st.cpu().numpy()
    F_r = np.concatenate([p[0].cpu().numpy() for p in parts])
    ok = st == 0
    assert np.all(np.isnan(F[~ok]))
    diag = np.abs(np.diagonal(F_r[ok], axis1=1, axis2=2))
    scale = np.sqrt(diag[:, :, None] * diag[:, None, :])
    assert np.all(np.abs(F[ok] - F_r[ok]) <= 1e-12 * scale)


def test_gamma2_above_one_branch(gpu):
    """A coefficient table with gamma2 > 1 for every source: the amplitude peak takes the
    no-stationary-point branch on both sides.  Strain, ln L with gradient, and Fisher matrices
    against the oracle."""
    import torch
    from paper_2302_05329_amd import api
    lam = W.lambda_gamma2_above_one()
    rows = W.draw_sources(12, 91, d_range=(100, 2000), tc_range=(-0.1, 0.1), phic_random=True)
    grid = W.Grid(20.0, 0.125, 16225)
    g = grid.as_tuple()
    psd = W.psd_aligo_zdhp_fit(grid.freqs())
    ip = 1.0 / psd
    data = W.complex_noise(psd, grid.df, 92) + O.waveform(rows[0], P, lam, g)
    _say(f"gamma2 > 1 table n=12 nb={g[2]}")
    h, st = api.waveform_eval(rows, P, grid, lam)
    lnl, grad, st2 = api.loglike_and_grad(rows, P, grid, lam, data, ip)
    F, st3 = api.fisher(rows, P, grid, lam, ip)
    torch.cuda.synchronize()
    h, lnl, grad, F = h.cpu().numpy(), lnl.cpu().numpy(), grad.cpu().numpy(), F.cpu().numpy()
    valid = 0
    for i, th in enumerate(rows):
        m = O.Model(th, P, lam, g[4])
        assert m.p["gamma2"] > 1.0
        if not m.valid:
            assert int(st[i]) != 0 and np.all(np.isnan(h[i]))
            continue
        valid += 1
        ref = O.waveform(th, P, lam, g)
        assert _strain_err(h[i], ref) <= 1e-10, i
        ref_l = O.loglike(th, P, lam, g, data, ip)
        assert abs(lnl[i] - ref_l) <= lnl_tolerance(th, P, lam, g, data, ip), (i, lnl[i], ref_l)
        Fr = O.fisher(th, P, lam, g, ip)
        r = data - ref
        scale = np.sqrt(O.inner(r, r, ip, g[1]) * np.diag(Fr))
        gref = O.loglike_grad(th, P, lam, g, data, ip)
        assert np.all(np.abs(grad[i] - gref) <= 1e-10 * scale), (i, grad[i], gref)
        fs = np.sqrt(np.outer(np.diag(Fr), np.diag(Fr)))
        assert np.all(np.abs(F[i] - Fr) <= 1e-10 * fs), i
    assert valid >= 8


def _mismatch_case(log2n, nt, seed, lam0):
    cfg = W.config4(n=nt, seed=seed, n_fft=1 << log2n)
    g = cfg["grid"].as_tuple()
    targets = np.stack([O.waveform(t, P, cfg["lam_star"], g) for t in cfg["theta"]])
    return cfg, g, targets


@pytest.mark.parametrize("log2n", [6, 7, 10, 11, 13, 15])
def test_mismatch_lengths_power_of_two(gpu, lam0, log2n):
    """Every supported FFT length (odd and even powers of two, so both the square and the
    2:1 four-step splits) against the oracle: mismatch, lag and the summed gradient; at 2^6 the
    overlap maximum is also taken from the brute-force DFT of the definition."""
    import torch
    cfg, g, targets = _mismatch_case(log2n, 3, 2000 + log2n, lam0)
    th, w = cfg["theta"], cfg["inv_psd"]
    _say(f"mismatch_grad nt=3 nb=2^{log2n}")
    mm, dl, lag = gpu.api.mismatch_grad(th, P, cfg["grid"], lam0, targets, w)
    torch.cuda.synchronize()
    mm, dl, lag = mm.cpu().numpy(), dl.cpu().numpy(), lag.cpu().numpy()
    gsum = np.zeros(209)
    wk = 4 * g[1] * w
    for i in range(len(th)):
        m_ref, j_ref, gap, gref = O.mismatch_grad_lambda(th[i], P, lam0, g, targets[i], wk)
        assert gap > 1e-12, "ambiguous lag in the fixture"
        assert lag[i] == j_ref, (lag[i], j_ref)
        assert abs(mm[i] - m_ref) <= 1e-12, (mm[i], m_ref)
        gsum += gref
        if log2n == 6:
            h = O.waveform(th[i], P, lam0, g)
            z = np.abs(O.overlap_series_bruteforce(h, targets[i], wk))
            a = math.fsum((wk * np.abs(h) ** 2).tolist())
            b = math.fsum((wk * np.abs(targets[i]) ** 2).tolist())
            assert lag[i] == int(np.argmax(z))
            assert abs(mm[i] - (1.0 - z.max() / math.sqrt(a * b))) <= 1e-12
    assert np.max(np.abs(dl - gsum)) <= 1e-8 * np.max(np.abs(gsum)), np.max(np.abs(dl - gsum)) / np.max(np.abs(gsum))


def test_mismatch_gradient_vs_gpu_finite_differences(gpu, lam0):
    """2 targets x 2^10 bins: the adjoint gradient against central differences of the GPU's own
    summed mismatch (the lag is the arg-max at every evaluation; the fixture keeps it unambiguous)."""
    import torch
    cfg, g, targets = _mismatch_case(10, 2, 2101, lam0)
    th, w = cfg["theta"], cfg["inv_psd"]
    _say("mismatch_grad finite differences nt=2 nb=2^10")
    mm, dl, lag = gpu.api.mismatch_grad(th, P, cfg["grid"], lam0, targets, w)
    torch.cuda.synchronize()
    dl, lag0 = dl.cpu().numpy(), lag.cpu().numpy()
    assert np.all(mm.cpu().numpy() > 1e-8)
    scale = np.max(np.abs(dl * np.abs(lam0)))
    for i in [0, 14, 47, 60, 77, 100, 133, 160, 171, 190, 208]:
        h = 1e-6 * abs(lam0[i])
        vals = []
        for sgn in (1.0, -1.0):
            lv = lam0.copy()
            lv[i] += sgn * h
            m, _, lg = gpu.api.mismatch_grad(th, P, cfg["grid"], lv, targets, w, want_grad=False)
            torch.cuda.synchronize()
            assert np.array_equal(lg.cpu().numpy(), lag0)
            vals.append(math.fsum(m.cpu().numpy().tolist()))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - dl[i]) <= 1e-5 * scale / abs(lam0[i]) + 1e-6 * abs(dl[i]), (i, fd, dl[i])


def test_mismatch_rejects_unsupported_lengths(gpu, lam0):
    from paper_2302_05329_amd import _lib as L
    for n in (32, 1000, 1 << 17):
        cfg = W.config4(n=1, n_fft=n)
        targets = np.zeros((1, n), dtype=np.complex128)
        with pytest.raises(L.PdError, match="FFT length"):
            gpu.api.mismatch_grad(cfg["theta"], P, cfg["grid"], lam0, targets, cfg["inv_psd"])
