"""Pins of the detector-network oracle (antenna patterns, delays, network likelihood)."""
import math

import numpy as np
import pytest

from oracle import network_oracle as N
from oracle import phenomd_oracle as O
from paper_2302_05329_amd import workloads as W

P = O.PARAM_M1M2


def test_site_geometry_inputs():
    """The site descriptions: unit, orthogonal arms, vertices on the Earth's surface, and the
    inter-site light travel times of the LIGO-Virgo network (10.0, 27.3 and 26.4 ms)."""
    for v, x, y in W.DETECTORS.values():
        v, x, y = map(np.asarray, (v, x, y))
        assert abs(np.linalg.norm(x) - 1) < 1e-9 and abs(np.linalg.norm(y) - 1) < 1e-9
        assert abs(x @ y) < 1e-6
        assert 6.35e6 < np.linalg.norm(v) < 6.39e6
    d = {k: np.asarray(v[0]) for k, v in W.DETECTORS.items()}
    for a, b, ms in (("H1", "L1", 10.01), ("H1", "V1", 27.29), ("L1", "V1", 26.45)):
        assert abs(np.linalg.norm(d[a] - d[b]) / N.C_SI * 1e3 - ms) < 0.01


def test_antenna_pattern_sum_closed_form():
    """Arms along x and y at the origin, gmst = 0: a source at polar angle t and azimuth p in that
    frame has F+^2 + Fx^2 = (1 + cos^2 t)^2 cos^2(2p) / 4 + cos^2 t sin^2(2p), for every psi."""
    det = ((0.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0))
    rng = np.random.default_rng(3)
    for _ in range(50):
        t, p, psi = rng.uniform(0, math.pi), rng.uniform(0, 2 * math.pi), rng.uniform(0, math.pi)
        fp, fx = N.antenna(det, p, math.pi / 2 - t, psi, 0.0)
        expect = (1 + math.cos(t) ** 2) ** 2 * math.cos(2 * p) ** 2 / 4 + math.cos(t) ** 2 * math.sin(2 * p) ** 2
        assert fp * fp + fx * fx == pytest.approx(expect, abs=1e-14)
    # overhead the response is optimal
    fp, fx = N.antenna(det, 0.3, math.pi / 2, 0.0, 0.0)
    assert fp * fp + fx * fx == pytest.approx(1.0, abs=1e-14)


def test_polarisation_rotation():
    """Rotating psi by pi/4 turns F+ into Fx; F+^2 + Fx^2 does not depend on psi."""
    rng = np.random.default_rng(4)
    for det in W.DETECTORS.values():
        for _ in range(10):
            a, d, psi, g = rng.uniform(0, 2 * math.pi), rng.uniform(-1.5, 1.5), rng.uniform(0, math.pi), 0.7
            fp, fx = N.antenna(det, a, d, psi, g)
            fp2, _ = N.antenna(det, a, d, psi + math.pi / 4, g)
            fp3, fx3 = N.antenna(det, a, d, psi + 0.9, g)
            assert fp2 == pytest.approx(fx, abs=1e-14)
            assert fp3 * fp3 + fx3 * fx3 == pytest.approx(fp * fp + fx * fx, abs=1e-14)


def test_delays_against_baselines():
    """Delay differences between two sites never exceed their baseline over c, and reach it for a
    source along the baseline; a source in the plane perpendicular to it arrives at once."""
    h, l = W.DETECTORS["H1"], W.DETECTORS["L1"]
    base = np.asarray(l[0]) - np.asarray(h[0])
    rng = np.random.default_rng(5)
    for _ in range(200):
        a, d = rng.uniform(0, 2 * math.pi), math.asin(rng.uniform(-1, 1))
        assert abs(N.delay(l, a, d, 0.0) - N.delay(h, a, d, 0.0)) <= np.linalg.norm(base) / N.C_SI * (1 + 1e-12)
    u = base / np.linalg.norm(base)
    a, d = math.atan2(u[1], u[0]), math.asin(u[2])
    # a source in direction u: the wave reaches L1 (further along u) first
    assert N.delay(l, a, d, 0.0) - N.delay(h, a, d, 0.0) == pytest.approx(-np.linalg.norm(base) / N.C_SI, rel=1e-12)
    perp = np.cross(u, [0.0, 0.0, 1.0])
    perp /= np.linalg.norm(perp)
    a, d = math.atan2(perp[1], perp[0]), math.asin(perp[2])
    assert abs(N.delay(l, a, d, 0.0) - N.delay(h, a, d, 0.0)) < 1e-16


def _problem(lam0, dets, seed, n_bins=2001, df=0.25):
    grid = W.Grid(20.0, df, n_bins, 20.0, 20.0)
    g = grid.as_tuple()
    psd = W.psd_aligo_zdhp_fit(grid.freqs())
    th = W.network_sources(1, seed)[0]
    th[4] = 400.0
    data = np.stack([W.complex_noise(psd, df, seed + k) for k in range(len(dets))])
    for k, det in enumerate(dets):
        data[k] = data[k] + N.strain(th * np.r_[1.01, 0.99, np.ones(9)], P, lam0, g, det, 0.4)
    return th, g, data, np.stack([1 / psd] * len(dets))


def test_single_optimal_detector_reduces_to_one_detector_likelihood(lam0):
    """A detector at the geocentre with the source overhead, face-on and psi chosen so that F+ = 1,
    Fx = 0 sees exactly the single-detector strain and likelihood."""
    det = ((0.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0))
    # overhead at gmst = 0: n = z and X = (sin(alpha + psi), -cos(alpha + psi), 0), so that
    # F+ = -cos 2(alpha + psi) and Fx = -sin 2(alpha + psi): psi = pi/2 - alpha gives F+ = 1
    a = 0.8
    fp, fx = N.antenna(det, a, math.pi / 2, math.pi / 2 - a, 0.0)
    assert fp == pytest.approx(1.0, abs=1e-15) and abs(fx) < 1e-15
    th, g, data, ip = _problem(lam0, [det], 21)
    th[7:11] = (0.0, math.pi / 2 - a, a, math.pi / 2)
    h = N.strain(th, P, lam0, g, det, 0.0)
    h0 = O.waveform(th[:7], P, lam0, g)
    assert np.max(np.abs(h - h0)) <= 1e-15 * np.max(np.abs(h0))
    assert N.loglike(th, P, lam0, g, [det], data, ip, 0.0) == pytest.approx(
        O.loglike(th[:7], P, lam0, g, data[0], ip[0]), rel=1e-13)


def test_detector_strain_is_the_model_at_effective_parameters(lam0):
    """The identity the network kernels are built on: h_d equals the single-detector strain with
    D -> D / |c|, tc -> tc + dt and phic -> phic + arg(c) / 2, c = F+ (1 + cos^2 i)/2 - i Fx cos i."""
    g = W.Grid(20.0, 0.25, 2001, 20.0, 20.0).as_tuple()
    for k, det in enumerate(W.DETECTORS.values()):
        th = W.network_sources(1, 30 + k)[0]
        iota, psi, a, d = th[7:11]
        fp, fx = N.antenna(det, a, d, psi, 1.1)
        c = fp * (1 + math.cos(iota) ** 2) / 2 - 1j * fx * math.cos(iota)
        eff = th[:7].copy()
        eff[4] = th[4] / abs(c)
        eff[5] = th[5] + N.delay(det, a, d, 1.1)
        eff[6] = th[6] + np.angle(c) / 2
        h = N.strain(th, P, lam0, g, det, 1.1)
        he = O.waveform(eff, P, lam0, g)
        assert np.max(np.abs(h - he)) <= 1e-9 * np.max(np.abs(h)), k


def test_network_gradient_against_central_differences(lam0):
    dets = [W.DETECTORS["H1"], W.DETECTORS["L1"], W.DETECTORS["V1"]]
    th, g, data, ip = _problem(lam0, dets, 41)
    grad = N.loglike_grad(th, P, lam0, g, dets, data, ip, 0.4)
    for p in range(11):
        h = 1e-6 * max(abs(th[p]), 1e-2) if p < 7 else 1e-6
        tp, tm = th.copy(), th.copy()
        tp[p] += h
        tm[p] -= h
        fd = (N.loglike(tp, P, lam0, g, dets, data, ip, 0.4) - N.loglike(tm, P, lam0, g, dets, data, ip, 0.4)) / (2 * h)
        assert abs(fd - grad[p]) <= 1e-5 * max(abs(grad[p]), 1.0), (p, fd, grad[p])


def test_network_fisher_is_negative_hessian_of_noise_free_loglike(lam0):
    """F = -Hessian of the network ln L at theta0 for noise-free data (Richardson-extrapolated
    central differences of the gradient); symmetric positive definite."""
    dets = [W.DETECTORS["H1"], W.DETECTORS["L1"], W.DETECTORS["V1"]]
    grid = W.Grid(20.0, 0.25, 2001, 20.0, 20.0)
    g = grid.as_tuple()
    psd = W.psd_aligo_zdhp_fit(grid.freqs())
    ip = np.stack([1 / psd] * 3)
    th = W.network_sources(1, 51)[0]
    th[4] = 400.0
    data = np.stack([N.strain(th, P, lam0, g, det, 0.9) for det in dets])
    F = N.fisher(th, P, lam0, g, dets, ip, 0.9)
    assert np.array_equal(F, F.T)
    assert np.all(np.linalg.eigvalsh(F / np.sqrt(np.outer(np.diag(F), np.diag(F)))) > 0)

    def central(p, h):
        tp, tm = th.copy(), th.copy()
        tp[p] += h
        tm[p] -= h
        return (N.loglike_grad(tp, P, lam0, g, dets, data, ip, 0.9) - N.loglike_grad(tm, P, lam0, g, dets, data, ip, 0.9)) / (2 * h)

    H = np.zeros((11, 11))
    for p in range(11):
        h = 1e-5 * max(abs(th[p]), 1.0)
        H[p] = (4.0 * central(p, h / 2) - central(p, h)) / 3.0
    scale = np.sqrt(np.outer(np.diag(F), np.diag(F)))
    assert np.max(np.abs(-H - F) / scale) < 1e-6


def test_network_fisher_one_optimal_site_is_the_single_detector_fisher(lam0):
    det = ((0.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0))
    grid = W.Grid(20.0, 0.25, 2001, 20.0, 20.0)
    g = grid.as_tuple()
    w = 1 / W.psd_aligo_zdhp_fit(grid.freqs())
    th = W.network_sources(1, 52)[0]
    a = 0.8
    th[7:11] = (0.0, math.pi / 2 - a, a, math.pi / 2)
    F = N.fisher(th, P, lam0, g, [det], w[None], 0.0)
    F7 = O.fisher(th[:7], P, lam0, g, w)
    assert np.max(np.abs(F[:7, :7] - F7) / np.sqrt(np.outer(np.diag(F7), np.diag(F7)))) < 1e-12
