"""Template-bank overlaps on the FP64 matrix cores against the oracle (GPU).

Tolerance: both sides accumulate ~10^3-10^4 FP64 products per entry in different orders; the
bound is 1e-11 sqrt((h|h)(d|d)), several hundred times the rounding of such a sum.
"""
import math
import sys

import numpy as np
import pytest

from oracle import phenomd_oracle as O
from paper_2302_05329_amd import workloads as W

pytestmark = pytest.mark.gpu
P = O.PARAM_M1M2


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _streams(grid, psd, ns, seed, inj=None):
    out = [W.complex_noise(psd, grid.df, seed + s) for s in range(ns)]
    if inj is not None:
        out[0] = out[0] + inj
    return np.stack(out)


def _check(O_gpu, hh_gpu, thetas, streams, lam, g, ip, rows):
    for i in rows:
        ref, hh = O.overlaps(thetas[i], P, lam, g, streams, ip)
        assert abs(hh_gpu[i] - hh) <= 1e-12 * max(hh, 1e-300), (i, hh_gpu[i], hh)
        for s in range(len(streams)):
            dd = O.inner(streams[s], streams[s], ip, g[1])
            tol = 1e-11 * math.sqrt(hh * dd) + 1e-300
            assert abs(O_gpu[i, s] - ref[s]) <= tol, (i, s, O_gpu[i, s], ref[s], tol)


@pytest.mark.parametrize("nt,ns,nb", [(1, 1, 257), (70, 5, 4017), (64, 64, 1000), (130, 9, 2049)])
def test_overlap_parity_ragged(gpu, lam0, nt, ns, nb):
    grid = W.Grid(20.0, 0.25, nb)
    g = grid.as_tuple()
    psd = W.psd_aligo_zdhp_fit(grid.freqs())
    ip = 1.0 / psd
    rows = W.draw_sources(nt, 300 + nt)
    rows = rows[np.argsort(rows[:, 0] + rows[:, 1])]
    inj = O.waveform(rows[nt // 2], P, lam0, g)
    streams = _streams(grid, psd, ns, 400, inj)
    _say(f"overlap nt={nt} ns={ns} nb={nb}")
    Og, hh, st = gpu.api.overlap(rows, P, grid, lam0, streams, ip)
    Og, hh, st = Og.cpu().numpy(), hh.cpu().numpy(), st.cpu().numpy()
    assert np.all(st == 0)
    check_rows = range(nt) if nt * ns <= 640 else sorted({0, nt - 1, nt // 2, 63 % nt, 64 % nt})
    _check(Og, hh, rows, streams, lam0, g, ip, check_rows)


def test_overlap_domain_errors_and_consistency_with_loglike(gpu, lam0):
    import torch
    grid = W.Grid(20.0, 0.125, 3001)
    g = grid.as_tuple()
    psd = W.psd_aligo_zdhp_fit(grid.freqs())
    ip = 1.0 / psd
    rows = W.draw_sources(20, 77)
    rows[3, 2] = 1.5            # |chi1| > 1: domain error
    streams = _streams(grid, psd, 3, 500, O.waveform(rows[0], P, lam0, g))
    _say("overlap domain errors + loglike consistency")
    Og, hh, st = gpu.api.overlap(rows, P, grid, lam0, streams, ip)
    Og, hh, st = Og.cpu().numpy(), hh.cpu().numpy(), st.cpu().numpy()
    assert st[3] != 0 and np.all(np.isnan(Og[3].real)) and np.isnan(hh[3])
    ok = np.array([i for i in range(20) if i != 3])
    assert np.all(st[ok] == 0) and np.all(np.isfinite(Og[ok]))
    for s in range(3):
        lnl, _, _ = gpu.api.loglike_and_grad(rows[ok], P, grid, lam0, streams[s], ip, want_grad=False)
        lnl = lnl.cpu().numpy()
        ref = Og[ok, s].real - 0.5 * hh[ok]
        scale = np.sqrt(hh[ok] * O.inner(streams[s], streams[s], ip, g[1]))
        assert np.all(np.abs(lnl - ref) <= 1e-11 * (scale + hh[ok]))


def test_overlap_full_c2_bank_sampled(gpu, lam0):
    """The benchmark's configuration: 65536 C2 templates (ordered by total mass) against 32
    noise streams on the 16225-bin grid; sampled rows against the oracle."""
    c2 = W.config2()
    grid = c2["grid"]
    g = grid.as_tuple()
    rows = c2["theta"][np.argsort(c2["theta"][:, 0] + c2["theta"][:, 1])]
    psd = W.psd_aligo_zdhp_fit(grid.freqs())
    streams = _streams(grid, psd, 32, 2000)
    _say("overlap full C2 bank 65536 x 32")
    Og, hh, st = gpu.api.overlap(rows, P, grid, lam0, streams, 1.0 / psd)
    Og, hh, st = Og.cpu().numpy(), hh.cpu().numpy(), st.cpu().numpy()
    assert np.all(st == 0) and np.all(np.isfinite(Og))
    rng = np.random.default_rng(3)
    pick = sorted({0, 65535, 32768} | set(int(i) for i in rng.choice(65536, 3, replace=False)))
    _check(Og, hh, rows, streams, lam0, g, 1.0 / psd, pick)
