"""Precision sweep shaped like the paper's Fig. 1: the GPU strain against the FP64 oracle over
masses (1, 100) Msun and spins (-1, 1) on a 79361-bin grid (32-1024 Hz, df = 0.0125 Hz), where the
inspiral phase reaches ~1e4 rad.  In place of the paper's comparison of two IMRPhenomD codes, the
mismatch of the GPU waveform against the oracle's is mapped over total mass and effective spin."""
import math
import sys

import numpy as np
import pytest

from oracle import phenomd_oracle as O
from paper_2302_05329_amd import workloads as W

P = O.PARAM_M1M2


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _mismatch(h1, h2, inv_psd, df):
    """1 - (h1|h2) / sqrt((h1|h1)(h2|h2)) without time or phase maximisation (an upper bound on the
    maximised mismatch of Eqs. 2-4), in a cancellation-free form: with d = h1 - h2, s = h1 + h2,
    a = |h1|, b = |h2|:  M = ((d|d) - (s|d)^2 / (a + b)^2) / (2 a b)."""
    d = h1 - h2
    a = math.sqrt(O.inner(h1, h1, inv_psd, df))
    b = math.sqrt(O.inner(h2, h2, inv_psd, df))
    dd = O.inner(d, d, inv_psd, df)
    sd = O.inner(h1 + h2, d, inv_psd, df)
    return max(0.0, (dd - sd * sd / (a + b) ** 2) / (2.0 * a * b))


def test_mismatch_form_is_exact():
    """The cancellation-free mismatch agrees with the direct formula where the latter is
    accurate (mismatch ~1e-3) and resolves a 1e-12 relative perturbation where it is not."""
    rng = np.random.default_rng(1)
    n = 2000
    ip = rng.uniform(0.5, 2.0, n)
    h = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    h2 = h * np.exp(1j * 0.05 * rng.standard_normal(n))
    direct = 1 - O.inner(h, h2, ip, 1.0) / math.sqrt(O.inner(h, h, ip, 1.0) * O.inner(h2, h2, ip, 1.0))
    assert _mismatch(h, h2, ip, 1.0) == pytest.approx(direct, rel=1e-9)
    eps = 1e-12 * (rng.standard_normal(n) + 1j * rng.standard_normal(n))
    m = _mismatch(h, h + eps * np.abs(h), ip, 1.0)
    assert 1e-27 < m < 1e-23


@pytest.mark.gpu
def test_fig1_sweep_against_oracle(gpu, lam0):
    import torch
    cfg = W.fig1_sweep()
    th, grid, ip = cfg["theta"], cfg["grid"], cfg["inv_psd"]
    g = grid.as_tuple()
    n = th.shape[0]
    _say(f"Fig. 1 sweep: waveform_eval n={n} nb={grid.n_bins} (one call, 12.7 GB of strain)")
    h, st = gpu.api.waveform_eval(th, P, grid, lam0)
    torch.cuda.synchronize()
    # sources outside the model's valid region (a large mass ratio with the heavier spin near 1
    # drives the closed-form final spin to 1 or above) are flagged on both sides, and only those
    st = st.cpu().numpy()
    with np.errstate(invalid="ignore"):
        bad_ref = sorted(i for i in range(n) if not O.Model(th[i], P, lam0, g[4]).valid)
    assert np.nonzero(st)[0].tolist() == bad_ref
    assert np.all(st[bad_ref] == -2) and len(bad_ref) < n // 100
    finite = torch.isfinite(torch.view_as_real(h)).flatten(1).all(dim=1).cpu().numpy()
    assert np.array_equal(finite, st == 0)
    _say(f"  {len(bad_ref)} sources outside the valid region, flagged identically")
    mt = th[:, 0] + th[:, 1]
    chi_eff = (th[:, 0] * th[:, 2] + th[:, 1] * th[:, 3]) / mt
    chi_eff[bad_ref] = 0.0
    order = np.array([i for i in np.argsort(mt) if st[i] == 0])
    q = np.where(st == 0, th[:, 0] / th[:, 1], 1.0)
    rows = set(order[np.linspace(0, order.size - 1, 56).astype(int)].tolist())
    rows |= {int(np.argmin(chi_eff)), int(np.argmax(chi_eff)), int(np.argmax(q)), int(np.argmin(q))}
    rows = sorted(rows)
    hs = h[torch.as_tensor(rows, device=h.device)].cpu().numpy()
    del h
    mm = []
    for r, hg in zip(rows, hs):
        ref = O.waveform(th[r], P, lam0, g)
        err = np.max(np.abs(hg - ref)) / np.max(np.abs(ref))
        assert err <= 1e-10, (r, th[r], err)
        assert np.all(hg[ref == 0] == 0), r
        mm.append(_mismatch(hg, ref, ip, g[1]))
    mm = np.array(mm)
    edges = [0, 25, 50, 100, 150, 201]
    for lo, hi in zip(edges[:-1], edges[1:]):
        sel = [(lo <= mt[r] < hi) for r in rows]
        if any(sel):
            _say(f"  total mass {lo:3d}-{hi:3d} Msun: {sum(sel):2d} points, mismatch max {mm[sel].max():.2e} "
                 f"median {np.median(mm[sel]):.2e}")
    ext = [int(np.argmin(chi_eff)), int(np.argmax(chi_eff))]
    _say(f"  effective spin {chi_eff[ext[0]]:.2f} and {chi_eff[ext[1]]:.2f}: mismatch "
         f"{mm[rows.index(ext[0])]:.2e} and {mm[rows.index(ext[1])]:.2e}; max over the sample {mm.max():.2e}")
    assert mm.max() < 1e-16
