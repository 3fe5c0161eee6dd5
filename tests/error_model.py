"""Rounding bounds for quantities computed in FP64 on two independent paths (GPU and oracle).

Log-likelihood.  ln L = (d|h) - (h|h)/2 with h_k = A_k exp(-i Psi_k).  To first order a phase
error dPsi_k and a relative amplitude error eA_k change it by

    d lnL = sum_k w_k [ Im(conj(d_k) h_k) dPsi_k + Re(conj(d_k - h_k) h_k) eA_k ]

(a common phase leaves (h|h) unchanged, so the phase term carries |d_k|, not |d_k - h_k|), and

    |d lnL| <= sum_k w_k |d_k| |h_k| |dPsi_k| + sum_k w_k (|d_k| + |h_k|) |h_k| |eA_k|.

Phase: each side assembles Psi_k in FP64 from summands of magnitude up to
S_k = max(|Phi(Mf_k)|, |t0 (Mf_k - Mf_ref)|, |Phi(Mf_ref)|, |2 pi f_k tc|, 2 |phic|)
(the three-region phase, the time and phase alignment, the tc and phic terms), so each side's
phase is good to about ulp(S_k): |dPsi_k| <= C_PSI ulp(S_k), C_PSI = 2 (one ulp per side).

Amplitude: a product of a few rounded factors on each side, |eA_k| <= C_AMP 2^-53 with
C_AMP = 8 (four roundings per side); plus, on the GPU, the merger-ringdown exponential
exp(-c (Mf - f_RD)) advances along a lane's bins (64 apart) by a rounded ratio and one rounded
multiply per step, a coherent drift of at most C_REC = 3 units of 2^-53 per step, with at most
n_k = (k - k_peak) / 64 steps at bin k past the first bin k_peak of that amplitude region.

    tol = 1e-10 + C_PSI sum_k w_k |d_k| |h_k| ulp(S_k)
                + 2^-53 sum_k w_k (|d_k| + |h_k|) |h_k| (C_AMP + C_REC n_k)

The sums over bins are the coherent worst case; 1e-10 is the absolute floor of the ln L parity target.

Network.  A site's strain is the model at effective parameters (D/|c|, tc + dt, phic + arg(c)/2),
so the network bound is the sum over sites of the bound above with S_k also covering
|2 pi f_k (tc + dt)|.  The network Fisher matrix is sum_d J_d^T F_d J_d; with each single-site
F_d good to 1e-10 sqrt(F_d,aa F_d,bb) (the single-detector bar) the propagated bound is
|dF_pq| <= 1e-10 sum_d u_d,p u_d,q, u_d,p = sum_a |J_d,ap| sqrt(F_d,aa).
"""
import math

import numpy as np

from oracle import network_oracle as N
from oracle import phenomd_oracle as O

C_PSI = 2.0
C_AMP = 8.0
C_REC = 3.0
FLOOR = 1e-10


def _terms(theta, param, lam, grid, data, inv_psd, extra_phase=None):
    """(E_psi, E_amp) of one detector: the two sums of the bound, constants included, for the
    model at theta (7) against `data`, with |extra_phase| (per active bin) joining the summands."""
    theta = np.asarray(theta, dtype=np.float64)
    model = O.Model(theta, param, lam, grid[4])
    amp, phase, act = O.amp_phase(theta, param, lam, grid)
    f = O.grid_freqs(grid)[act]
    mf = model.Ms * f
    s = O.source(theta, param)
    summands = [np.abs(model.phase_raw(mf)), np.abs(model.t0 * (mf - model.mf_ref)),
                np.full(mf.shape, abs(model.phi_ref)), np.abs(2.0 * math.pi * f * s["tc"]),
                np.full(mf.shape, 2.0 * abs(s["phic"]))]
    if extra_phase is not None:
        summands.append(np.abs(extra_phase))
    S = np.max(np.stack(summands), axis=0)
    w = 4.0 * grid[1] * np.asarray(inv_psd)[act]
    dk = np.abs(np.asarray(data)[act])
    k = np.nonzero(act)[0]
    mrd = mf >= np.real(model.f_peak)
    n_rec = np.zeros(k.shape)
    if np.any(mrd):
        n_rec[mrd] = (k[mrd] - k[mrd][0]) // 64
    e_psi = C_PSI * float(np.sum(w * dk * amp * np.spacing(S)))
    e_amp = 2.0**-53 * float(np.sum(w * (dk + amp) * amp * (C_AMP + C_REC * n_rec)))
    return e_psi, e_amp


def lnl_tolerance(theta, param, lam, grid, data, inv_psd):
    """Bound on |ln L(GPU) - ln L(oracle)| for one detector."""
    e_psi, e_amp = _terms(theta, param, lam, grid, data, inv_psd)
    return FLOOR + e_psi + e_amp


def effective_rows(theta11, param, dets, gmst):
    """Per site, the 7 single-detector parameters whose strain is the site's strain:
    (D / |c|, tc + dt, phic + arg(c) / 2) with c = F+ (1 + cos^2 iota)/2 - i Fx cos iota;
    None for a site with no response (c = 0), which records no signal."""
    theta11 = np.asarray(theta11, dtype=np.float64)
    iota, psi, alpha, delta = theta11[7:11]
    rows = []
    for det in dets:
        fp, fx = N.antenna(det, alpha, delta, psi, gmst)
        c = complex(fp * (1.0 + math.cos(iota) ** 2) / 2.0, -fx * math.cos(iota))
        if c == 0:
            rows.append(None)
            continue
        r = theta11[:7].copy()
        dist_index = 4
        if param == O.PARAM_LNMC_ETA_LND:
            r[dist_index] -= math.log(abs(c))
        else:
            r[dist_index] /= abs(c)
        r[5] += N.delay(det, alpha, delta, gmst)
        r[6] += 0.5 * math.atan2(c.imag, c.real)
        rows.append(r)
    return rows


def network_lnl_tolerance(theta11, param, lam, grid, dets, data, inv_psd, gmst):
    """Bound on the network ln L difference: the single-detector bound summed over sites, with the
    site's delay term among the phase summands."""
    f = O.grid_freqs(grid)
    tol = FLOOR
    for k, (det, row) in enumerate(zip(dets, effective_rows(theta11, param, dets, gmst))):
        if row is None:
            continue
        act = O.active_mask(row, param, grid)
        extra = 2.0 * math.pi * f[act] * row[5]
        e_psi, e_amp = _terms(row, param, lam, grid, data[k], inv_psd[k], extra_phase=extra)
        tol += e_psi + e_amp
    return tol


def network_fisher_tolerance(theta11, param, lam, grid, dets, inv_psd, gmst):
    """[11][11] bound on |F_network(GPU) - F_network(oracle)| propagated from the single-site
    Fisher bar through the Jacobian of the effective parameters (central differences)."""
    theta11 = np.asarray(theta11, dtype=np.float64)
    tol = np.zeros((11, 11))
    for k, det in enumerate(dets):
        row = effective_rows(theta11, param, [det], gmst)[0]
        if row is None:
            continue
        F = O.fisher(row, param, lam, grid, inv_psd[k])
        J = np.zeros((7, 11))
        for p in range(11):
            e = 1e-6 * max(abs(theta11[p]), 1e-2)
            tp, tm = theta11.copy(), theta11.copy()
            tp[p] += e
            tm[p] -= e
            J[:, p] = (effective_rows(tp, param, [det], gmst)[0] - effective_rows(tm, param, [det], gmst)[0]) / (2 * e)
        u = np.abs(J).T @ np.sqrt(np.abs(np.diag(F)))
        tol += FLOOR * np.outer(u, u)
    return tol
