"""Detector-network response and likelihood: the CPU oracle of the network kernels.

TEST INFRASTRUCTURE ONLY: used by the tests (and nothing in the product path).  It shares no
code with the GPU library.

The paper's sampling example (Sec. 3.3) analyses an injection in the two LIGO detectors, with
inclination, polarisation and sky position held at fixed values, and its Fisher forecasts
(Sec. 3.2) use a network of detectors.  The response of a ground-based interferometer to the
dominant (2,2) mode is not printed in the paper; it is restated here from the standard
definitions (e.g. Schutz 2011, Anderson et al. 2001), with these readings:
  * Earth-fixed Cartesian frame; the source lies in the direction
    n = (cos d cos l, cos d sin l, sin d), l = alpha - gmst (right ascension minus the
    Greenwich sidereal angle at the reference time, which is an input);
  * wave-frame axes a = (sin l, -cos l, 0) and b = n x a; rotated by the polarisation angle:
    X = cos psi a + sin psi b,  Y = -sin psi a + cos psi b;
  * polarisation tensors e+ = X X^T - Y Y^T, ex = X Y^T + Y X^T; detector tensor
    D = (x x^T - y y^T) / 2 for unit arm vectors x, y;  F+ = D : e+,  Fx = D : ex;
  * the signal reaches a site at r later than the geocentre by dt = -(r . n) / c;
  * (2,2)-mode polarisations: h+ = h0 (1 + cos^2 iota) / 2, hx = -i cos iota h0, with h0 the
    face-on, optimally oriented strain of the single-detector model;
  * detector strain h_d(f) = (F+ h+ + Fx hx) exp(-2 pi i f dt_d);
  * network log-likelihood: the sum over detectors of (d_d|h_d) - (h_d|h_d)/2 (Eq. 1 per
    detector, each with its own noise PSD);
  * network Fisher matrix: the sum over detectors of (d_p h_d | d_q h_d) (Eq. 8 per detector).
Parameters: the 7 of the single-detector model (layout `param`) followed by (iota, psi, alpha,
delta).  Pinned by tests/test_network_oracle.py (the antenna-pattern sum against its closed form
for a detector with arms along x and y, polarisation-rotation identities, arrival delays against
the site baselines, reduction to the single-detector likelihood, the effective-parameter identity,
gradients against central differences, the Fisher matrix against minus the Hessian of the
noise-free network likelihood).
"""
import math

import numpy as np

from . import phenomd_oracle as O

C_SI = 299792458.0


def frame(alpha, delta, psi, gmst):
    """(n, X, Y): source direction and the two polarisation axes, Earth-fixed."""
    lam = alpha - gmst
    cd, sd, cl, sl = np.cos(delta), np.sin(delta), np.cos(lam), np.sin(lam)
    n = np.array([cd * cl, cd * sl, sd])
    a = np.array([sl, -cl, 0.0 * sl])
    b = np.cross(n, a)
    cp, sp = np.cos(psi), np.sin(psi)
    return n, cp * a + sp * b, -sp * a + cp * b


def antenna(det, alpha, delta, psi, gmst):
    """(F+, Fx) of a detector (vertex, x arm, y arm)."""
    _, xa, ya = (np.asarray(v, dtype=np.float64) for v in det)
    D = 0.5 * (np.outer(xa, xa) - np.outer(ya, ya))
    _, X, Y = frame(alpha, delta, psi, gmst)
    ep = np.outer(X, X) - np.outer(Y, Y)
    ex = np.outer(X, Y) + np.outer(Y, X)
    return np.sum(D * ep), np.sum(D * ex)


def delay(det, alpha, delta, gmst):
    """Arrival time at the site minus arrival time at the geocentre (s)."""
    r = np.asarray(det[0], dtype=np.float64)
    n, _, _ = frame(alpha, delta, 0.0, gmst)
    return -np.dot(r, n) / C_SI


def strain(theta, param, lam, grid, det, gmst):
    """Complex strain of one detector, h_d(f) = (F+ h+ + Fx hx) exp(-2 pi i f dt)."""
    theta = np.asarray(theta, dtype=np.float64)
    iota, psi, alpha, delta = theta[7:11]
    h0 = O.waveform(theta[:7], param, lam, grid)
    fp, fx = antenna(det, alpha, delta, psi, gmst)
    hp = h0 * (1.0 + math.cos(iota) ** 2) / 2.0
    hx = -1j * math.cos(iota) * h0
    f = O.grid_freqs(grid)
    return (fp * hp + fx * hx) * np.exp(-2j * math.pi * f * delay(det, alpha, delta, gmst))


def loglike(theta, param, lam, grid, dets, data, inv_psd, gmst):
    """Network ln L: sum over detectors of (d|h) - (h|h)/2, each summed with exact rounding."""
    df = grid[1]
    total = 0.0
    for k, det in enumerate(dets):
        h = strain(theta, param, lam, grid, det, gmst)
        total += O.inner(data[k], h, inv_psd[k], df) - 0.5 * O.inner(h, h, inv_psd[k], df)
    return total


def _strain_parts(tp, param, lam, grid, act, det, gmst):
    """Real and imaginary parts of one detector's strain on the active bins, written in
    real-analytic form so that complex-step perturbations of tp pass through:
    with c = F+ (1 + cos^2 iota)/2 - i Fx cos iota = cr + i ci and Phi = Psi + 2 pi f dt,
    Re h_d = A (cr cos Phi + ci sin Phi) and Im h_d = A (ci cos Phi - cr sin Phi)."""
    a_c, ph_c, _ = O.amp_phase(tp[:7], param, lam, grid, act)
    iota, psi, alpha, delta = tp[7:11]
    f = O.grid_freqs(grid)[act]
    fp, fx = antenna(det, alpha, delta, psi, gmst)
    cr = fp * (1.0 + np.cos(iota) ** 2) / 2.0
    ci = -fx * np.cos(iota)
    phi = ph_c + 2.0 * math.pi * f * delay(det, alpha, delta, gmst)
    return a_c * (cr * np.cos(phi) + ci * np.sin(phi)), a_c * (ci * np.cos(phi) - cr * np.sin(phi))


def fisher(theta, param, lam, grid, dets, inv_psd, gmst):
    """F_pq = sum over detectors of (d_p h_d | d_q h_d), the strain derivatives by complex step
    (11 x 11)."""
    theta = np.asarray(theta, dtype=np.float64)
    act = O.active_mask(theta[:7], param, grid)
    df = grid[1]
    F = np.zeros((11, 11))
    for k, det in enumerate(dets):
        dh = []
        for p in range(11):
            hstep = O._cs_step(theta[p])
            tp = theta.astype(np.complex128)
            tp[p] += 1j * hstep
            hr, hi = _strain_parts(tp, param, lam, grid, act, det, gmst)
            dh.append(np.imag(hr) / hstep + 1j * (np.imag(hi) / hstep))
        w = inv_psd[k][act]
        for p in range(11):
            for q in range(p, 11):
                F[p, q] += O.inner(dh[p], dh[q], w, df)
    return np.triu(F) + np.triu(F, 1).T


def loglike_grad(theta, param, lam, grid, dets, data, inv_psd, gmst):
    """d lnL / d theta (11) by complex step through the real-analytic strain of each detector."""
    theta = np.asarray(theta, dtype=np.float64)
    act = O.active_mask(theta[:7], param, grid)
    df = grid[1]
    g = np.zeros(11)
    for p in range(11):
        hstep = O._cs_step(theta[p])
        tp = theta.astype(np.complex128)
        tp[p] += 1j * hstep
        lnl = 0.0
        for k, det in enumerate(dets):
            hr, hi = _strain_parts(tp, param, lam, grid, act, det, gmst)
            w = inv_psd[k][act]
            d = data[k][act]
            lnl = lnl + 4.0 * df * np.sum(w * (d.real * hr + d.imag * hi)) - 2.0 * df * np.sum(w * (hr * hr + hi * hi))
        g[p] = np.imag(lnl) / hstep
    return g
