"""Torch-facing wrappers of the C ABI (marshalling only; every step runs in the HIP kernels).

Tensors live on the GPU; calls are enqueued on torch's current stream.
"""
import ctypes

import torch

from . import _lib as L

FP64 = L.PD_FP64
PD_TARGET_GW_NETWORK = L.PD_TARGET_GW_NETWORK
MIXED = L.PD_MIXED
PARAM_MC_ETA = L.PD_PARAM_MC_ETA
PARAM_LNMC_ETA_LND = L.PD_PARAM_LNMC_ETA_LND
PARAM_MC_Q = L.PD_PARAM_MC_Q
PARAM_M1M2 = L.PD_PARAM_M1M2


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev(t, dtype=torch.float64):
    """Contiguous float64 tensor on the GPU (copies host data)."""
    if not torch.is_tensor(t):
        t = torch.as_tensor(t)
    if t.is_complex():
        t = torch.view_as_real(t.to(torch.complex128))
    return t.to(device="cuda", dtype=dtype).contiguous()


def _need(cond, msg):
    if not cond:
        raise ValueError(msg)


def _check_shapes(th, lam, nb, data=None, inv_psd=None, targets=None):
    """Host-side shape checks: the kernels index these arrays without bounds checks."""
    _need(th.dim() == 2 and th.shape[1] == 7 and th.shape[0] > 0, f"theta must be [n, 7], got {tuple(th.shape)}")
    _need(lam.numel() == 209, f"lambda must hold 209 coefficients, got {lam.numel()}")
    if data is not None:
        _need(tuple(data.shape) == (nb, 2), f"data must be complex [{nb}], got {tuple(data.shape)}")
    if inv_psd is not None:
        _need(tuple(inv_psd.shape) == (nb,), f"inv_psd must be [{nb}], got {tuple(inv_psd.shape)}")
    if targets is not None:
        _need(tuple(targets.shape) == (th.shape[0], nb, 2),
              f"targets must be complex [{th.shape[0]}, {nb}], got {tuple(targets.shape)}")


def _grid(grid):
    if isinstance(grid, L.PdGrid):
        return grid
    if hasattr(grid, "as_tuple"):
        grid = grid.as_tuple()
    return L.make_grid(*grid)


class Workspace:
    """Caller-owned, reusable device scratch (grown on demand, 256-byte aligned)."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes, device="cuda"):
        nbytes = max(int(nbytes), 256)
        if self.buf is None or self.buf.numel() < nbytes + 256:
            self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        addr = self.buf.data_ptr()
        off = (-addr) % 256
        return ctypes.c_void_p(addr + off), nbytes


_default_ws = Workspace()


def workspace_bytes(op, n, n_bins):
    return L.lib().pd_workspace_bytes(op, int(n), int(n_bins))


def waveform_eval(theta, param, grid, lam, precision=FP64, ws=None):
    """Complex128 strain [n, n_bins] and int32 status [n]."""
    ws = ws or _default_ws
    g = _grid(grid)
    th = _dev(theta)
    lam = _dev(lam)
    _check_shapes(th, lam, g.n_bins)
    n = th.shape[0]
    h = torch.empty((n, g.n_bins, 2), dtype=torch.float64, device="cuda")
    status = torch.empty(n, dtype=torch.int32, device="cuda")
    wp, wb = ws.get(workspace_bytes(L.PD_OP_WAVEFORM, n, g.n_bins))
    L.check(L.lib().pd_waveform_eval(_ptr(th), n, param, ctypes.byref(g), _ptr(lam), precision, _ptr(h),
                                     _ptr(status), wp, wb, _stream()))
    return torch.view_as_complex(h), status


def loglike_and_grad(theta, param, grid, lam, data, inv_psd, want_grad=True, precision=FP64, ws=None):
    """ln L [n], d lnL / d theta [n, 7] (or None), status [n]."""
    ws = ws or _default_ws
    g = _grid(grid)
    th = _dev(theta)
    lam = _dev(lam)
    d = _dev(data)
    ip = _dev(inv_psd)
    _check_shapes(th, lam, g.n_bins, data=d, inv_psd=ip)
    n = th.shape[0]
    lnl = torch.empty(n, dtype=torch.float64, device="cuda")
    grad = torch.empty((n, 7), dtype=torch.float64, device="cuda") if want_grad else None
    status = torch.empty(n, dtype=torch.int32, device="cuda")
    op = L.PD_OP_LOGLIKE_GRAD if want_grad else L.PD_OP_LOGLIKE
    wp, wb = ws.get(workspace_bytes(op, n, g.n_bins))
    L.check(L.lib().pd_loglike_and_grad(_ptr(th), n, param, ctypes.byref(g), _ptr(lam), _ptr(d), _ptr(ip),
                                        precision, _ptr(lnl), _ptr(grad), _ptr(status), wp, wb, _stream()))
    return lnl, grad, status


def _net_args(theta, lam, grid, detectors, inv_psd):
    g = _grid(grid)
    th = _dev(theta)
    lam = _dev(lam)
    ip = None if inv_psd is None else _dev(inv_psd)
    nd = len(detectors)
    _need(1 <= nd <= L.PD_NETWORK_MAX_DETECTORS, f"1..{L.PD_NETWORK_MAX_DETECTORS} detectors, got {nd}")
    _need(th.dim() == 2 and th.shape[1] == 11 and th.shape[0] > 0, f"theta must be [n, 11], got {tuple(th.shape)}")
    _need(lam.numel() == 209, f"lambda must hold 209 coefficients, got {lam.numel()}")
    _need(ip is None or tuple(ip.shape) == (nd, g.n_bins), f"inv_psd must be [{nd}, {g.n_bins}]")
    dets = (L.PdDetector * nd)()
    for k, (v, x, y) in enumerate(detectors):
        for j in range(3):
            dets[k].vertex[j], dets[k].xarm[j], dets[k].yarm[j] = float(v[j]), float(x[j]), float(y[j])
    return g, th, lam, ip, nd, dets


def network_strain(theta, param, grid, lam, detector, gmst, ws=None):
    """Strain recorded at one site: complex128 [n, n_bins] (theta [n, 11])."""
    ws = ws or _default_ws
    g, th, lam, _, _, dets = _net_args(theta, lam, grid, [detector], None)
    n = th.shape[0]
    h = torch.empty((n, g.n_bins, 2), dtype=torch.float64, device="cuda")
    wp, wb = ws.get(L.lib().pd_network_strain_workspace_bytes(n, g.n_bins))
    L.check(L.lib().pd_network_strain(_ptr(th), n, param, ctypes.byref(g), _ptr(lam), dets, float(gmst), _ptr(h), None,
                                      wp, wb, _stream()))
    return torch.view_as_complex(h)


def network_fisher(theta, param, grid, lam, detectors, gmst, inv_psd, ws=None):
    """Network Fisher matrices [n, 11, 11] and status [n] (theta [n, 11], inv_psd [n_det, n_bins])."""
    ws = ws or _default_ws
    g, th, lam, ip, nd, dets = _net_args(theta, lam, grid, detectors, inv_psd)
    n = th.shape[0]
    F = torch.empty((n, 11, 11), dtype=torch.float64, device="cuda")
    status = torch.empty(n, dtype=torch.int32, device="cuda")
    wp, wb = ws.get(L.lib().pd_network_fisher_workspace_bytes(n, g.n_bins, nd))
    L.check(L.lib().pd_network_fisher(_ptr(th), n, param, ctypes.byref(g), _ptr(lam), nd, dets, float(gmst), _ptr(ip),
                                      _ptr(F), _ptr(status), wp, wb, _stream()))
    return F, status


def network_loglike_and_grad(theta, param, grid, lam, detectors, gmst, data, inv_psd, want_grad=True, ws=None):
    """Detector-network ln L [n], d lnL / d theta [n, 11] (or None) and status [n].  theta: [n, 11]
    (the 7 entries of `param`, then iota, psi, ra, dec); detectors: sequence of (vertex, x arm,
    y arm); data: complex [n_det, n_bins]; inv_psd: [n_det, n_bins]."""
    ws = ws or _default_ws
    g, th, lam, ip, nd, dets = _net_args(theta, lam, grid, detectors, inv_psd)
    d = _dev(data)
    _need(tuple(d.shape) == (nd, g.n_bins, 2), f"data must be complex [{nd}, {g.n_bins}], got {tuple(d.shape)}")
    n = th.shape[0]
    lnl = torch.empty(n, dtype=torch.float64, device="cuda")
    grad = torch.empty((n, 11), dtype=torch.float64, device="cuda") if want_grad else None
    status = torch.empty(n, dtype=torch.int32, device="cuda")
    wp, wb = ws.get(L.lib().pd_network_workspace_bytes(n, g.n_bins, nd))
    L.check(L.lib().pd_network_loglike_and_grad(_ptr(th), n, param, ctypes.byref(g), _ptr(lam), nd, dets,
                                                float(gmst), _ptr(d), _ptr(ip), _ptr(lnl), _ptr(grad), _ptr(status),
                                                wp, wb, _stream()))
    return lnl, grad, status


def fisher(theta, param, grid, lam, inv_psd, ws=None):
    """Fisher matrices [n, 7, 7] and status [n]."""
    ws = ws or _default_ws
    g = _grid(grid)
    th = _dev(theta)
    lam = _dev(lam)
    ip = _dev(inv_psd)
    _check_shapes(th, lam, g.n_bins, inv_psd=ip)
    n = th.shape[0]
    F = torch.empty((n, 7, 7), dtype=torch.float64, device="cuda")
    status = torch.empty(n, dtype=torch.int32, device="cuda")
    wp, wb = ws.get(workspace_bytes(L.PD_OP_FISHER, n, g.n_bins))
    L.check(L.lib().pd_fisher(_ptr(th), n, param, ctypes.byref(g), _ptr(lam), _ptr(ip), _ptr(F), _ptr(status),
                              wp, wb, _stream()))
    return F, status


def mismatch_grad(theta, param, grid, lam, targets, inv_psd, want_grad=True, ws=None):
    """Mismatch [nt], sum over targets of d M / d lambda [209] (or None), lag [nt]."""
    ws = ws or _default_ws
    g = _grid(grid)
    th = _dev(theta)
    lam = _dev(lam)
    tg = _dev(targets)
    ip = _dev(inv_psd)
    _check_shapes(th, lam, g.n_bins, inv_psd=ip, targets=tg)
    nt = th.shape[0]
    mm = torch.empty(nt, dtype=torch.float64, device="cuda")
    dl = torch.empty(209, dtype=torch.float64, device="cuda") if want_grad else None
    lag = torch.empty(nt, dtype=torch.int32, device="cuda")
    wp, wb = ws.get(workspace_bytes(L.PD_OP_MISMATCH_GRAD, nt, g.n_bins))
    L.check(L.lib().pd_mismatch_grad(_ptr(th), nt, param, ctypes.byref(g), _ptr(lam), _ptr(tg), _ptr(ip),
                                     _ptr(mm), _ptr(dl), _ptr(lag), wp, wb, _stream()))
    return mm, dl, lag


class LambdaFit:
    """Gradient descent on the 209 fit coefficients against fixed targets (Sec. 3.1): each
    `step` is one library call that evaluates the mismatches and their summed gradient at the
    current coefficients and then updates them in place on the device.  `precond` [209] (or
    None) multiplies each coefficient's step; relative=True sets it to lam0^2, which is Eq. 6 in
    the coordinates u = lam / lam0 - 1."""

    def __init__(self, theta, param, grid, lam0, targets, inv_psd, alpha, ws=None, precond=None, relative=False):
        self.ws = ws or Workspace()
        self.g = _grid(grid)
        self.th = _dev(theta)
        self.lam = _dev(lam0).clone().contiguous()
        self.tg = _dev(targets)
        self.ip = _dev(inv_psd)
        _check_shapes(self.th, self.lam, self.g.n_bins, inv_psd=self.ip, targets=self.tg)
        self.param = int(param)
        self.alpha = float(alpha)
        self.nt = self.th.shape[0]
        self.mismatch = torch.empty(self.nt, dtype=torch.float64, device="cuda")
        self.dsum = torch.empty(209, dtype=torch.float64, device="cuda")
        if relative:
            precond = self.lam.square()
        self.precond = None if precond is None else _dev(precond).clone().contiguous()
        if self.precond is not None and tuple(self.precond.shape) != (209,):
            raise ValueError("precond must have 209 entries")

    def _mean_grad(self, lam):
        _, d, _ = mismatch_grad(self.th, self.param, self.g, lam, self.tg, self.ip, ws=self.ws)
        return d / self.nt

    def max_curvature(self, iters=25, rel_eps=1e-5, seed=0):
        """Largest eigenvalue of P^1/2 H P^1/2 at the current coefficients (H the Hessian of the
        mean mismatch, P the preconditioner or the identity) by power iteration, each
        Hessian-vector product a difference of two gradients.  Eq. 6 decreases the local quadratic
        model monotonically for alpha <= 1 / that value."""
        lam = self.lam.clone()
        ps = torch.ones_like(lam) if self.precond is None else self.precond.clamp_min(0.0).sqrt()
        g0 = self._mean_grad(lam)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(seed)
        v = torch.randn(209, dtype=torch.float64, device="cuda", generator=gen)
        v /= v.norm()
        lmax = 0.0
        for _ in range(iters):
            w = ps * v
            e = rel_eps * float(lam.norm()) / max(float(w.norm()), 1e-300)
            hv = ps * (self._mean_grad(lam + e * w) - g0) / e
            lmax = float(v @ hv)
            v = hv / hv.norm()
        return lmax

    def step(self):
        """One descent step; afterwards `mismatch` and `dsum` hold the values at the coefficients
        before the update and `lam` the updated coefficients."""
        wp, wb = self.ws.get(workspace_bytes(L.PD_OP_MISMATCH_GRAD, self.nt, self.g.n_bins))
        L.check(L.lib().pd_fit_lambda_step(_ptr(self.th), self.nt, self.param, ctypes.byref(self.g), _ptr(self.lam),
                                           _ptr(self.tg), _ptr(self.ip), self.alpha, _ptr(self.precond),
                                           _ptr(self.mismatch), _ptr(self.dsum), wp, wb, _stream()))


def overlap(theta, param, grid, lam, streams, inv_psd, want_hh=True, ws=None):
    """Template-bank overlaps: O [nt, ns] complex128 with O[t, s] = sum_k w_k conj(h_t,k) d_s,k,
    (h_t|h_t) [nt] (or None) and status [nt].  streams: [ns, n_bins] complex, ns <= 64."""
    ws = ws or _default_ws
    g = _grid(grid)
    th = _dev(theta)
    lam = _dev(lam)
    d = torch.as_tensor(streams)
    if not d.is_complex():
        raise ValueError("streams must be complex [ns, n_bins]")
    d = torch.view_as_real(d.to(device="cuda", dtype=torch.complex128)).contiguous()
    ip = _dev(inv_psd)
    _check_shapes(th, lam, g.n_bins, inv_psd=ip)
    _need(d.dim() == 3 and d.shape[1] == g.n_bins and 1 <= d.shape[0] <= L.PD_OVERLAP_MAX_STREAMS,
          f"streams must be complex [ns <= {L.PD_OVERLAP_MAX_STREAMS}, {g.n_bins}], got {tuple(d.shape[:2])}")
    nt, ns = th.shape[0], d.shape[0]
    out = torch.empty((nt, ns, 2), dtype=torch.float64, device="cuda")
    hh = torch.empty(nt, dtype=torch.float64, device="cuda") if want_hh else None
    status = torch.empty(nt, dtype=torch.int32, device="cuda")
    wp, wb = ws.get(L.lib().pd_overlap_workspace_bytes(nt, ns, g.n_bins))
    L.check(L.lib().pd_overlap(_ptr(th), nt, param, ctypes.byref(g), _ptr(lam), _ptr(d), ns, _ptr(ip), _ptr(out),
                               _ptr(hh), _ptr(status), wp, wb, _stream()))
    return torch.view_as_complex(out), hh, status


class LogLike(torch.autograd.Function):
    """ln L(theta) with its gradient from the hand-written forward-mode kernels.

    forward computes value and gradient in one fused pass and saves the gradient;
    backward scales it by the incoming gradient.
    """

    @staticmethod
    def forward(ctx, theta, param, grid, lam, data, inv_psd):
        lnl, grad, _ = loglike_and_grad(theta.detach(), param, grid, lam, data, inv_psd, want_grad=True)
        ctx.save_for_backward(grad)
        return lnl

    @staticmethod
    def backward(ctx, g_out):
        (grad,) = ctx.saved_tensors
        return g_out[:, None] * grad, None, None, None, None, None


class Mismatch(torch.autograd.Function):
    """Mismatch of each target [nt] as a function of the 209 coefficients lambda (Sec. 3.1).

    forward evaluates the mismatches only; backward recomputes them with the adjoint pass, which
    returns the gradient summed over targets.  The incoming gradient must therefore weight every
    target equally (as the mean or the sum of the mismatches does); other weightings raise.
    """

    @staticmethod
    def forward(ctx, lam, theta, param, grid, targets, inv_psd):
        mm, _, _ = mismatch_grad(theta, param, grid, lam.detach(), targets, inv_psd, want_grad=False)
        ctx.save_for_backward(lam.detach())
        ctx.args = (theta, param, grid, targets, inv_psd)
        return mm

    @staticmethod
    def backward(ctx, g_out):
        (lam,) = ctx.saved_tensors
        theta, param, grid, targets, inv_psd = ctx.args
        w = g_out.detach()
        if not bool(torch.all(w == w[0])):
            raise NotImplementedError("Mismatch.backward: the adjoint sums over targets; weight them equally")
        _, dsum, _ = mismatch_grad(theta, param, grid, lam, targets, inv_psd, want_grad=True)
        return w[0] * dsum, None, None, None, None, None


def transition_frequencies(theta, param, grid, lam, ws=None):
    """Per point: (M T_sun [s], Mf of the phase join f_RD/2, Mf of the amplitude join f_peak, valid)."""
    ws = ws or _default_ws
    g = _grid(grid)
    th = _dev(theta)
    lam = _dev(lam)
    _check_shapes(th, lam, g.n_bins)
    n = th.shape[0]
    out = torch.empty((n, 4), dtype=torch.float64, device="cuda")
    wp, wb = ws.get(workspace_bytes(L.PD_OP_WAVEFORM, n, g.n_bins))
    L.check(L.lib().pd_transition_frequencies(_ptr(th), n, param, ctypes.byref(g), _ptr(lam), _ptr(out), wp, wb,
                                              _stream()))
    return out


def profile_enable(on=True):
    L.check(L.lib().pd_profile_enable(1 if on else 0))


def profile_read(kernel):
    """(total ms, launches) of one kernel id since the last read (waits for its events)."""
    ms = ctypes.c_double(0.0)
    cnt = ctypes.c_int64(0)
    L.check(L.lib().pd_profile_read(int(kernel), ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value
