"""Samplers of Sec. 3.3 on the GPU: posterior log-density, HMC transitions, the random-walk
Metropolis-Hastings baseline, independence Metropolis-Hastings.  Marshalling only; the
transitions run in the HIP library.
"""
import ctypes

import numpy as np
import torch

from . import _lib as L
from .api import Workspace, _grid, _ptr, _stream


class Posterior:
    """A pd_posterior description plus the device arrays it points at."""

    def __init__(self, kind, grid=None, lam=None, data=None, inv_psd=None, lo=None, hi=None, mu=None, isig2=None,
                 detectors=None, gmst=0.0, orient=None):
        self.kind = kind
        self._keep = []
        st = L.PdPosterior()
        st.kind = kind
        if kind in (L.PD_TARGET_GW, L.PD_TARGET_GW_NETWORK):
            g = _grid(grid)
            lam = torch.as_tensor(lam, dtype=torch.float64, device="cuda").contiguous()
            d = torch.as_tensor(data, device="cuda")
            if d.is_complex():
                d = torch.view_as_real(d.to(torch.complex128))
            d = d.to(torch.float64).contiguous()
            ip = torch.as_tensor(inv_psd, dtype=torch.float64, device="cuda").contiguous()
            lead = ()
            if kind == L.PD_TARGET_GW_NETWORK:
                nd = len(detectors)
                if not 1 <= nd <= L.PD_NETWORK_MAX_DETECTORS or orient is None or len(orient) != 4:
                    raise ValueError("network posterior: 1..8 detectors and orient = (iota, psi, ra, dec)")
                lead = (nd,)
                st.n_det = nd
                st.gmst = float(gmst)
                for k, (v, x, y) in enumerate(detectors):
                    for j in range(3):
                        st.detectors[k].vertex[j] = float(v[j])
                        st.detectors[k].xarm[j] = float(x[j])
                        st.detectors[k].yarm[j] = float(y[j])
                for j in range(4):
                    st.orient[j] = float(orient[j])
            if lam.numel() != 209 or tuple(d.shape) != lead + (g.n_bins, 2) or tuple(ip.shape) != lead + (g.n_bins,):
                raise ValueError("posterior arrays do not match the grid")
            self._keep += [lam, d, ip]
            st.grid = g
            st.lam, st.data, st.inv_psd = lam.data_ptr(), d.data_ptr(), ip.data_ptr()
            if len(lo) != 7 or len(hi) != 7:
                raise ValueError("lo and hi bound all 7 parameters (Mc, q, chi1, chi2, D, tc, phic)")
            for j in range(7):
                st.lo[j], st.hi[j] = float(lo[j]), float(hi[j])
        else:
            for j in range(7):
                st.mu[j], st.isig2[j] = float(mu[j]), float(isig2[j])
        self.st = st
        self.lo = None if lo is None else np.asarray(lo, dtype=np.float64)
        self.hi = None if hi is None else np.asarray(hi, dtype=np.float64)

    def ref(self):
        return ctypes.byref(self.st)

    # ---- coordinate maps (host-side helpers for initialisation and reporting) ----------
    def to_x(self, theta):
        """theta rows (Mc, q, chi1, chi2, D, tc, phic) -> unconstrained x (inverse sigmoid)."""
        th = np.asarray(theta, dtype=np.float64)
        x = th.copy()
        s = (th - self.lo) / (self.hi - self.lo)
        x = np.log(s) - np.log1p(-s)
        return x

    def to_theta(self, x):
        x = np.asarray(x, dtype=np.float64)
        th = x.copy()
        th = self.lo + (self.hi - self.lo) / (1.0 + np.exp(-x))
        return th


def logp(post, x, want_grad=True, ws=None):
    ws = ws or Workspace()
    x = torch.as_tensor(x, dtype=torch.float64, device="cuda").contiguous()
    if x.dim() != 2 or x.shape[1] != 7:
        raise ValueError("x must be [n, 7]")
    n = x.shape[0]
    lp = torch.empty(n, dtype=torch.float64, device="cuda")
    g = torch.empty((n, 7), dtype=torch.float64, device="cuda") if want_grad else None
    wp, wb = ws.get(L.lib().pd_posterior_workspace_bytes(post.ref(), n))
    L.check(L.lib().pd_posterior_logp(post.ref(), _ptr(x), n, _ptr(lp), _ptr(g), wp, wb, _stream()))
    return lp, g


class HMC:
    """n parallel HMC chains with cached log-density and gradient (all tensors on the GPU).

    The metric is a diagonal mass matrix `mass` [7], or, when `chol` is given, the dense inverse
    mass matrix L L^T with chol = L [7][7] lower triangular (pd_hmc_step_dense)."""

    def __init__(self, post, x0, eps, n_leapfrog, mass=None, chol=None):
        self.post = post
        self.x = torch.as_tensor(x0, dtype=torch.float64, device="cuda").clone().contiguous()
        self.n = self.x.shape[0]
        self.eps = float(eps)
        self.L = int(n_leapfrog)
        if chol is not None:
            c = np.tril(np.asarray(chol, dtype=np.float64))
            if c.shape != (7, 7) or not np.all(np.diag(c) > 0) or not np.all(np.isfinite(c)):
                raise ValueError("chol must be a finite 7 x 7 lower-triangular matrix with a positive diagonal")
            self.chol = (ctypes.c_double * 49)(*c.reshape(-1).tolist())
            self.mass = None
        else:
            self.mass = (ctypes.c_double * 7)(*[float(m) for m in mass])
            self.chol = None
        self.ws = Workspace()
        self.logp, self.grad = logp(post, self.x, ws=self.ws)
        self.accepted = torch.empty(self.n, dtype=torch.int32, device="cuda")
        self.dh = torch.empty(self.n, dtype=torch.float64, device="cuda")

    def step(self, xi, u):
        """One transition; xi [n, 7] standard normals, u [n] uniforms (device tensors)."""
        if tuple(xi.shape) != (self.n, 7) or tuple(u.shape) != (self.n,):
            raise ValueError("random draws have the wrong shape")
        wp, wb = self.ws.get(L.lib().pd_hmc_workspace_bytes(self.post.ref(), self.n))
        if self.chol is not None:
            L.check(L.lib().pd_hmc_step_dense(self.post.ref(), self.n, _ptr(self.x), _ptr(self.logp), _ptr(self.grad),
                                              _ptr(xi), _ptr(u), self.L, self.eps, self.chol, _ptr(self.accepted),
                                              _ptr(self.dh), wp, wb, _stream()))
        else:
            L.check(L.lib().pd_hmc_step(self.post.ref(), self.n, _ptr(self.x), _ptr(self.logp), _ptr(self.grad),
                                        _ptr(xi), _ptr(u), self.L, self.eps, self.mass, _ptr(self.accepted),
                                        _ptr(self.dh), wp, wb, _stream()))
        return self.accepted


class RWMH:
    """n parallel random-walk Metropolis-Hastings chains (Gaussian steps of standard deviation
    `scale` per coordinate, or correlated steps L xi with `chol` = L) with cached log-density (all
    tensors on the GPU)."""

    def __init__(self, post, x0, scale=None, chol=None):
        self.post = post
        self.x = torch.as_tensor(x0, dtype=torch.float64, device="cuda").clone().contiguous()
        if self.x.dim() != 2 or self.x.shape[1] != 7:
            raise ValueError("x0 must be [n, 7]")
        self.n = self.x.shape[0]
        self.set_step(scale, chol)
        self.ws = Workspace()
        self.logp, _ = logp(post, self.x, want_grad=False, ws=self.ws)
        self.accepted = torch.empty(self.n, dtype=torch.int32, device="cuda")

    def set_step(self, scale=None, chol=None):
        if chol is not None:
            c = np.tril(np.asarray(chol, dtype=np.float64))
            if c.shape != (7, 7) or not np.all(np.isfinite(c)):
                raise ValueError("chol must be a finite 7 x 7 lower-triangular matrix")
            self.chol = (ctypes.c_double * 49)(*c.reshape(-1).tolist())
            self.scale = None
        else:
            self.scale = (ctypes.c_double * 7)(*[float(s) for s in scale])
            self.chol = None

    def step(self, xi, u):
        """One transition; xi [n, 7] standard normals, u [n] uniforms (FP64 device tensors)."""
        for t, shape in ((xi, (self.n, 7)), (u, (self.n,))):
            if tuple(t.shape) != shape or t.dtype != torch.float64 or not t.is_contiguous() or not t.is_cuda:
                raise ValueError("random draws have the wrong shape or type")
        wp, wb = self.ws.get(L.lib().pd_rwmh_workspace_bytes(self.post.ref(), self.n))
        if self.chol is not None:
            L.check(L.lib().pd_rwmh_step_dense(self.post.ref(), self.n, _ptr(self.x), _ptr(self.logp), _ptr(xi),
                                               _ptr(u), self.chol, _ptr(self.accepted), wp, wb, _stream()))
        else:
            L.check(L.lib().pd_rwmh_step(self.post.ref(), self.n, _ptr(self.x), _ptr(self.logp), _ptr(xi), _ptr(u),
                                         self.scale, _ptr(self.accepted), wp, wb, _stream()))
        return self.accepted


def independence_mh(x, lp, lq, xp, lp_p, lq_p, u, accepted=None, grad=None, grad_p=None):
    """In-place accept of proposals xp for the chains x (all device tensors); grad / grad_p, if
    given, are carried along with the state."""
    n = x.shape[0]
    if (grad is None) != (grad_p is None):
        raise ValueError("independence_mh: give both grad and grad_p or neither")
    checks = [(x, (n, 7)), (lp, (n,)), (lq, (n,)), (xp, (n, 7)), (lp_p, (n,)), (lq_p, (n,)), (u, (n,))]
    if grad is not None:
        checks += [(grad, (n, 7)), (grad_p, (n, 7))]
    for t, shape in checks:
        if tuple(t.shape) != shape or t.dtype != torch.float64 or not t.is_contiguous() or not t.is_cuda:
            raise ValueError("independence_mh: bad tensor")
    if accepted is None:
        accepted = torch.empty(n, dtype=torch.int32, device="cuda")
    L.check(L.lib().pd_independence_mh(n, _ptr(x), _ptr(lp), _ptr(lq), _ptr(grad), _ptr(xp), _ptr(lp_p), _ptr(lq_p),
                                       _ptr(grad_p), _ptr(u), _ptr(accepted), _stream()))
    return accepted
