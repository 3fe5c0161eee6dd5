"""The learned independence proposal: a RealNVP flow trained on the GPU, and the sampler that
interleaves flow-proposal Metropolis-Hastings with HMC (the flow + GPU + gradient-sampler
combination the paper points to at the end of Sec. 3.3).  Marshalling only: forward, inverse,
backward, gradient reduction and Adam run in the HIP library.
"""
import numpy as np
import torch

from . import _lib as L
from .api import Workspace, _ptr, _stream
from . import sampling


def param_count():
    return int(L.lib().pd_flow_param_count())


def _x(t):
    t = torch.as_tensor(t, dtype=torch.float64, device="cuda").contiguous()
    if t.dim() != 2 or t.shape[1] != 7 or t.shape[0] == 0:
        raise ValueError(f"expected [n, 7] rows, got {tuple(t.shape)}")
    return t


class Flow:
    """Parameters (float32, device) plus Adam state; the layout is the library's.  mode "fp32"
    runs every layer in FP32; "bf16" runs the hidden and output layers (and their gradient
    products) on the bfloat16 matrix cores with FP32 accumulation."""

    def __init__(self, params, mode="fp32"):
        if mode not in ("fp32", "bf16"):
            raise ValueError("mode must be 'fp32' or 'bf16'")
        self.mode = L.PD_FLOW_BF16 if mode == "bf16" else L.PD_FLOW_FP32
        p = torch.as_tensor(params, dtype=torch.float32, device="cuda").contiguous()
        if p.dim() != 1 or p.numel() != param_count():
            raise ValueError(f"flow parameters must be a vector of {param_count()} floats")
        self.params = p
        self.m = torch.zeros_like(p)
        self.v = torch.zeros_like(p)
        self.grad = torch.zeros_like(p)
        self.loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        self.t = 0
        self.ws = Workspace()

    def forward(self, x, want_z=True):
        """x [n, 7] -> (z [n, 7] or None, log q(x) [n])."""
        x = _x(x)
        n = x.shape[0]
        z = torch.empty_like(x) if want_z else None
        lq = torch.empty(n, dtype=torch.float64, device="cuda")
        L.check(L.lib().pd_flow_forward(_ptr(self.params), _ptr(x), n, _ptr(z), _ptr(lq), self.mode, _stream()))
        return z, lq

    def sample(self, z):
        """Standard-normal draws z [n, 7] -> (x [n, 7], log q(x) [n])."""
        z = _x(z)
        n = z.shape[0]
        x = torch.empty_like(z)
        lq = torch.empty(n, dtype=torch.float64, device="cuda")
        L.check(L.lib().pd_flow_sample(_ptr(self.params), _ptr(z), n, _ptr(x), _ptr(lq), self.mode, _stream()))
        return x, lq

    def loss_grad(self, x, want_loss=True):
        """Fills self.grad with d(-mean log q)/d params and, if want_loss, self.loss with the loss."""
        x = _x(x)
        n = x.shape[0]
        wp, wb = self.ws.get(L.lib().pd_flow_workspace_bytes(n))
        L.check(L.lib().pd_flow_loss_grad(_ptr(self.params), _ptr(x), n, _ptr(self.grad),
                                          _ptr(self.loss) if want_loss else None, wp, wb, self.mode, _stream()))
        return self.loss

    def adam(self, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        L.check(L.lib().pd_adam_step(_ptr(self.params), _ptr(self.grad), _ptr(self.m), _ptr(self.v),
                                     self.params.numel(), float(lr), float(b1), float(b2), float(eps), self.t,
                                     _stream()))

    def fit(self, x, steps, batch, lr, generator, log_every=0):
        """Maximum-likelihood training on the rows of x with minibatches drawn by `generator`;
        returns the loss history (host floats, one per log_every steps)."""
        x = _x(x)
        hist = []
        for k in range(steps):
            idx = torch.randint(0, x.shape[0], (batch,), device="cuda", generator=generator)
            logged = bool(log_every) and (k % log_every == 0 or k == steps - 1)
            self.loss_grad(x.index_select(0, idx), want_loss=logged)
            self.adam(lr)
            if logged:
                hist.append(float(self.loss.item()))
        return hist


def standardisation(x):
    """(mean, standard deviation) of training rows, computed on the host from a copy."""
    a = np.asarray(x.cpu().numpy() if torch.is_tensor(x) else x, dtype=np.float64)
    return a.mean(axis=0), np.maximum(a.std(axis=0), 1e-6)


class FlowHMC:
    """HMC chains whose transitions alternate with flow-proposal independence MH: every
    `mh_every`-th transition draws x' = f^{-1}(z), z ~ N(0, I), and accepts it with probability
    min(1, pi(x') q(x) / (pi(x) q(x'))); the chain's gradient is carried along for HMC."""

    def __init__(self, hmc, flow):
        self.hmc = hmc
        self.flow = flow
        self.lq = None
        self.ws = Workspace()

    def refresh(self):
        """log q at the current states (after the flow changed)."""
        self.lq = self.flow.forward(self.hmc.x, want_z=False)[1]

    def mh_step(self, z, u):
        if self.lq is None:
            self.refresh()
        xp, lqp = self.flow.sample(z)
        lpp, gp = sampling.logp(self.hmc.post, xp, ws=self.ws)
        return sampling.independence_mh(self.hmc.x, self.hmc.logp, self.lq, xp, lpp, lqp, u, grad=self.hmc.grad,
                                        grad_p=gp)

    def hmc_step(self, xi, u):
        acc = self.hmc.step(xi, u)
        self.lq = None
        return acc
