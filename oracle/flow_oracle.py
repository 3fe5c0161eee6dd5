"""Plain PyTorch (CPU, float64) RealNVP flow and Adam: the CPU oracle of the GPU flow kernels.

TEST INFRASTRUCTURE ONLY: used by the tests, smoke() and the CPU leg of the benchmark, never by
the product path.

The paper closes Sec. 3.3 by pointing at normalising flows trained on the fly as proposals
for a gradient-based sampler on the GPU.  The flow here is a RealNVP (Dinh, Sohl-Dickstein &
Bengio 2017) on R^7 with a fixed shape:
  * standardisation y = (x - mu) * isd (mu, isd fixed, not trained);
  * 8 affine couplings; layer l keeps the dims in C_l (C_l = {0,1,2} for even l, {3,...,6}
    for odd l) and maps the others: with m the indicator of C_l,
        h1 = tanh((m y) W1 + b1),  h2 = tanh(h1 W2 + b2),  o = h2 W3 + b3   (o in R^14)
        s = 2 tanh(o[:7] / 2) * (1 - m),  t = o[7:] * (1 - m)
        y <- m y + (1 - m) (y exp(s) + t)
  * z = y after the last layer; by the change of variables
        log q(x) = sum_d log N(z_d; 0, 1) + sum_l sum_d s_l,d + sum_d log isd_d.
Training minimises -mean log q over the samples with Adam (Kingma & Ba 2015).
Parameter layout (the library's, float values as given): per layer W1[7][128] b1[128]
W2[128][128] b2[128] W3[128][14] b3[14]; 8 layers; then mu[7], isd[7].

Pinned by tests/test_flow_oracle.py: inverse(forward(x)) = x; log q against log N(z) plus
the log-determinant of a brute-force finite-difference Jacobian; zero output weights give
the closed-form Gaussian N(mu, diag(1/isd^2)); the gradient against central differences;
the first Adam steps against their closed form.
"""
import math

import numpy as np
import torch

D, H, O, LAYERS = 7, 128, 14, 8
LAYER_P = D * H + H + H * H + H + H * O + O
P = LAYERS * LAYER_P + 2 * D
S_BOUND = 2.0


def mask(layer):
    m = torch.zeros(D, dtype=torch.float64)
    if layer % 2 == 0:
        m[:3] = 1.0
    else:
        m[3:] = 1.0
    return m


def unpack(params):
    """Flat parameter vector -> (list of per-layer (W1, b1, W2, b2, W3, b3), mu, isd)."""
    p = torch.as_tensor(np.asarray(params, dtype=np.float64)) if not torch.is_tensor(params) else params
    if p.numel() != P:
        raise ValueError(f"expected {P} parameters, got {p.numel()}")
    layers = []
    off = 0
    for _ in range(LAYERS):
        shapes = [(D, H), (H,), (H, H), (H,), (H, O), (O,)]
        ts = []
        for sh in shapes:
            k = int(np.prod(sh))
            ts.append(p[off:off + k].reshape(sh))
            off += k
        layers.append(ts)
    mu = p[off:off + D]
    isd = p[off + D:off + 2 * D]
    return layers, mu, isd


def _net(ws, y_cond):
    W1, b1, W2, b2, W3, b3 = ws
    h1 = torch.tanh(y_cond @ W1 + b1)
    h2 = torch.tanh(h1 @ W2 + b2)
    o = h2 @ W3 + b3
    return o


def _scale_shift(ws, y, m):
    o = _net(ws, y * m)
    s = S_BOUND * torch.tanh(o[:, :D] / S_BOUND) * (1.0 - m)
    t = o[:, D:] * (1.0 - m)
    return s, t


def log_normal(z):
    return -0.5 * (z * z).sum(dim=1) - 0.5 * D * math.log(2.0 * math.pi)


def forward(params, x):
    """x [n, 7] -> (z [n, 7], log q(x) [n]), float64 torch tensors."""
    layers, mu, isd = unpack(params)
    x = torch.as_tensor(x, dtype=torch.float64)
    y = (x - mu) * isd
    logdet = torch.log(isd).sum().expand(x.shape[0]).clone()
    for l in range(LAYERS):
        m = mask(l)
        s, t = _scale_shift(layers[l], y, m)
        y = m * y + (1.0 - m) * (y * torch.exp(s) + t)
        logdet = logdet + s.sum(dim=1)
    return y, log_normal(y) + logdet


def inverse(params, z):
    """z [n, 7] -> (x [n, 7], log q(x) [n]): the layers undone in reverse order."""
    layers, mu, isd = unpack(params)
    y = torch.as_tensor(z, dtype=torch.float64)
    z = y
    logdet = torch.log(isd).sum().expand(y.shape[0]).clone()
    for l in reversed(range(LAYERS)):
        m = mask(l)
        s, t = _scale_shift(layers[l], y, m)   # depends on the kept dims only, unchanged here
        y = m * y + (1.0 - m) * (y - t) * torch.exp(-s)
        logdet = logdet + s.sum(dim=1)
    return y / isd + mu, log_normal(z) + logdet


def loss(params, x):
    return -forward(params, x)[1].mean()


def loss_grad(params, x):
    """(loss, d loss / d params [P]) by reverse-mode autodiff in float64; the standardisation
    entries (not trained) get zero."""
    p = torch.tensor(np.asarray(params, dtype=np.float64), requires_grad=True)
    val = loss(p, x)
    (g,) = torch.autograd.grad(val, p)
    g = g.detach().clone()
    g[LAYERS * LAYER_P:] = 0.0
    return float(val.detach()), g.numpy()


def adam(params, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected), float64 numpy; returns (params, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mhat = m / (1.0 - b1**t)
    vhat = v / (1.0 - b2**t)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v
