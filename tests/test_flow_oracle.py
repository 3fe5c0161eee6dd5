"""Pins of the flow oracle (CPU only): invertibility, change of variables against a brute-force
Jacobian, the closed-form Gaussian at zero output weights, the gradient against finite
differences, Adam's first steps against their closed form."""
import math

import numpy as np
import torch

from oracle import flow_oracle as F
from paper_2302_05329_amd import workloads as W


def _params(seed=3, out_scale=0.5, bias_scale=0.1):
    mean, cov, _ = W.correlated_gaussian(2, 40 + seed)
    return W.flow_init_params(seed, mu=mean, sd=np.sqrt(np.diag(cov)), out_scale=out_scale,
                              bias_scale=bias_scale)


def test_layout_size():
    assert F.P == 8 * 19342 + 14
    assert _params().size == F.P


def test_inverse_undoes_forward():
    p = _params()
    _, _, x = W.correlated_gaussian(64, 5)
    z, lq = F.forward(p, x)
    x2, lq2 = F.inverse(p, z)
    assert torch.max(torch.abs(x2 - torch.as_tensor(x))) < 1e-10
    assert torch.max(torch.abs(lq2 - lq)) < 1e-10
    # the flow is not the identity at these weights
    assert torch.max(torch.abs(z - (torch.as_tensor(x) - torch.as_tensor(p[-14:-7], dtype=torch.float64))
                               * torch.as_tensor(p[-7:], dtype=torch.float64))) > 0.1


def test_logq_matches_bruteforce_jacobian():
    """log q(x) = log N(f(x)) + log |det df/dx| with df/dx by central differences."""
    p = _params(seed=4, out_scale=0.8)
    _, _, x = W.correlated_gaussian(6, 6)
    z, lq = F.forward(p, x)
    h = 1e-6
    for i in range(x.shape[0]):
        J = np.zeros((7, 7))
        for j in range(7):
            xp, xm = x[i].copy(), x[i].copy()
            xp[j] += h
            xm[j] -= h
            J[:, j] = ((F.forward(p, xp[None])[0] - F.forward(p, xm[None])[0]) / (2 * h)).numpy()[0]
        sign, logdet = np.linalg.slogdet(J)
        ref = -0.5 * float(z[i] @ z[i]) - 3.5 * math.log(2 * math.pi) + logdet
        assert sign > 0
        assert abs(float(lq[i]) - ref) < 1e-7


def test_zero_output_weights_give_the_standardisation_gaussian():
    mu = np.array([1.0, -2.0, 0.5, 3.0, 0.0, -1.0, 2.0])
    sd = np.array([0.5, 2.0, 1.0, 0.1, 3.0, 1.5, 0.7])
    p = W.flow_init_params(9, mu=mu, sd=sd, out_scale=0.0, bias_scale=0.0)
    x = np.random.default_rng(1).standard_normal((20, 7)) * sd + mu
    _, lq = F.forward(p, x)
    mu32, sd32 = p[-14:-7].astype(np.float64), 1.0 / p[-7:].astype(np.float64)
    ref = np.sum(-0.5 * ((x - mu32) / sd32) ** 2 - np.log(sd32) - 0.5 * math.log(2 * math.pi), axis=1)
    assert np.max(np.abs(lq.numpy() - ref)) < 1e-12


def test_gradient_matches_central_differences():
    p = _params(seed=5, out_scale=0.7, bias_scale=0.2).astype(np.float64)
    _, _, x = W.correlated_gaussian(16, 7)
    val, g = F.loss_grad(p, x)
    assert abs(val - float(F.loss(torch.as_tensor(p), x))) < 1e-12
    rng = np.random.default_rng(2)
    # a sample of entries from every block of the first and the last layer
    offs = [0, 7 * 128, 7 * 128 + 128, 7 * 128 + 256 + 128 * 128, F.LAYER_P - 14 - 128 * 14, F.LAYER_P - 14]
    lens = [7 * 128, 128, 128 * 128, 128, 128 * 14, 14]
    idx = []
    for layer in (0, 7):
        for o, n in zip(offs, lens):
            idx += list(layer * F.LAYER_P + o + rng.choice(n, 3, replace=False))
    for k in idx:
        h = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (float(F.loss(torch.as_tensor(pp), x)) - float(F.loss(torch.as_tensor(pm), x))) / (2 * h)
        assert abs(fd - g[k]) < 1e-7 * max(1.0, abs(g[k])), (k, fd, g[k])
    assert np.all(g[-14:] == 0.0)
    # rows of W1 that multiply transformed dims see a zero input and get no gradient
    W1g = g[:7 * 128].reshape(7, 128)
    assert np.all(W1g[3:] == 0.0) and np.any(W1g[:3] != 0.0)


def test_adam_first_steps_closed_form():
    rng = np.random.default_rng(3)
    p0 = rng.standard_normal(50)
    g1, g2 = rng.standard_normal(50), rng.standard_normal(50)
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    p1, m, v = F.adam(p0, g1, np.zeros(50), np.zeros(50), 1, lr, b1, b2, eps)
    # step 1: m_hat = g, v_hat = g^2
    assert np.allclose(p1, p0 - lr * g1 / (np.abs(g1) + eps), rtol=0, atol=1e-15)
    p2, _, _ = F.adam(p1, g2, m, v, 2, lr, b1, b2, eps)
    mh = (b1 * (1 - b1) * g1 + (1 - b1) * g2) / (1 - b1**2)
    vh = (b2 * (1 - b2) * g1**2 + (1 - b2) * g2**2) / (1 - b2**2)
    assert np.allclose(p2, p1 - lr * mh / (np.sqrt(vh) + eps), rtol=0, atol=1e-15)
