"""GPU flow kernels against the float64 flow oracle; training and flow-proposal MH on the GPU.

The GPU flow computes in float32 (parameters and activations); the oracle in float64 on the
same float32 parameter values.  Tolerances: a float32 emulation of the same network gives
|dz| ~ 1.5e-6 and |d log q| ~ 7e-6 on these inputs (8 layers of 128-term sums, rounding
2^-24 each); the tests allow 20 times that.  Gradients: float32 sums over tiles of 32
samples; allowed 1e-3 of the largest entry of each parameter block, and 2e-4 in norm.
"""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import flow_oracle as F
from paper_2302_05329_amd import workloads as W

pytestmark = pytest.mark.gpu

Z_TOL = 3e-5
LQ_TOL = 1.5e-4


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _setup(n, seed=11, out_scale=0.5):
    mean, cov, x = W.correlated_gaussian(n, seed)
    sd = np.sqrt(np.diag(cov))
    p = W.flow_init_params(seed + 10, mu=mean, sd=sd, out_scale=out_scale, bias_scale=0.1)
    return p, x, sd


@pytest.mark.parametrize("n", [1, 16, 100, 1000, 4096])
def test_forward_and_sample_parity(gpu, n):
    from paper_2302_05329_amd import flow
    p, x, sd = _setup(n)
    fl = flow.Flow(p)
    _say(f"flow forward/sample n={n}")
    z, lq = fl.forward(x)
    zr, lqr = F.forward(p, x)
    z, lq = z.cpu().numpy(), lq.cpu().numpy()
    assert np.all(np.abs(z - zr.numpy()) <= Z_TOL * (1 + np.abs(zr.numpy())))
    assert np.all(np.abs(lq - lqr.numpy()) <= LQ_TOL * (1 + np.abs(lqr.numpy()) / 10))
    zs = np.random.default_rng(n).standard_normal((n, 7))
    xs, lqs = fl.sample(torch.as_tensor(zs, device="cuda"))
    xr, lqsr = F.inverse(p, zs)
    xs, lqs = xs.cpu().numpy(), lqs.cpu().numpy()
    assert np.all(np.abs(xs - xr.numpy()) <= Z_TOL * sd * (1 + np.abs(zs)) * 4)
    assert np.all(np.abs(lqs - lqsr.numpy()) <= LQ_TOL * (1 + np.abs(lqsr.numpy()) / 10))


@pytest.mark.parametrize("n", [7, 100, 513, 4096])
def test_loss_and_gradient_parity(gpu, n):
    from paper_2302_05329_amd import flow
    p, x, _ = _setup(n, seed=12, out_scale=0.7)
    fl = flow.Flow(p)
    _say(f"flow loss/grad n={n}")
    loss = float(fl.loss_grad(x).item())
    g = fl.grad.cpu().numpy().astype(np.float64)
    lr, gr = F.loss_grad(p, x)
    assert abs(loss - lr) <= LQ_TOL * (1 + abs(lr) / 10)
    assert np.all(g[-14:] == 0.0)
    assert np.linalg.norm(g - gr) <= 2e-4 * np.linalg.norm(gr)
    blocks = [7 * 128, 128, 128 * 128, 128, 128 * 14, 14]
    off = 0
    for _layer in range(8):
        for b in blocks:
            ref = gr[off:off + b]
            assert np.max(np.abs(g[off:off + b] - ref)) <= 1e-3 * max(np.max(np.abs(ref)), 1e-6), (off, b)
            off += b


def test_adam_parity(gpu):
    from paper_2302_05329_amd import flow
    p, _, _ = _setup(64, seed=13)
    fl = flow.Flow(p)
    pr = p.astype(np.float64)
    m = np.zeros_like(pr)
    v = np.zeros_like(pr)
    rng = np.random.default_rng(5)
    _say("adam 3 steps")
    for t in range(1, 4):
        g = rng.standard_normal(pr.size).astype(np.float32)
        g[-14:] = 0
        fl.grad.copy_(torch.as_tensor(g, device="cuda"))
        fl.adam(1e-3)
        pr, m, v = F.adam(pr, g.astype(np.float64), m, v, t, 1e-3)
    got = fl.params.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - pr)) <= 1e-6 * (1 + np.max(np.abs(pr)))
    assert np.array_equal(got[-14:], p[-14:].astype(np.float64))


def test_training_fits_a_gaussian(gpu):
    """Maximum likelihood on 16384 draws of a correlated Gaussian: the held-out loss ends within
    0.05 nats of the target's entropy (the minimum possible) and well below the start."""
    from paper_2302_05329_amd import flow
    mean, cov, xa = W.correlated_gaussian(16384 + 4096, 21)
    x, xt = xa[:16384], xa[16384:]
    m0, s0 = flow.standardisation(x)
    fl = flow.Flow(W.flow_init_params(23, mu=m0, sd=s0))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(23)
    _, lq0 = fl.forward(xt, want_z=False)
    _say("flow training 400 steps")
    fl.fit(x, 400, 512, 2e-3, gen)
    _, lq1 = fl.forward(xt, want_z=False)
    entropy = 0.5 * np.linalg.slogdet(2 * math.pi * math.e * cov)[1]
    l0, l1 = -float(lq0.mean()), -float(lq1.mean())
    assert l1 < l0 - 0.1
    assert l1 - entropy < 0.05, (l0, l1, entropy)


def test_flow_proposal_mh_keeps_the_target(gpu):
    """Flow-proposal independence MH on a Gaussian posterior (the library's Gaussian target).
    The flow starts from a wrong standardisation (shifted mean, widened scales); training on
    draws of the target raises the stationary acceptance rate; MH steps from exact draws keep
    the target's moments; and HMC alternating with flow MH from a start far out reaches them
    (independence MH alone can stall in tails that the proposal under-covers)."""
    from paper_2302_05329_amd import flow, sampling
    mu = np.array([0.3, -1.0, 2.0, 0.0, 0.5, -0.2, 1.1])
    sig = np.array([0.5, 1.0, 2.0, 0.1, 1.5, 0.7, 0.3])
    post = sampling.Posterior(1, mu=mu, isig2=1 / sig**2)
    rng = np.random.default_rng(31)
    train = mu + sig * rng.standard_normal((16384, 7))
    fl = flow.Flow(W.flow_init_params(31, mu=mu + 0.5 * sig, sd=1.5 * sig))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(31)
    n = 4096

    def run(x0, steps, keep_from, with_hmc):
        hmc = sampling.HMC(post, x0, 0.2, 8, 1 / sig**2)
        fh = flow.FlowHMC(hmc, fl)
        acc, draws = 0, []
        for t in range(steps):
            if with_hmc:
                xi = torch.randn((n, 7), dtype=torch.float64, device="cuda", generator=gen)
                fh.hmc_step(xi, torch.rand(n, dtype=torch.float64, device="cuda", generator=gen))
            z = torch.randn((n, 7), dtype=torch.float64, device="cuda", generator=gen)
            u = torch.rand(n, dtype=torch.float64, device="cuda", generator=gen)
            a = fh.mh_step(z, u)
            if t >= keep_from:
                acc += int((a == 1).sum())
                draws.append(hmc.x.cpu().numpy())
        return acc / ((steps - keep_from) * n), np.concatenate(draws), hmc

    stationary = mu + sig * rng.standard_normal((n, 7))
    _say("flow-MH gaussian: untrained acceptance")
    a0, _, _ = run(stationary, 5, 0, False)
    _say("flow-MH gaussian: train 300 steps")
    fl.fit(train, 300, 1024, 5e-4, gen)
    a1, s, _ = run(stationary, 10, 0, False)
    assert a1 > 0.6 and a1 > a0 + 0.2, (a0, a1)
    se = sig / np.sqrt(n * 10 * a1)
    assert np.all(np.abs(s.mean(axis=0) - mu) < 6 * se)
    assert np.all(np.abs(s.std(axis=0) / sig - 1) < 0.03)
    _say("flow-MH gaussian: 30 HMC + MH steps from an overdispersed start")
    acc, s, hmc = run(mu + 4 * sig * rng.standard_normal((n, 7)), 30, 10, True)
    se = sig / np.sqrt(n * 20 * acc)
    assert np.all(np.abs(s.mean(axis=0) - mu) < 6 * se)
    assert np.all(np.abs(s.std(axis=0) / sig - 1) < 0.03)
    # the carried gradient is the target's at the current state
    g = hmc.grad.cpu().numpy()
    xs = hmc.x.cpu().numpy()
    assert np.allclose(g, -(xs - mu) / sig**2, rtol=1e-12, atol=1e-12)


# ---- bfloat16 matrix-core mode -------------------------------------------------------------
# Operands of the hidden and output layers are rounded to bfloat16 (unit roundoff 2^-8) and
# accumulated in FP32.  A float32 emulation of this rounding on these inputs gives relative z
# errors up to ~1e-2 and log q errors up to ~0.3 (mean ~0.02) through the 8 layers, so parity
# with the float64 oracle is checked at those scales; the mode's own consistency (inverse then
# forward returns z and the same log q) is checked at float32 scale, since that is what makes
# the bf16 flow an exact proposal.


@pytest.mark.parametrize("n", [1, 33, 1000, 4096])
def test_bf16_forward_sample_parity_and_self_consistency(gpu, n):
    from paper_2302_05329_amd import flow
    p, x, sd = _setup(n)
    fl = flow.Flow(p, mode="bf16")
    _say(f"bf16 flow forward/sample n={n}")
    z, lq = fl.forward(x)
    zr, lqr = F.forward(p, x)
    z, lq, zr, lqr = z.cpu().numpy(), lq.cpu().numpy(), zr.numpy(), lqr.numpy()
    assert np.all(np.abs(z - zr) <= 5e-2 * (1 + np.abs(zr)))
    assert np.all(np.abs(lq - lqr) <= 1.0 + 0.02 * np.abs(lqr))
    assert np.mean(np.abs(lq - lqr)) <= 0.1
    zs = np.random.default_rng(n).standard_normal((n, 7))
    xs, lqs = fl.sample(torch.as_tensor(zs, device="cuda"))
    z2, lq2 = fl.forward(xs)
    z2, lq2, lqs = z2.cpu().numpy(), lq2.cpu().numpy(), lqs.cpu().numpy()
    # inverse then forward: the same map up to float32 rounding of the data coordinates, which can
    # move an operand across a bfloat16 rounding boundary for a small fraction of points
    close = np.all(np.abs(z2 - zs) <= 1e-4 * (1 + np.abs(zs)), axis=1) & (np.abs(lq2 - lqs) <= 1e-3 * (1 + np.abs(lqs) / 10))
    _say(f"bf16 inverse/forward agreement at float32 scale: {close.mean():.4f}")
    assert close.mean() >= 0.9
    assert np.all(np.abs(z2 - zs) <= 5e-2 * (1 + np.abs(zs)))
    assert np.all(np.abs(lq2 - lqs) <= 0.5)


@pytest.mark.parametrize("n", [7, 100, 513, 4096])
def test_bf16_loss_and_gradient_parity(gpu, n):
    from paper_2302_05329_amd import flow
    p, x, _ = _setup(n, seed=12, out_scale=0.7)
    fl = flow.Flow(p, mode="bf16")
    _say(f"bf16 flow loss/grad n={n}")
    loss = float(fl.loss_grad(x).item())
    g = fl.grad.cpu().numpy().astype(np.float64)
    lr, gr = F.loss_grad(p, x)
    assert abs(loss - lr) <= 0.1 + 0.02 * abs(lr)
    assert np.all(g[-14:] == 0.0)
    rel = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    _say(f"bf16 gradient relative error {rel:.3e}")
    assert rel <= 2e-2


def test_bf16_training_fits_a_gaussian(gpu):
    from paper_2302_05329_amd import flow
    mean, cov, xa = W.correlated_gaussian(16384 + 4096, 21)
    x, xt = xa[:16384], xa[16384:]
    m0, s0 = flow.standardisation(x)
    fl = flow.Flow(W.flow_init_params(23, mu=m0, sd=s0), mode="bf16")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(23)
    _, lq0 = fl.forward(xt, want_z=False)
    _say("bf16 flow training 400 steps")
    fl.fit(x, 400, 512, 2e-3, gen)
    _, lq1 = fl.forward(xt, want_z=False)
    entropy = 0.5 * np.linalg.slogdet(2 * math.pi * math.e * cov)[1]
    l0, l1 = -float(lq0.mean()), -float(lq1.mean())
    assert l1 < l0 - 0.1
    assert l1 - entropy < 0.1, (l0, l1, entropy)
