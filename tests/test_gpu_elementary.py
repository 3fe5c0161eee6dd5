"""The kernels' own FP64 elementary functions against 50-digit mpmath values (GPU).

Measured on the arguments the kernels see: sincos of phases up to 1e5 rad (and beyond, the
library fallback), atan of the merger-ringdown argument (the two-level and the table-reduced forms), exp of the amplitude and f^-7/6
arguments, reciprocals.  Bound: 2 ulp of the exact result (the polynomials alone are about
1 ulp; the Cody-Waite reduction and the final rounding add at most one more).
"""
import ctypes

import mpmath as mp
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

mp.mp.dps = 50


def _ulp_err(got, exact):
    ex = np.array([float(e) for e in exact])
    err = np.array([abs(mp.mpf(float(g)) - e) for g, e in zip(got, exact)], dtype=object)
    return np.array([float(e) for e in err]) / np.spacing(np.abs(ex))


def _args(rng):
    return {
        0: np.concatenate([rng.uniform(-4, 4, 1500), rng.uniform(-1e5, 1e5, 1500), rng.uniform(-1e9, 1e9, 200)]),
        2: np.concatenate([rng.uniform(-1, 1, 1000), rng.uniform(-50, 50, 1000), 10 ** rng.uniform(-8, 8, 1000)]),
        3: np.concatenate([rng.uniform(-700, 700, 1500), rng.uniform(-5, 5, 1500)]),
        4: np.concatenate([10 ** rng.uniform(-10, 10, 1500), -(10 ** rng.uniform(-5, 5, 500))]),
        # table atan: the merger-ringdown range, every octave of the table and beyond it, and the
        # bucket edges (powers of two and their sixteenths, and the next doubles on either side)
        5: np.concatenate([rng.uniform(-1, 1, 800), rng.uniform(-50, 50, 800), 10 ** rng.uniform(-8, 8, 800),
                           -(10 ** rng.uniform(-4, 4, 300)), _edges()]),
    }


def _edges():
    e = np.array([2.0**k * (1 + m / 16) for k in range(-11, 11) for m in range(16)])
    return np.concatenate([e, np.nextafter(e, 0), np.nextafter(e, np.inf), [0.0, -0.0, 5e-324, 1e300]])


@pytest.mark.parametrize("fn,name", [(0, "sin"), (1, "cos"), (2, "atan"), (3, "exp"), (4, "rcp"), (5, "atan_table")])
def test_elementary_ulp(gpu, fn, name):
    import torch
    from paper_2302_05329_amd import _lib as L
    rng = np.random.default_rng(40 + fn)
    x = _args(rng)[0 if fn == 1 else fn]
    xt = torch.as_tensor(x, device="cuda")
    out = torch.empty_like(xt)
    print(f"elementary {name} n={x.size}", flush=True)
    L.check(L.lib().pd_elementary_eval(fn, ctypes.c_void_p(xt.data_ptr()), x.size, ctypes.c_void_p(out.data_ptr()),
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    got = out.cpu().numpy()
    f = {0: mp.sin, 1: mp.cos, 2: mp.atan, 3: mp.exp, 4: lambda v: 1 / v, 5: mp.atan}[fn]
    exact = [f(mp.mpf(float(v))) for v in x]
    e = _ulp_err(got, exact)
    print(f"{name}: max {e.max():.3f} ulp, mean {e.mean():.3f}", flush=True)
    assert e.max() <= 2.0, (name, e.max(), x[np.argmax(e)])
