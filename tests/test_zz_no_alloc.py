"""The allocation-free likelihood entry point (workspace in the library's fixed device array)
against pd_loglike_and_grad with a caller-owned workspace: same kernels, so the results must
agree bit for bit.  Two calls in a row, the second with a smaller batch, so that the second
reads an array holding the first call's contents."""
import ctypes
import sys

import numpy as np
import pytest

from paper_2302_05329_amd import _lib as L
from paper_2302_05329_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _noalloc(th, grid, lam, d, ip, want_grad):
    import torch
    n = th.shape[0]
    lnl = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    grad = torch.full((n, 7), float("nan"), dtype=torch.float64, device="cuda") if want_grad else None
    st = torch.full((n,), 7, dtype=torch.int32, device="cuda")
    g = L.make_grid(grid.f0, grid.df, grid.n_bins, grid.f_min, grid.f_ref)
    ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None  # noqa: E731
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.lib().pd_loglike_and_grad_noalloc(ptr(th), n, W.PARAM_M1M2, ctypes.byref(g), ptr(lam), ptr(d), ptr(ip),
                                             L.PD_FP64, ptr(lnl), ptr(grad), ptr(st), stream)
    L.check(rc)
    return lnl, grad, st


@pytest.mark.parametrize("want_grad", [True, False])
def test_noalloc_matches_workspace_entry(gpu, lam0, want_grad):
    import torch
    from paper_2302_05329_amd import api
    lam = torch.as_tensor(lam0, device="cuda")
    # 4096 chains on the sampler grid (the graph-capture use), then a smaller ragged batch with an
    # invalid row, on the same array
    for n, nb, seed in ((4096, 8033, 11), (777, 4017, 12)):
        rows = W.draw_sources(n, seed, d_range=(100, 2000), tc_range=(-0.1, 0.1), phic_random=True)
        if n == 777:
            rows[5, 2] = 1.5      # |chi1| > 1: outside the model's domain
        grid = W.Grid(20.0, 0.125 if nb == 8033 else 0.25, nb)
        psd = W.psd_aligo_zdhp_fit(grid.freqs())
        data = W.complex_noise(psd, grid.df, 1000 + seed)
        th = torch.as_tensor(rows, device="cuda")
        d = torch.view_as_real(torch.as_tensor(data, device="cuda")).contiguous()
        ip = torch.as_tensor(1.0 / psd, device="cuda")
        _say(f"noalloc lnl grad={want_grad} n={n} nb={nb}")
        l1, g1, s1 = _noalloc(th, grid, lam, d, ip, want_grad)
        l2, g2, s2 = api.loglike_and_grad(th, W.PARAM_M1M2, grid, lam, d, ip, want_grad=want_grad)
        torch.cuda.synchronize()
        assert torch.equal(s1, s2)
        assert int((s1 != 0).sum()) == (1 if n == 777 else 0)
        ok = s1 == 0
        assert torch.equal(l1[ok], l2[ok])
        assert bool(torch.isnan(l1[~ok]).all())
        if want_grad:
            assert torch.equal(g1[ok], g2[ok])
            assert bool(torch.isnan(g1[~ok]).all())


def test_noalloc_rejects_oversized_batch(gpu, lam0):
    import torch
    lam = torch.as_tensor(lam0, device="cuda")
    grid = W.Grid(20.0, 0.125, 16225)
    n = 65536
    need = L.lib().pd_workspace_bytes(L.PD_OP_LOGLIKE_GRAD, n, grid.n_bins)
    assert need > L.PD_NOALLOC_SCRATCH_BYTES
    th = torch.zeros((n, 7), dtype=torch.float64, device="cuda")
    d = torch.zeros((grid.n_bins, 2), dtype=torch.float64, device="cuda")
    ip = torch.ones(grid.n_bins, dtype=torch.float64, device="cuda")
    with pytest.raises(L.PdError) as e:
        _noalloc(th, grid, lam, d, ip, True)
    assert e.value.code == L.PD_EUNSUPPORTED
