"""The C ABI library loads, exports every symbol include/phenomd.h declares, and its
host-side validation rejects bad batches before anything is launched (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2302_05329_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(pd_[a-z0-9_]+)\s*\(", src))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("library not built")
    return L.lib()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert {"pd_waveform_eval", "pd_loglike_and_grad", "pd_fisher", "pd_mismatch_grad"} <= names
    for name in sorted(names):
        assert hasattr(lib, name), name
    assert lib.pd_version().startswith(b"phenomd")


def test_workspace_queries(lib):
    for op in range(5):
        a = lib.pd_workspace_bytes(op, 1000, 65536)
        b = lib.pd_workspace_bytes(op, 2000, 65536)
        assert a > 0 and b > a and a % 256 == 0
    assert lib.pd_workspace_bytes(0, 0, 100) == 0
    assert lib.pd_workspace_bytes(9, 10, 100) == 0


def _call_waveform(lib, theta=1, n=1, param=3, grid=None, lam=1, prec=0, out=1, ws=1, wsb=1 << 40):
    g = grid or L.make_grid(20.0, 0.25, 100, 20.0, 20.0)
    vp = lambda x: ctypes.c_void_p(x) if x else None  # noqa: E731
    return lib.pd_waveform_eval(vp(theta and 256), n, param, ctypes.byref(g), vp(lam and 512), prec,
                                vp(out and 768), None, vp(ws and 1024), wsb, None)


@pytest.mark.parametrize("kw,code", [
    (dict(theta=0), L.PD_EINVAL),
    (dict(lam=0), L.PD_EINVAL),
    (dict(out=0), L.PD_EINVAL),
    (dict(ws=0), L.PD_EINVAL),
    (dict(n=0), L.PD_EINVAL),
    (dict(param=7), L.PD_EINVAL),
    (dict(prec=5), L.PD_EINVAL),
    (dict(wsb=16), L.PD_ENOMEM),
    (dict(grid=L.make_grid(20.0, 0.0, 100, 20.0, 20.0)), L.PD_EINVAL),
    (dict(grid=L.make_grid(20.0, 0.25, 0, 20.0, 20.0)), L.PD_EINVAL),
    (dict(grid=L.make_grid(20.0, 0.25, (1 << 28) + 1, 20.0, 20.0)), L.PD_EINVAL),
    (dict(grid=L.make_grid(20.0, 0.25, 100, 0.0, 20.0)), L.PD_EINVAL),
    (dict(grid=L.make_grid(20.0, 0.25, 100, 20.0, float("nan"))), L.PD_EINVAL),
])
def test_batch_level_errors(lib, kw, code):
    assert _call_waveform(lib, **kw) == code
    assert len(lib.pd_last_error()) > 0


def test_mismatch_requires_fft_length(lib):
    g = L.make_grid(0.0, 0.01, 1000, 1.0, 20.0)
    vp = ctypes.c_void_p
    rc = lib.pd_mismatch_grad(vp(256), 1, 3, ctypes.byref(g), vp(512), vp(768), vp(1024), vp(1280), None, None,
                              vp(2048), 1 << 40, None)
    assert rc == L.PD_EUNSUPPORTED


def _gauss_post():
    st = L.PdPosterior()
    st.kind = L.PD_TARGET_GAUSS
    for j in range(7):
        st.mu[j], st.isig2[j] = 0.0, 1.0
    return st


@pytest.mark.parametrize("bad", ["scale_neg", "scale_nan", "xi", "n", "ws", "wsb"])
def test_rwmh_rejects_bad_arguments(lib, bad):
    st = _gauss_post()
    vp = ctypes.c_void_p
    n = 0 if bad == "n" else 16
    need = lib.pd_rwmh_workspace_bytes(ctypes.byref(st), 16)
    assert need > 0 and need % 256 == 0
    sc = [0.1] * 7
    if bad == "scale_neg":
        sc[3] = -0.1
    if bad == "scale_nan":
        sc[6] = float("nan")
    scale = (ctypes.c_double * 7)(*sc)
    rc = lib.pd_rwmh_step(ctypes.byref(st), n, vp(256), vp(512), None if bad == "xi" else vp(768), vp(1024), scale,
                          None, None if bad == "ws" else vp(2048), 16 if bad == "wsb" else need, None)
    assert rc == (L.PD_ENOMEM if bad == "wsb" else L.PD_EINVAL)
    assert len(lib.pd_last_error()) > 0


@pytest.mark.parametrize("bad", ["ndet0", "ndet9", "gmst", "dets", "wsb"])
def test_network_rejects_bad_arguments(lib, bad):
    vp = ctypes.c_void_p
    g = L.make_grid(20.0, 0.25, 100, 20.0, 20.0)
    nd = {"ndet0": 0, "ndet9": 9}.get(bad, 2)
    dets = (L.PdDetector * 2)()
    for k in range(2):
        dets[k].xarm[0], dets[k].yarm[1] = 1.0, 1.0
    need = lib.pd_network_workspace_bytes(4, 100, 2)
    assert need > lib.pd_workspace_bytes(2, 4, 100) and need % 256 == 0
    assert lib.pd_network_workspace_bytes(4, 100, 0) == 0
    rc = lib.pd_network_loglike_and_grad(vp(256), 4, 3, ctypes.byref(g), vp(512), nd, None if bad == "dets" else dets,
                                         float("nan") if bad == "gmst" else 0.5, vp(768), vp(1024), vp(1280), None,
                                         None, vp(2048), 16 if bad == "wsb" else need, None)
    assert rc == (L.PD_ENOMEM if bad == "wsb" else L.PD_EINVAL)
    assert len(lib.pd_last_error()) > 0


@pytest.mark.parametrize("bad", ["alpha_neg", "alpha_nan", "dsum", "alias", "precond_alias"])
def test_fit_lambda_step_rejects_bad_arguments(lib, bad):
    vp = ctypes.c_void_p
    g = L.make_grid(0.0, 0.01, 65536, 1.0, 20.0)
    alpha = {"alpha_neg": -1e-6, "alpha_nan": float("nan")}.get(bad, 1e-6)
    dsum = None if bad == "dsum" else (512 if bad == "alias" else 4096)
    precond = vp(512) if bad == "precond_alias" else None
    rc = lib.pd_fit_lambda_step(vp(256), 1, 3, ctypes.byref(g), vp(512), vp(768), vp(1024), alpha, precond,
                                vp(1280), vp(dsum) if dsum else None, vp(2048), 1 << 40, None)
    assert rc == L.PD_EINVAL
    assert len(lib.pd_last_error()) > 0


def test_network_posterior_validation(lib):
    """A network posterior needs 1..8 sites and finite geometry, sidereal angle and orientation;
    its workspace holds the network likelihood's."""
    st = L.PdPosterior()
    st.kind = L.PD_TARGET_GW_NETWORK
    st.grid = L.make_grid(20.0, 0.25, 100, 20.0, 20.0)
    st.lam, st.data, st.inv_psd = 256, 512, 768
    for j, (lo, hi) in enumerate([(20, 40), (0.125, 1), (-0.9, 0.9), (-0.9, 0.9), (100, 900), (-0.1, 0.1), (-1.6, 1.6)]):
        st.lo[j], st.hi[j] = lo, hi
    st.n_det = 2
    for k in range(2):
        st.detectors[k].xarm[0], st.detectors[k].yarm[1] = 1.0, 1.0
    need = lib.pd_posterior_workspace_bytes(ctypes.byref(st), 10)
    assert need >= lib.pd_network_workspace_bytes(10, 100, 2)
    assert lib.pd_hmc_workspace_bytes(ctypes.byref(st), 10) > need
    for field, bad in (("n_det", 0), ("n_det", 9), ("gmst", float("nan"))):
        old = getattr(st, field)
        setattr(st, field, bad)
        assert lib.pd_posterior_workspace_bytes(ctypes.byref(st), 10) == 0
        setattr(st, field, old)
    st.orient[2] = float("inf")
    assert lib.pd_posterior_workspace_bytes(ctypes.byref(st), 10) == 0
