import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def lam0():
    from paper_2302_05329_amd import workloads
    return workloads.load_lambda()


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def gpu():
    if not gpu_available():
        pytest.skip("no GPU")
    import paper_2302_05329_amd as pd
    return pd


def rel_err_strain(h_gpu, h_ref):
    """max_k |dh_k| / max_k |h_k| (normwise per point)."""
    h_gpu = np.asarray(h_gpu)
    h_ref = np.asarray(h_ref)
    return np.max(np.abs(h_gpu - h_ref)) / np.max(np.abs(h_ref))
