"""MI355X (gfx950) implementation of the batched IMRPhenomD-structured waveform hot path of
arXiv:2302.05329 (ripple): strain, fused likelihood and gradient, Fisher matrices,
mismatch adjoint over the 209 fit coefficients, and the samplers built on them.

The compute path is the HIP library libphenomd_hip.so behind the C ABI in
include/phenomd.h; this package holds its Python binding.
"""
from . import workloads  # noqa: F401  (pure numpy, importable without a GPU)

__all__ = ["workloads", "api"]


def __getattr__(name):
    if name == "api":
        import importlib
        return importlib.import_module(__name__ + ".api")
    raise AttributeError(name)
