"""MI355X (gfx950) hot path of rank-adaptive matrix-free atomic quantum state
tomography: the batched forward map from pure-state atoms to per-setting Born
probabilities over Pauli measurement settings, its adjoint (atom and weight
gradients), the FP64 coefficient step with pruning and the Lanczos spectral
refactorisation, behind the C ABI of include/qst.h (``libqst.so``).
"""
from . import _lib  # noqa: F401

__all__ = ["api", "autograd", "build"]


def __getattr__(name):
    if name in ("api", "autograd"):
        import importlib

        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
