"""DEAM hot path on MI355X (gfx950): metal-trace data substitution for
dual-energy alternating minimisation (Ge et al.).  Kernels live in libdeam.so
(C ABI, include/deam.h); this package only marshals torch tensors into it."""
from ._lib import (FAN2D, HELICAL3D, W_AM, W_GRAD, W_VJP, DeamError, load)  # noqa: F401


def __getattr__(name):
    if name == "Plan":
        from .plan import Plan
        return Plan
    if name == "DEAMNLL":
        from .autograd import DEAMNLL
        return DEAMNLL
    raise AttributeError(name)
