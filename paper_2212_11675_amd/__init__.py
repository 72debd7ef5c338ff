"""MI355X (gfx950) PC-LSQR hot path of the Gaia AVU-GSR solver (arXiv 2212.11675).

``gsr``      ctypes binding of libgsr.so (C ABI in include/gsr.h), same entry-point names.
``autograd`` torch.autograd.Function through the least-squares solve (one handle per index
             map, refreshed in place when the coefficients change).
``build``    compiles libgsr.so with hipcc for gfx950.
"""
from . import gsr  # noqa: F401

__all__ = ["gsr"]
