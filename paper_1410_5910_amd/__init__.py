"""MI355X-native online solver of the method of polarized traces (2D Helmholtz).

The compute path is libpolar.so (HIP for gfx950, C-ABI in include/polar.h);
``polar`` is its thin Python binding and ``build`` compiles it in-tree;
``spectral`` assembles the preconditioned operator on the GPU for eigenvalue
diagnostics.
"""
from .polar import (Solver, Learned, PolarError, lib, solve_batch, setup_batch, tune_cache_save, tune_cache_load, OP_A, OP_R, OP_DINV, OP_PRECOND,  # noqa: F401
                    OP_A_EXTRAP, OP_R_EXTRAP, OP_DINV_EXTRAP, OP_PRECOND_EXTRAP, EXPORTS)

__all__ = ["Solver", "Learned", "PolarError", "solve_batch", "setup_batch", "tune_cache_save", "tune_cache_load", "lib", "OP_A", "OP_R", "OP_DINV", "OP_PRECOND",
           "OP_A_EXTRAP", "OP_R_EXTRAP", "OP_DINV_EXTRAP", "OP_PRECOND_EXTRAP", "EXPORTS"]
