"""Sparse direct solve of the PML-padded Helmholtz system (oracle; test infrastructure only).

This is the plain definition of what the method of polarized traces computes:
by the paper's Theorem 1 and Proposition 1 the polarized solve reproduces the
solution of eq. discrete_Helmholtz_equation exactly (up to the GMRES
tolerance), so the reference result is u* = A^{-1} (h^2 f) with A = h^2 H.
The paper factors with UMFPACK (Section 7.1); any exact sparse LU is
equivalent -- SciPy's SuperLU is used here.

Pinned by tests/test_oracle_direct.py: residual of the solve, dense
brute-force solves on tiny grids, and second-order convergence to the
free-space Green's function (i/4) H0^(1)(omega r) in a constant medium.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .assemble import global_operator


class DirectSolver:
    """u = A^{-1} h^2 f for one problem; factor once, solve many right-hand sides."""

    def __init__(self, prob):
        self.prob = prob
        self.A = global_operator(prob).tocsc()
        self.lu = spla.splu(self.A)

    def solve(self, f: np.ndarray) -> np.ndarray:
        """f: (NZ, NX) or (nrhs, NZ, NX) complex -> u of the same shape."""
        p = self.prob
        NX, NZ = p.NX, p.NZ
        f = np.asarray(f, dtype=np.complex128)
        single = f.ndim == 2
        F = f.reshape(-1, NZ * NX).T * (p.h * p.h)
        U = self.lu.solve(np.ascontiguousarray(F))
        U = U.T.reshape(-1, NZ, NX)
        return U[0] if single else U


def direct_solve(prob, f: np.ndarray) -> np.ndarray:
    return DirectSolver(prob).solve(f)
