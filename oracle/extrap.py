"""The polarized system completed with extrapolation relations (oracle; test
infrastructure only).

Section 3.4 ("Extrapolation conditions"), Def. polarized_out_going and
eq. splitting_out_going, written in the unknown layout of oracle.polarized
(d = down-going traces at rows n, n+1 of layer k; a = up-going traces at rows
0, 1 of layer k+1; interface k between layers k and k+1):

  * the integral rows at row n of layer k and row 1 of layer k+1 (the
    regularised equations, with the annihilated incomplete Green's integrals
    of the polarized traces dropped) are the jump system's rows jump_2 and
    jump_1 of oracle.polarized.apply_A;
  * the other two rows are the extrapolation relations of Lemma
    extrapolator, u^down_{n+1} = E^down u^down_n and u^up_0 = E^up u^up_1,
    with the one-sided extrapolators of Def. extrapolator,
        E^down = G(z_n, z_n)^-1 G(z_n, z_{n+1}) = K_{n,n}^-1 K_{n,n+1}  (layer k),
        E^up   = G(z_1, z_1)^-1 G(z_1, z_0)     = K_{1,1}^-1 K_{1,0}     (layer k+1),
    taken here with dense solves (the inversion of small dense blocks the
    paper names as this closure's cost); their right-hand side is zero;
  * D^extrap keeps, per half, the couplings among the traces of the same
    polarization (block-triangular with identity diagonal blocks) and
    R^extrap = A^extrap - D^extrap the couplings across polarizations;
    D^extrap^-1 is a top-down sweep for d and a bottom-up sweep for a;
  * the Gauss-Seidel preconditioner of Alg. 4 on this splitting, and
    flexible GMRES (oracle.polarized.PolarizedSolver.fgmres) on A^extrap.

Rows are scaled so every diagonal block is +I (the paper's 1/h factor and
row signs do not change the solution).  The solution of this system is the
polarized traces of the jump system (both are the unique polarized
decomposition of the traces of the solution).
"""
from __future__ import annotations

import numpy as np

from .polarized import PolarizedSolver


class ExtrapSystem:
    """A^extrap, its splitting and its solve on top of a PolarizedSolver's blocks."""

    def __init__(self, ps: PolarizedSolver):
        self.ps = ps
        self.L = ps.L
        K = [lp.K for lp in ps.loc]
        # E_down of layer k (interface k), E_up of layer k+1 (interface k)
        self.E_dn = [np.linalg.solve(K[k][("n", "n")], K[k][("n", "n+1")]) for k in range(ps.L - 1)]
        self.E_up = [np.linalg.solve(K[k + 1][("1", "1")], K[k + 1][("1", "0")]) for k in range(ps.L - 1)]

    @staticmethod
    def _mul(E, v):
        return v @ E.T

    # ------------------------------------------------------------ the system
    def rhs(self, w: list) -> np.ndarray:
        """Newton-potential rows at row n of layer k and row 1 of layer k+1; zero on the extrapolation rows."""
        s = self.ps.rhs(w)
        s[:, 0, :, 1] = 0.0
        s[:, 1, :, 0] = 0.0
        return s

    def apply_A(self, x: np.ndarray) -> np.ndarray:
        d, a = x[:, 0], x[:, 1]
        y = self.ps.apply_A(x)  # rows jump_2 (row n) and jump_1 (row 1) are kept
        for k in range(self.L - 1):
            y[:, 0, k, 1] = d[:, k, 1] - self._mul(self.E_dn[k], d[:, k, 0])
            y[:, 1, k, 0] = a[:, k, 0] - self._mul(self.E_up[k], a[:, k, 1])
        return y

    def apply_D(self, x: np.ndarray) -> np.ndarray:
        d, a = x[:, 0], x[:, 1]
        y = np.zeros_like(x)
        L = self.L
        for k in range(L - 1):
            y[:, 0, k, 0] = d[:, k, 0]
            if k >= 1:
                y[:, 0, k, 0] -= self.ps.loc[k].g_down("n", d[:, k - 1, 0], d[:, k - 1, 1])
            y[:, 0, k, 1] = d[:, k, 1] - self._mul(self.E_dn[k], d[:, k, 0])
            y[:, 1, k, 1] = a[:, k, 1]
            if k + 1 <= L - 2:
                y[:, 1, k, 1] -= self.ps.loc[k + 1].g_up("1", a[:, k + 1, 0], a[:, k + 1, 1])
            y[:, 1, k, 0] = a[:, k, 0] - self._mul(self.E_up[k], a[:, k, 1])
        return y

    def apply_R(self, x: np.ndarray) -> np.ndarray:
        d, a = x[:, 0], x[:, 1]
        y = np.zeros_like(x)
        L = self.L
        for k in range(L - 1):
            up, lo = self.ps.loc[k], self.ps.loc[k + 1]
            # down row n: the up-going traces of interfaces k and k-1
            y[:, 0, k, 0] = a[:, k, 0] - up.g_up("n", a[:, k, 0], a[:, k, 1])
            if k >= 1:
                y[:, 0, k, 0] -= up.g_down("n", a[:, k - 1, 0], a[:, k - 1, 1])
            # up row 1: the down-going traces of interfaces k and k+1
            y[:, 1, k, 1] = d[:, k, 1] - lo.g_down("1", d[:, k, 0], d[:, k, 1])
            if k + 1 <= L - 2:
                y[:, 1, k, 1] -= lo.g_up("1", d[:, k + 1, 0], d[:, k + 1, 1])
        return y

    def apply_D_inv(self, r: np.ndarray) -> np.ndarray:
        """Block forward substitution: top-down for d, bottom-up for a."""
        L = self.L
        u = np.zeros_like(r)
        for k in range(L - 1):
            u[:, 0, k, 0] = r[:, 0, k, 0]
            if k >= 1:
                u[:, 0, k, 0] += self.ps.loc[k].g_down("n", u[:, 0, k - 1, 0], u[:, 0, k - 1, 1])
            u[:, 0, k, 1] = r[:, 0, k, 1] + self._mul(self.E_dn[k], u[:, 0, k, 0])
        for k in range(L - 2, -1, -1):
            u[:, 1, k, 1] = r[:, 1, k, 1]
            if k + 1 <= L - 2:
                u[:, 1, k, 1] += self.ps.loc[k + 1].g_up("1", u[:, 1, k + 1, 0], u[:, 1, k + 1, 1])
            u[:, 1, k, 0] = r[:, 1, k, 0] + self._mul(self.E_up[k], u[:, 1, k, 1])
        return u

    def precondition(self, r: np.ndarray, n_it: int | None = None) -> np.ndarray:
        """Gauss-Seidel on the extrapolation splitting (Alg. 4): u^{i+1} = D^-1 (r - R u^i), u^0 = 0."""
        n_it = self.ps.n_it if n_it is None else n_it
        u = np.zeros_like(r)
        for _ in range(n_it):
            u = self.apply_D_inv(r - self.apply_R(u))
        return u

    def dense(self, which: str = "A") -> np.ndarray:
        ps = self.ps
        n = 4 * (ps.L - 1) * ps.NX
        op = {"A": self.apply_A, "D": self.apply_D, "R": self.apply_R, "Dinv": self.apply_D_inv}[which]
        E = np.eye(n, dtype=np.complex128).reshape(n, 2, ps.L - 1, 2, ps.NX)
        return op(E).reshape(n, n).T

    def solve(self, f: np.ndarray, tol: float = 1e-10, maxit: int = 50, n_it: int | None = None):
        """Alg. 2 with the trace solve on the extrapolation-closed system."""
        ps = self.ps
        f = np.asarray(f, dtype=np.complex128).reshape(-1, ps.NZ, ps.NX)
        s = self.rhs(ps.newton(f))
        x, info = ps.fgmres(s, tol=tol, maxit=maxit, op=self.apply_A,
                            prec=lambda v: self.precondition(v, n_it))
        return ps.reconstruct(f, x), x, info
