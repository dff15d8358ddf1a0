"""Naive polarized-traces solve (oracle; test infrastructure only).

Follows the paper step by step, in FP64, with no blocking, fusion or reordering:

  * local problems and their sparse LU (Alg. 1: partition, set local
    problems, factorize);
  * local Green's trace blocks K_{j,k} = (A^ell)^{-1}_{j,k} for local rows
    j, k in {0, 1, n, n+1}, by solving against identity columns (Alg. 1,
    'extract Green's functions'; Section 7.1).  With A = h^2 H,
    G^ell(z_j, z_k) = (1/h)(H^ell)^{-1}_{j,k} = h K_{j,k} (Def. 1 with the
    1/h^2 delta of eq. definition_local_helmholtz_problem), so the 1/h factor
    of the matrix form of the incomplete Green's integrals (Def. 2) leaves
        G^down_j(v0, v1) = K_{j,1} v0 - K_{j,0} v1,
        G^up_j(vn, vn1)  = -K_{j,n+1} vn + K_{j,n} vn1;
  * Newton potential N f = (H^ell)^{-1} f^ell = (A^ell)^{-1} h^2 f^ell
    (Alg. 2, 'solve local problems');
  * the polarized system closed by jump conditions (Def. 9), written from
    eqs. jump_1 .. jump_4 with the reading u^down_{n+1} on the right of
    jump_4 (the matrix forms printed after them carry misplaced identity
    blocks; the equations are used instead);
  * its splitting into D (two block-triangular halves, identity diagonal)
    and R = A - D (eq. splitting_jump), D^-1 by a top-down and a bottom-up
    block back-substitution (Section 4.1);
  * the Gauss-Seidel preconditioner with n_it iterations (Alg. 4);
  * GMRES (Section 4.2 / Section 7.1: Saad's algorithm, no restart), used
    here in its flexible right-preconditioned form with modified Gram-Schmidt;
  * total traces u = u^down + u^up and the reconstruction of every layer by a
    local solve with interface forcing (eq. PDE_version_green_formula; Alg. 2,
    'reconstruct local solutions', 'concatenate').

Unknown layout: a polarized vector is an array (..., 2, L-1, 2, NX): index 0
of the second-to-last-but-two axis is the down-going part d, 1 the up-going
part a; then the interface k = 0..L-2 (between layers k and k+1, 0-based);
then the two trace rows (row n and n+1 of layer k, which are rows 0 and 1 of
layer k+1); then x.

Pinned by tests/test_oracle_polarized.py: discrete GRF (Lemma 1, zero outside
the layer), extrapolator and jump identities of the blocks (Lemma 4),
reciprocity of the blocks (appendix, symmetric PML form), the traces of the
direct solution satisfying the integral system (Def. 4) and the polarized
system (Prop. 1), the eigenvalue structure of D^-1 A (Section 4.2), L = 1 and
L = 2 special cases, the 1D tridiagonal closed form (appendix, Usmani), and
agreement of the full solve with the direct solve.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .assemble import layer_split, local_operator, restrict_source

KEYS = ("0", "1", "n", "n+1")


class LocalProblem:
    """Local operator of one layer, its sparse LU and its Green's trace blocks."""

    def __init__(self, prob, slab, extract=True):
        self.prob = prob
        self.slab = slab
        self.NX = prob.NX
        self.A = local_operator(prob, slab).tocsc()
        self.lu = spla.splu(self.A)
        self.rows = slab.trace_rows()
        self.K = self._extract() if extract else {}

    def solve(self, b: np.ndarray) -> np.ndarray:
        """(A^ell)^{-1} b for b of shape (k, R, NX)."""
        k = b.shape[0]
        B = b.reshape(k, -1).T
        X = self.lu.solve(np.ascontiguousarray(B, dtype=np.complex128))
        return X.T.reshape(b.shape)

    def _extract(self) -> dict:
        """K[(j, k)] = (A^ell)^{-1}_{row j, row k}: solve with identity columns at source row k."""
        NX, R = self.NX, self.slab.R
        K = {}
        for kk, rk in self.rows.items():
            E = np.zeros((NX, R, NX), dtype=np.complex128)
            E[np.arange(NX), rk, np.arange(NX)] = 1.0
            X = self.solve(E)  # X[c] = column c of the inverse restricted to the local grid
            for jj, rj in self.rows.items():
                K[(jj, kk)] = X[:, rj, :].T.copy()  # rows: target x; cols: source x
        return K

    # incomplete Green's integrals (Def. 2, matrix form), vectors (..., NX)
    def g_down(self, j: str, v0, v1):
        K = self.K
        return v0 @ K[(j, "1")].T - v1 @ K[(j, "0")].T

    def g_up(self, j: str, vn, vn1):
        K = self.K
        return -(vn @ K[(j, "n+1")].T) + vn1 @ K[(j, "n")].T


class PolarizedSolver:
    """The method of polarized traces on one problem (Algs. 1, 2 and 4, Def. 9)."""

    def __init__(self, prob, n_it: int = 2, extract=True):
        self.prob = prob
        self.NX = prob.NX
        self.NZ = prob.NZ
        self.slabs = layer_split(prob)
        self.L = len(self.slabs)
        self.loc = [LocalProblem(prob, s, extract=extract) for s in self.slabs]
        self.n_it = n_it

    # ------------------------------------------------------------------ shapes
    def zeros(self, nrhs: int = 1):
        return np.zeros((nrhs, 2, self.L - 1, 2, self.NX), dtype=np.complex128)

    # ------------------------------------------------------------- Newton pot.
    def newton(self, f: np.ndarray) -> list:
        """w^ell = (A^ell)^{-1} h^2 f^ell for every layer; f (nrhs, NZ, NX)."""
        h2 = self.prob.h ** 2
        return [lp.solve(h2 * restrict_source(self.prob, lp.slab, f)) for lp in self.loc]

    def rhs(self, w: list) -> np.ndarray:
        """Right-hand side of the polarized system: N_{n}, N_{n+1} f of layer k for the down rows,
        N_0, N_1 f of layer k+1 for the up rows (eqs. jump_1..jump_4)."""
        nrhs = w[0].shape[0]
        s = self.zeros(nrhs)
        for k in range(self.L - 1):
            top, bot = self.loc[k], self.loc[k + 1]
            s[:, 0, k, 0] = w[k][:, top.rows["n"]]
            s[:, 0, k, 1] = w[k][:, top.rows["n+1"]]
            s[:, 1, k, 0] = w[k + 1][:, bot.rows["0"]]
            s[:, 1, k, 1] = w[k + 1][:, bot.rows["1"]]
        return s

    # ------------------------------------------------------- the jump system
    def apply_A(self, x: np.ndarray) -> np.ndarray:
        """The polarized system closed by jump conditions (Def. 9), row-permuted as in eq. splitting_jump."""
        d, a = x[:, 0], x[:, 1]
        y = np.zeros_like(x)
        L = self.L
        for k in range(L - 1):
            up = self.loc[k]          # layer above interface k; its rows n, n+1
            lo = self.loc[k + 1]      # layer below interface k; its rows 0, 1
            # down rows: eq. jump_2 (j = n) and jump_4 (j = n+1) of layer k
            y[:, 0, k, 0] = d[:, k, 0] + a[:, k, 0] - up.g_up("n", a[:, k, 0], a[:, k, 1])
            y[:, 0, k, 1] = d[:, k, 1] - up.g_up("n+1", a[:, k, 0], a[:, k, 1])
            if k >= 1:
                t0 = d[:, k - 1, 0] + a[:, k - 1, 0]
                t1 = d[:, k - 1, 1] + a[:, k - 1, 1]
                y[:, 0, k, 0] -= up.g_down("n", t0, t1)
                y[:, 0, k, 1] -= up.g_down("n+1", t0, t1)
            # up rows: eq. jump_3 (j = 0) and jump_1 (j = 1) of layer k+1
            y[:, 1, k, 0] = a[:, k, 0] - lo.g_down("0", d[:, k, 0], d[:, k, 1])
            y[:, 1, k, 1] = a[:, k, 1] + d[:, k, 1] - lo.g_down("1", d[:, k, 0], d[:, k, 1])
            if k + 1 <= L - 2:
                b0 = a[:, k + 1, 0] + d[:, k + 1, 0]
                b1 = a[:, k + 1, 1] + d[:, k + 1, 1]
                y[:, 1, k, 0] -= lo.g_up("0", b0, b1)
                y[:, 1, k, 1] -= lo.g_up("1", b0, b1)
        return y

    def apply_D(self, x: np.ndarray) -> np.ndarray:
        """Block-triangular part D = diag(D^down, D^up) of eq. def_permuted_system_jump."""
        d, a = x[:, 0], x[:, 1]
        y = x.copy()
        L = self.L
        for k in range(L - 1):
            if k >= 1:
                up = self.loc[k]
                y[:, 0, k, 0] -= up.g_down("n", d[:, k - 1, 0], d[:, k - 1, 1])
                y[:, 0, k, 1] -= up.g_down("n+1", d[:, k - 1, 0], d[:, k - 1, 1])
            if k + 1 <= L - 2:
                lo = self.loc[k + 1]
                y[:, 1, k, 0] -= lo.g_up("0", a[:, k + 1, 0], a[:, k + 1, 1])
                y[:, 1, k, 1] -= lo.g_up("1", a[:, k + 1, 0], a[:, k + 1, 1])
        return y

    def apply_R(self, x: np.ndarray) -> np.ndarray:
        """R = [[0, U], [L, 0]] (eq. def_permuted_system_jump): the couplings of A not in D."""
        d, a = x[:, 0], x[:, 1]
        y = np.zeros_like(x)
        L = self.L
        for k in range(L - 1):
            up = self.loc[k]
            lo = self.loc[k + 1]
            # U: up-going traces feeding the down rows
            y[:, 0, k, 0] = a[:, k, 0] - up.g_up("n", a[:, k, 0], a[:, k, 1])
            y[:, 0, k, 1] = -up.g_up("n+1", a[:, k, 0], a[:, k, 1])
            if k >= 1:
                y[:, 0, k, 0] -= up.g_down("n", a[:, k - 1, 0], a[:, k - 1, 1])
                y[:, 0, k, 1] -= up.g_down("n+1", a[:, k - 1, 0], a[:, k - 1, 1])
            # L: down-going traces feeding the up rows
            y[:, 1, k, 0] = -lo.g_down("0", d[:, k, 0], d[:, k, 1])
            y[:, 1, k, 1] = d[:, k, 1] - lo.g_down("1", d[:, k, 0], d[:, k, 1])
            if k + 1 <= L - 2:
                y[:, 1, k, 0] -= lo.g_up("0", d[:, k + 1, 0], d[:, k + 1, 1])
                y[:, 1, k, 1] -= lo.g_up("1", d[:, k + 1, 0], d[:, k + 1, 1])
        return y

    def apply_D_inv(self, r: np.ndarray) -> np.ndarray:
        """D^-1 r by block back-substitution: a top-down sweep for d, a bottom-up sweep for a (Section 4.1)."""
        L = self.L
        u = np.zeros_like(r)
        for k in range(L - 1):  # down sweep
            u[:, 0, k] = r[:, 0, k]
            if k >= 1:
                up = self.loc[k]
                u[:, 0, k, 0] += up.g_down("n", u[:, 0, k - 1, 0], u[:, 0, k - 1, 1])
                u[:, 0, k, 1] += up.g_down("n+1", u[:, 0, k - 1, 0], u[:, 0, k - 1, 1])
        for k in range(L - 2, -1, -1):  # up sweep
            u[:, 1, k] = r[:, 1, k]
            if k + 1 <= L - 2:
                lo = self.loc[k + 1]
                u[:, 1, k, 0] += lo.g_up("0", u[:, 1, k + 1, 0], u[:, 1, k + 1, 1])
                u[:, 1, k, 1] += lo.g_up("1", u[:, 1, k + 1, 0], u[:, 1, k + 1, 1])
        return u

    def precondition(self, r: np.ndarray, n_it: int | None = None) -> np.ndarray:
        """Gauss-Seidel preconditioner (Alg. 4): u^0 = 0, u^{i+1} = D^-1 (r - R u^i), n_it times.

        n_it = 0 is read as GMRES on the polarized system with no preconditioner
        (Section 4.2 runs GMRES on the system itself before preconditioning it):
        the identity, not the zero map that a loop of no passes would leave."""
        n_it = self.n_it if n_it is None else n_it
        if n_it == 0:
            return r.copy()
        u = np.zeros_like(r)
        for _ in range(n_it):
            u = self.apply_D_inv(r - self.apply_R(u))
        return u

    def gauss_seidel(self, s: np.ndarray, tol: float = 1e-10, maxit: int = 500):
        """Alg. 3: the Gauss-Seidel iteration as a stand-alone solver (stops on the relative update)."""
        u = np.zeros_like(s)
        hist = []
        for it in range(1, maxit + 1):
            un = self.apply_D_inv(s - self.apply_R(u))
            num = np.linalg.norm((un - u).reshape(un.shape[0], -1), axis=1)
            den = np.linalg.norm(un.reshape(un.shape[0], -1), axis=1)
            u = un
            hist.append(float(np.max(num / np.maximum(den, 1e-300))))
            if hist[-1] < tol:
                break
        return u, hist

    # ---------------------------------------------------------------- FGMRES
    def fgmres(self, s: np.ndarray, tol: float = 1e-10, maxit: int = 50, precond=True, op=None, prec=None):
        """Flexible right-preconditioned GMRES with modified Gram-Schmidt, x0 = 0, no restart.

        op / prec (default: this system's apply_A / precondition) select the
        operator and the preconditioner.  Returns (x, info) with info a list of
        dicts per right-hand side: iterations, residual history (least-squares
        estimates) and the true relative residual ||s - A x|| / ||s||.
        """
        apply_A = op or self.apply_A
        precondition = prec or self.precondition
        nrhs = s.shape[0]
        shape = s.shape[1:]
        x = np.zeros_like(s)
        infos = []
        for r in range(nrhs):
            b = s[r:r + 1]
            beta = np.linalg.norm(b)
            if beta == 0.0:
                infos.append({"iters": 0, "hist": [0.0], "relres": 0.0})
                continue
            V = [b / beta]
            Z = []
            H = np.zeros((maxit + 1, maxit), dtype=np.complex128)
            hist = [1.0]
            y = np.zeros(0, dtype=np.complex128)
            for j in range(maxit):
                z = precondition(V[j]) if precond else V[j].copy()
                Z.append(z)
                w = apply_A(z)
                for i in range(j + 1):
                    H[i, j] = np.vdot(V[i], w)
                    w = w - H[i, j] * V[i]
                H[j + 1, j] = np.linalg.norm(w)
                e1 = np.zeros(j + 2, dtype=np.complex128)
                e1[0] = beta
                y, *_ = np.linalg.lstsq(H[: j + 2, : j + 1], e1, rcond=None)
                res = np.linalg.norm(e1 - H[: j + 2, : j + 1] @ y) / beta
                hist.append(float(res))
                if res < tol or H[j + 1, j] == 0.0:
                    break
                V.append(w / H[j + 1, j])
            xr = sum(y[i] * Z[i] for i in range(len(y)))
            x[r] = xr[0]
            true = np.linalg.norm(b - apply_A(xr)) / beta
            infos.append({"iters": len(y), "hist": hist, "relres": float(true)})
        return x, infos

    # -------------------------------------------------------- reconstruction
    def reconstruct(self, f: np.ndarray, x: np.ndarray) -> np.ndarray:
        """u from the total traces t = d + a (Section 4.1) by one forced local solve per layer
        (eq. PDE_version_green_formula; Alg. 2), concatenating the owned rows."""
        nrhs = f.shape[0]
        t = x[:, 0] + x[:, 1]  # (nrhs, L-1, 2, NX)
        u = np.zeros((nrhs, self.NZ, self.NX), dtype=np.complex128)
        h2 = self.prob.h ** 2
        for l, lp in enumerate(self.loc):
            b = h2 * restrict_source(self.prob, lp.slab, f)
            if l >= 1:  # top interface l-1: + e_1 v_0 - e_0 v_1
                b[:, lp.rows["1"]] += t[:, l - 1, 0]
                b[:, lp.rows["0"]] -= t[:, l - 1, 1]
            if l <= self.L - 2:  # bottom interface l: - e_{n+1} v_n + e_n v_{n+1}
                b[:, lp.rows["n+1"]] -= t[:, l, 0]
                b[:, lp.rows["n"]] += t[:, l, 1]
            ul = lp.solve(b)
            s = lp.slab
            u[:, s.own_start:s.own_start + s.n] = ul[:, s.top_ext:s.top_ext + s.n]
        return u

    def solve(self, f: np.ndarray, tol: float = 1e-10, maxit: int = 50):
        """Alg. 2 with the trace solve of Section 4: u for f (nrhs, NZ, NX)."""
        f = np.asarray(f, dtype=np.complex128).reshape(-1, self.NZ, self.NX)
        if self.L == 1:  # a single layer is one local solve
            u = self.loc[0].solve(self.prob.h ** 2 * restrict_source(self.prob, self.slabs[0], f))
            return u, []
        w = self.newton(f)
        s = self.rhs(w)
        x, info = self.fgmres(s, tol=tol, maxit=maxit)
        return self.reconstruct(f, x), info

    # ------------------------------------------------ Def. 4 integral system
    def apply_M(self, t: np.ndarray) -> np.ndarray:
        """The discrete integral system of Def. 4 (without the 1/h scaling): rows
        G^down_j(t_top) + G^up_j(t_bot) - t_j at j = 1 and j = n of each layer,
        ordered as in eq. integral_formulation.  t: (nrhs, L-1, 2, NX)."""
        rows = []
        L = self.L
        for l, lp in enumerate(self.loc):
            for j in ("1", "n"):
                if j == "1" and l == 0:
                    continue
                if j == "n" and l == L - 1:
                    continue
                acc = -(t[:, l - 1, 1] if j == "1" else t[:, l, 0])
                if l >= 1:
                    acc = acc + lp.g_down(j, t[:, l - 1, 0], t[:, l - 1, 1])
                if l <= L - 2:
                    acc = acc + lp.g_up(j, t[:, l, 0], t[:, l, 1])
                rows.append(acc)
        return np.stack(rows, axis=1)

    def newton_rows(self, w: list) -> np.ndarray:
        """(N_j f) at j = 1 and j = n of each layer, ordered as eq. integral_formulation."""
        rows = []
        L = self.L
        for l, lp in enumerate(self.loc):
            if l >= 1:
                rows.append(w[l][:, lp.slab.row(1)])
            if l <= L - 2:
                rows.append(w[l][:, lp.slab.row(lp.slab.n)])
        return np.stack(rows, axis=1)

    def traces_of(self, u: np.ndarray) -> np.ndarray:
        """Interface traces (rows n, n+1 of layer k) of a volume field u (nrhs, NZ, NX)."""
        t = np.zeros((u.shape[0], self.L - 1, 2, self.NX), dtype=np.complex128)
        for k in range(self.L - 1):
            s = self.slabs[k]
            g = s.own_start + s.n - 1
            t[:, k, 0] = u[:, g]
            t[:, k, 1] = u[:, g + 1]
        return t

    # ---------------------------------------------------------- dense forms
    def dense(self, which: str = "A") -> np.ndarray:
        """The operator as one dense matrix (tiny problems only), by applying it to unit vectors."""
        n = 4 * (self.L - 1) * self.NX
        op = {"A": self.apply_A, "D": self.apply_D, "R": self.apply_R, "Dinv": self.apply_D_inv}[which]
        E = np.eye(n, dtype=np.complex128).reshape(n, 2, self.L - 1, 2, self.NX)
        return op(E).reshape(n, n).T
