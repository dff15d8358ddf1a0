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



def _worker() -> None:
    """Child-process entry of direct_solve_jobs: argv = job file, result file."""
    import pickle
    import sys

    with open(sys.argv[1], "rb") as fh:
        prob, f = pickle.load(fh)
    np.save(sys.argv[2], DirectSolver(prob).solve(f))


def direct_solve_jobs(jobs, workers: int = 8) -> list:
    """u* = A^{-1} h^2 f for a list of independent (problem, sources) jobs.

    Each job is factored and solved on its own in a separate Python process
    (at most `workers` at a time), with exactly the arithmetic of DirectSolver;
    this only bounds the wall time of checking every source of a large batch.
    """
    import os
    import pickle
    import subprocess
    import sys
    import tempfile

    jobs = list(jobs)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ)
    env["PYTHONPATH"] = root + (os.pathsep + env["PYTHONPATH"] if env.get("PYTHONPATH") else "")
    env["OMP_NUM_THREADS"] = "1"
    out = [None] * len(jobs)
    with tempfile.TemporaryDirectory(prefix="oracle_direct_") as tmp:
        todo = list(range(len(jobs)))
        running = []
        while todo or running:
            while todo and len(running) < max(1, workers):
                i = todo.pop(0)
                jf, rf = os.path.join(tmp, f"job{i}.pkl"), os.path.join(tmp, f"u{i}.npy")
                with open(jf, "wb") as fh:
                    pickle.dump(jobs[i], fh, protocol=pickle.HIGHEST_PROTOCOL)
                cmd = [sys.executable, "-c", "import sys; from oracle.direct import _worker; _worker()", jf, rf]
                running.append((i, rf, subprocess.Popen(cmd, env=env)))
            i, rf, p = running.pop(0)
            if p.wait() != 0:
                for _, _, q in running:
                    q.kill()
                raise RuntimeError(f"oracle direct-solve worker for job {i} failed (exit {p.returncode})")
            out[i] = np.load(rf)
            os.remove(rf)
    return out


def direct_solve_parallel(prob, f: np.ndarray, workers: int = 8) -> np.ndarray:
    """direct_solve for (nrhs, NZ, NX) sources, the sources split evenly over `workers` processes."""
    f = np.asarray(f, dtype=np.complex128)
    parts = [p for p in np.array_split(np.arange(f.shape[0]), max(1, min(workers, f.shape[0]))) if p.size]
    return np.concatenate(direct_solve_jobs([(prob, f[p]) for p in parts], workers), axis=0)
