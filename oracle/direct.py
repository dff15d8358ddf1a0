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
    """Child-process entry of DirectSolveJobs: argv = job file, result file, niceness."""
    import os
    import pickle
    import sys

    if int(sys.argv[3]):
        os.nice(int(sys.argv[3]))
    with open(sys.argv[1], "rb") as fh:
        prob, f = pickle.load(fh)
    np.save(sys.argv[2], DirectSolver(prob).solve(f))
    print(f"[oracle] direct solve of {getattr(prob, 'name', 'problem')}, {f.shape[0]} sources: done",
          file=sys.stderr, flush=True)


class DirectSolveJobs:
    """u* = A^{-1} h^2 f for a list of independent (problem, sources) jobs, each factored and solved in a
    separate Python process, all started at once; results() waits for them.

    The arithmetic is exactly DirectSolver's; the processes only bound the wall time of checking every source
    of a large batch.  Start them before the calling process initialises a GPU runtime (a process that holds
    one should not spawn programs).  `nice` lowers their scheduling priority.
    """

    def __init__(self, jobs, nice: int = 0):
        import os
        import pickle
        import subprocess
        import sys
        import tempfile

        self.n = len(jobs)
        self._tmp = tempfile.TemporaryDirectory(prefix="oracle_direct_")
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        env = dict(os.environ)
        env["PYTHONPATH"] = root + (os.pathsep + env["PYTHONPATH"] if env.get("PYTHONPATH") else "")
        env["OMP_NUM_THREADS"] = "1"
        self._procs = []
        for i, job in enumerate(jobs):
            jf, rf = os.path.join(self._tmp.name, f"job{i}.pkl"), os.path.join(self._tmp.name, f"u{i}.npy")
            with open(jf, "wb") as fh:
                pickle.dump(job, fh, protocol=pickle.HIGHEST_PROTOCOL)
            cmd = [sys.executable, "-c", "from oracle.direct import _worker; _worker()", jf, rf, str(int(nice))]
            self._procs.append((rf, subprocess.Popen(cmd, env=env)))

    def results(self, timeout: float | None = None) -> list:
        import time

        t_end = None if timeout is None else time.monotonic() + timeout
        out = []
        try:
            for i, (rf, p) in enumerate(self._procs):
                left = None if t_end is None else max(1.0, t_end - time.monotonic())
                if p.wait(timeout=left) != 0:
                    raise RuntimeError(f"oracle direct-solve worker for job {i} failed (exit {p.returncode})")
                out.append(np.load(rf))
        finally:
            for _, p in self._procs:
                if p.poll() is None:
                    p.kill()
                    p.wait()
            self._tmp.cleanup()
        return out


def direct_solve_jobs(jobs, workers: int = 8) -> list:
    """DirectSolveJobs over `jobs`, at most `workers` processes at a time."""
    jobs = list(jobs)
    out = []
    for k in range(0, len(jobs), max(1, workers)):
        out += DirectSolveJobs(jobs[k:k + max(1, workers)]).results()
    return out


def split_sources(prob, f: np.ndarray, parts: int) -> list:
    """(problem, sources) jobs of about equal size covering f's sources in order."""
    f = np.asarray(f, dtype=np.complex128)
    idx = [p for p in np.array_split(np.arange(f.shape[0]), max(1, min(parts, f.shape[0]))) if p.size]
    return [(prob, f[p]) for p in idx]


def direct_solve_parallel(prob, f: np.ndarray, workers: int = 8) -> np.ndarray:
    """direct_solve for (nrhs, NZ, NX) sources, the sources split evenly over `workers` processes."""
    return np.concatenate(direct_solve_jobs(split_sources(prob, f, workers), workers), axis=0)
