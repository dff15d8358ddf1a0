"""Spectral diagnostics of the preconditioned polarized system.

Section 4.2: with the splitting A = D + R, the preconditioned operator
D^-1 A = I + D^-1 R has at least half of its eigenvalues at 1 and the others
in pairs 1 +- sqrt(mu), mu the eigenvalues of the "double reflection"
operator (D_up^-1 L)(D_dn^-1 U).  The eigenvalue figures of the numerical
section read this as a clustering claim: tight around 1 in media without
resonances (closer as the PML improves), spread towards 0 in a resonant
cavity (more eigenvalues far from 1 as the frequency grows).

The dense operator is assembled on the GPU, column block by column block,
by applying the library's operators (``pt_apply``: A, R, D^-1 by the two
sweeps, the Gauss-Seidel preconditioner) to unit vectors held in device
memory; only the final eigenvalue decomposition of the (small) assembled
matrix runs on the host (``numpy.linalg.eigvals``).
"""
from __future__ import annotations

import numpy as np

from .polar import OP_A, OP_DINV, OP_PRECOND, OP_R

# operator name -> chain of pt_apply codes, applied right to left
CHAINS = {
    "A": (OP_A,),
    "R": (OP_R,),
    "Dinv": (OP_DINV,),
    "DinvA": (OP_DINV, OP_A),      # D^-1 A (Section 4.2)
    "DinvR": (OP_DINV, OP_R),      # the Gauss-Seidel iteration matrix up to sign (Alg. 3)
    "MinvA": (OP_PRECOND, OP_A),   # the preconditioned operator GMRES sees (Alg. 4, gs_iters sweeps)
}


def operator_matrix(solver, op: str = "DinvA"):
    """The dense ntrace x ntrace matrix of `op` (a key of CHAINS) as a complex128
    device tensor: column i is op applied to the i-th unit polarized vector,
    max_nrhs columns per library call."""
    import torch

    chain = CHAINS[op]
    n = solver.ntrace
    nb = max(1, solver.max_nrhs)
    shape = (2, solver.L - 1, 2, solver.NX)
    out = torch.empty((n, n), dtype=torch.complex128, device="cuda")
    for b0 in range(0, n, nb):
        k = min(nb, n - b0)
        x = torch.zeros((k, n), dtype=torch.complex128, device="cuda")
        idx = torch.arange(k, device="cuda")
        x[idx, b0 + idx] = 1.0
        y = x.reshape((k,) + shape)
        for code in reversed(chain):
            y = solver.apply(code, y)
        out[:, b0:b0 + k] = y.reshape(k, n).transpose(0, 1)
    torch.cuda.synchronize()
    return out


def eigenvalues(solver, op: str = "DinvA") -> np.ndarray:
    """Eigenvalues of the assembled operator (host LAPACK on the small dense matrix)."""
    return np.linalg.eigvals(operator_matrix(solver, op).cpu().numpy())


def cluster_summary(ev: np.ndarray, radius: float = 0.2) -> dict:
    """How tightly eigenvalues cluster around 1: the largest distance, how many lie
    outside the disc of `radius` around 1, and the smallest modulus."""
    d = np.abs(np.asarray(ev) - 1.0)
    return {"n": int(d.size), "max_dist_from_1": float(d.max()), "outside": int(np.sum(d > radius)),
            "radius": float(radius), "min_modulus": float(np.abs(ev).min())}
