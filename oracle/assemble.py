"""Discretisation and domain decomposition (oracle; test infrastructure only).

Follows the paper's Section 2.1 (PML, 5-point stencil, eqs.
Helmholtz_pml / discrete_helmholtz_equation_by_point / pml_partial_z) and
Section 2.2 (layered decomposition, PML-extended local problems with the
normally extended model m~).

Conventions (readings of the paper where it is silent or garbled):
  * nodes x_p = p h, physical p = 1..nx, PML p = -npml+1..0 and nx+1..nx+npml,
    homogeneous Dirichlet one node beyond (so L_x = (nx+1) h);
  * sigma(d) = (C/delta)(d/delta)^2 with d the distance beyond [0, L_x],
    evaluated at nodes and at half nodes; delta = npml h;
  * the operator assembled is A = h^2 H (so the right-hand side is h^2 f):
      (A u)_{p,q} = -a_x(p)[a_x(p+1/2)(u_{p+1}-u_p) - a_x(p-1/2)(u_p-u_{p-1})]
                    -a_z(q)[a_z(q+1/2)(u_{q+1}-u_q) - a_z(q-1/2)(u_q-u_{q-1})]
                    - h^2 omega^2 m_{p,q} u_{p,q},  a = 1/(1 + i sigma/omega);
  * layers split the nz physical rows evenly (the first nz mod L layers get one
    more); layer 1 also owns the top npml PML rows and layer L the bottom ones;
  * interior sides of a layer get npml extension rows whose PML distance is
    measured from the first extension node (so the couplings across the
    interface rows are exactly -1), with the model extended normally.

Pinned by tests/test_oracle_assembly.py: two independent assemblies agree,
hand-computed stencil rows (tests/golden/stencil_3x3.json), complex symmetry
of diag(a_x a_z)^-1 A (the symmetric PML form of the appendix), local
operators equal the global one on owned rows, dense brute-force solves.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


# ----------------------------------------------------------------------------
# PML profile (Section 2.1)
# ----------------------------------------------------------------------------

def pml_sigma(d_len, C: float, delta: float):
    """sigma = (C/delta) (d/delta)^2 for a distance d >= 0 into the PML, 0 outside."""
    d_len = np.asarray(d_len, dtype=np.float64)
    return np.where(d_len > 0.0, (C / delta) * (d_len / delta) ** 2, 0.0)


def pml_alpha(d_len, C: float, delta: float, omega: float):
    """alpha = 1 / (1 + i sigma/omega) (Section 2.1)."""
    return 1.0 / (1.0 + 1j * pml_sigma(d_len, C, delta) / omega)


def global_distance(pos, n: int):
    """Distance (in units of h) of grid position `pos` beyond the physical segment [0, n+1]."""
    pos = np.asarray(pos, dtype=np.float64)
    return np.maximum(0.0, np.maximum(-pos, pos - (n + 1)))


def axis_alphas(n: int, npml: int, h: float, C: float, omega: float, npml_profile: int | None = None):
    """alpha at every padded node and at the half nodes on either side.

    Returns (a_node, a_minus, a_plus), each of length n + 2 npml, for nodes
    p = -npml+1 .. n+npml (array index i = p + npml - 1).  The profile's
    delta is npml_profile * h (default npml * h).
    """
    p = np.arange(-npml + 1, n + npml + 1, dtype=np.float64)
    delta = (npml if npml_profile is None else npml_profile) * h
    a_node = pml_alpha(global_distance(p, n) * h, C, delta, omega)
    a_minus = pml_alpha(global_distance(p - 0.5, n) * h, C, delta, omega)
    a_plus = pml_alpha(global_distance(p + 0.5, n) * h, C, delta, omega)
    return a_node, a_minus, a_plus


# ----------------------------------------------------------------------------
# 5-point operator on a (rows x NX) grid from per-row z data
# ----------------------------------------------------------------------------

def _five_point(ax, axm, axp, az, azm, azp, m, h, omega):
    """Sparse A = h^2 H on a grid whose z rows carry (az, azm, azp) and model m (rows, NX)."""
    nrow, NX = m.shape
    N = nrow * NX
    idx = np.arange(N).reshape(nrow, NX)
    diag = (ax[None, :] * (axp[None, :] + axm[None, :])
            + az[:, None] * (azp[:, None] + azm[:, None])
            - (h * h * omega * omega) * m)
    rows = [idx.ravel()]
    cols = [idx.ravel()]
    vals = [diag.ravel()]
    # west / east couplings (Dirichlet beyond the padded grid: dropped)
    w = -(ax * axm)[None, :] * np.ones((nrow, 1))
    e = -(ax * axp)[None, :] * np.ones((nrow, 1))
    rows += [idx[:, 1:].ravel(), idx[:, :-1].ravel()]
    cols += [idx[:, :-1].ravel(), idx[:, 1:].ravel()]
    vals += [w[:, 1:].ravel(), e[:, :-1].ravel()]
    # up / down couplings
    up = -(az * azm)[:, None] * np.ones((1, NX))
    dn = -(az * azp)[:, None] * np.ones((1, NX))
    rows += [idx[1:, :].ravel(), idx[:-1, :].ravel()]
    cols += [idx[:-1, :].ravel(), idx[1:, :].ravel()]
    vals += [up[1:, :].ravel(), dn[:-1, :].ravel()]
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    return A


def global_operator(prob) -> sp.csr_matrix:
    """A = h^2 H for the whole PML-padded grid (eq. discrete_Helmholtz_equation), x fastest."""
    ax, axm, axp = axis_alphas(prob.nx, prob.px, prob.h, prob.C, prob.omega, prob.npml)
    az, azm, azp = axis_alphas(prob.nz, prob.npml, prob.h, prob.C, prob.omega)
    m = 1.0 / np.asarray(prob.c, dtype=np.float64) ** 2
    return _five_point(ax, axm, axp, az, azm, azp, m, prob.h, prob.omega)


def global_operator_loops(prob) -> np.ndarray:
    """Dense A built node by node with plain loops (independent second assembly; tiny grids only)."""
    NX, NZ = prob.NX, prob.NZ
    h, w, npml, C = prob.h, prob.omega, prob.npml, prob.C
    px = prob.px
    delta = npml * h

    def alpha_at(pos, n):
        d = max(0.0, -pos, pos - (n + 1)) * h
        s = (C / delta) * (d / delta) ** 2 if d > 0 else 0.0
        return 1.0 / (1.0 + 1j * s / w)

    A = np.zeros((NX * NZ, NX * NZ), dtype=np.complex128)
    for iz in range(NZ):
        q = iz - npml + 1
        for ix in range(NX):
            p = ix - px + 1
            r = iz * NX + ix
            a0x, amx, apx = alpha_at(p, prob.nx), alpha_at(p - 0.5, prob.nx), alpha_at(p + 0.5, prob.nx)
            a0z, amz, apz = alpha_at(q, prob.nz), alpha_at(q - 0.5, prob.nz), alpha_at(q + 0.5, prob.nz)
            m = 1.0 / prob.c[iz, ix] ** 2
            A[r, r] = a0x * (apx + amx) + a0z * (apz + amz) - h * h * w * w * m
            if ix > 0:
                A[r, r - 1] = -a0x * amx
            if ix < NX - 1:
                A[r, r + 1] = -a0x * apx
            if iz > 0:
                A[r, r - NX] = -a0z * amz
            if iz < NZ - 1:
                A[r, r + NX] = -a0z * apz
    return A


def symmetric_scaling(prob) -> np.ndarray:
    """diag(a_x a_z) over the padded grid (appendix, eq. Helmholtz_pml_symmetric)."""
    ax, _, _ = axis_alphas(prob.nx, prob.px, prob.h, prob.C, prob.omega, prob.npml)
    az, _, _ = axis_alphas(prob.nz, prob.npml, prob.h, prob.C, prob.omega)
    return (az[:, None] * ax[None, :]).ravel()


# ----------------------------------------------------------------------------
# layered decomposition (Section 2.2)
# ----------------------------------------------------------------------------

@dataclass
class Slab:
    """Layer ell (0-based `index`) of the decomposition.

    own_start: padded-grid row index of the first owned row
    n:         number of owned rows (the paper's n^ell, including global PML rows for the end layers)
    top_ext / bot_ext: extension rows added above / below (npml on interior sides, 0 on outer sides)
    Local rows r = 0..R-1; the paper's local index is j = r - top_ext + 1.
    """

    index: int
    own_start: int
    n: int
    top_ext: int
    bot_ext: int

    @property
    def R(self) -> int:
        return self.top_ext + self.n + self.bot_ext

    def row(self, j: int) -> int:
        """Local row r of the paper's local index j."""
        return j - 1 + self.top_ext

    def trace_rows(self) -> dict:
        """Local rows of j in {0, 1, n, n+1} that exist for this layer."""
        out = {}
        if self.top_ext:
            out["0"] = self.row(0)
            out["1"] = self.row(1)
        if self.bot_ext:
            out["n"] = self.row(self.n)
            out["n+1"] = self.row(self.n + 1)
        return out


def layer_split(prob) -> list[Slab]:
    """Even split of the nz physical rows into L layers (Section 2.2 with an even n_c^ell)."""
    L, nz, npml = prob.L, prob.nz, prob.npml
    if L < 1:
        raise ValueError("L must be >= 1")
    base, extra = divmod(nz, L)
    counts = [base + (1 if l < extra else 0) for l in range(L)]
    if min(counts) < 2:
        raise ValueError("every layer needs at least 2 physical rows")
    slabs = []
    start = 0
    for l in range(L):
        n = counts[l] + (npml if l == 0 else 0) + (npml if l == L - 1 else 0)
        slabs.append(Slab(l, start, n, npml if l > 0 else 0, npml if l < L - 1 else 0))
        start += n
    return slabs


def local_z_profile(prob, slab: Slab):
    """(az, azm, azp) and the model rows m~ (R, NX) of the local problem of `slab`.

    Owned rows inherit the global discretisation; extension rows carry a PML
    whose distance is measured from the first extension node (local j = 0 or
    n+1) and the normally extended model (Section 2.2, m~).
    """
    h, npml, C, w = prob.h, prob.npml, prob.C, prob.omega
    delta = npml * h
    q_start = slab.own_start - npml + 1  # global q of local j = 1
    n = slab.n

    def dist(zeta):
        if slab.top_ext and zeta < 1:
            return max(0.0, -zeta)
        if slab.bot_ext and zeta > n:
            return max(0.0, zeta - (n + 1))
        return float(global_distance(q_start + zeta - 1, prob.nz))

    js = np.arange(slab.R) - slab.top_ext + 1
    az = pml_alpha(np.array([dist(j) for j in js]) * h, C, delta, w)
    azm = pml_alpha(np.array([dist(j - 0.5) for j in js]) * h, C, delta, w)
    azp = pml_alpha(np.array([dist(j + 0.5) for j in js]) * h, C, delta, w)
    mg = 1.0 / np.asarray(prob.c, dtype=np.float64) ** 2
    rows = np.clip(slab.own_start + js - 1, slab.own_start, slab.own_start + n - 1)
    return az, azm, azp, mg[rows, :]


def local_operator(prob, slab: Slab) -> sp.csr_matrix:
    """A^ell = h^2 H^ell of eq. def_local_Green_function on the (R x NX) local grid."""
    ax, axm, axp = axis_alphas(prob.nx, prob.px, prob.h, prob.C, prob.omega, prob.npml)
    az, azm, azp, m = local_z_profile(prob, slab)
    return _five_point(ax, axm, axp, az, azm, azp, m, prob.h, prob.omega)


def restrict_source(prob, slab: Slab, f: np.ndarray) -> np.ndarray:
    """f^ell = f chi_{Omega^ell}, zero on the extension rows (Alg. 2, 'partition the source')."""
    NX = prob.NX
    f = np.asarray(f).reshape(-1, prob.NZ, NX)
    out = np.zeros((f.shape[0], slab.R, NX), dtype=np.complex128)
    out[:, slab.top_ext:slab.top_ext + slab.n, :] = f[:, slab.own_start:slab.own_start + slab.n, :]
    return out
