"""Partitioned low-rank (PLR) compression and matrix-vector product (oracle; test infrastructure only).

Follows the paper's Section 5.1: Alg. 5 (adaptive quadtree compression: a
block becomes a leaf when its (r_max+1)-th singular value is below eps,
otherwise it is split into four and each quarter is compressed) and Alg. 6
(recursive matrix-vector product over the tree, computed in the paper in a
sparse-factorised form).

Readings (the paper leaves these open):
  * eps is absolute on the singular values; a leaf keeps the k <= r_max
    singular triplets with sigma_i >= eps (the paper stores U*Sigma and V^t
    of the r_max+1 leading triplets); its error is then sigma_{k+1} < eps in
    the 2-norm;
  * a block whose smaller side is <= r_max cannot be tested this way and is
    kept as a dense leaf;
  * an odd side is split into ceil/floor halves;
  * the printed matvec recursion has garbled index ranges; the product is
    y_i += sum_j H_ij x_j over the quarters.
The partition is not unique near thresholds, so other implementations are
compared on products, not trees.

Pinned by tests/test_oracle_plr.py: exact low-rank inputs become one leaf of
that rank, full-rank inputs end in dense leaves, the leaves tile the block
exactly once, every discarded singular value is below eps, the product is
within the sum-of-leaf-error bound of the dense product, and the
sparse-factorised form gives the same product as the recursion.
"""
from __future__ import annotations

import numpy as np


class Node:
    """kind 'c' (leaf: low-rank 'lr' or 'dense'), or 'h' (branch with 2x2 children)."""

    __slots__ = ("kind", "r0", "c0", "m", "n", "U", "V", "D", "children", "sigma_next")

    def __init__(self, kind, r0, c0, m, n):
        self.kind, self.r0, self.c0, self.m, self.n = kind, r0, c0, m, n
        self.U = self.V = self.D = None
        self.children = None
        self.sigma_next = 0.0


def compress(M: np.ndarray, rmax: int, eps: float, r0: int = 0, c0: int = 0) -> Node:
    """Alg. 5: PLR tree of M (m x n)."""
    m, n = M.shape
    if min(m, n) <= rmax:
        nd = Node("dense", r0, c0, m, n)
        nd.D = M.copy()
        return nd
    U, s, Vh = np.linalg.svd(M, full_matrices=False)
    if s[rmax] < eps:  # the (r_max+1)-th singular value
        k = int(np.sum(s >= eps))
        nd = Node("lr", r0, c0, m, n)
        nd.U = U[:, :k] * s[:k]      # U Sigma
        nd.V = Vh[:k, :]             # V^t (conjugate-transposed right factor)
        nd.sigma_next = float(s[k]) if k < len(s) else 0.0
        return nd
    m1, n1 = (m + 1) // 2, (n + 1) // 2
    nd = Node("h", r0, c0, m, n)
    nd.children = [[compress(M[:m1, :n1], rmax, eps, r0, c0), compress(M[:m1, n1:], rmax, eps, r0, c0 + n1)],
                   [compress(M[m1:, :n1], rmax, eps, r0 + m1, c0), compress(M[m1:, n1:], rmax, eps, r0 + m1, c0 + n1)]]
    return nd


def matvec(H: Node, x: np.ndarray) -> np.ndarray:
    """Alg. 6: y = H x for x of shape (n,) or (n, k) (local indexing of H)."""
    if H.kind == "lr":
        return H.U @ (H.V @ x)
    if H.kind == "dense":
        return H.D @ x
    n1 = H.children[0][0].n
    m1 = H.children[0][0].m
    y = np.zeros((H.m,) + x.shape[1:], dtype=np.result_type(x, np.complex128))
    for i in range(2):
        rows = slice(0, m1) if i == 0 else slice(m1, H.m)
        y[rows] += matvec(H.children[i][0], x[:n1])
        y[rows] += matvec(H.children[i][1], x[n1:])
    return y


def leaves(H: Node) -> list:
    if H.kind != "h":
        return [H]
    return [lf for row in H.children for ch in row for lf in leaves(ch)]


def to_dense(H: Node) -> np.ndarray:
    """The matrix the tree represents."""
    M = np.zeros((H.m, H.n), dtype=np.complex128)
    for lf in leaves(H):
        blk = lf.D if lf.kind == "dense" else lf.U @ lf.V
        M[lf.r0 - H.r0:lf.r0 - H.r0 + lf.m, lf.c0 - H.c0:lf.c0 - H.c0 + lf.n] = blk
    return M


def sparse_factorized_matvec(H: Node, x: np.ndarray) -> np.ndarray:
    """The sparse-factorised form of the product (Section 5.1): t = blockdiag(V_leaf) x over the
    leaves' column ranges, then y = blockdiag(U_leaf) t scattered to their row ranges."""
    lv = leaves(H)
    ts = []
    for lf in lv:
        xs = x[lf.c0 - H.c0:lf.c0 - H.c0 + lf.n]
        ts.append(lf.D @ xs if lf.kind == "dense" else lf.V @ xs)
    y = np.zeros((H.m,) + x.shape[1:], dtype=np.complex128)
    for lf, t in zip(lv, ts):
        y[lf.r0 - H.r0:lf.r0 - H.r0 + lf.m] += t if lf.kind == "dense" else lf.U @ t
    return y


def stored_entries(H: Node) -> int:
    """Complex entries stored by the tree: (m + n) k per low-rank leaf, m n per dense leaf."""
    return sum(lf.m * lf.n if lf.kind == "dense" else (lf.m + lf.n) * lf.U.shape[1] for lf in leaves(H))
