"""The oracle's extrapolation-closed polarized system (Section 3.4, Def.
polarized_out_going, eq. splitting_out_going) against what the paper and the
mathematics fix:

- the one-sided extrapolators (Def. extrapolator) reproduce the Green's
  functions one row further (Lemma extrapolator_def):
  E_down K_{n,j} = K_{n+1,j} for j = 0, 1 and E_up K_{1,j} = K_{0,j} for
  j = n, n+1;
- the polarized traces of the sparse direct solution satisfy the system with
  its right-hand side (zero on the extrapolation rows);
- A = D + R, D has identity diagonal blocks and is block-triangular per
  half, its sweeps invert it, and D^extrap^-1 = D_jump^-1 T with
  T r = (r_n, r_{n+1} + E_down r_n; r_0 + E_up r_1, r_1) (the route the GPU
  takes, by Lemma extrapolator_def);
- flexible GMRES on it (Gauss-Seidel with 1 and 2 sweeps) gives the same
  traces and volume field as the jump-closed system and the direct solve.
"""
import numpy as np
import pytest

import synth
from oracle.direct import DirectSolver
from oracle.extrap import ExtrapSystem
from oracle.polarized import PolarizedSolver


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.fixture(scope="module")
def sys4():
    prob, f = synth.config_small(nx=20, nz=36, npml=5, L=4, nrhs=2, seed=33)
    ps = PolarizedSolver(prob)
    ex = ExtrapSystem(ps)
    u = DirectSolver(prob).solve(f)
    return prob, f, ps, ex, u


def _traces(ps, u, f):
    """Polarized traces of the direct solution: the jump system's solution (pinned in
    test_oracle_polarized), from the jump FGMRES at tight tolerance."""
    x, _ = ps.fgmres(ps.rhs(ps.newton(f)), tol=1e-13, maxit=200)
    return x


def test_extrapolators_reproduce_green_rows(sys4):
    prob, f, ps, ex, u = sys4
    for k in range(ps.L - 1):
        Kt, Kb = ps.loc[k].K, ps.loc[k + 1].K
        checked = 0
        for j in ("0", "1"):  # sources above row n (layers with a top interface)
            if ("n", j) in Kt:
                assert rel(ex.E_dn[k] @ Kt[("n", j)], Kt[("n+1", j)]) < 1e-10, (k, j)
                checked += 1
        for j in ("n", "n+1"):  # sources below row 1 (layers with a bottom interface)
            if ("1", j) in Kb:
                assert rel(ex.E_up[k] @ Kb[("1", j)], Kb[("0", j)]) < 1e-10, (k, j)
                checked += 1
        assert checked >= 2
    # and not one row further the other way: the extrapolator does not reach past its source rows
    Kt = ps.loc[1].K
    assert rel(ex.E_dn[1] @ Kt[("n", "n+1")], Kt[("n+1", "n+1")]) > 1e-3


def test_extrapolators_reach_every_owned_source(sys4):
    """Lemma extrapolator_def over all owned source rows (not only the trace rows):
    row n+1 of a layer's inverse is E_down times row n on the columns of rows j <= n,
    row 0 is E_up times row 1 on the columns of rows j >= 1."""
    prob, f, ps, ex, u = sys4
    NX = ps.NX
    for k in range(ps.L - 1):
        for lay, E, tgt, src, cols in ((ps.loc[k], ex.E_dn[k], "n+1", "n", "le_n"),
                                      (ps.loc[k + 1], ex.E_up[k], "0", "1", "ge_1")):
            s = lay.slab
            R = s.R
            inv = lay.solve(np.eye(R * NX, dtype=np.complex128).reshape(R * NX, R, NX))  # columns of the inverse
            inv = inv.reshape(R * NX, R * NX).T  # inv[i, c] = (A^l)^-1 entry (row i, column c)
            rt, rs = lay.rows[tgt], lay.rows[src]
            own = slice(s.top_ext * NX, (s.top_ext + s.n) * NX)  # owned rows j = 1..n
            rows_t = inv[rt * NX:(rt + 1) * NX, own]
            rows_s = inv[rs * NX:(rs + 1) * NX, own]
            assert rel(E @ rows_s, rows_t) < 1e-9, (k, tgt)


def test_polarized_traces_solve_the_system(sys4):
    prob, f, ps, ex, u = sys4
    x = _traces(ps, u, f)
    assert rel(x[:, 0] + x[:, 1], ps.traces_of(u)) < 1e-9
    s = ex.rhs(ps.newton(f))
    assert rel(ex.apply_A(x), s) < 1e-9
    # the jump closure's second rows are not satisfied by the extrapolation system's operator
    assert rel(ex.apply_A(x), ps.rhs(ps.newton(f))) > 1e-3


def test_splitting_structure_and_sweeps(sys4):
    prob, f, ps, ex, u = sys4
    A, D, R = ex.dense("A"), ex.dense("D"), ex.dense("R")
    assert rel(D + R, A) < 1e-14
    n = A.shape[0]
    h = n // 2
    NX = ps.NX
    # identity diagonal blocks (NX x NX) and no coupling across polarizations in D
    for b in range(n // NX):
        assert np.allclose(D[b * NX:(b + 1) * NX, b * NX:(b + 1) * NX], np.eye(NX), atol=1e-14)
    assert np.abs(D[:h, h:]).max() == 0.0 and np.abs(D[h:, :h]).max() == 0.0
    # down half block lower triangular, up half block upper triangular
    assert np.abs(np.triu(D[:h, :h], NX)).max() == 0.0
    assert np.abs(np.tril(D[h:, h:], -NX)).max() == 0.0
    Dinv = ex.dense("Dinv")
    assert rel(Dinv @ D, np.eye(n)) < 1e-12
    # D^extrap^-1 = D_jump^-1 T
    T = np.eye(n, dtype=np.complex128).reshape(n, 2, ps.L - 1, 2, NX).copy()
    Tm = np.eye(n, dtype=np.complex128)
    blk = lambda hh, k, r: ((hh * (ps.L - 1) + k) * 2 + r) * NX
    for k in range(ps.L - 1):
        i, j = blk(0, k, 1), blk(0, k, 0)
        Tm[i:i + NX, j:j + NX] = ex.E_dn[k]
        i, j = blk(1, k, 0), blk(1, k, 1)
        Tm[i:i + NX, j:j + NX] = ex.E_up[k]
    assert rel(ps.dense("Dinv") @ Tm, Dinv) < 1e-10


@pytest.mark.parametrize("n_it", [1, 2])
def test_fgmres_matches_jump_and_direct(sys4, n_it):
    prob, f, ps, ex, u = sys4
    ue, xe, info = ex.solve(f, tol=1e-11, maxit=80, n_it=n_it)
    assert rel(ue, u) < 1e-8
    xj = _traces(ps, u, f)
    assert rel(xe, xj) < 1e-8
    assert all(i["relres"] < 1e-10 for i in info)
