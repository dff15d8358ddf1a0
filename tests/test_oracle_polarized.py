"""Pins of the oracle's polarized-traces solve (CPU only).

Lemma 1 (discrete GRF), Lemma 4 (extrapolator / jump identities), the
symmetric PML form of the appendix (reciprocity), Def. 4 / Thm. 1 (integral
system), Def. 9 / Prop. 1 (polarized system), Section 4.2 (spectral
structure), Alg. 3 / Alg. 4 (Gauss-Seidel), appendix B (Usmani's closed form
of the tridiagonal inverse).
"""
import numpy as np
import pytest

import synth
from oracle import assemble as asm
from oracle.direct import DirectSolver
from oracle.polarized import PolarizedSolver, LocalProblem


@pytest.fixture(scope="module")
def small3():
    prob, f = synth.config_small(nx=20, nz=27, npml=4, L=3, nrhs=2, seed=11)
    ps = PolarizedSolver(prob)
    u = DirectSolver(prob).solve(f)
    return prob, f, ps, u


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_grf_reproduces_traces_and_vanishes_outside(small3):
    # Lemma 1: with the traces of the global solution, the GRF gives u on rows 1..n
    # and 0 at rows 0 and n+1 (eqs. discrete_GRF_inside / discrete_GRF_outside)
    prob, f, ps, u = small3
    w = ps.newton(f)
    t = ps.traces_of(u)
    for l, lp in enumerate(ps.loc):
        s = lp.slab
        for j, r in lp.rows.items():
            acc = w[l][:, r].copy()
            if l >= 1:
                acc += lp.g_down(j, t[:, l - 1, 0], t[:, l - 1, 1])
            if l <= ps.L - 2:
                acc += lp.g_up(j, t[:, l, 0], t[:, l, 1])
            jj = {"0": 0, "1": 1, "n": s.n, "n+1": s.n + 1}[j]
            if j in ("1", "n"):
                ref = u[:, s.own_start + jj - 1]
                assert rel(acc, ref) < 1e-11, (l, j)
            else:
                assert np.linalg.norm(acc) < 1e-11 * np.linalg.norm(u), (l, j)


def test_grf_full_layer_as_forced_solve(small3):
    # eq. PDE_version_green_formula: one forced local solve gives u on owned rows, 0 on extension rows
    prob, f, ps, u = small3
    t = ps.traces_of(u)
    for l, lp in enumerate(ps.loc):
        s = lp.slab
        b = prob.h ** 2 * asm.restrict_source(prob, s, f)
        if l >= 1:
            b[:, lp.rows["1"]] += t[:, l - 1, 0]
            b[:, lp.rows["0"]] -= t[:, l - 1, 1]
        if l <= ps.L - 2:
            b[:, lp.rows["n+1"]] -= t[:, l, 0]
            b[:, lp.rows["n"]] += t[:, l, 1]
        v = lp.solve(b)
        assert rel(v[:, s.top_ext:s.top_ext + s.n], u[:, s.own_start:s.own_start + s.n]) < 1e-11
        outside = np.concatenate([v[:, :s.top_ext], v[:, s.top_ext + s.n:]], axis=1)
        assert np.linalg.norm(outside) < 1e-11 * np.linalg.norm(u)


def test_extrapolator_and_jump_identities(small3):
    # Lemma 4 (A scaling): K_{n+1,j} = E_dn K_{n,j} (j <= n), K_{0,j} = E_up K_{1,j} (j >= 1),
    # K_{n+1,n+1} - E_dn = E_dn K_{n,n+1}, K_{0,0} - E_up = E_up K_{1,0}
    prob, f, ps, u = small3
    for lp in ps.loc:
        K = lp.K
        if "n" in lp.rows:
            E = np.linalg.solve(K[("n", "n")], K[("n", "n+1")])
            for j in [k for k in ("0", "1", "n") if k in lp.rows]:
                assert rel(E @ K[("n", j)], K[("n+1", j)]) < 1e-10
            assert rel(K[("n+1", "n+1")] - E, E @ K[("n", "n+1")]) < 1e-10
        if "0" in lp.rows:
            E = np.linalg.solve(K[("1", "1")], K[("1", "0")])
            for j in [k for k in ("1", "n", "n+1") if k in lp.rows]:
                assert rel(E @ K[("1", j)], K[("0", j)]) < 1e-10
            assert rel(K[("0", "0")] - E, E @ K[("1", "0")]) < 1e-10


def test_block_reciprocity(small3):
    # appendix: G(x,y) alpha(y) = G^s(x,y) with G^s symmetric => K_jk diag(a_x) = diag(a_x) K_kj^T
    prob, f, ps, u = small3
    ax, _, _ = asm.axis_alphas(prob.nx, prob.npml, prob.h, prob.C, prob.omega)
    for lp in ps.loc:
        for (j, k), Kjk in lp.K.items():
            lhs = Kjk * ax[None, :]
            rhs = ax[:, None] * lp.K[(k, j)].T
            assert rel(lhs, rhs) < 1e-10


def test_integral_system_satisfied_by_direct_traces(small3):
    # Def. 4 / Thm. 1: M t* = -f with t* the traces of the direct solution
    prob, f, ps, u = small3
    t = ps.traces_of(u)
    lhs = ps.apply_M(t)
    rhs = -ps.newton_rows(ps.newton(f))
    assert rel(lhs, rhs) < 1e-11


def test_polarized_system_gives_direct_traces(small3):
    # Prop. 1: the solution of the jump-closed polarized system sums to the global traces
    prob, f, ps, u = small3
    s = ps.rhs(ps.newton(f))
    A = ps.dense("A")
    x = np.linalg.solve(A, s.reshape(s.shape[0], -1).T).T.reshape(s.shape)
    assert rel(x[:, 0] + x[:, 1], ps.traces_of(u)) < 1e-10
    # and the operator is the sum of its block-triangular part and the rest
    assert rel(ps.dense("D") + ps.dense("R"), A) < 1e-14
    # D^-1 by the two sweeps inverts D
    Dinv = ps.dense("Dinv")
    assert rel(Dinv @ ps.dense("D"), np.eye(A.shape[0])) < 1e-12


def test_spectral_structure(small3):
    # Section 4.2: U and L carry the extrapolation structure, so R has rank <= half;
    # D^-1 A = I + D^-1 R has >= half its eigenvalues at 1 and the others in 1 +- sqrt(mu) pairs
    prob, f, ps, u = small3
    n = 4 * (ps.L - 1) * ps.NX
    R = ps.dense("R")
    sv = np.linalg.svd(R, compute_uv=False)
    assert np.sum(sv < 1e-9 * sv[0]) >= n // 2
    T = ps.dense("Dinv") @ R
    nu = np.linalg.eigvals(T)
    big = nu[np.abs(nu) > 1e-6]
    # +- pairing of the non-zero eigenvalues of the Gauss-Seidel iteration matrix
    for z in big:
        assert np.min(np.abs(big + z)) < 1e-6 * max(1.0, abs(z))
    # mu = nu^2 are the eigenvalues of (D_up^-1 L)(D_dn^-1 U)
    h = n // 2
    mu = np.linalg.eigvals(T[h:, :h] @ T[:h, h:])
    mub = np.sort_complex(mu[np.abs(mu) > 1e-10])
    nu2 = np.sort_complex((big ** 2)[::1])
    # each mu appears twice among nu^2 (from +nu and -nu)
    for m in mub:
        assert np.sum(np.abs(nu2 - m) < 1e-6 * max(1.0, abs(m))) >= 2


def test_L2_means_D_is_identity():
    prob, f = synth.config_small(nx=12, nz=16, npml=3, L=2, nrhs=1)
    ps = PolarizedSolver(prob)
    D = ps.dense("D")
    assert np.array_equal(D, np.eye(D.shape[0]))


def test_L1_is_a_direct_solve():
    prob, f = synth.config_small(nx=12, nz=16, npml=3, L=1, nrhs=2)
    u1, _ = PolarizedSolver(prob).solve(f)
    u0 = DirectSolver(prob).solve(f)
    assert rel(u1, u0) < 1e-12


def _usmani_inverse(b, a, c):
    """Inverse of the tridiagonal with diagonal b, sub-diagonal a (a[i] = H[i+1, i]) and
    super-diagonal c (c[i] = H[i, i+1]) from the theta/phi minor recurrences (appendix B)."""
    n = len(b)
    th = np.zeros(n + 1, dtype=complex)
    th[0] = 1.0
    th[1] = b[0]
    for i in range(2, n + 1):
        th[i] = b[i - 1] * th[i - 1] - a[i - 2] * c[i - 2] * th[i - 2]
    ph = np.zeros(n + 2, dtype=complex)
    ph[n + 1] = 1.0
    ph[n] = b[n - 1]
    for i in range(n - 1, 0, -1):
        ph[i] = b[i - 1] * ph[i + 1] - c[i - 1] * a[i - 1] * ph[i + 2]
    G = np.zeros((n, n), dtype=complex)
    for i in range(1, n + 1):
        for j in range(1, n + 1):
            if i == j:
                G[i - 1, j - 1] = th[i - 1] * ph[i + 1] / th[n]
            elif i < j:
                G[i - 1, j - 1] = (-1) ** (i + j) * np.prod(c[i - 1:j - 1]) * th[i - 1] * ph[j + 1] / th[n]
            else:
                G[i - 1, j - 1] = (-1) ** (i + j) * np.prod(a[j - 1:i - 1]) * th[j - 1] * ph[i + 1] / th[n]
    return G


def test_one_dimensional_blocks_match_usmani_closed_form():
    # a single column (n' = 1): every trace block is one entry of a tridiagonal inverse
    nz, npml = 14, 4
    c = np.ones((nz + 2 * npml, 1)) * 1.3
    prob = synth.Problem("col", 1, nz, npml, 1.0 / 15, 7.0, 2, 20.0, c, npml_x=0)
    ps = PolarizedSolver(prob)
    for lp in ps.loc:
        T = lp.A.toarray()
        b, a, cc = np.diag(T), np.diag(T, -1), np.diag(T, 1)
        G = _usmani_inverse(b, a, cc)
        assert rel(G, np.linalg.inv(T)) < 1e-10  # the closed form itself
        for (j, k), Kjk in lp.K.items():
            assert Kjk.shape == (1, 1)
            assert abs(Kjk[0, 0] - G[lp.rows[j], lp.rows[k]]) < 1e-10 * abs(G[lp.rows[j], lp.rows[k]])


@pytest.mark.parametrize("L", [2, 3, 4])
def test_full_solve_matches_direct(L):
    prob, f = synth.config_small(nx=18, nz=28, npml=4, L=L, nrhs=2, seed=5)
    ps = PolarizedSolver(prob)
    u, info = ps.solve(f, tol=1e-12)
    assert rel(u, DirectSolver(prob).solve(f)) < 1e-10
    for it in info:
        h = it["hist"]
        assert all(b <= a * (1 + 1e-12) for a, b in zip(h, h[1:]))  # GMRES residual is non-increasing
        assert it["relres"] < 1e-10


def test_preconditioner_is_two_gauss_seidel_updates(small3):
    # Alg. 4 with n_it = 2: u1 = D^-1 r, u2 = D^-1 (r - R u1)
    prob, f, ps, u = small3
    r = np.random.default_rng(0).standard_normal(ps.zeros(1).shape) + 0j
    u1 = ps.apply_D_inv(r)
    u2 = ps.apply_D_inv(r - ps.apply_R(u1))
    assert rel(ps.precondition(r, 2), u2) < 1e-15
    assert rel(ps.precondition(r, 1), u1) < 1e-15


def test_gauss_seidel_iteration_converges():
    # Alg. 3 as a stand-alone solver on a smooth medium
    prob, f = synth.config_small(nx=20, nz=30, npml=5, L=3, nrhs=1, seed=2)
    ps = PolarizedSolver(prob)
    s = ps.rhs(ps.newton(f))
    x, hist = ps.gauss_seidel(s, tol=1e-10, maxit=200)
    assert hist[-1] < 1e-10
    u = ps.reconstruct(f, x)
    assert rel(u, DirectSolver(prob).solve(f)) < 1e-8


def test_operator_rows_by_extrapolation(small3):
    # Lemma 4 turns the second row of each interface pair of y = A x into one extrapolation of
    # the first: y_dn[k, n+1] = d_k[n+1] - E_dn(k) (d_k[n] - y_dn[k, n]) and
    # y_up[k, 0] = a_k[0] - E_up(k+1) (a_k[1] - y_up[k, 1]); with general couplings the
    # identities K_{n+1,n+1} - E_dn K_{n,n+1} = Sigma^-1 and K_{0,0} - E_up K_{1,0} = Delta^-1 (the
    # one-row Schur complements) add (Sigma^-1 - E_dn) a_k[n] resp. (Delta^-1 - E_up) d_k[n+1],
    # which vanish in the A scaling (couplings -1 at the trace rows).
    prob, f, ps, u = small3
    rng = np.random.default_rng(5)
    x = rng.standard_normal(ps.zeros(3).shape) + 1j * rng.standard_normal(ps.zeros(3).shape)
    y = ps.apply_A(x)
    d, a = x[:, 0], x[:, 1]
    for k in range(ps.L - 1):
        up, lo = ps.loc[k], ps.loc[k + 1]
        Kt, Kb = up.K, lo.K
        Edn = np.linalg.solve(Kt[("n", "n")], Kt[("n", "n+1")])
        Eup = np.linalg.solve(Kb[("1", "1")], Kb[("1", "0")])
        Sig = Kt[("n+1", "n+1")] - Edn @ Kt[("n", "n+1")]
        Dlt = Kb[("0", "0")] - Eup @ Kb[("1", "0")]
        y1 = d[:, k, 1] - (d[:, k, 0] - y[:, 0, k, 0] + a[:, k, 0]) @ Edn.T + a[:, k, 0] @ Sig.T
        y0 = a[:, k, 0] - (a[:, k, 1] - y[:, 1, k, 1] + d[:, k, 1]) @ Eup.T + d[:, k, 1] @ Dlt.T
        assert rel(y1, y[:, 0, k, 1]) < 1e-10, k
        assert rel(y0, y[:, 1, k, 0]) < 1e-10, k
        # A scaling: the one-row Schur complements are the extrapolators themselves
        assert rel(Sig, Edn) < 1e-10 and rel(Dlt, Eup) < 1e-10
        assert rel(d[:, k, 1] - (d[:, k, 0] - y[:, 0, k, 0]) @ Edn.T, y[:, 0, k, 1]) < 1e-10
        assert rel(a[:, k, 0] - (a[:, k, 1] - y[:, 1, k, 1]) @ Eup.T, y[:, 1, k, 0]) < 1e-10
