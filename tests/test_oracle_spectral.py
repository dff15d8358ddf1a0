"""The oracle against the spectral claims of Section 4.2 and of the eigenvalue
figures of the numerical section (parity pins for the spectral diagnostics).

- D^-1 A = I + D^-1 R; the Gauss-Seidel preconditioner with n_it sweeps from
  zero (Alg. 4) gives M^-1 A = I - (-D^-1 R)^n_it, so for n_it = 2 every
  eigenvalue of M^-1 A is 1 - (lambda - 1)^2 for an eigenvalue lambda of
  D^-1 A (a pin between two independent assemblies of the oracle).
- Homogeneous medium: every reflection comes from the PML, so the eigenvalues
  of D^-1 A tighten around 1 as the PML widens (the figure with 5, 30 and 100
  PML points; here 4, 8 and 16 on a 24 x 24 grid).
- Resonant cavity (ring of speed 5 in a smooth background; the ring shape is
  invented, see synth.cavity_medium): the count of eigenvalues outside the
  disc of radius 0.2 around 1 grows with the frequency (the figure at
  omega = 8, 16, 32).
"""
import numpy as np
from scipy.optimize import linear_sum_assignment

import synth
from oracle.polarized import PolarizedSolver


def _spec(ps, which="DinvA"):
    if which == "DinvA":
        M = ps.dense("Dinv") @ ps.dense("A")
    else:
        n = 4 * (ps.L - 1) * ps.NX
        E = np.eye(n, dtype=np.complex128).reshape(n, 2, ps.L - 1, 2, ps.NX)
        M = ps.precondition(ps.apply_A(E), n_it=2).reshape(n, n).T
    return np.linalg.eigvals(M)


def test_gauss_seidel_spectrum_is_one_minus_square():
    ps = PolarizedSolver(synth.cavity_problem(32, 16.0, npml=5, L=4))
    e_d = _spec(ps, "DinvA")
    e_m = _spec(ps, "MinvA")
    pred = 1.0 - (e_d - 1.0) ** 2
    C = np.abs(e_m[:, None] - pred[None, :])
    r, c = linear_sum_assignment(C)
    assert C[r, c].max() < 1e-9
    # and a plausible slip (one sweep, n_it = 1, i.e. M^-1 = D^-1) fails the pin
    C1 = np.abs(e_d[:, None] - pred[None, :])
    r1, c1 = linear_sum_assignment(C1)
    assert C1[r1, c1].max() > 1e-3


def test_homogeneous_spectrum_tightens_with_pml_width():
    spread = []
    for npml in (4, 8, 16):
        ev = _spec(PolarizedSolver(synth.homogeneous_problem(24, npml, L=3)))
        spread.append(float(np.abs(ev - 1.0).max()))
    assert spread[0] < 0.1  # clustered around 1 already at 4 points
    assert spread[0] > 5 * spread[1] > 25 * spread[2]


def test_cavity_spectrum_spreads_with_frequency():
    outside, dist = [], []
    for om in (8.0, 16.0, 32.0):
        ev = _spec(PolarizedSolver(synth.cavity_problem(48, om, npml=6, L=4)))
        d = np.abs(ev - 1.0)
        outside.append(int(np.sum(d > 0.2)))
        dist.append(float(d.max()))
    assert 0 < outside[0] < outside[1] < outside[2]
    assert dist[0] < dist[1] < dist[2]


def test_gauss_seidel_with_n_sweeps_is_a_truncated_neumann_series():
    # Alg. 4 from u^0 = 0 with n sweeps: M_n^-1 = sum_{j<n} (-D^-1 R)^j D^-1, so M_n^-1 A = I - (-D^-1 R)^n;
    # pins the oracle's sweep loop for every n the GPU path is compared at
    ps = PolarizedSolver(synth.config_small(nx=12, nz=24, npml=4, L=3, nrhs=1, seed=5)[0])
    n = 4 * (ps.L - 1) * ps.NX
    E = np.eye(n, dtype=np.complex128).reshape(n, 2, ps.L - 1, 2, ps.NX)
    G = -ps.dense("Dinv") @ ps.dense("R")
    AE = ps.apply_A(E)
    for n_it in (1, 3, 4, 8):
        M = ps.precondition(AE, n_it=n_it).reshape(n, n).T
        ref = np.eye(n) - np.linalg.matrix_power(G, n_it)
        assert np.abs(M - ref).max() < 1e-10 * max(1.0, np.abs(ref).max()), n_it
        # an off-by-one in the sweep count fails it (where G^n is not yet negligible)
        if np.abs(ref - np.eye(n)).max() > 1e-5:
            assert np.abs(M - (np.eye(n) - np.linalg.matrix_power(G, n_it + 1))).max() > 1e-6, n_it
    assert np.abs(np.linalg.matrix_power(G, 4)).max() > 1e-5  # the off-by-one check ran for n = 1, 3 and 4
    # no sweeps: no preconditioner, so the preconditioned operator is A itself
    assert np.abs(ps.precondition(AE, n_it=0).reshape(n, n).T - ps.dense("A")).max() == 0.0
