"""Spectral diagnostics on the GPU path against the oracle.

The preconditioned operators are assembled on the GPU from the library's own
applies (paper_1410_5910_amd.spectral) and compared entry by entry with the
oracle's dense forms; their spectra then reproduce the oracle-pinned claims
(the Gauss-Seidel relation eig(M^-1 A) = 1 - (eig(D^-1 A) - 1)^2 for n_it = 2,
tightening with the PML width in a homogeneous medium, spreading with the
frequency in a resonant cavity).
"""
import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

import synth
from oracle.polarized import PolarizedSolver

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1410_5910_amd")
from paper_1410_5910_amd import spectral  # noqa: E402


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _flush(msg):
    print(msg, flush=True)


def _solver(prob, nrhs=48):
    return P.Solver.from_problem(prob, max_nrhs=nrhs, tol=1e-10, maxit=60)


def test_assembled_operators_match_oracle():
    prob = synth.cavity_problem(32, 16.0, npml=5, L=4)
    _flush(f"[gpu] spectral assembly {prob.name}")
    gs, ps = _solver(prob), PolarizedSolver(prob)
    ref = {"A": ps.dense("A"), "R": ps.dense("R"), "Dinv": ps.dense("Dinv")}
    ref["DinvA"] = ref["Dinv"] @ ref["A"]
    for op, M in ref.items():
        G = spectral.operator_matrix(gs, op).cpu().numpy()
        assert G.shape == M.shape
        assert rel(G, M) < 1e-10, op
    gs.close()


def test_spectra_match_oracle_and_gauss_seidel_relation():
    prob = synth.cavity_problem(48, 16.0, npml=6, L=4)
    _flush(f"[gpu] spectral relation {prob.name}")
    gs, ps = _solver(prob, 64), PolarizedSolver(prob)
    e_d = spectral.eigenvalues(gs, "DinvA")
    e_m = spectral.eigenvalues(gs, "MinvA")
    pred = 1.0 - (e_d - 1.0) ** 2
    C = np.abs(e_m[:, None] - pred[None, :])
    r, c = linear_sum_assignment(C)
    assert C[r, c].max() < 1e-8
    e_o = np.linalg.eigvals(ps.dense("Dinv") @ ps.dense("A"))
    C = np.abs(e_d[:, None] - e_o[None, :])
    r, c = linear_sum_assignment(C)
    assert C[r, c].max() < 1e-8
    so, sg = spectral.cluster_summary(e_o), spectral.cluster_summary(e_d)
    assert so["outside"] == sg["outside"]
    gs.close()


def test_homogeneous_spectrum_tightens_with_pml_width():
    spread = []
    for npml in (4, 8, 16):
        prob = synth.homogeneous_problem(32, npml, L=3)
        _flush(f"[gpu] spectral {prob.name}")
        gs = _solver(prob, 64)
        spread.append(spectral.cluster_summary(spectral.eigenvalues(gs))["max_dist_from_1"])
        gs.close()
    assert spread[0] < 0.1
    assert spread[0] > 5 * spread[1] > 25 * spread[2]


def test_cavity_spectrum_spreads_with_frequency():
    outside = []
    for om in (8.0, 16.0, 32.0):
        prob = synth.cavity_problem(64, om, npml=8, L=4)
        _flush(f"[gpu] spectral {prob.name}")
        gs = _solver(prob, 64)
        outside.append(spectral.cluster_summary(spectral.eigenvalues(gs))["outside"])
        gs.close()
    assert 0 < outside[0] < outside[1] < outside[2]
