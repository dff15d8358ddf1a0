"""Pins of the oracle's direct solve (CPU only): residual, brute force, free-space Green's function."""
import math

import numpy as np
import pytest
import scipy.special

import synth
from oracle import assemble as asm
from oracle.direct import DirectSolver


def test_direct_residual_and_bruteforce():
    prob, f = synth.config_small(nx=8, nz=8, npml=3, L=1, nrhs=2)
    ds = DirectSolver(prob)
    u = ds.solve(f)
    A = asm.global_operator(prob)
    b = (prob.h ** 2 * f).reshape(2, -1)
    r = np.linalg.norm(A @ u.reshape(2, -1).T - b.T) / np.linalg.norm(b)
    assert r < 1e-12
    # brute force: dense solve of the loop-assembled matrix
    Ad = asm.global_operator_loops(prob)
    ud = np.linalg.solve(Ad, b.T).T.reshape(u.shape)
    assert np.linalg.norm(ud - u) / np.linalg.norm(u) < 1e-12


def _hankel_error(nint, omega=2 * math.pi * 2, delta=0.25):
    # unit-size physical box: L_x = (nx+1) h = 1, source at the centre node
    h = 1.0 / (nint + 1)
    npml = int(round(delta / h))
    c = np.ones((nint + 2 * npml, nint + 2 * npml))
    prob = synth.Problem("hankel", nint, nint, npml, h, omega, 1, 30.0, c)
    f = np.zeros((prob.NZ, prob.NX), dtype=complex)
    pc = (nint + 1) // 2
    ic = pc + npml - 1
    f[ic, ic] = 1.0 / h ** 2  # discrete delta (Section 2.3)
    u = DirectSolver(prob).solve(f)
    p = np.arange(-npml + 1, nint + npml + 1) * h
    X, Z = np.meshgrid(p, p)
    r = np.hypot(X - pc * h, Z - pc * h)
    mask = (r >= 0.2) & (r <= 0.4)
    g = 0.25j * scipy.special.hankel1(0, omega * r[mask])
    return np.max(np.abs(u[mask] - g)) / np.max(np.abs(g))


@pytest.mark.slow
def test_second_order_convergence_to_hankel():
    # constant medium: u -> (i/4) H0^(1)(omega r) at second order (5-point stencil)
    errs = [_hankel_error(n) for n in (39, 79, 159)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert errs[2] < 2e-3
    assert 3.5 <= r1 <= 4.5 and 3.5 <= r2 <= 4.5, (errs, r1, r2)


def test_parallel_direct_solve_equals_serial():
    # splitting the sources over separate processes changes nothing: each process factors the same matrix
    # with the same SuperLU and solves its share (bitwise equal to one process solving them all)
    import synth
    from oracle.direct import DirectSolver, direct_solve_jobs, direct_solve_parallel
    prob, f = synth.config_small(nx=20, nz=24, npml=4, L=2, nrhs=5, seed=9)
    ref = DirectSolver(prob).solve(f)
    assert np.array_equal(direct_solve_parallel(prob, f, 3), ref)
    prob2, f2 = synth.config_small(nx=16, nz=18, npml=3, L=2, nrhs=2, seed=10)
    out = direct_solve_jobs([(prob, f[:2]), (prob2, f2)], 2)
    assert np.array_equal(out[0], ref[:2]) and np.array_equal(out[1], DirectSolver(prob2).solve(f2))
