"""Pre-solve by interface Green's functions (presolve="green") against the
line-by-line local solves (presolve="local") and the oracle.

The rows j = 1 and n of each layer's inverse over its owned rows are built at
setup from the extraction solves (the columns at those rows) and the diagonal
scaling that makes the local operator symmetric; rows 0 and n+1 of the
pre-solve follow by one-sided extrapolation (Lemma extrapolator_def: the
sources lie on the owned rows).  The pre-solve is
then one product per (layer, trace row) instead of ~R dependent launches, so
the trace right-hand side must match the oracle's N^l f^l at the trace rows
(Alg. 2, Def. 3) to float64 rounding, for dense, sparse and single sources,
through the streaming (<= 4 columns) and the MFMA (> 4 columns) kernels.
"""
import numpy as np
import pytest

import synth
from oracle.direct import DirectSolver
from oracle.polarized import PolarizedSolver

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1410_5910_amd")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _flush(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def pair():
    # 4 layers of 12 physical rows (NX = 42: one ragged 64-row MFMA tile, 6 streaming row tiles)
    prob, _ = synth.config_small(nx=30, nz=48, npml=6, L=4, seed=51)
    _flush("[gpu] green setup")
    g = P.Solver.from_problem(prob, max_nrhs=8, tol=1e-12, maxit=60, presolve="green")
    loc = P.Solver.from_problem(prob, max_nrhs=8, tol=1e-12, maxit=60, presolve="local")
    yield prob, g, loc, PolarizedSolver(prob)
    g.close()
    loc.close()


def _compact(prob, spec, seed):
    rng = np.random.default_rng(seed)
    f = np.zeros((len(spec), prob.NZ, prob.NX), dtype=np.complex128)
    for r, (z0, z1) in enumerate(spec):
        f[r, z0:z1, prob.npml:prob.npml + prob.nx] = rng.standard_normal((z1 - z0, prob.nx))
    return f


def test_green_layout(pair):
    prob, g, loc, ps = pair
    lay = g.layout()
    want = 0
    for s in ps.slabs:  # rows 1 and n only: rows 0 and n+1 follow by extrapolation
        ntr = (1 if s.top_ext else 0) + (1 if s.bot_ext else 0)
        want += ntr * prob.NX * s.n * prob.NX * 16
    assert lay["green_bytes"] == want
    assert loc.layout()["green_bytes"] == 0


def _points(prob, nsrc, npts, seed):
    """Sources nonzero at a few scattered nodes: most 16-entry chunks of a layer's inputs are zero."""
    rng = np.random.default_rng(seed)
    f = np.zeros((nsrc, prob.NZ, prob.NX), dtype=np.complex128)
    for r in range(nsrc):
        zs = rng.integers(prob.npml, prob.npml + prob.nz, npts)
        xs = rng.integers(prob.npml, prob.npml + prob.nx, npts)
        f[r, zs, xs] = rng.standard_normal(npts) + 1j * rng.standard_normal(npts)
    # the last physical node of a row and of the section: ragged chunk ends
    f[0, prob.npml + prob.nz - 1, prob.npml + prob.nx - 1] = 1.0 - 0.5j
    f[1, prob.npml + 11, prob.npml + prob.nx - 1] = 0.25
    return f


@pytest.mark.parametrize("kind", ["dense3", "dense6", "sparse", "single", "points"])
def test_green_trace_rhs_matches_oracle(pair, kind):
    prob, g, loc, ps = pair
    _flush(f"[gpu] green trace rhs {kind}")
    rng = np.random.default_rng(7)
    if kind.startswith("dense"):
        k = int(kind[5:])  # 3: streaming kernel; 6: MFMA kernel (every layer, every source)
        f = rng.standard_normal((k, prob.NZ, prob.NX)) + 1j * rng.standard_normal((k, prob.NZ, prob.NX))
    elif kind == "sparse":
        f = _compact(prob, [(8, 10), (20, 23), (28, 32), (12, 14), (44, 47), (33, 35)], seed=3)
    elif kind == "points":  # MFMA form with most chunks skipped
        f = _points(prob, 6, 12, seed=11)
    else:
        f = _compact(prob, [(28, 32)], seed=5)  # straddles layers 1 and 2: a two-layer range
    ref = ps.rhs(ps.newton(f))
    sg = g.trace_rhs(f)
    sl = loc.trace_rhs(f)
    assert rel(sg, ref) < 1e-10
    assert rel(sl, ref) < 1e-10
    for r in range(f.shape[0]):
        assert rel(sg[r], ref[r]) < 1e-10, r


def test_green_solves_match_direct(pair):
    prob, g, loc, ps = pair
    _flush("[gpu] green full solves")
    h = prob.h
    zs = [10, 17, 24, 31, 40, 50]
    f = np.stack([synth.gaussian_source(prob, (prob.nx / 2 + 2 * i) * h, z * h, h) for i, z in enumerate(zs)])
    ud = DirectSolver(prob).solve(f)
    ug, _ = g.solve(f)
    ul, _ = loc.solve(f)
    for r in range(len(zs)):
        assert rel(ug[r], ud[r]) < 1e-8, r
        assert rel(ug[r], ul[r]) < 1e-9, r
    u1, _ = g.solve(f[2])
    assert rel(u1, ud[2]) < 1e-8


def test_green_in_the_float32_form():
    # every precision form keeps float64 factors, so the float32 form (float32 preconditioner blocks) forms
    # its pre-solve from the same float64 Green's functions and meets the float64 bar
    prob, f = synth.config_small(nx=24, nz=31, npml=5, L=3, nrhs=2, seed=21)
    _flush("[gpu] green f32")
    s = P.Solver.from_problem(prob, precision="f32", max_nrhs=2, tol=1e-10, maxit=60, presolve="green")
    g = P.Solver.from_problem(prob, precision="f64", max_nrhs=2, tol=1e-10, maxit=60, presolve="green")
    assert s.layout()["green_bytes"] == g.layout()["green_bytes"] > 0
    u, info = s.solve(f)
    assert all(i["converged"] for i in info)
    assert rel(u, DirectSolver(prob).solve(f)) < 1e-8
    s.close()
    g.close()
    with pytest.raises(ValueError):
        P.Solver.from_problem(prob, presolve="nope")


def test_green_bumps440_single_source():
    prob, f = synth.config2()
    _flush("[gpu] green bumps-440x440-L8 single source")
    g = P.Solver.from_problem(prob, tol=1e-10, maxit=50, presolve="green")
    assert g.layout()["green_bytes"] > 0
    u, info = g.solve(f)
    g.close()
    err = rel(u, DirectSolver(prob).solve(f))
    _flush(f"[gpu] green bumps440 rel err {err:.2e}")
    assert err < 1e-8 and info[0]["converged"]
