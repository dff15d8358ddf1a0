"""The system closed by extrapolation relations (closure="extrap") on the GPU
against the oracle's ExtrapSystem (Def. polarized_out_going, eq.
splitting_out_going) and the direct solve.

The GPU forms D^-1 as the jump system's sweeps after one extrapolation step
(pinned on the oracle: D^extrap^-1 = D_jump^-1 T) and the extrapolation rows
from the layers' one-row Schur complements; here every operator is compared
with the oracle's dense-extrapolator form.
"""
import numpy as np
import pytest

import synth
from oracle.direct import DirectSolver
from oracle.extrap import ExtrapSystem
from oracle.polarized import PolarizedSolver

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1410_5910_amd")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _flush(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def small():
    prob, f = synth.config_small(nx=20, nz=36, npml=5, L=4, nrhs=6, seed=33)
    _flush(f"[gpu] extrap setup {prob.name}")
    ps = PolarizedSolver(prob)
    ex = ExtrapSystem(ps)
    gx = P.Solver.from_problem(prob, max_nrhs=8, tol=1e-11, maxit=80, closure="extrap")
    return prob, f, ps, ex, gx


@pytest.mark.parametrize("op", ["A", "R", "Dinv", "precond"])
@pytest.mark.parametrize("nrhs", [3, 6])  # streaming kernel / MFMA kernel
def test_operators_match_oracle(small, op, nrhs):
    prob, f, ps, ex, gx = small
    rng = np.random.default_rng(nrhs)
    x = rng.standard_normal(ps.zeros(nrhs).shape) + 1j * rng.standard_normal(ps.zeros(nrhs).shape)
    code = {"A": P.OP_A_EXTRAP, "R": P.OP_R_EXTRAP, "Dinv": P.OP_DINV_EXTRAP, "precond": P.OP_PRECOND_EXTRAP}[op]
    y = gx.apply(code, x)
    ref = {"A": ex.apply_A, "R": ex.apply_R, "Dinv": ex.apply_D_inv, "precond": ex.precondition}[op](x)
    assert rel(y, ref) < 1e-10, (op, rel(y, ref))


@pytest.mark.parametrize("n_it", [1, 4])
def test_preconditioner_sweep_counts(small, n_it):
    prob, f, ps, ex, gx = small
    g = P.Solver.from_problem(prob, max_nrhs=8, tol=1e-11, maxit=80, closure="extrap", gs_iters=n_it)
    rng = np.random.default_rng(10 + n_it)
    x = rng.standard_normal(ps.zeros(6).shape) + 1j * rng.standard_normal(ps.zeros(6).shape)
    err = rel(g.apply(P.OP_PRECOND_EXTRAP, x), ex.precondition(x, n_it))
    assert err < 1e-10, err
    g.close()


def test_solves_match_direct(small):
    prob, f, ps, ex, gx = small
    _flush("[gpu] extrap solves")
    ud = DirectSolver(prob).solve(f)
    u, info = gx.solve(f)
    for r in range(f.shape[0]):
        assert rel(u[r], ud[r]) < 1e-8, r
        assert info[r]["converged"]
    # the oracle's extrapolation solve takes the same number of iterations
    _, _, oinfo = ex.solve(f[:1], tol=1e-11, maxit=80)
    assert abs(info[0]["iters"] - oinfo[0]["iters"]) <= 1


def test_mixed_form_and_bumps():
    prob, f = synth.config_small(nx=60, nz=90, npml=8, L=6, nrhs=24, seed=12)
    _flush(f"[gpu] extrap mixed {prob.name}")
    ud = DirectSolver(prob).solve(f)
    for prec, bar in (("split-bf16", 1e-6), ("f64", 1e-8)):
        gj = P.Solver.from_problem(prob, precision=prec, max_nrhs=24, tol=1e-10, maxit=80)
        gx = P.Solver.from_problem(prob, precision=prec, max_nrhs=24, tol=1e-10, maxit=80, closure="extrap")
        uj, ij = gj.solve(f)
        ux, ix = gx.solve(f)
        _flush(f"[gpu]   {prec}: iterations jump {max(i['iters'] for i in ij)}, "
               f"extrap {max(i['iters'] for i in ix)}")
        assert rel(ux, ud) < bar and rel(uj, ud) < bar
        assert max(i["iters"] for i in ix) <= max(i["iters"] for i in ij) + 2
        gj.close()
        gx.close()


def test_closure_validation():
    prob, f = synth.config_small(nx=16, nz=24, npml=4, L=3, nrhs=1, seed=2)
    with pytest.raises(ValueError):
        P.Solver.from_problem(prob, closure="annihilation")
    with pytest.raises(P.PolarError):
        P.Solver.from_problem(prob, precision="f32", closure="extrap")
    g = P.Solver.from_problem(prob, max_nrhs=1)
    with pytest.raises(P.PolarError):
        g.apply(P.OP_A_EXTRAP, np.zeros((1, 2, 2, 2, g.NX), dtype=np.complex128))
    g.close()
