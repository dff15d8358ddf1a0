"""The offline state written by pt_save and read back by pt_load (Alg. 1's output, reused by Alg. 2 for
every right-hand side), and several problems set up at once by pt_setup_batch.  A loaded solver must give
bit-identical fields (the same factors, blocks, Green's functions, compressed blocks and tuned launch shapes
feed the same kernels); a batch-set-up solver the same fields as one set up alone."""
import os

import numpy as np
import pytest

import synth
from oracle.direct import DirectSolver

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1410_5910_amd")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.mark.parametrize("kw,nrhs", [
    (dict(precision="f64"), 3),                       # float64, Green's-function pre-solve (auto)
    (dict(precision="f64", presolve="local"), 20),    # line-by-line pre-solve, MFMA tiles, tuned
    (dict(precision="split-bf16"), 40),               # split-bfloat16 planes rebuilt from the loaded blocks
    (dict(precision="split-f16", closure="extrap"), 40),  # split-float16 planes and scale rebuilt likewise
    (dict(precision="f32"), 20),                      # float32 preconditioner copies rebuilt from the loaded blocks
    (dict(precision="f64", plr=True, plr_eps=1e-10), 3),  # compressed blocks stored
    (dict(precision="f64", closure="extrap"), 5),     # extrapolation closure
])
def test_save_load_roundtrip_is_bitwise(tmp_path, kw, nrhs):
    prob, f = synth.config_small(nx=40, nz=48, npml=6, L=4, nrhs=nrhs, seed=101)
    print(f"[gpu] save/load {kw} nrhs={nrhs}", flush=True)
    a = P.Solver.from_problem(prob, max_nrhs=nrhs, tol=1e-10, maxit=60, **kw)
    if nrhs > 4:
        a.tune(nrhs)
    u1, i1 = a.solve(f)
    path = str(tmp_path / "solver.pts")
    a.save(path)
    assert os.path.getsize(path) > 0
    b = P.Solver.load(path)
    la, lb = a.layout(), b.layout()
    for k in ("NX", "NZ", "L", "sumR", "ntrace", "block_bytes", "factor_bytes", "green_bytes", "plr_leaves",
              "max_nrhs", "precision"):
        assert la[k] == lb[k], k
    u2, i2 = b.solve(f)
    assert np.array_equal(u1.view(np.float64), u2.view(np.float64))
    assert [i["iters"] for i in i1] == [i["iters"] for i in i2]
    bar = 1e-8
    assert rel(u2, DirectSolver(prob).solve(f)) < bar
    a.close()
    b.close()


def test_load_rejects_bad_files(tmp_path):
    prob, f = synth.config_small(nx=24, nz=30, npml=5, L=3, nrhs=1, seed=102)
    a = P.Solver.from_problem(prob, tol=1e-10)
    path = str(tmp_path / "s.pts")
    a.save(path)
    data = open(path, "rb").read()
    a.close()
    bad = str(tmp_path / "bad.pts")
    for blob in (b"", b"not a solver file at all", data[: len(data) // 2], data[:-7]):
        open(bad, "wb").write(blob)
        with pytest.raises(P.PolarError) as e:
            P.Solver.load(bad)
        assert e.value.status == P.polar.PT_EINVAL
    with pytest.raises(P.PolarError):
        P.Solver.load(str(tmp_path / "missing.pts"))


def test_setup_batch_matches_separate_setups():
    import torch
    probs = [synth.config_small(nx=nx, nz=nz, npml=5, L=L, nrhs=k, seed=110 + i)
             for i, (nx, nz, L, k) in enumerate([(24, 30, 3, 2), (40, 48, 4, 5), (56, 40, 5, 3), (30, 24, 1, 2)])]
    print("[gpu] setup_batch: 4 problems", flush=True)
    streams = [torch.cuda.Stream() for _ in probs]
    batch = P.setup_batch([p for p, _ in probs], streams=[s.cuda_stream for s in streams],
                          max_nrhs=[f.shape[0] for _, f in probs], tol=1e-11, maxit=60)
    for (p, f), sv in zip(probs, batch):
        alone = P.Solver.from_problem(p, max_nrhs=f.shape[0], tol=1e-11, maxit=60)
        ua, _ = alone.solve(f)
        ub, info = sv.solve(f)
        assert np.array_equal(ua.view(np.float64), ub.view(np.float64)), p.name
        assert rel(ub, DirectSolver(p).solve(f)) < 1e-8
        alone.close()
    res = P.solve_batch(batch, [f for _, f in probs])  # the batch solve on the batch-set-up solvers
    for (p, f), (u, infos) in zip(probs, res):
        assert all(i["converged"] for i in infos)
    for sv in batch:
        sv.close()
    # an invalid problem in the batch: nothing is returned, the error names it
    bad = synth.config_small(nx=24, nz=30, npml=5, L=3, nrhs=1, seed=120)[0]
    bad.L = 50
    with pytest.raises(P.PolarError) as e:
        P.setup_batch([probs[0][0], bad], tol=1e-10)
    assert "problem 1" in str(e.value)


def test_tune_cache_reuse_and_file_roundtrip(tmp_path):
    prob, f = synth.config_small(nx=40, nz=48, npml=6, L=4, nrhs=24, seed=130)
    a = P.Solver.from_problem(prob, max_nrhs=24, tol=1e-10, maxit=60, precision="split-bf16")
    t1 = a.tune(24)
    u1, _ = a.solve(f)
    b = P.Solver.from_problem(prob, max_nrhs=24, tol=1e-10, maxit=60, precision="split-bf16")
    t2 = b.tune(24)  # same shape and form: every timed class comes from the cache
    for cls, e in t1.items():
        if e["tried"] > 0:
            assert t2[cls]["cached"] and t2[cls]["tile_rhs"] == e["tile_rhs"] and t2[cls]["ksplit"] == e["ksplit"]
    u2, _ = b.solve(f)
    assert np.array_equal(u1.view(np.float64), u2.view(np.float64))
    path = str(tmp_path / "tune.txt")
    P.tune_cache_save(path)
    lines = [ln for ln in open(path) if not ln.startswith("#")]
    assert len(lines) >= sum(1 for e in t1.values() if e["tried"] > 0)
    P.tune_cache_load(path)  # merging the same entries back changes nothing
    c = P.Solver.from_problem(prob, max_nrhs=24, tol=1e-10, maxit=60, precision="split-bf16")
    c.tune(24)
    u3, _ = c.solve(f)
    assert np.array_equal(u1.view(np.float64), u3.view(np.float64))
    for s in (a, b, c):
        s.close()


def test_tuner_picks_plr_rank():
    prob, f = synth.config_small(nx=90, nz=60, npml=8, L=4, nrhs=1, seed=131)
    s = P.Solver.from_problem(prob, plr=True, plr_eps=1e-10, max_nrhs=2, tol=1e-10, maxit=60)
    r0 = s.layout()["plr_rmax"]
    root = int(np.ceil(np.sqrt(prob.NX)))
    assert r0 == root
    s.tune(1)
    r1 = s.layout()["plr_rmax"]
    assert r1 in {max(1, root // 2), root, 2 * root, 4 * root}
    u, info = s.solve(f)
    assert rel(u, DirectSolver(prob).solve(f)) < 1e-8
    # a second solver of the same shape takes the cached rank without timing
    s2 = P.Solver.from_problem(prob, plr=True, plr_eps=1e-10, max_nrhs=2, tol=1e-10, maxit=60)
    s2.tune(1)
    assert s2.layout()["plr_rmax"] == r1
    u2, _ = s2.solve(f)
    assert np.array_equal(u.view(np.float64), u2.view(np.float64))
    s.close()
    s2.close()
