"""Parity of the HIP path (through the C-ABI) with the CPU oracle, stage by stage and end to end.

Tolerances: float64 stages agree with the oracle to ~1e-11 relative (the two
sides differ only in rounding order: sparse LU vs dense Schur inverses);
full solves match the direct solve to <= 1e-8 relative L2 over the whole
padded grid at GMRES tol 1e-10 (the float64 bar).
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
def small():
    # NX = 34 (< 64: one ragged row tile), nz = 31 split 11/10/10 (uneven layers)
    prob, f = synth.config_small(nx=24, nz=31, npml=5, L=3, nrhs=3, seed=21)
    _flush(f"[gpu] setup small {prob.name}")
    gs = P.Solver.from_problem(prob, max_nrhs=20, tol=1e-12, maxit=40)
    ps = PolarizedSolver(prob)
    return prob, f, gs, ps


def test_layout_matches_oracle(small):
    prob, f, gs, ps = small
    lay = gs.layout()
    assert lay["L"] == ps.L
    for l, s in enumerate(ps.slabs):
        assert (lay["own_start"][l], lay["n_own"][l], lay["top_ext"][l], lay["bot_ext"][l], lay["R"][l]) == \
            (s.own_start, s.n, s.top_ext, s.bot_ext, s.R)


def test_trace_blocks(small):
    prob, f, gs, ps = small
    for l, lp in enumerate(ps.loc):
        for (j, k), K in lp.K.items():
            Kg = gs.get_block(l, j, k)
            assert rel(Kg, K) < 1e-10, (l, j, k, rel(Kg, K))


def _random_local(ps, nrhs, seed):
    rng = np.random.default_rng(seed)
    sumR = sum(s.R for s in ps.slabs)
    return rng.standard_normal((nrhs, sumR, ps.NX)) + 1j * rng.standard_normal((nrhs, sumR, ps.NX))


def test_local_solve(small):
    prob, f, gs, ps = small
    # 1 / 3: 1- and 4-column streaming passes; 6 / 13: 8- and 16-column passes; 20: MFMA tiles
    for nrhs in (1, 3, 6, 13, 20):
        b = _random_local(ps, nrhs, nrhs)
        x = gs.local_solve(b)
        r0 = 0
        for lp in ps.loc:
            R = lp.slab.R
            ref = lp.solve(b[:, r0:r0 + R])
            assert rel(x[:, r0:r0 + R], ref) < 1e-10, (nrhs, lp.slab.index)
            r0 += R


def test_trace_rhs(small):
    prob, f, gs, ps = small
    s = gs.trace_rhs(f)
    ref = ps.rhs(ps.newton(f))
    assert rel(s, ref) < 1e-10


@pytest.mark.parametrize("op", ["A", "R", "Dinv", "precond"])
def test_operators(small, op):
    prob, f, gs, ps = small
    rng = np.random.default_rng(3)
    x = rng.standard_normal(ps.zeros(5).shape) + 1j * rng.standard_normal(ps.zeros(5).shape)
    code = {"A": P.OP_A, "R": P.OP_R, "Dinv": P.OP_DINV, "precond": P.OP_PRECOND}[op]
    y = gs.apply(code, x)
    ref = {"A": ps.apply_A, "R": ps.apply_R, "Dinv": ps.apply_D_inv, "precond": ps.precondition}[op](x)
    assert rel(y, ref) < 1e-10, rel(y, ref)


@pytest.mark.parametrize("n_it", [0, 1, 3, 4, 8])
@pytest.mark.parametrize("precision", ["f64", "split-bf16", "split-f16"])
def test_preconditioner_sweep_counts(small, n_it, precision):
    # Alg. 4 with n_it Gauss-Seidel sweeps from u^0 = 0 (the bench runs the mixed form with 4); n_it = 0 is no
    # preconditioner (the identity), which both sides give exactly
    prob, f, gs, ps = small
    g = P.Solver.from_problem(prob, precision=precision, gs_iters=n_it, max_nrhs=20, tol=1e-12, maxit=40)
    rng = np.random.default_rng(n_it)
    for nrhs in (3, 20):  # the 16-column and the wide split-bfloat16 kernels
        x = rng.standard_normal(ps.zeros(nrhs).shape) + 1j * rng.standard_normal(ps.zeros(nrhs).shape)
        err = rel(g.apply(P.OP_PRECOND, x), ps.precondition(x, n_it))
        bar = {"f64": 1e-10, "split-bf16": 1e-4, "split-f16": 1e-5}[precision]
        assert err < (1e-10 if n_it == 0 else bar), (nrhs, err)
    g.close()


@pytest.mark.parametrize("precision", ["f64", "split-bf16", "split-f16"])
def test_unpreconditioned_solve_matches_direct(small, precision):
    # gs_iters = 0: plain GMRES on the polarized system (no sweeps); more iterations, the same field
    prob, f, gs, ps = small
    g = P.Solver.from_problem(prob, precision=precision, gs_iters=0, max_nrhs=3, tol=1e-12, maxit=200)
    u, info = g.solve(f)
    ref = DirectSolver(prob).solve(f)
    assert all(i["converged"] for i in info)
    assert max(rel(u[r], ref[r]) for r in range(f.shape[0])) < 1e-8
    u2, info2 = gs.solve(f)  # the same problem with n_it = 2
    assert min(i["iters"] for i in info) > max(i["iters"] for i in info2)
    g.close()


def test_maxit_reports_noconv_and_last_iterate(small):
    # GMRES stopped at maxit = 2: PT_ENOCONV, converged = 0 for every source, and u is the field of the
    # second iterate (GMRES iterates are unique up to rounding: the residual minimiser over the Krylov space)
    prob, f, gs, ps = small
    g = P.Solver.from_problem(prob, max_nrhs=3, tol=1e-14, maxit=2)
    u, info = g.solve(f)
    assert all(not i["converged"] and i["iters"] == 2 for i in info)
    fc = np.ascontiguousarray(f)
    uc = np.empty_like(fc)  # kept alive: the call writes the field into it
    with pytest.raises(P.PolarError) as e:
        P.polar._check(g._lib.pt_solve(g._h, 3, fc.ctypes.data, uc.ctypes.data, 0, None))
    assert e.value.status == P.polar.PT_ENOCONV
    s = ps.rhs(ps.newton(f))
    x, oinfo = ps.fgmres(s, tol=1e-14, maxit=2)
    assert all(i["iters"] == 2 for i in oinfo)
    ref = ps.reconstruct(f, x)
    assert max(rel(u[r], ref[r]) for r in range(3)) < 1e-9
    for r in range(3):
        assert abs(info[r]["relres"] - oinfo[r]["relres"]) <= 1e-6 * oinfo[r]["relres"]
    g.close()


@pytest.mark.parametrize("precision,nrhs", [("f64", 3), ("f64", 20), ("split-bf16", 20), ("split-f16", 20),
                                            ("f32", 20)])
def test_reruns_are_bitwise_identical(precision, nrhs):
    # no atomics and a fixed reduction order: the same call gives the same bits
    prob, f = synth.config_small(nx=40, nz=48, npml=6, L=4, nrhs=nrhs, seed=91)
    _flush(f"[gpu] determinism {precision} nrhs={nrhs}")
    g = P.Solver.from_problem(prob, precision=precision, max_nrhs=nrhs, tol=1e-10, maxit=60)
    u1, i1 = g.solve(f)
    u2, i2 = g.solve(f)
    assert np.array_equal(u1.view(np.float64), u2.view(np.float64))
    assert [i["iters"] for i in i1] == [i["iters"] for i in i2]
    g.close()


@pytest.mark.parametrize("L", [1, 3])
def test_nan_source_without_info_is_noconv(L):
    # the convergence decision does not depend on the caller asking for per-source info
    prob, f = synth.config_small(nx=24, nz=30, npml=5, L=L, nrhs=2, seed=93)
    f = np.ascontiguousarray(f, dtype=np.complex128)
    g = P.Solver.from_problem(prob, max_nrhs=2, tol=1e-10, maxit=40)
    fb = f.copy()
    fb[1, prob.npml + 10, prob.npml + 5] = np.nan
    u = np.empty_like(fb)
    st = g._lib.pt_solve(g._h, 2, fb.ctypes.data, u.ctypes.data, 0, None)
    assert st == P.polar.PT_ENOCONV
    st = g._lib.pt_solve(g._h, 2, f.ctypes.data, u.ctypes.data, 0, None)
    assert st == P.polar.PT_OK
    assert rel(u, DirectSolver(prob).solve(f)) < 1e-8
    g.close()


def test_streams_are_ordered_with_torch_work():
    # sources produced by torch kernels on the default stream, solved by solvers on their own (non-blocking)
    # streams, and the fields consumed by torch kernels on the default stream again
    import torch
    probs = [synth.config_small(nx=nx, nz=nz, npml=5, L=L, nrhs=4, seed=95 + i)
             for i, (nx, nz, L) in enumerate([(40, 48, 4), (56, 40, 5)])]
    streams = [torch.cuda.Stream() for _ in probs]
    solvers = [P.Solver.from_problem(p, max_nrhs=4, tol=1e-11, maxit=60, stream=st.cuda_stream)
               for (p, _), st in zip(probs, streams)]
    for rep in range(3):
        fds = []
        for p, f in probs:
            big = torch.ones(1 << 24, dtype=torch.float64, device="cuda:0")
            for _ in range(8):  # keep the default stream busy before the source is written
                big = big * 1.0000001
            fd = torch.from_numpy(f).to("cuda:0") * 0.5 + (big[0] - big[0])
            fds.append(fd * 2.0)
        res = P.solve_batch(solvers, fds)
        outs = [u * 1.0 for u, _ in res]  # consumed on the default stream
        for (p, f), u in zip(probs, outs):
            ud = DirectSolver(p).solve(f)
            assert max(rel(u[r].cpu().numpy(), ud[r]) for r in range(4)) < 1e-8, (rep, p.name)
        u1, _ = solvers[0].solve(fds[0] + 0.0)
        assert rel((u1 * 1.0).cpu().numpy(), DirectSolver(probs[0][0]).solve(probs[0][1])) < 1e-8
    for sv in solvers:
        sv.close()


def test_reconstruct(small):
    prob, f, gs, ps = small
    rng = np.random.default_rng(4)
    x = rng.standard_normal(ps.zeros(3).shape) + 1j * rng.standard_normal(ps.zeros(3).shape)
    u = gs.reconstruct(f, x)
    assert rel(u, ps.reconstruct(f, x)) < 1e-10


def test_reconstruct_in_place_and_aliased(small):
    """The reconstruction addresses f and u in place; with u overlapping f
    (the C-ABI allows one buffer for both) it takes copies first."""
    import ctypes as C
    import torch
    prob, f, gs, ps = small
    rng = np.random.default_rng(5)
    x = rng.standard_normal(ps.zeros(3).shape) + 1j * rng.standard_normal(ps.zeros(3).shape)
    ref = ps.reconstruct(f, x)
    fd = torch.from_numpy(np.ascontiguousarray(f)).cuda()
    xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    ud = gs.reconstruct(fd, xd)  # device arrays: f and u distinct
    assert rel(ud.cpu().numpy(), ref) < 1e-10
    assert torch.equal(fd.cpu(), torch.from_numpy(np.ascontiguousarray(f)))  # f left untouched
    buf = fd.clone()
    rc = gs._lib.pt_reconstruct(gs._h, f.shape[0], C.c_void_p(buf.data_ptr()), C.c_void_p(xd.data_ptr()),
                                C.c_void_p(buf.data_ptr()), 1)
    assert rc == 0
    assert rel(buf.cpu().numpy(), ref) < 1e-10


def test_solve_small_matches_direct(small):
    prob, f, gs, ps = small
    u, info = gs.solve(f)
    ud = DirectSolver(prob).solve(f)
    assert rel(u, ud) < 1e-8
    for i in info:
        assert i["converged"] and i["relres"] < 1e-10
    # per-RHS results do not depend on the batch they were solved in
    u1, _ = gs.solve(f[1:2])
    assert rel(u1[0], u[1]) < 1e-10


@pytest.mark.parametrize("L", [1, 2, 4])
def test_solve_edge_layer_counts(L):
    prob, f = synth.config_small(nx=20, nz=24, npml=4, L=L, nrhs=2, seed=30 + L)
    _flush(f"[gpu] edge L={L}")
    gs = P.Solver.from_problem(prob, max_nrhs=2, tol=1e-12)
    u, info = gs.solve(f)
    assert rel(u, DirectSolver(prob).solve(f)) < 1e-8
    gs.close()


def test_zero_source_gives_zero_field(small):
    prob, f, gs, ps = small
    u, info = gs.solve(np.zeros_like(f[:1]))
    assert np.all(u == 0)
    assert info[0]["iters"] == 0


def test_config1_full_solve():
    prob, f = synth.config1()
    _flush("[gpu] config1 constant-100x100-L4")
    gs = P.Solver.from_problem(prob, tol=1e-10)
    u, info = gs.solve(f)
    ud = DirectSolver(prob).solve(f)
    assert rel(u, ud) < 1e-8, rel(u, ud)
    assert info[0]["converged"]
    gs.close()


def test_device_arrays_roundtrip(small):
    torch = pytest.importorskip("torch")
    prob, f, gs, ps = small
    fd = torch.from_numpy(f).to("cuda")
    ud, info = gs.solve(fd)
    uh, _ = gs.solve(f)
    assert rel(ud.cpu().numpy(), uh) < 1e-14


def test_bad_nrhs_is_rejected(small):
    prob, f, gs, ps = small
    with pytest.raises(P.PolarError):
        gs.solve(np.zeros((21, prob.NZ, prob.NX), dtype=complex))


# ---------------------------------------------------------------- precision forms
def test_f32_blocks_and_factors_small():
    prob, f = synth.config_small(nx=24, nz=31, npml=5, L=3, nrhs=3, seed=21)
    _flush("[gpu] f32 small")
    gs = P.Solver.from_problem(prob, precision="f32", max_nrhs=3, tol=1e-10, maxit=60)
    u, info = gs.solve(f)
    err = rel(u, DirectSolver(prob).solve(f))
    _flush(f"[gpu] f32 small rel err {err:.2e}, iters {[i['iters'] for i in info]}")
    # float32 blocks in the preconditioner only: flexible GMRES with the float64 operator converges
    # to the float64 solution, so the float64 bar holds
    assert err < 1e-8
    assert all(i["converged"] and i["relres"] < 1e-9 for i in info)
    gs.close()


def test_f32_thirteen_sources():
    # float32 blocks with 13 right-hand sides: the 16-column streaming pass
    prob, f = synth.config_small(nx=24, nz=31, npml=5, L=3, nrhs=13, seed=23)
    _flush("[gpu] f32 13 sources")
    gs = P.Solver.from_problem(prob, precision="f32", max_nrhs=13, tol=1e-10, maxit=60)
    u, info = gs.solve(f)
    ud = DirectSolver(prob).solve(f)
    assert max(rel(u[r], ud[r]) for r in range(13)) < 1e-8
    gs.close()


def test_f32_bumps440_single_source():
    prob, f = synth.config2()
    _flush("[gpu] f32 bumps-440x440-L8")
    gs = P.Solver.from_problem(prob, precision="f32", tol=1e-10, maxit=60)
    u, info = gs.solve(f)
    err = rel(u, DirectSolver(prob).solve(f))
    _flush(f"[gpu] f32 bumps440 rel err {err:.2e}, iters {info[0]['iters']}")
    assert err < 1e-8
    gs.close()


# ---------------------------------------------------------------- full-size, bench launch configuration
def test_bumps440_f64_matches_direct():
    # the launch configuration bench.py times: one source, FP64, tol 1e-10
    prob, f = synth.config2()
    _flush("[gpu] f64 bumps-440x440-L8")
    gs = P.Solver.from_problem(prob, tol=1e-10, maxit=50)
    u, info = gs.solve(f)
    assert rel(u, DirectSolver(prob).solve(f)) < 1e-8
    assert info[0]["converged"] and info[0]["relres"] < 1e-9
    gs.close()


def test_batched_many_sources_match_single():
    # many right-hand sides in one call (NR = 16 path, ragged last chunk) vs the same sources one by one
    prob, f = synth.config_small(nx=40, nz=48, npml=6, L=4, nrhs=37, seed=8)
    _flush("[gpu] batched 37 sources")
    gs = P.Solver.from_problem(prob, max_nrhs=37, tol=1e-11, maxit=60)
    u, info = gs.solve(f)
    ud = DirectSolver(prob).solve(f)
    errs = [rel(u[i], ud[i]) for i in range(37)]
    assert max(errs) < 1e-8, max(errs)
    u5, _ = gs.solve(f[5:6])
    assert rel(u5[0], u[5]) < 1e-9
    gs.close()


# ---------------------------------------------------------------- partitioned low-rank blocks
@pytest.mark.parametrize("nrhs", [3, 40])  # 16 waves per tile (few workgroups) / 4 waves
def test_plr_operator_matches_dense_oracle(nrhs):
    prob, f = synth.config_small(nx=90, nz=60, npml=8, L=3, nrhs=2, seed=12)
    _flush(f"[gpu] plr operator small, {nrhs} sources")
    gs = P.Solver.from_problem(prob, plr=True, plr_eps=1e-10, max_nrhs=nrhs, tol=1e-12)
    lay = gs.layout()
    assert lay["plr_leaves"] > 0 and lay["block_bytes"] < lay["dense_block_bytes"]
    ps = PolarizedSolver(prob)
    rng = np.random.default_rng(9)
    x = rng.standard_normal(ps.zeros(nrhs).shape) + 1j * rng.standard_normal(ps.zeros(nrhs).shape)
    for code, fn in ((P.OP_A, ps.apply_A), (P.OP_R, ps.apply_R), (P.OP_DINV, ps.apply_D_inv),
                     (P.OP_PRECOND, ps.precondition)):
        err = rel(gs.apply(code, x), fn(x))
        assert err < 1e-8, (code, err)
    u, info = gs.solve(f)
    assert rel(u, DirectSolver(prob).solve(f)) < 1e-7
    gs.close()


def test_plr_bumps440_single_source():
    prob, f = synth.config2()
    _flush("[gpu] plr bumps-440x440-L8")
    gs = P.Solver.from_problem(prob, plr=True, plr_eps=1e-9, tol=1e-10)
    lay = gs.layout()
    _flush(f"[gpu] plr ratio {lay['block_bytes'] / lay['dense_block_bytes']:.3f}, leaves {lay['plr_leaves']}, "
           f"setup {lay['setup_ms'] / 1e3:.1f} s")
    u, info = gs.solve(f)
    err = rel(u, DirectSolver(prob).solve(f))
    _flush(f"[gpu] plr bumps440 rel err {err:.2e}, iters {info[0]['iters']}")
    assert err < 1e-6
    gs.close()


# ---------------------------------------------------------------- sources touching few layers
def _compact_sources(prob, spec, seed):
    """spec: list of (z0, z1) padded-grid row ranges (None: dense everywhere); random complex values there."""
    rng = np.random.default_rng(seed)
    f = np.zeros((len(spec), prob.NZ, prob.NX), dtype=np.complex128)
    for r, zr in enumerate(spec):
        if zr is None:
            f[r, prob.npml:prob.npml + prob.nz, prob.npml:prob.npml + prob.nx] = rng.standard_normal((prob.nz, prob.nx))
        else:
            z0, z1 = zr
            x0 = prob.npml + 2 + 3 * r % (prob.nx - 6)
            f[r, z0:z1, x0:x0 + 3] = rng.standard_normal((z1 - z0, 3)) + 1j * rng.standard_normal((z1 - z0, 3))
    return f


@pytest.fixture(scope="module")
def layered4():
    # 4 layers of 12 physical rows; owned padded rows: [0, 18), [18, 30), [30, 42), [42, 60)
    prob, _ = synth.config_small(nx=30, nz=48, npml=6, L=4, seed=51)
    gs = P.Solver.from_problem(prob, max_nrhs=8, tol=1e-12, maxit=60)
    return prob, gs, PolarizedSolver(prob)


def test_sparse_presolve_trace_rhs_matches_oracle(layered4):
    prob, gs, ps = layered4
    _flush("[gpu] sparse pre-solve trace rhs")
    # one layer each, one straddling 29/30, two in layer 0 (ragged slot counts), one in the last layer
    spec = [(8, 10), (20, 23), (28, 32), (12, 14), (44, 47), (33, 35)]
    f = _compact_sources(prob, spec, seed=3)
    s = gs.trace_rhs(f)
    ref = ps.rhs(ps.newton(f))
    assert rel(s, ref) < 1e-10
    for r in range(len(spec)):
        assert rel(s[r], ref[r]) < 1e-10, r


def test_sparse_presolve_solves_match_direct(layered4):
    prob, gs, ps = layered4
    _flush("[gpu] sparse pre-solve full solves")
    spec = [(8, 10), (20, 23), None, (28, 32), (44, 47), (33, 35), (40, 44)]
    f = _compact_sources(prob, spec, seed=4)
    u, info = gs.solve(f)
    ud = DirectSolver(prob).solve(f)
    for r in range(len(spec)):
        assert rel(u[r], ud[r]) < 1e-8, r
    # the same sources one by one (single-source calls take the dense path)
    for r in (0, 3):
        u1, _ = gs.solve(f[r])
        assert rel(u1, u[r]) < 1e-10


def test_sparse_presolve_zero_and_mixed_zero_sources(layered4):
    prob, gs, ps = layered4
    _flush("[gpu] sparse pre-solve zero sources")
    f = np.zeros((3, prob.NZ, prob.NX), dtype=np.complex128)
    s = gs.trace_rhs(f)
    assert np.all(s == 0)
    u, info = gs.solve(f)
    assert np.all(u == 0)
    f[1] = _compact_sources(prob, [(20, 23)], seed=5)[0]
    u, info = gs.solve(f)
    assert np.all(u[0] == 0) and np.all(u[2] == 0)
    assert rel(u[1], DirectSolver(prob).solve(f[1])) < 1e-8


def test_sparse_presolve_gaussian_tails_match_direct(layered4):
    # Gaussians (sigma = h) stay nonzero in float64 about 38 widths out, i.e. over several 12-row layers;
    # layers where a source is below 2^-80 of its peak are skipped, far below float64 rounding of u
    prob, gs, ps = layered4
    _flush("[gpu] sparse pre-solve gaussian sources")
    h = prob.h
    zs = [10, 17, 24, 31, 40, 50]
    f = np.stack([synth.gaussian_source(prob, (prob.nx / 2 + 2 * i) * h, z * h, h) for i, z in enumerate(zs)])
    tail_layers = [(np.abs(f[r]).max(axis=1) > 0).sum() for r in range(len(zs))]
    assert max(tail_layers) > 30  # the float64 tails really do span several layers
    u, info = gs.solve(f)
    ud = DirectSolver(prob).solve(f)
    for r in range(len(zs)):
        assert rel(u[r], ud[r]) < 1e-8, r
    s = gs.trace_rhs(f)
    assert rel(s, ps.rhs(ps.newton(f))) < 1e-10


# ---------------------------------------------------------------- autotuner
@pytest.mark.parametrize("precision,nrhs", [("f64", 40), ("split-bf16", 40), ("f64", 3)])
def test_tune_keeps_results(precision, nrhs):
    prob, f = synth.config_small(nx=60, nz=60, npml=6, L=5, nrhs=nrhs, seed=61)
    _flush(f"[gpu] tune {precision} nrhs={nrhs}")
    gs = P.Solver.from_problem(prob, precision=precision, max_nrhs=nrhs, tol=1e-11, maxit=60)
    u0, _ = gs.solve(f)
    res = gs.tune(nrhs)
    _flush(f"[gpu]   {res}")
    assert set(res) == {"local", "sweep", "reflect", "operator", "presolve"}
    assert res.pop("presolve")["tried"] == 0  # the pre-solve products keep the rule's shape
    for cls, e in res.items():
        assert e["tried"] >= 1 and e["best_us"] > 0 and e["best_us"] <= e["default_us"]
        if nrhs > 4 and precision == "f64":
            assert e["tried"] > 1, cls  # float64 MFMA shapes were timed
        if e["tried"] > 1:
            # the shape in use is reported, the rule's included; a candidate replaces the rule's shape
            # only when at least 2% faster
            assert e["tile_rhs"] in (16, 32, 64) and e["ksplit"] >= 1, (cls, e)
            assert e["best_us"] == e["default_us"] or e["best_us"] < 0.98 * e["default_us"], (cls, e)
    if res["local"]["tile_rhs"] in (32, 64) and not precision.startswith("split"):
        assert res["local"]["ksplit"] == 1, res["local"]  # the local passes are not offered k-slices
    s = gs.layout()  # the solver is still usable
    assert s["L"] == prob.L
    u1, info = gs.solve(f)
    ud = DirectSolver(prob).solve(f)
    for r in range(nrhs):
        assert rel(u1[r], ud[r]) < 1e-8, r
    assert rel(u1, u0) < 1e-9
    gs.close()


@pytest.mark.parametrize("precision", ["f64", "f32", "split-bf16"])
def test_mfma_kslices_match_the_unsliced_apply(tmp_path, precision):
    # the local solves' passes and operator A (every form), the sweep steps and reflection terms (float64
    # and float32 blocks) forced onto 32-source MFMA tiles split over 4 workgroups (partial tiles summed by a
    # second kernel) through the tuning cache: the solve must match the rules' shapes and the direct solve
    # (a grid size no other test uses, so the forced cache entries touch nothing else)
    prob, f = synth.config_small(nx=62, nz=60, npml=6, L=5, nrhs=40, seed=63)
    _flush(f"[gpu] MFMA k-slices {precision}")
    sv = P.Solver.from_problem(prob, precision=precision, max_nrhs=40, tol=1e-11, maxit=60)
    u0, _ = sv.solve(f)  # the rules' shapes
    sv.tune(40)
    path = tmp_path / "tune.txt"
    P.tune_cache_save(str(path))
    lines = path.read_text().splitlines()
    names = ["local", "sweep", "reflect", "operator"]  # tuning classes 0..3
    forced = {0, 3} if precision.startswith("split") else {0, 1, 2, 3}
    out, hit = [lines[0]], set()
    for line in lines[1:]:
        x = line.split()  # NX L precision closure plr class nrhs njobs | has_cfg tn ks mks ...
        if int(x[0]) == sv.NX and int(x[1]) == prob.L and int(x[5]) in forced and int(x[6]) == 40:
            x[8], x[9], x[10], x[11] = "1", "32", "1", "4"
            hit.add(int(x[5]))
        out.append(" ".join(x))
    assert hit == forced
    path.write_text("\n".join(out) + "\n")
    P.tune_cache_load(str(path))
    t = sv.tune(40)
    for cls in (names[c] for c in forced):
        assert t[cls]["cached"] and t[cls]["tile_rhs"] == 32 and t[cls]["ksplit"] == 4, (cls, t[cls])
    u1, info = sv.solve(f)
    assert all(i["converged"] for i in info)
    assert rel(u1, u0) < 1e-9
    ud = DirectSolver(prob).solve(f)  # reduced-precision forms too: the outer solve is float64 to 1e-11
    assert max(rel(u1[r], ud[r]) for r in range(f.shape[0])) < 1e-8
    sv.close()


# ---------------------------------------------------------------- several problems at once
def test_solve_batch_uneven_problems():
    import torch
    probs = [synth.config_small(nx=nx, nz=nz, npml=5, L=L, nrhs=k, seed=70 + i)
             for i, (nx, nz, L, k) in enumerate([(24, 30, 3, 2), (40, 48, 4, 5), (30, 24, 2, 1), (56, 40, 5, 3)])]
    _flush("[gpu] solve_batch: 4 uneven problems")
    streams = [torch.cuda.Stream() for _ in probs]
    solvers = [P.Solver.from_problem(p, max_nrhs=f.shape[0], tol=1e-11, maxit=60, stream=st.cuda_stream)
               for (p, f), st in zip(probs, streams)]
    res = P.solve_batch(solvers, [f for _, f in probs])
    for (p, f), sv, (u, infos) in zip(probs, solvers, res):
        ud = DirectSolver(p).solve(f)
        assert max(rel(u[r], ud[r]) for r in range(f.shape[0])) < 1e-8
        assert all(i["converged"] for i in infos)
        u1, _ = sv.solve(f)  # the same problem alone: the same result
        assert rel(u1, u) < 1e-13
    # device arrays
    dres = P.solve_batch(solvers, [torch.from_numpy(f).to("cuda:0") for _, f in probs])
    for (u, _), (ud, _) in zip(res, dres):
        assert rel(ud.cpu().numpy(), u) < 1e-13
    with pytest.raises(P.PolarError):
        P.solve_batch([solvers[0], solvers[0]], [probs[0][1], probs[0][1]])
    for sv in solvers:
        sv.close()


# ---------------------------------------------------------------- Gauss-Seidel as a solver (Alg. 3)
def test_gauss_seidel_solver_matches_oracle_iteration(small):
    prob, f, gs, ps = small
    _flush("[gpu] gauss-seidel solver")
    s = ps.rhs(ps.newton(f))
    for k in (1, 2, 5):
        u, it, ru, conv = gs.gauss_seidel(f, tol=0.0, maxit=k)  # exactly k iterations
        assert it == k and not conv
        x_ref, hist = ps.gauss_seidel(s, tol=0.0, maxit=k)
        u_ref = ps.reconstruct(f, x_ref)
        assert rel(u, u_ref) < 1e-10, k
        assert abs(max(ru) - hist[-1]) <= 1e-8 * max(1.0, hist[-1])
    u, it, ru, conv = gs.gauss_seidel(f, tol=1e-11, maxit=400)
    assert conv and max(ru) < 1e-11
    assert rel(u, DirectSolver(prob).solve(f)) < 1e-8
    _flush(f"[gpu]   Gauss-Seidel alone: {it} iterations to 1e-11")


# ---------------------------------------------------------------- graph-captured iterations
@pytest.mark.parametrize("precision", ["f64", "split-bf16"])
def test_graph_replays_match_plain_launches(precision):
    import torch
    prob, f = synth.config_small(nx=40, nz=48, npml=6, L=4, nrhs=24, seed=81)
    _flush(f"[gpu] graphs {precision}")
    st = torch.cuda.Stream()
    g = P.Solver.from_problem(prob, precision=precision, max_nrhs=24, tol=1e-11, maxit=60,
                              stream=st.cuda_stream, use_graph=True)
    p = P.Solver.from_problem(prob, precision=precision, max_nrhs=24, tol=1e-11, maxit=60)
    ud = DirectSolver(prob).solve(f)
    fd = torch.from_numpy(f).to("cuda:0")
    torch.cuda.synchronize()
    for rep, k in enumerate([24, 24, 5, 24, 5, 1]):  # capture on first use of each nrhs, then replays
        ref, _ = p.solve(f[:k])
        junk = torch.randn(1 << 20, dtype=torch.float64, device="cuda:0").sum()  # eager work in between
        torch.cuda.synchronize()
        u, info = g.solve(fd[:k] if rep % 2 else f[:k])
        torch.cuda.synchronize()
        u = u.cpu().numpy() if hasattr(u, "cpu") else u
        assert rel(u, ref) < 1e-14, (rep, k, rel(u, ref))
        assert max(rel(u[r], ud[r]) for r in range(k)) < 1e-8
        assert all(i["converged"] for i in info)
        del junk
    g.tune(24)  # drops the graphs; the next solve captures again with the tuned shapes
    u, _ = g.solve(f)
    assert max(rel(u[r], ud[r]) for r in range(24)) < 1e-8
    g.close()
    p.close()


# ---------------------------------------------------------------- a source with a NaN
@pytest.mark.parametrize("nrhs", [3, 20])  # streaming kernel / MFMA kernel paths
def test_nan_source_stays_in_its_column(nrhs):
    """A NaN in one source touches every layer of that source only: the other
    sources of the batch are solved as without it, and the NaN source is
    reported not converged with a non-finite field."""
    prob, f = synth.config_small(nx=40, nz=48, npml=6, L=4, nrhs=nrhs, seed=77)
    _flush(f"[gpu] nan source, {nrhs} sources")
    gs = P.Solver.from_problem(prob, max_nrhs=nrhs, tol=1e-10, maxit=40)
    bad = nrhs // 2
    fb = f.copy()
    fb[bad, prob.npml + 20, prob.npml + 7] = np.nan
    u, info = gs.solve(fb)
    ref = DirectSolver(prob).solve(f)
    assert not np.all(np.isfinite(u[bad]))
    assert not info[bad]["converged"]
    for r in range(nrhs):
        if r != bad:
            assert np.all(np.isfinite(u[r])) and info[r]["converged"], r
            assert rel(u[r], ref[r]) < 1e-8, r
    gs.close()
