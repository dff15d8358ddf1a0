"""pt_apply_noalloc: the variant of pt_apply whose scratch (Gauss-Seidel iterates, staged input, k-slice
partial tiles) lives in the library's fixed device array instead of the solver's buffers.  Its output must
equal pt_apply's bit for bit (the same kernels and launch shapes on the same inputs), on two calls in a row,
the second with fewer sources, and sizes beyond the fixed array are rejected."""
import ctypes as C

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1410_5910_amd")

MAX_SCRATCH = 64 << 20


def _noalloc(lib):
    f = lib.pt_apply_noalloc
    f.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]
    f.restype = C.c_int32
    return f


@pytest.mark.parametrize("precision,closure", [("f64", "jump"), ("split-bf16", "jump"), ("f64", "extrap"),
                                               ("split-bf16", "extrap")])
def test_noalloc_apply_matches_apply(precision, closure):
    torch = pytest.importorskip("torch")
    prob, _ = synth.config_small(nx=200, nz=66, npml=8, L=6, seed=33, nrhs=1)
    print(f"[gpu] noalloc {precision} {closure} NX={prob.NX}", flush=True)
    s = P.Solver.from_problem(prob, precision=precision, max_nrhs=64, tol=1e-10, maxit=40, closure=closure,
                              stream=torch.cuda.current_stream().cuda_stream)
    fn = _noalloc(P.lib())
    ops = [P.OP_A, P.OP_R, P.OP_DINV, P.OP_PRECOND]
    if closure == "extrap":
        ops += [P.OP_A_EXTRAP, P.OP_R_EXTRAP, P.OP_DINV_EXTRAP, P.OP_PRECOND_EXTRAP]
    g = torch.Generator(device="cuda:0").manual_seed(7)
    for tuned in (False, True):  # the rules' launch shapes, then pt_tune's (MFMA k-slices where it picks them)
        if tuned:
            s.tune(40)
        for nrhs in (40, 7):  # two calls in a row, the second smaller
            shape = (nrhs, 2, prob.L - 1, 2, prob.NX)
            x = torch.complex(torch.randn(shape, dtype=torch.float64, device="cuda:0", generator=g),
                              torch.randn(shape, dtype=torch.float64, device="cuda:0", generator=g))
            for op in ops:
                ref = s.apply(op, x)
                y = torch.full_like(x, complex(np.nan, np.nan))
                torch.cuda.synchronize()
                st = fn(s._h, op, nrhs, x.data_ptr(), y.data_ptr())
                assert st == 0, P.lib().pt_last_error().decode()
                torch.cuda.synchronize()
                assert torch.equal(torch.view_as_real(y), torch.view_as_real(ref)), (tuned, nrhs, op)
    s.close()


def test_noalloc_rejects_sizes_beyond_the_scratch():
    torch = pytest.importorskip("torch")
    prob, _ = synth.config_small(nx=200, nz=66, npml=8, L=6, seed=33, nrhs=1)
    s = P.Solver.from_problem(prob, max_nrhs=400, tol=1e-10, maxit=20)
    fn = _noalloc(P.lib())
    ntrace = 4 * (prob.L - 1) * prob.NX
    big = 3 * 400 * ntrace * 16
    assert big > MAX_SCRATCH  # three vectors of 400 sources do not fit
    x = torch.zeros((400, ntrace), dtype=torch.complex128, device="cuda:0")
    y = torch.empty_like(x)
    assert fn(s._h, P.OP_PRECOND, 400, x.data_ptr(), y.data_ptr()) == P.polar.PT_EINVAL
    assert b"scratch" in P.lib().pt_last_error()
    assert fn(s._h, 99, 4, x.data_ptr(), y.data_ptr()) == P.polar.PT_EINVAL
    # a size that fits still works after the rejection
    assert fn(s._h, P.OP_PRECOND, 4, x.data_ptr(), y.data_ptr()) == 0
    torch.cuda.synchronize()
    assert torch.count_nonzero(y[:4]) == 0
    s.close()
