"""Thin ctypes binding of libpolar (include/polar.h).

Argument marshalling only: every step of the solve runs in the HIP library.
Arrays may be NumPy complex128 arrays (host; the library copies and
synchronises) or torch complex128 CUDA tensors on the solver's device
(on_device; results are written in place of a tensor this module allocates
on the same device).  With device tensors the solver's stream first waits for
the caller's current torch stream (so inputs produced there are complete and
the output's memory is free), and the current stream then waits for the
solver's stream (so the results are ordered before later work on it).
The library must be built (paper_1410_5910_amd.build); importing this module
without it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpolar.so")

PT_OK, PT_EINVAL, PT_ENOMEM, PT_EHIP, PT_ESINGULAR, PT_ENOCONV = range(6)
PT_F64, PT_F32, PT_SPLIT_BF16, PT_SPLIT_F16 = 0, 1, 2, 3
PT_LEARN_CORRECT, PT_LEARN_AUGMENT = 0, 1
OP_A, OP_R, OP_DINV, OP_PRECOND = 0, 1, 2, 3
# the same operators of the system closed by extrapolation (closure="extrap")
OP_A_EXTRAP, OP_R_EXTRAP, OP_DINV_EXTRAP, OP_PRECOND_EXTRAP = 4, 5, 6, 7
ROWS = {"0": 0, "1": 1, "n": 2, "n+1": 3}

EXPORTS = ("pt_setup", "pt_solve", "pt_free", "pt_status_str", "pt_last_error", "pt_get_layout", "pt_get_block",
           "pt_get_plr_block",
           "pt_apply", "pt_local_solve", "pt_trace_rhs", "pt_reconstruct", "pt_profile", "pt_profile_read",
           "pt_learned_create", "pt_learned_free", "pt_learned_num_params", "pt_learned_get_params",
           "pt_learned_set_params", "pt_learned_gradient", "pt_learned_forward", "pt_learned_collect",
           "pt_learned_samples", "pt_learned_train", "pt_solver_set_learned", "pt_learned_save", "pt_learned_load",
           "pt_profile_read_class", "pt_tune", "pt_solve_batch", "pt_solve_batch_merged", "pt_gauss_seidel",
           "pt_apply_noalloc",
           "pt_setup_batch", "pt_save", "pt_load", "pt_tune_cache_save", "pt_tune_cache_load")
CLASSES = ("local", "sweep", "reflect", "operator", "presolve")


class PtProblem(C.Structure):
    _fields_ = [("nx", C.c_int32), ("nz", C.c_int32), ("npml", C.c_int32), ("h", C.c_double),
                ("omega", C.c_double), ("pml_C", C.c_double), ("L", C.c_int32), ("c", C.POINTER(C.c_double))]


class PtOptions(C.Structure):
    _fields_ = [("precision", C.c_int32), ("gs_iters", C.c_int32), ("tol", C.c_double), ("maxit", C.c_int32),
                ("max_nrhs", C.c_int32), ("plr", C.c_int32), ("plr_eps", C.c_double), ("plr_rmax", C.c_int32),
                ("use_graph", C.c_int32), ("presolve", C.c_int32), ("closure", C.c_int32)]


class PtRhsInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("est", C.c_double), ("relres", C.c_double),
                ("learned", C.c_int32), ("learned_steps", C.c_int32)]


class PtLayout(C.Structure):
    _fields_ = [("NX", C.c_int32), ("NZ", C.c_int32), ("L", C.c_int32), ("sumR", C.c_int32), ("ntrace", C.c_int64),
                ("R", C.c_int32 * 64), ("own_start", C.c_int32 * 64), ("n_own", C.c_int32 * 64),
                ("top_ext", C.c_int32 * 64), ("bot_ext", C.c_int32 * 64), ("setup_ms", C.c_double),
                ("block_bytes", C.c_int64), ("factor_bytes", C.c_int64), ("dense_block_bytes", C.c_int64),
                ("plr_leaves", C.c_int64), ("green_bytes", C.c_int64), ("plr_ms", C.c_double),
                ("max_nrhs", C.c_int32), ("plr_rmax", C.c_int32), ("precision", C.c_int32)]


class PtKernelStats(C.Structure):
    _fields_ = [("launches", C.c_int64), ("kernel_ms", C.c_double), ("alg_bytes", C.c_double),
                ("alg_flops", C.c_double)]


class PtTuneEntry(C.Structure):
    _fields_ = [("cls", C.c_int32), ("tried", C.c_int32), ("tile_rhs", C.c_int32), ("ksplit", C.c_int32),
                ("best_us", C.c_double), ("default_us", C.c_double), ("cached", C.c_int32)]


class PolarError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libpolar status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libpolar.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # One HIP runtime per process: when torch is present, load it first so that
        # libpolar's libamdhip64.so.7 dependency resolves to the runtime torch uses.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1410_5910_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, dp = C.c_void_p, C.c_int32, C.POINTER(C.c_double)
        L.pt_setup.argtypes = [C.POINTER(PtProblem), C.POINTER(PtOptions), vp, C.POINTER(vp)]
        L.pt_solve.argtypes = [vp, i32, vp, vp, i32, C.POINTER(PtRhsInfo)]
        L.pt_setup_batch.argtypes = [i32, C.POINTER(PtProblem), C.POINTER(PtOptions), C.POINTER(vp), C.POINTER(vp)]
        L.pt_save.argtypes = [vp, C.c_char_p]
        L.pt_tune_cache_save.argtypes = [C.c_char_p]
        L.pt_tune_cache_load.argtypes = [C.c_char_p]
        L.pt_load.argtypes = [C.c_char_p, vp, C.POINTER(vp)]
        L.pt_free.argtypes = [vp]
        L.pt_free.restype = None
        L.pt_status_str.argtypes = [i32]
        L.pt_status_str.restype = C.c_char_p
        L.pt_last_error.argtypes = []
        L.pt_last_error.restype = C.c_char_p
        L.pt_get_layout.argtypes = [vp, C.POINTER(PtLayout)]
        L.pt_get_block.argtypes = [vp, i32, i32, i32, dp]
        L.pt_get_plr_block.argtypes = [vp, i32, i32, i32, dp, C.POINTER(i32), C.POINTER(C.c_int64)]
        L.pt_apply.argtypes = [vp, i32, i32, vp, vp, i32]
        L.pt_apply_noalloc.argtypes = [vp, i32, i32, vp, vp]
        L.pt_local_solve.argtypes = [vp, i32, vp, vp, i32]
        L.pt_trace_rhs.argtypes = [vp, i32, vp, vp, i32]
        L.pt_reconstruct.argtypes = [vp, i32, vp, vp, vp, i32]
        L.pt_profile.argtypes = [vp, i32]
        L.pt_profile_read.argtypes = [vp, C.POINTER(PtKernelStats)]
        L.pt_profile_read_class.argtypes = [vp, i32, C.POINTER(PtKernelStats)]
        L.pt_tune.argtypes = [vp, i32, C.POINTER(PtTuneEntry)]
        L.pt_gauss_seidel.argtypes = [vp, i32, vp, vp, i32, C.c_double, i32, C.POINTER(i32), dp]
        L.pt_solve_batch.argtypes = [i32, C.POINTER(vp), C.POINTER(i32), C.POINTER(vp), C.POINTER(vp), i32,
                                     C.POINTER(C.POINTER(PtRhsInfo))]
        L.pt_solve_batch_merged.argtypes = L.pt_solve_batch.argtypes
        fp = C.POINTER(C.c_float)
        L.pt_learned_create.argtypes = [i32, C.c_uint64, vp, C.POINTER(vp)]
        L.pt_learned_free.argtypes = [vp]
        L.pt_learned_free.restype = None
        L.pt_learned_num_params.argtypes = []
        L.pt_learned_num_params.restype = C.c_int64
        L.pt_learned_get_params.argtypes = [vp, fp]
        L.pt_learned_set_params.argtypes = [vp, fp]
        L.pt_learned_gradient.argtypes = [vp, i32, i32, fp, fp, dp, fp]
        L.pt_learned_forward.argtypes = [vp, i32, i32, fp, fp]
        L.pt_learned_collect.argtypes = [vp, vp, i32, vp, i32, C.POINTER(i32)]
        L.pt_learned_samples.argtypes = [vp, C.POINTER(i32), C.POINTER(i32)]
        L.pt_learned_train.argtypes = [vp, i32, i32, C.c_double, dp]
        L.pt_solver_set_learned.argtypes = [vp, vp, i32]
        L.pt_learned_save.argtypes = [vp, C.c_char_p]
        L.pt_learned_load.argtypes = [vp, C.c_char_p]
        for name in EXPORTS:
            f = getattr(L, name)
            if f.restype is C.c_int:  # default
                f.restype = C.c_int32
        _lib = L
    return _lib


def _check(st: int, allow=()):
    if st != PT_OK and st not in allow:
        raise PolarError(st, lib().pt_last_error().decode())
    return st


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def _problem_options(nx, nz, npml, h, omega, C_pml, L, c, *, precision="f64", gs_iters=2, tol=1e-10, maxit=50,
                     max_nrhs=1, plr=False, plr_eps=1e-9, plr_rmax=0, use_graph=False, presolve="auto",
                     closure="jump"):
    """(PtProblem, PtOptions, the contiguous velocity the problem points at)."""
    c = np.ascontiguousarray(c, dtype=np.float64)
    NX, NZ = nx + 2 * npml, nz + 2 * npml
    if c.size != NX * NZ:
        raise ValueError(f"c must have (nz+2npml)*(nx+2npml) = {NZ * NX} values")
    prob = PtProblem(int(nx), int(nz), int(npml), float(h), float(omega), float(C_pml), int(L),
                     c.ctypes.data_as(C.POINTER(C.c_double)))
    prec = {"f64": PT_F64, "f32": PT_F32, "split-bf16": PT_SPLIT_BF16, "split-f16": PT_SPLIT_F16}[precision]
    if presolve not in ("local", "green", "auto"):
        raise ValueError(f"presolve must be 'local', 'green' or 'auto', not {presolve!r}")
    if closure not in ("jump", "extrap"):
        raise ValueError(f"closure must be 'jump' or 'extrap', not {closure!r}")
    opt = PtOptions(prec, int(gs_iters), float(tol), int(maxit), int(max_nrhs), 1 if plr else 0,
                    float(plr_eps), int(plr_rmax), 1 if use_graph else 0, {"local": 0, "green": 1, "auto": 2}[presolve],
                    {"jump": 0, "extrap": 1}[closure])
    return prob, opt, c


class Solver:
    """Offline setup on construction (Alg. 1), online solves with solve() (Alg. 2)."""

    def __init__(self, nx, nz, npml, h, omega, C_pml, L, c, *, precision="f64", gs_iters=2, tol=1e-10, maxit=50,
                 max_nrhs=1, stream=None, plr=False, plr_eps=1e-9, plr_rmax=0, use_graph=False, presolve="auto",
                 closure="jump"):
        self._lib = lib()
        prob, opt, self._c = _problem_options(nx, nz, npml, h, omega, C_pml, L, c, precision=precision,
                                              gs_iters=gs_iters, tol=tol, maxit=maxit, max_nrhs=max_nrhs, plr=plr,
                                              plr_eps=plr_eps, plr_rmax=plr_rmax, use_graph=use_graph,
                                              presolve=presolve, closure=closure)
        h_ = C.c_void_p()
        _check(self._lib.pt_setup(C.byref(prob), C.byref(opt), C.c_void_p(stream or 0), C.byref(h_)))
        self._adopt(h_, stream)

    def _adopt(self, handle, stream):
        """Take ownership of a set-up solver handle."""
        self._lib = lib()
        self._h = handle
        self._stream = int(stream or 0)
        lay = self.layout()
        self.NX, self.NZ, self.L = lay["NX"], lay["NZ"], lay["L"]
        self.max_nrhs = lay["max_nrhs"]
        self.sumR = lay["sumR"]
        self.ntrace = lay["ntrace"]

    @classmethod
    def load(cls, path: str, stream=None) -> "Solver":
        """A solver read back from a file written by save() (no factorisation, extraction or compression)."""
        h_ = C.c_void_p()
        _check(lib().pt_load(os.fsencode(path), C.c_void_p(stream or 0), C.byref(h_)))
        self = cls.__new__(cls)
        self._adopt(h_, stream)
        return self

    def save(self, path: str):
        """Write the offline state (factors, blocks, Green's functions, compressed blocks, tuned shapes)."""
        _check(self._lib.pt_save(self._h, os.fsencode(path)))

    @classmethod
    def from_problem(cls, prob, **kw):
        """Build from any object with nx, nz, npml, h, omega, C, L, c attributes."""
        return cls(prob.nx, prob.nz, prob.npml, prob.h, prob.omega, prob.C, prob.L, prob.c, **kw)

    # ----------------------------------------------------------------- admin
    def close(self):
        if getattr(self, "_h", None):
            self._lib.pt_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def layout(self) -> dict:
        o = PtLayout()
        _check(self._lib.pt_get_layout(self._h, C.byref(o)))
        L = o.L
        return {"NX": o.NX, "NZ": o.NZ, "L": L, "sumR": o.sumR, "ntrace": o.ntrace, "R": list(o.R[:L]),
                "own_start": list(o.own_start[:L]), "n_own": list(o.n_own[:L]), "top_ext": list(o.top_ext[:L]),
                "bot_ext": list(o.bot_ext[:L]), "setup_ms": o.setup_ms, "block_bytes": o.block_bytes,
                "factor_bytes": o.factor_bytes, "dense_block_bytes": o.dense_block_bytes,
                "plr_leaves": o.plr_leaves, "green_bytes": o.green_bytes,
                "plr_ms": o.plr_ms, "max_nrhs": o.max_nrhs, "plr_rmax": o.plr_rmax, "precision": o.precision}

    def profile(self, enable: bool):
        """Start (reset) / stop recording HIP events around every block-apply launch."""
        _check(self._lib.pt_profile(self._h, 1 if enable else 0))

    def profile_read(self) -> dict:
        o = PtKernelStats()
        _check(self._lib.pt_profile_read(self._h, C.byref(o)))
        return {"launches": o.launches, "kernel_ms": o.kernel_ms, "alg_bytes": o.alg_bytes, "alg_flops": o.alg_flops}

    def profile_read_class(self, cls: str) -> dict:
        """Counters of one launch class: 'local', 'sweep', 'reflect', 'operator' or 'presolve'."""
        o = PtKernelStats()
        _check(self._lib.pt_profile_read_class(self._h, CLASSES.index(cls), C.byref(o)))
        return {"launches": o.launches, "kernel_ms": o.kernel_ms, "alg_bytes": o.alg_bytes, "alg_flops": o.alg_flops}

    def tune(self, nrhs: int) -> dict:
        """Time every candidate tile shape of each launch class for nrhs sources and keep the fastest."""
        arr = (PtTuneEntry * len(CLASSES))()
        _check(self._lib.pt_tune(self._h, int(nrhs), arr))
        return {CLASSES[e.cls]: {"tried": e.tried, "tile_rhs": e.tile_rhs, "ksplit": e.ksplit,
                                 "best_us": e.best_us, "default_us": e.default_us, "cached": bool(e.cached)}
                for e in arr}

    def get_block(self, layer: int, j: str, k: str) -> np.ndarray:
        """K^layer_{j,k} (NX x NX, rows: target x) for j, k in {'0', '1', 'n', 'n+1'}."""
        out = np.empty((self.NX, self.NX), dtype=np.complex128)
        _check(self._lib.pt_get_block(self._h, layer, ROWS[j], ROWS[k],
                                      out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def get_plr_block(self, layer: int, j: str, k: str):
        """The same block expanded from its compressed (PLR) form: (matrix, leaves, stored complex entries)."""
        out = np.empty((self.NX, self.NX), dtype=np.complex128)
        nl, ns = C.c_int32(0), C.c_int64(0)
        _check(self._lib.pt_get_plr_block(self._h, layer, ROWS[j], ROWS[k],
                                          out.ctypes.data_as(C.POINTER(C.c_double)), C.byref(nl), C.byref(ns)))
        return out, int(nl.value), int(ns.value)

    # -------------------------------------------------------------- marshalling
    def _prep(self, a, shape_tail):
        """-> (pointer, on_device, array kept alive, nrhs)"""
        if _is_torch(a):
            import torch
            if not a.is_cuda:
                a = a.numpy()
            else:
                if a.dtype != torch.complex128:
                    raise TypeError("device arrays must be complex128")
                a = a.contiguous()
                n = a.numel() // int(np.prod(shape_tail))
                return C.c_void_p(a.data_ptr()), 1, a, n
        a = np.ascontiguousarray(a, dtype=np.complex128)
        n = a.size // int(np.prod(shape_tail))
        return C.c_void_p(a.ctypes.data), 0, a, n

    def _out(self, like, on_device, shape):
        if on_device:
            import torch
            return torch.empty(shape, dtype=torch.complex128, device=like.device)
        return np.empty(shape, dtype=np.complex128)

    @staticmethod
    def _ptr(a, on_device):
        return C.c_void_p(a.data_ptr()) if on_device else C.c_void_p(a.ctypes.data)

    def _enter(self, like, on_device):
        """Order the solver's stream after the caller's current torch stream; returns what _leave needs."""
        if not on_device:
            return None
        import torch
        cur = torch.cuda.current_stream(like.device)
        if cur.cuda_stream == self._stream:
            return None
        mine = (torch.cuda.ExternalStream(self._stream, device=like.device) if self._stream
                else torch.cuda.default_stream(like.device))
        mine.wait_stream(cur)
        return cur, mine

    @staticmethod
    def _leave(pair):
        """Order the caller's current stream after the solver's stream."""
        if pair is not None:
            pair[0].wait_stream(pair[1])

    def _call(self, like, on_device, fn, *args, allow=()):
        pair = self._enter(like, on_device)
        try:
            return _check(fn(*args), allow=allow)
        finally:
            self._leave(pair)

    # ------------------------------------------------------------------ online
    def solve(self, f):
        """u = H^{-1} f for f of shape (nrhs, NZ, NX) or (NZ, NX).  Returns (u, info list)."""
        single = f.ndim == 2
        p, dev, keep, n = self._prep(f, (self.NZ, self.NX))
        u = self._out(keep, dev, (n, self.NZ, self.NX))
        info = (PtRhsInfo * n)()
        self._call(keep, dev, self._lib.pt_solve, self._h, n, p, self._ptr(u, dev), dev, info, allow=(PT_ENOCONV,))
        infos = [{"iters": i.iters, "converged": bool(i.converged), "est": i.est, "relres": i.relres,
                  "learned": bool(i.learned), "learned_steps": i.learned_steps} for i in info]
        return (u[0] if single else u), infos

    def gauss_seidel(self, f, tol=1e-10, maxit=500):
        """Alg. 3 as a stand-alone solver: (u, iterations, last relative update per source, converged)."""
        single = f.ndim == 2
        p, dev, keep, n = self._prep(f, (self.NZ, self.NX))
        u = self._out(keep, dev, (n, self.NZ, self.NX))
        it = C.c_int32()
        ru = np.zeros(n)
        st = self._call(keep, dev, self._lib.pt_gauss_seidel, self._h, n, p, self._ptr(u, dev), dev, float(tol),
                        int(maxit), C.byref(it), ru.ctypes.data_as(C.POINTER(C.c_double)), allow=(PT_ENOCONV,))
        return (u[0] if single else u), it.value, ru, st == PT_OK

    def apply(self, op: int, x):
        """y = op(x) for polarized vectors x (nrhs, 2, L-1, 2, NX)."""
        p, dev, keep, n = self._prep(x, (self.ntrace,))
        y = self._out(keep, dev, (n, 2, self.L - 1, 2, self.NX))
        self._call(keep, dev, self._lib.pt_apply, self._h, op, n, p, self._ptr(y, dev), dev)
        return y

    def local_solve(self, b):
        """x = (A^l)^{-1} b on layer-local fields (nrhs, sumR, NX)."""
        p, dev, keep, n = self._prep(b, (self.sumR * self.NX,))
        x = self._out(keep, dev, (n, self.sumR, self.NX))
        self._call(keep, dev, self._lib.pt_local_solve, self._h, n, p, self._ptr(x, dev), dev)
        return x

    def trace_rhs(self, f):
        p, dev, keep, n = self._prep(f, (self.NZ, self.NX))
        s = self._out(keep, dev, (n, 2, self.L - 1, 2, self.NX))
        self._call(keep, dev, self._lib.pt_trace_rhs, self._h, n, p, self._ptr(s, dev), dev)
        return s

    def reconstruct(self, f, x):
        pf, dev, kf, n = self._prep(f, (self.NZ, self.NX))
        px, dev2, kx, _ = self._prep(x, (self.ntrace,))
        if dev != dev2:
            raise TypeError("f and x must both be host or both device arrays")
        u = self._out(kf, dev, (n, self.NZ, self.NX))
        self._call(kf, dev, self._lib.pt_reconstruct, self._h, n, pf, px, self._ptr(u, dev), dev)
        return u


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_float))


class Learned:
    """The learned preconditioner stage: a 1D CNN along the interfaces (8 -> 32 -> 32 -> 32 -> 8 channels,
    kernel 5, dilations 1, 2, 4, 8), trained on the GPU from the solver's own Krylov vectors and applied as
    z = GS(v) + N(v)."""

    def __init__(self, capacity: int = 4096, seed: int = 0, stream=None):
        self._lib = lib()
        h_ = C.c_void_p()
        _check(self._lib.pt_learned_create(int(capacity), int(seed), C.c_void_p(stream or 0), C.byref(h_)))
        self._h = h_
        self.nparams = int(self._lib.pt_learned_num_params())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.pt_learned_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def params(self) -> np.ndarray:
        """float32 master weights in the order w1, b1, w2, b2, w3, b3, w4, b4 (w: c_out x c_in x 5)."""
        out = np.empty(self.nparams, dtype=np.float32)
        _check(self._lib.pt_learned_get_params(self._h, _fptr(out)))
        return out

    @params.setter
    def params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        if p.size != self.nparams:
            raise ValueError(f"expected {self.nparams} parameters")
        _check(self._lib.pt_learned_set_params(self._h, _fptr(p)))

    def forward(self, x):
        """Network output for samples x (batch, 8, n) float32 (host)."""
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.empty_like(x)
        _check(self._lib.pt_learned_forward(self._h, x.shape[0], x.shape[2], _fptr(x), _fptr(y)))
        return y

    def gradient(self, x, t):
        """(loss, gradient of every parameter) for samples x and targets t (batch, 8, n)."""
        x = np.ascontiguousarray(x, dtype=np.float32)
        t = np.ascontiguousarray(t, dtype=np.float32)
        g = np.empty(self.nparams, dtype=np.float32)
        loss = C.c_double()
        _check(self._lib.pt_learned_gradient(self._h, x.shape[0], x.shape[2], _fptr(x), _fptr(t), C.byref(loss),
                                             _fptr(g)))
        return loss.value, g

    def collect(self, solver: "Solver", f) -> int:
        """Add training pairs from the Krylov vectors of a sweep-only solve of the sources f."""
        p, dev, keep, n = solver._prep(f, (solver.NZ, solver.NX))
        added = C.c_int32()
        solver._call(keep, dev, self._lib.pt_learned_collect, self._h, solver._h, n, p, dev, C.byref(added))
        return added.value

    def samples(self):
        cnt, n = C.c_int32(), C.c_int32()
        _check(self._lib.pt_learned_samples(self._h, C.byref(cnt), C.byref(n)))
        return cnt.value, n.value

    def train(self, steps: int, batch: int = 32, lr: float = 1e-3) -> np.ndarray:
        losses = np.empty(max(int(steps), 1), dtype=np.float64)
        _check(self._lib.pt_learned_train(self._h, int(steps), int(batch), float(lr),
                                          losses.ctypes.data_as(C.POINTER(C.c_double))))
        return losses[:steps]

    def attach(self, solver: "Solver", mode: str = "correct"):
        """Use this network as the learned stage of `solver`: mode 'augment' (extra GMRES directions)
        or 'correct' (guarded correction of every sweep step)."""
        m = {"correct": PT_LEARN_CORRECT, "augment": PT_LEARN_AUGMENT}[mode]
        _check(self._lib.pt_solver_set_learned(solver._h, self._h, m))
        solver._learned = self

    @staticmethod
    def detach(solver: "Solver"):
        _check(solver._lib.pt_solver_set_learned(solver._h, None, PT_LEARN_CORRECT))
        solver._learned = None

    def save(self, path: str):
        _check(self._lib.pt_learned_save(self._h, os.fsencode(path)))

    def load(self, path: str):
        _check(self._lib.pt_learned_load(self._h, os.fsencode(path)))


def solve_batch(solvers, fs, merged: bool = False):
    """Solve independent problems at once (pt_solve_batch): solvers[i] on fs[i] (all host arrays or all device
    tensors).  Returns [(u_i, infos_i)].  Give each solver its own stream for the problems to overlap.
    merged: one launch sequence for all problems (pt_solve_batch_merged)."""
    n = len(solvers)
    if n != len(fs):
        raise ValueError("one source array per solver")
    L = lib()
    preps, outs, infos = [], [], []
    dev0 = None
    for sv, f in zip(solvers, fs):
        p, dev, keep, k = sv._prep(f, (sv.NZ, sv.NX))
        if dev0 is None:
            dev0 = dev
        elif dev != dev0:
            raise TypeError("all host arrays or all device tensors")
        preps.append((p, keep, k))
        outs.append(sv._out(keep, dev, (k, sv.NZ, sv.NX)))
        infos.append((PtRhsInfo * k)())
    hs = (C.c_void_p * n)(*[sv._h for sv in solvers])
    ks = (C.c_int32 * n)(*[k for _, _, k in preps])
    fp = (C.c_void_p * n)(*[p for p, _, _ in preps])
    up = (C.c_void_p * n)(*[Solver._ptr(u, dev0) for u in outs])
    ip = (C.POINTER(PtRhsInfo) * n)(*[C.cast(i, C.POINTER(PtRhsInfo)) for i in infos])
    pairs = [sv._enter(keep, dev0) for sv, (_, keep, _) in zip(solvers, preps)]
    try:
        call = L.pt_solve_batch_merged if merged else L.pt_solve_batch
        _check(call(n, hs, ks, fp, up, dev0 or 0, ip), allow=(PT_ENOCONV,))
    finally:
        for pr in pairs:
            Solver._leave(pr)
    return [(u, [{"iters": i.iters, "converged": bool(i.converged), "est": i.est, "relres": i.relres,
                  "learned": bool(i.learned), "learned_steps": i.learned_steps} for i in inf])
            for u, inf in zip(outs, infos)]


def setup_batch(probs, streams=None, **kw):
    """Set up several problems at once (pt_setup_batch): one host thread per problem, each on its stream
    (streams[i], or the null stream), so their factorisations overlap on the GPU.  probs: objects with nx, nz,
    npml, h, omega, C, L, c; kw: the Solver options, shared by all (max_nrhs may be a list).  -> [Solver]"""
    n = len(probs)
    mx = kw.pop("max_nrhs", 1)
    mx = list(mx) if isinstance(mx, (list, tuple)) else [mx] * n
    made = [_problem_options(p.nx, p.nz, p.npml, p.h, p.omega, p.C, p.L, p.c, max_nrhs=m, **kw)
            for p, m in zip(probs, mx)]
    pa = (PtProblem * n)(*[m[0] for m in made])
    oa = (PtOptions * n)(*[m[1] for m in made])
    sa = (C.c_void_p * n)(*[int(s or 0) for s in (streams or [0] * n)])
    out = (C.c_void_p * n)()
    _check(lib().pt_setup_batch(n, pa, oa, sa, out))
    res = []
    for i in range(n):
        sv = Solver.__new__(Solver)
        sv._c = made[i][2]
        sv._adopt(C.c_void_p(out[i]), streams[i] if streams else None)
        res.append(sv)
    return res


def tune_cache_save(path: str):
    """Write the process-wide tuning cache (every choice pt_tune made or loaded) to a text file."""
    _check(lib().pt_tune_cache_save(os.fsencode(path)))


def tune_cache_load(path: str):
    """Merge a tuning cache written by tune_cache_save into this process's cache."""
    _check(lib().pt_tune_cache_load(os.fsencode(path)))
