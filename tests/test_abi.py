"""The C-ABI library loads and exports every entry point include/polar.h declares (CPU only),
and host-side validation rejects invalid problems before touching the GPU."""
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "polar.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pt_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("pt_setup", "pt_solve", "pt_free", "pt_apply", "pt_local_solve", "pt_trace_rhs", "pt_reconstruct",
              "pt_get_block", "pt_get_layout", "pt_status_str", "pt_last_error"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    P = pytest.importorskip("paper_1410_5910_amd")
    L = P.lib()
    for s in declared_symbols():
        assert hasattr(L, s), s
    assert L.pt_status_str(0) == b"ok"


@pytest.mark.parametrize("change,msg", [
    (dict(L=50), "physical rows"),
    (dict(omega=-1.0), "omega"),
    (dict(h=0.0), "h and omega"),
    (dict(npml=0), "npml"),
    (dict(C=-1.0), "pml_C"),
])
def test_invalid_problems_rejected(change, msg):
    P = pytest.importorskip("paper_1410_5910_amd")
    prob, f = synth.config_small(nx=12, nz=16, npml=3, L=2)
    kw = dict(nx=prob.nx, nz=prob.nz, npml=prob.npml, h=prob.h, omega=prob.omega, C_pml=prob.C, L=prob.L, c=prob.c)
    if "C" in change:
        kw["C_pml"] = change.pop("C")
    kw.update(change)
    if kw["npml"] != prob.npml:
        kw["c"] = np.ones(((prob.nz + 2 * kw["npml"]), (prob.nx + 2 * kw["npml"])))
    with pytest.raises(P.PolarError) as e:
        P.Solver(**kw)
    assert e.value.status == 1 and msg in str(e.value)


def test_nonpositive_velocity_rejected():
    P = pytest.importorskip("paper_1410_5910_amd")
    prob, f = synth.config_small(nx=12, nz=16, npml=3, L=2)
    c = prob.c.copy()
    c[3, 4] = 0.0
    with pytest.raises(P.PolarError) as e:
        P.Solver(prob.nx, prob.nz, prob.npml, prob.h, prob.omega, prob.C, prob.L, c)
    assert e.value.status == 1


@pytest.mark.parametrize("opt,msg", [
    (dict(gs_iters=9), "gs_iters"),
    (dict(gs_iters=-1), "gs_iters"),
    (dict(plr=True, plr_rmax=65), "plr_rmax"),
    (dict(plr=True, plr_eps=0.0), "plr_eps"),
    (dict(plr=True, precision="f32"), "float64 only"),
])
def test_invalid_options_rejected(opt, msg):
    # option checks run before any device work (no GPU needed)
    P = pytest.importorskip("paper_1410_5910_amd")
    prob, f = synth.config_small(nx=12, nz=16, npml=3, L=2)
    with pytest.raises(P.PolarError) as e:
        P.Solver(prob.nx, prob.nz, prob.npml, prob.h, prob.omega, prob.C, prob.L, prob.c, **opt)
    assert e.value.status == 1 and msg in str(e.value)


def test_load_rejects_non_solver_files_without_a_gpu(tmp_path):
    # pt_load checks the file's magic before any device call
    P = pytest.importorskip("paper_1410_5910_amd")
    L = P.lib()
    import ctypes as C
    bad = tmp_path / "x.pts"
    bad.write_bytes(b"definitely not a saved solver")
    out = C.c_void_p()
    assert L.pt_load(str(bad).encode(), None, C.byref(out)) == P.polar.PT_EINVAL
    assert out.value is None
    assert L.pt_load(str(tmp_path / "missing").encode(), None, C.byref(out)) == P.polar.PT_EINVAL
    assert L.pt_setup_batch(0, None, None, None, None) == P.polar.PT_OK


def test_tune_cache_files_without_a_gpu(tmp_path):
    # the tuning cache is host data: saving, loading and rejecting foreign files need no device
    P = pytest.importorskip("paper_1410_5910_amd")
    path = str(tmp_path / "tune.txt")
    P.tune_cache_save(path)
    assert open(path).readline().startswith("# libpolar tuning cache v2")
    P.tune_cache_load(path)
    bad = tmp_path / "bad.txt"
    bad.write_text("# libpolar tuning cache v2\n1 2 3\n")
    with pytest.raises(P.PolarError):
        P.tune_cache_load(str(bad))
    # a file of the previous format (no k-slice column for the MFMA tiles) is rejected whole
    bad.write_text("# libpolar tuning cache v1\n440 16 2 0 0 1 128 4 1 0 0 32 4 0 0 20.6 30.9 21\n")
    with pytest.raises(P.PolarError):
        P.tune_cache_load(str(bad))
    # MFMA tile widths and wave-group counts the kernel does not have
    for cfg in ("1 48 1 1", "1 16 3 1"):
        bad.write_text("# libpolar tuning cache v2\n440 16 2 0 0 1 128 4 " + cfg + " 0 0 0 0 20.6 30.9 21\n")
        with pytest.raises(P.PolarError):
            P.tune_cache_load(str(bad))
    bad.write_text("# libpolar tuning cache v2\n440 16 2 0 0 1 128 4 1 16 4 2 0 0 0 0 20.6 30.9 21\n")
    P.tune_cache_load(str(bad))  # a shape the kernel has
    bad.write_text("something else\n")
    with pytest.raises(P.PolarError):
        P.tune_cache_load(str(bad))
