#!/usr/bin/env python3
"""Online Helmholtz solves/s of the polarized-traces solver on one MI355X.

One step = one pt_solve call (pre local solves, trace right-hand side,
flexible GMRES with the Gauss-Seidel sweep preconditioner, reconstruction)
over one batch of synthetic sources already resident in HBM.

Default workload: the smooth 20-bump medium, 400x400 interior + 20-point PML
(440x440 padded grid), h = 1/400, omega at 10 points per wavelength of the
minimum velocity, L = 8 layers, one Gaussian source (sigma = 0.01) at
(0.5, 0.125), dense float64 trace blocks and local factors.

Prints one JSON line (see --help); progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "online Helmholtz solves/s on 1 MI355X at rel err<=1e-6: mixed+batched vs FP64"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def workload(name):
    import synth
    if name == "bumps440":
        prob, f = synth.config2()
        desc = ("bumps-440x440-L8: smooth 20-bump medium, 400x400 interior + 20-point PML, h=1/400, "
                "10 points/wavelength at min c, one Gaussian source (sigma 0.01) at (0.5, 0.125)")
        return prob, f, desc, 1e-10
    if name == "constant100":
        prob, f = synth.config1()
        desc = ("constant-100x100-L4: c=1, 80x80 interior + 10-point PML, h=1/80, omega=2pi*8, "
                "one Gaussian source (sigma 0.01) at (0.5, 0.125)")
        return prob, f, desc, 1e-10
    if name == "layered1240":
        prob, f = synth.config3()
        desc = ("layered-1240x440-L16: 12 dipping layers 1.5-4.5 km/s, 3 faults, log-normal 5% noise, "
                "1200x400 nodes (h=10 m) + 20-point PML, f=10 Hz, layers cut along the 1200-node axis, "
                "128 Gaussian sources (sigma=h) on the first physical depth row, solved in one call")
        return prob, f, desc, 1e-10
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(prob, f, budget_s=10.0):
    """The oracle's sparse direct solve timed on this host: factorisation excluded (offline),
    repeated per-source triangular solves for about budget_s seconds."""
    import numpy as np
    from oracle.direct import DirectSolver
    t0 = time.perf_counter()
    ds = DirectSolver(prob)
    t_fact = time.perf_counter() - t0
    nsol = 0
    t0 = time.perf_counter()
    while True:
        ds.solve(f[nsol % f.shape[0]])
        nsol += 1
        el = time.perf_counter() - t0
        if el > budget_s:
            break
    return ds, {
        "value": nsol / el, "unit": "solves/s", "cores": 1, "kind": "oracle",
        "sample": (f"SuperLU factorisation of the {prob.NZ}x{prob.NX} padded system ({t_fact:.2f} s, offline, "
                   f"excluded), then {nsol} single-source solves in {el:.1f} s"),
        "cpu": _cpu_model(), "host_cpus": os.cpu_count(),
    }


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="bumps440", choices=["bumps440", "constant100", "layered1240"])
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"])
    ap.add_argument("--nrhs", type=int, default=0, help="sources per step (default: all of the workload's)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-check", action="store_true", help="skip the parity check against the oracle")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the polarized-traces layers are batched inside one device "
              "and there is no multi-GPU path; run with --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    import paper_1410_5910_amd as P

    assert torch.cuda.is_available(), "no GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    prob, f, desc, tol = workload(args.workload)
    if args.nrhs:
        f = f[: args.nrhs]
    nrhs = f.shape[0]
    log(f"workload {prob.name}: grid {prob.NZ}x{prob.NX}, L={prob.L}, nrhs={nrhs}, precision={args.precision}")

    t0 = time.perf_counter()
    s = P.Solver.from_problem(prob, precision=args.precision, tol=tol, maxit=50, max_nrhs=nrhs,
                              stream=stream.cuda_stream)
    lay = s.layout()
    log(f"setup {time.perf_counter() - t0:.1f} s (library {lay['setup_ms'] / 1e3:.1f} s); "
        f"blocks {lay['block_bytes'] / 1e6:.0f} MB, factors {lay['factor_bytes'] / 1e6:.0f} MB")
    fd = torch.from_numpy(f).to(dev)

    for i in range(args.warmup):
        u, info = s.solve(fd)
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps); iterations {sorted(set(i['iters'] for i in info))}")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        u, info = s.solve(fd)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    value = args.steps * nrhs / el
    log(f"timed {args.steps} steps in {el:.3f} s -> {value:.1f} solves/s")

    # live kernel timing of the block-apply launches (HIP events on the solver stream)
    s.profile(True)
    nprof = max(1, min(args.steps, 5))
    for i in range(nprof):
        s.solve(fd)
    st = s.profile_read()
    s.profile(False)
    kern_s = st["kernel_ms"] / 1e3
    achieved_gbs = st["alg_bytes"] / kern_s / 1e9 if kern_s > 0 else 0.0
    achieved_tf = st["alg_flops"] / kern_s / 1e12 if kern_s > 0 else 0.0
    batched = nrhs >= 16
    if batched:
        roof = {"bound": "alu", "achieved": achieved_tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved_tf / FP64_PEAK_TFLOPS}
    else:
        roof = {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved_gbs / HBM_PEAK_GBS}
    roof.update({"traffic": None, "kernel": "block_apply_kernel", "launches_per_step": st["launches"] / nprof,
                 "avg_launch_us": 1e3 * st["kernel_ms"] / max(1, st["launches"]),
                 "alg_bytes_per_launch": st["alg_bytes"] / max(1, st["launches"]),
                 "kernel_share_of_step": kern_s / nprof / (el / args.steps)})
    log(f"block_apply: {st['launches'] / nprof:.0f} launches/step, avg {roof['avg_launch_us']:.2f} us, "
        f"{achieved_gbs:.0f} GB/s, {achieved_tf:.2f} TFLOP/s")

    out = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "f64" else "f32", "data": "synthetic",
        "config": {"workload": desc, "grid": [prob.NZ, prob.NX], "L": prob.L, "nrhs": nrhs,
                   "precision": args.precision, "gmres_tol": tol, "gs_iters": 2,
                   "iterations": sorted(set(i["iters"] for i in info))},
        "roofline": roof,
    }

    ds = None
    if not args.no_cpu:
        log("cpu baseline (oracle direct solve)")
        ds, out["cpu_baseline"] = cpu_baseline(prob, f[:1])
    if not args.no_check:
        from oracle.direct import DirectSolver
        if ds is None:
            ds = DirectSolver(prob)
        k = min(nrhs, 4)
        ref = ds.solve(f[:k])
        got = u[:k].cpu().numpy()
        errs = [float(np.linalg.norm(got[i] - ref[i]) / np.linalg.norm(ref[i])) for i in range(k)]
        out["rel_err_vs_oracle"] = max(errs)
        out["rel_err_checked_rhs"] = k
        log(f"parity vs oracle direct solve: max rel err {max(errs):.2e} over {k} sources")
    print(json.dumps(out), flush=True)
    s.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
