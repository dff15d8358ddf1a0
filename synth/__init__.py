"""Seeded synthetic inputs for the polarized-traces Helmholtz solver.

This module only *makes inputs*: velocity models on the PML-padded grid,
frequencies, layer counts and right-hand sides.  It holds none of the
method's arithmetic (no stencil, no PML profile, no solve), so both the CPU
oracle and the GPU library can consume what it produces without sharing any
code of the method.

Grid convention (the paper's discretisation section): physical nodes are
x_p = p*h, p = 1..nx (and z_q = q*h, q = 1..nz); the padded grid adds npml
nodes on every side, so arrays have shape (nz + 2*npml, nx + 2*npml) with x
fastest.  Array index ix corresponds to p = ix - npml + 1.

Every array is float64 / complex128.  Randomness is NumPy PCG64 seeded per
workload, so a workload is fully determined by its name and seed.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

__all__ = [
    "Problem",
    "normal_extend",
    "gaussian_source",
    "config1",
    "config2",
    "config3",
    "config4",
    "config_small",
    "bump_medium",
    "layered_medium",
    "homogeneous_problem",
    "cavity_medium",
    "cavity_problem",
]


@dataclass
class Problem:
    """One Helmholtz problem: -Lap u - omega^2 m u = f with m = 1/c^2.

    c is given on the padded grid (nz+2npml, nx+2npml), x fastest.  C is the
    PML strength constant of sigma(d) = (C/delta)(d/delta)^2.  L is the number
    of layers the z axis is split into.
    """

    name: str
    nx: int
    nz: int
    npml: int
    h: float
    omega: float
    L: int
    C: float
    c: np.ndarray
    meta: dict = field(default_factory=dict)
    npml_x: int | None = None   # PML width along x if different from npml (oracle-only special cases)

    @property
    def px(self) -> int:
        return self.npml if self.npml_x is None else self.npml_x

    @property
    def NX(self) -> int:
        return self.nx + 2 * self.px

    @property
    def NZ(self) -> int:
        return self.nz + 2 * self.npml

    def replace(self, **kw) -> "Problem":
        d = dict(self.__dict__)
        d.update(kw)
        return Problem(**d)


def normal_extend(c_phys: np.ndarray, npml: int) -> np.ndarray:
    """Pad a physical (nz, nx) model by edge replication (normal extension)."""
    return np.pad(np.asarray(c_phys, dtype=np.float64), npml, mode="edge")


def _phys_coords(nx: int, nz: int, h: float):
    x = np.arange(1, nx + 1, dtype=np.float64) * h
    z = np.arange(1, nz + 1, dtype=np.float64) * h
    return np.meshgrid(x, z)  # (nz, nx) each


def gaussian_source(prob: Problem, x0: float, z0: float, sigma: float) -> np.ndarray:
    """exp(-|x-x0|^2/(2 sigma^2)) on physical nodes, zero in the PML."""
    X, Z = _phys_coords(prob.nx, prob.nz, prob.h)
    g = np.exp(-((X - x0) ** 2 + (Z - z0) ** 2) / (2.0 * sigma * sigma))
    f = np.zeros((prob.NZ, prob.NX), dtype=np.complex128)
    f[prob.npml : prob.npml + prob.nz, prob.npml : prob.npml + prob.nx] = g
    return f


def random_sources(prob: Problem, nrhs: int, seed: int, cplx: bool = True) -> np.ndarray:
    """Dense random right-hand sides on physical nodes (zero in the PML)."""
    rng = np.random.default_rng(seed)
    f = np.zeros((nrhs, prob.NZ, prob.NX), dtype=np.complex128)
    sl = (slice(None), slice(prob.npml, prob.npml + prob.nz), slice(prob.npml, prob.npml + prob.nx))
    re = rng.standard_normal((nrhs, prob.nz, prob.nx))
    im = rng.standard_normal((nrhs, prob.nz, prob.nx)) if cplx else 0.0
    f[sl] = re + 1j * im
    return f


# ----------------------------------------------------------------------------
# media
# ----------------------------------------------------------------------------

def bump_medium(nx: int, nz: int, h: float, rng: np.random.Generator, nbumps: int = 20) -> np.ndarray:
    """c = 1 + sum_b A_b exp(-|x-x_b|^2/(2 w_b^2)), A~U[-.3,.3], w~U[.03,.1], x_b~U[0,1]^2; c >= 0.3."""
    X, Z = _phys_coords(nx, nz, h)
    c = np.ones_like(X)
    A = rng.uniform(-0.3, 0.3, nbumps)
    w = rng.uniform(0.03, 0.1, nbumps)
    cx = rng.uniform(0.0, 1.0, nbumps)
    cz = rng.uniform(0.0, 1.0, nbumps)
    for b in range(nbumps):
        c += A[b] * np.exp(-((X - cx[b]) ** 2 + (Z - cz[b]) ** 2) / (2.0 * w[b] ** 2))
    return np.maximum(c, 0.3)


def layered_medium(width: int, depth: int, h: float, rng: np.random.Generator,
                   nlayers: int = 12, nfaults: int = 3, lognormal_sigma: float = 0.05) -> np.ndarray:
    """Dipping, faulted layered section (depth, width) in m/s, 1.5 -> 4.5 km/s with depth.

    Layer i (0 = top) has velocity 1500 + 3000 i/(nlayers-1) + U[-100, 100].
    Interfaces sit at evenly spaced depths, dip by U[-10, 10] degrees about the
    section's centre, and are shifted by U[-200, 200] m on the right of each of
    nfaults vertical faults at x ~ U(2, 10) km.  Finally c *= exp(s * xi),
    xi ~ N(0, 1) i.i.d. per node.
    """
    X = np.arange(1, width + 1, dtype=np.float64) * h
    Zd = np.arange(1, depth + 1, dtype=np.float64) * h
    vel = 1500.0 + 3000.0 * np.arange(nlayers) / (nlayers - 1) + rng.uniform(-100.0, 100.0, nlayers)
    base = np.arange(1, nlayers) * (depth * h) / nlayers
    dips = np.deg2rad(rng.uniform(-10.0, 10.0, nlayers - 1))
    xf = rng.uniform(2000.0, 10000.0, nfaults)
    throw = rng.uniform(-200.0, 200.0, nfaults)
    shift = np.zeros_like(X)
    for k in range(nfaults):
        shift += np.where(X > xf[k], throw[k], 0.0)
    xm = 0.5 * width * h
    ifz = base[:, None] + np.tan(dips)[:, None] * (X[None, :] - xm) + shift[None, :]  # (nl-1, width)
    layer = (Zd[None, :, None] > ifz[:, None, :]).sum(axis=0)  # (depth, width)
    c = vel[layer]
    c = c * np.exp(lognormal_sigma * rng.standard_normal(c.shape))
    return c


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def _pml_C(c_pad: np.ndarray) -> float:
    # PML strength: 30 * max velocity gives a continuous normal-incidence
    # round-trip reflection exp(-2C/(3c)) <= exp(-20).
    return 30.0 * float(np.max(c_pad))


def config1() -> tuple[Problem, np.ndarray]:
    """Constant c = 1, 80x80 interior, h = 1/80, 10-point PML, omega = 2 pi 8, L = 4.

    One Gaussian source (sigma = 0.01) at (0.5, 0.125) = physical node (40, 10).
    """
    nx = nz = 80
    npml = 10
    h = 1.0 / 80.0
    c = np.ones((nz + 2 * npml, nx + 2 * npml))
    prob = Problem("constant-100x100-L4", nx, nz, npml, h, 2 * math.pi * 8.0, 4, _pml_C(c), c)
    f = gaussian_source(prob, 0.5, 0.125, 0.01)
    return prob, f[None]


def config2(seed: int = 2, n: int = 400, npml: int = 20, L: int = 8) -> tuple[Problem, np.ndarray]:
    """20 Gaussian bumps, n x n interior (default 400), h = 1/n, 20-point PML, 10 ppw at min c, L = 8."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    cp = bump_medium(n, n, h, rng)
    c = normal_extend(cp, npml)
    omega = 2 * math.pi * float(cp.min()) / (10.0 * h)
    prob = Problem(f"bumps-{n + 2 * npml}x{n + 2 * npml}-L{L}", n, n, npml, h, omega, L, _pml_C(c), c,
                   meta={"seed": seed, "c_min": float(cp.min()), "c_max": float(cp.max())})
    f = gaussian_source(prob, 0.5, 0.125, 0.01)
    return prob, f[None]


def config3(seed: int = 3, nrhs: int = 128, width: int = 1200, depth: int = 400, npml: int = 20,
            L: int = 16) -> tuple[Problem, np.ndarray]:
    """Layered faulted section (width x depth, h = 10 m), f = 10 Hz, L = 16, nrhs Gaussian sources.

    Layers are cut across the wide axis: the solver's layer axis (z) is the
    section's horizontal axis and the solver's x axis is depth, so the model
    is stored transposed, shape (width + 2 npml, depth + 2 npml).  Sources
    (sigma = h) sit on the first physical depth row at horizontal nodes
    round((i + 1/2) width / nrhs), i = 0..nrhs-1.
    """
    rng = np.random.default_rng(seed)
    h = 10.0
    geo = layered_medium(width, depth, h, rng)      # (depth, width)
    cp = geo.T.copy()                               # solver (z = width, x = depth)
    c = normal_extend(cp, npml)
    prob = Problem(f"layered-{width + 2 * npml}x{depth + 2 * npml}-L{L}", depth, width, npml, h,
                   2 * math.pi * 10.0, L, _pml_C(c), c,
                   meta={"seed": seed, "orientation": "layers cut along the 1200-node horizontal axis"})
    f = np.zeros((nrhs, prob.NZ, prob.NX), dtype=np.complex128)
    for i in range(nrhs):
        q = int(round((i + 0.5) * width / nrhs))
        q = min(max(q, 1), width)
        f[i] = gaussian_source(prob, 1 * h, q * h, h)
    return prob, f


def config4(seed: int = 4, nprob: int = 8, nrhs: int = 32, nmin: int = 200, nmax: int = 800,
            npml: int = 20) -> list[tuple[Problem, np.ndarray]]:
    """nprob independent square problems, n ~ U{nmin..nmax}, L ~ U{4..16}, nrhs Gaussian sources each."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(nprob):
        n = int(rng.integers(nmin, nmax + 1))
        L = int(rng.integers(4, 17))
        h = 1.0 / n
        if i % 2 == 0:
            cp = np.ones((n, n))
        else:
            cp = bump_medium(n, n, h, np.random.default_rng(seed * 1000 + i))
        c = normal_extend(cp, npml)
        omega = 2 * math.pi * float(cp.min()) / (10.0 * h)
        prob = Problem(f"p{i}-{n + 2 * npml}sq-L{L}", n, n, npml, h, omega, L, _pml_C(c), c,
                       meta={"seed": seed, "index": i})
        sig = 2 * h
        lo, hi = 3 * sig + h, (n + 1) * h - 3 * sig - h
        f = np.zeros((nrhs, prob.NZ, prob.NX), dtype=np.complex128)
        xs = rng.uniform(lo, hi, nrhs)
        zs = rng.uniform(lo, hi, nrhs)
        for j in range(nrhs):
            f[j] = gaussian_source(prob, xs[j], zs[j], sig)
        out.append((prob, f))
    return out


def config_small(nx: int = 24, nz: int = 30, npml: int = 5, L: int = 3, seed: int = 7,
                 ppw: float = 8.0, bumps: bool = True, nrhs: int = 1) -> tuple[Problem, np.ndarray]:
    """Small heterogeneous problem for tests (h = 1/max(nx, nz))."""
    rng = np.random.default_rng(seed)
    h = 1.0 / max(nx, nz)
    cp = bump_medium(nx, nz, h, rng, nbumps=5) if bumps else np.ones((nz, nx))
    c = normal_extend(cp, npml)
    omega = 2 * math.pi * float(cp.min()) / (ppw * h)
    prob = Problem(f"small-{nx}x{nz}-L{L}", nx, nz, npml, h, omega, L, _pml_C(c), c, meta={"seed": seed})
    f = random_sources(prob, nrhs, seed + 1)
    return prob, f


def learned_model(index: int, n: int = 256, L: int = 8, npml: int = 20, nrhs: int = 16,
                  seed: int = 5) -> tuple[Problem, np.ndarray]:
    """One model of the learned-stage workload: n x n interior, L layers, nrhs Gaussian sources.

    Even indices draw a smooth-bump medium (as config2: h = 1/n, c ~ 1), odd
    indices a dipping, faulted layered section (as config3, scaled to a 12 km
    square: h = 12000/n m).  omega gives 10 points per wavelength at the
    minimum velocity.  Sources (sigma = 2h) sit at uniform random interior
    positions at least 3 sigma + h from the PML.  Model i uses the generator
    seeded with (seed, i): training and held-out sets take disjoint index ranges.
    """
    rng = np.random.default_rng([seed, index])
    if index % 2 == 0:
        h = 1.0 / n
        cp = bump_medium(n, n, h, rng)
        kind = "bumps"
    else:
        h = 12000.0 / n
        cp = layered_medium(n, n, h, rng)
        kind = "layered"
    c = normal_extend(cp, npml)
    omega = 2 * math.pi * float(cp.min()) / (10.0 * h)
    prob = Problem(f"{kind}{index}-{n + 2 * npml}sq-L{L}", n, n, npml, h, omega, L, _pml_C(c), c,
                   meta={"seed": seed, "index": index, "kind": kind})
    sig = 2 * h
    lo, hi = 3 * sig + h, (n + 1) * h - 3 * sig - h
    xs = rng.uniform(lo, hi, nrhs)
    zs = rng.uniform(lo, hi, nrhs)
    f = np.zeros((nrhs, prob.NZ, prob.NX), dtype=np.complex128)
    for j in range(nrhs):
        f[j] = gaussian_source(prob, xs[j], zs[j], sig)
    return prob, f


def homogeneous_problem(n: int = 32, npml: int = 8, L: int = 3, ppw: float = 10.0) -> Problem:
    """c = 1 on [0, 1]^2 (n x n nodes, h = 1/n), ppw points per wavelength, npml-point PML.

    The spectral workload for PML quality: with no heterogeneity every
    reflection comes from the truncation of the PML.
    """
    h = 1.0 / n
    c = normal_extend(np.ones((n, n)), npml)
    return Problem(f"homogeneous-{n}-pml{npml}-L{L}", n, n, npml, h, 2 * math.pi / (ppw * h), L, _pml_C(c), c,
                   meta={"ppw": ppw})


def cavity_medium(n: int, c_red: float = 5.0) -> np.ndarray:
    """A resonant wave-guide on [0, 1]^2 (n x n nodes, h = 1/n): smooth background
    c = 1 + 0.1 x + 0.1 z and a ring of speed c_red (radii 0.18-0.30 around the
    centre) with a 60-degree opening facing +x.  The ring shape is invented for
    this workload; only the background and c_red follow the cavity experiment.
    """
    h = 1.0 / n
    X, Z = _phys_coords(n, n, h)
    c = 1.0 + 0.1 * X + 0.1 * Z
    r = np.hypot(X - 0.5, Z - 0.5)
    ang = np.arctan2(Z - 0.5, X - 0.5)
    ring = (r > 0.18) & (r < 0.30) & (np.abs(ang) > math.pi / 6)
    return np.where(ring, c_red, c)


def cavity_problem(n: int = 64, omega: float = 16.0, npml: int = 8, L: int = 4, c_red: float = 5.0) -> Problem:
    """The cavity medium of `cavity_medium` at angular frequency omega, L layers."""
    c = normal_extend(cavity_medium(n, c_red), npml)
    return Problem(f"cavity-{n}-w{omega:g}-L{L}", n, n, npml, 1.0 / n, float(omega), L, _pml_C(c), c,
                   meta={"c_red": c_red})
