"""Pins of the oracle's discretisation and decomposition (CPU only).

Section 2.1 (stencil + PML), Section 2.2 (layers, local problems), appendix
(symmetric PML form).
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import assemble as asm

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def tiny(nx=4, nz=5, npml=2, L=2, seed=3):
    rng = np.random.default_rng(seed)
    h = 1.0 / 6
    c = synth.normal_extend(0.8 + 0.4 * rng.random((nz, nx)), npml)
    return synth.Problem("tiny", nx, nz, npml, h, 9.0, L, 25.0, c)


def test_two_assemblies_agree():
    p = tiny()
    A1 = asm.global_operator(p).toarray()
    A2 = asm.global_operator_loops(p)
    assert A1.shape == A2.shape == (p.NX * p.NZ,) * 2
    assert np.max(np.abs(A1 - A2)) <= 1e-14 * np.max(np.abs(A1))


def test_hand_computed_stencil_rows():
    g = json.load(open(os.path.join(GOLD, "stencil_3x3.json")))
    q = g["problem"]
    p = synth.Problem("golden", q["nx"], q["nz"], q["npml"], q["h"], q["omega"], 1, q["C"],
                      np.full((3, 3), q["c"]))
    A = asm.global_operator(p).toarray()
    for r, entries in g["rows"].items():
        row = np.zeros(9, dtype=complex)
        for c, (re, im) in entries.items():
            row[int(c)] = re + 1j * im
        assert np.allclose(A[int(r)], row, atol=1e-14), (r, A[int(r)], row)


def test_symmetric_pml_form():
    # diag(a_x a_z)^-1 A is complex symmetric (appendix, eq. Helmholtz_pml_symmetric)
    p = tiny(nx=6, nz=7, npml=3)
    A = asm.global_operator(p).toarray()
    S = A / asm.symmetric_scaling(p)[:, None]
    assert np.max(np.abs(S - S.T)) <= 1e-13 * np.max(np.abs(S))
    # and A itself is not symmetric inside the PML (the paper's remark)
    assert np.max(np.abs(A - A.T)) > 1e-3


def test_pml_profile_values():
    # sigma = (C/delta)(d/delta)^2, zero on [0, L]; alpha = 1/(1 + i sigma/omega)
    n, npml, h, C, w = 10, 4, 0.1, 5.0, 3.0
    a, am, ap = asm.axis_alphas(n, npml, h, C, w)
    assert a.shape == (n + 2 * npml,)
    phys = slice(npml - 1, npml + n + 1)  # nodes p = 0..n+1 have d = 0
    assert np.all(a[phys] == 1.0)
    d = 3 * h  # node p = -3 is array index npml-1-3
    sig = (C / (npml * h)) * (d / (npml * h)) ** 2
    assert np.isclose(a[npml - 4], 1 / (1 + 1j * sig / w), rtol=1e-15)
    # half node p - 1/2 of p = 0 sits at d = h/2
    sig = (C / (npml * h)) * (0.5 * h / (npml * h)) ** 2
    assert np.isclose(am[npml - 1], 1 / (1 + 1j * sig / w), rtol=1e-15)
    assert ap[npml - 1] == 1.0


@pytest.mark.parametrize("L", [1, 2, 3, 5])
def test_layer_split(L):
    p = tiny(nx=4, nz=17, npml=3, L=L)
    slabs = asm.layer_split(p)
    assert len(slabs) == L
    assert slabs[0].own_start == 0
    assert sum(s.n for s in slabs) == p.NZ
    for a, b in zip(slabs[:-1], slabs[1:]):
        assert b.own_start == a.own_start + a.n
        # interface rows (n, n+1 of a) are physical rows
        assert a.own_start + a.n - 1 >= p.npml and a.own_start + a.n <= p.npml + p.nz - 1
    assert slabs[0].top_ext == 0 and slabs[-1].bot_ext == 0
    assert all(s.top_ext == p.npml for s in slabs[1:])
    assert all(s.bot_ext == p.npml for s in slabs[:-1])


def test_layer_split_rejects_thin_layers():
    p = tiny(nx=4, nz=5, npml=2, L=3)
    with pytest.raises(ValueError):
        asm.layer_split(p)


@pytest.mark.parametrize("L", [2, 3])
def test_local_equals_global_on_owned_rows(L):
    # Section 2.2: the local and global equations coincide on the owned rows
    p = tiny(nx=5, nz=12, npml=3, L=L)
    A = asm.global_operator(p).toarray()
    NX = p.NX
    for s in asm.layer_split(p):
        Al = asm.local_operator(p, s).toarray()
        g0 = s.own_start * NX
        l0 = s.top_ext * NX
        n = s.n * NX
        assert np.array_equal(Al[l0:l0 + n, l0:l0 + n], A[g0:g0 + n, g0:g0 + n])
        # couplings across the interface rows are exactly -1 (identity blocks)
        if s.top_ext:
            r0, r1 = s.row(0) * NX, s.row(1) * NX
            assert np.array_equal(Al[r1:r1 + NX, r0:r0 + NX], -np.eye(NX))
            assert np.array_equal(Al[r0:r0 + NX, r1:r1 + NX], -np.eye(NX))
        if s.bot_ext:
            rn, rn1 = s.row(s.n) * NX, s.row(s.n + 1) * NX
            assert np.array_equal(Al[rn:rn + NX, rn1:rn1 + NX], -np.eye(NX))
            assert np.array_equal(Al[rn1:rn1 + NX, rn:rn + NX], -np.eye(NX))


def test_local_extension_model_is_normal_extension():
    p = tiny(nx=5, nz=12, npml=3, L=3)
    for s in asm.layer_split(p):
        az, azm, azp, m = asm.local_z_profile(p, s)
        mg = 1.0 / p.c ** 2
        for r in range(s.R):
            j = r - s.top_ext + 1
            jj = min(max(j, 1), s.n)
            assert np.array_equal(m[r], mg[s.own_start + jj - 1])
        # first extension node carries no damping, deeper ones do
        if s.top_ext:
            assert az[s.row(0)] == 1.0 and abs(az[s.row(-1)] - 1) > 0


@pytest.mark.parametrize("L", [2, 3])
def test_local_inverse_rows_from_columns(L):
    # The local operator is a diagonal times a symmetric matrix, A^l = diag(s) A_sym with
    # s = a_x a_z (its own z profile, extension PML included), so the rows of (A^l)^-1 follow
    # from its columns: K[p, q] = K[q, p] s_p / s_q.  The GPU pre-solve builds the rows of the
    # inverse at the trace rows from the columns its extraction solves compute.
    prob = tiny(nx=5, nz=9, npml=2, L=L, seed=11)
    ax, _, _ = asm.axis_alphas(prob.nx, prob.px, prob.h, prob.C, prob.omega, prob.npml)
    for slab in asm.layer_split(prob):
        A = asm.local_operator(prob, slab).toarray()
        K = np.linalg.inv(A)
        az, _, _, _ = asm.local_z_profile(prob, slab)
        s = (az[:, None] * ax[None, :]).ravel()
        assert np.abs(K - K.T).max() > 1e-3 * np.abs(K).max()  # not symmetric by itself
        assert np.allclose(K, K.T * s[:, None] / s[None, :], rtol=0, atol=1e-12 * np.abs(K).max())
        # and A_sym = diag(1/s) A is symmetric (a planted transpose of the scaling would fail)
        As = A / s[:, None]
        assert np.allclose(As, As.T, rtol=0, atol=1e-13 * np.abs(As).max())
