"""Partitioned low-rank compression on the GPU (Alg. 5) against the dense
blocks and the oracle's compression of the same blocks.

The compressed form is not unique (a randomized sketch decides the leaves;
near the threshold eps the oracle's exact SVD may split where the sketch does
not), so the checks are: every expanded block is within the leaf error bound
of the dense block (each leaf drops only singular values below eps, and the
probes bound the sketch's own error by eps); and the tree, seen through the
stored entries per block, is the oracle's for almost every block.
"""
import math

import numpy as np
import pytest

import synth
from oracle import plr
from oracle.polarized import PolarizedSolver

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1410_5910_amd")


def _flush(msg):
    print(msg, flush=True)


# the blocks stored with an identity added (their trees differ from those of K)
SHIFTED = {("1", "0"), ("n", "n+1")}


# NX = 106: rmax 0 -> ceil(sqrt(NX)) = 11 (22-column sketches); 64: the widest sketch (70 columns).
# NX = 34 with rmax 2: odd halves down to 2-3 rows, six levels deep, 13-column sketches.
@pytest.mark.parametrize("nx,nz,npml,eps,rmax", [(90, 60, 8, 1e-10, 0), (90, 60, 8, 1e-6, 0), (90, 60, 8, 1e-10, 64),
                                                 (24, 30, 5, 1e-10, 2)])
def test_compressed_blocks_within_bound_and_match_oracle_tree(nx, nz, npml, eps, rmax):
    prob, _ = synth.config_small(nx=nx, nz=nz, npml=npml, L=3, nrhs=1, seed=12)
    _flush(f"[gpu] plr compression, NX {nx + 2 * npml}, eps {eps:g}, rmax {rmax}")
    gs = P.Solver.from_problem(prob, plr=True, plr_eps=eps, plr_rmax=rmax)
    ps = PolarizedSolver(prob)
    rmax = rmax or math.ceil(math.sqrt(ps.NX))
    total = same = 0
    st_gpu = st_or = 0
    leaves = 0
    for l, lp in enumerate(ps.loc):
        for (j, k), K in lp.K.items():
            Kd = gs.get_block(l, j, k)
            Kp, nl, ns = gs.get_plr_block(l, j, k)
            leaves += nl
            assert nl >= 1
            err = float(np.abs(Kp - Kd).max())
            assert err <= 4 * eps, (l, j, k, err)
            if (j, k) in SHIFTED:
                continue
            H = plr.compress(K, rmax, eps)
            so = plr.stored_entries(H)
            total += 1
            same += int(so == ns)
            st_gpu += ns
            st_or += so
    lay = gs.layout()
    _flush(f"[gpu] blocks {total}: same tree {same}, stored {st_gpu} vs oracle {st_or}, leaves {leaves}")
    assert lay["plr_leaves"] == leaves
    assert same >= 0.9 * total
    assert abs(st_gpu - st_or) <= 0.05 * st_or
    gs.close()


def test_plr_needs_compressed_solver():
    prob, _ = synth.config_small(nx=40, nz=30, npml=6, L=2, nrhs=1, seed=3)
    gs = P.Solver.from_problem(prob)
    with pytest.raises(P.PolarError):
        gs.get_plr_block(0, "n", "n")
    gs.close()
