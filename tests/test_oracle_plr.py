"""Pins of the oracle's PLR compression (Alg. 5) and product (Alg. 6), CPU only."""
import numpy as np
import pytest

from oracle import plr


def rand_lowrank(m, n, r, rng):
    A = rng.standard_normal((m, r)) + 1j * rng.standard_normal((m, r))
    B = rng.standard_normal((r, n)) + 1j * rng.standard_normal((r, n))
    return A @ B


def check_tiling(H):
    cover = np.zeros((H.m, H.n), dtype=int)
    for lf in plr.leaves(H):
        cover[lf.r0 - H.r0:lf.r0 - H.r0 + lf.m, lf.c0 - H.c0:lf.c0 - H.c0 + lf.n] += 1
    assert np.all(cover == 1)


def test_exact_low_rank_is_one_leaf():
    rng = np.random.default_rng(0)
    M = rand_lowrank(70, 50, 3, rng)
    H = plr.compress(M, rmax=5, eps=1e-9)
    assert H.kind == "lr" and H.U.shape[1] == 3
    assert np.allclose(plr.to_dense(H), M, atol=1e-10 * np.abs(M).max())


def test_full_rank_splits_to_dense_leaves():
    rng = np.random.default_rng(1)
    M = rng.standard_normal((33, 33)) + 0j
    H = plr.compress(M, rmax=4, eps=1e-9)
    lv = plr.leaves(H)
    assert all(lf.kind == "dense" for lf in lv)
    assert all(min(lf.m, lf.n) <= 4 for lf in lv)
    check_tiling(H)
    assert np.array_equal(plr.to_dense(H), M)


def smooth_kernel(n, rng):
    # oscillatory kernel with a near-diagonal singularity: low rank away from the diagonal
    x = np.sort(rng.uniform(0, 1, n))
    d = np.abs(x[:, None] - x[None, :]) + 1.0 / n
    return np.exp(10j * d) / d


@pytest.mark.parametrize("eps", [1e-6, 1e-9])
def test_leaves_tile_and_errors_are_bounded(eps):
    rng = np.random.default_rng(2)
    M = smooth_kernel(96, rng)
    H = plr.compress(M, rmax=8, eps=eps)
    check_tiling(H)
    lv = plr.leaves(H)
    assert any(lf.kind == "lr" for lf in lv) and any(lf.kind == "dense" for lf in lv)
    for lf in lv:
        if lf.kind == "lr":
            assert lf.U.shape[1] <= 8 and lf.sigma_next < eps
            # the leaf's 2-norm error is its first discarded singular value
            blk = M[lf.r0:lf.r0 + lf.m, lf.c0:lf.c0 + lf.n]
            assert np.linalg.norm(blk - lf.U @ lf.V, 2) <= lf.sigma_next * (1 + 1e-6) + 1e-13
    # product error within the sum of leaf errors
    x = rng.standard_normal(96) + 1j * rng.standard_normal(96)
    err = np.linalg.norm(plr.matvec(H, x) - M @ x)
    bound = sum(lf.sigma_next for lf in lv if lf.kind == "lr") * np.linalg.norm(x) + 1e-12 * np.linalg.norm(M @ x)
    assert err <= bound
    assert plr.stored_entries(H) < M.size


def test_recursive_and_sparse_factorized_products_agree():
    rng = np.random.default_rng(3)
    M = smooth_kernel(77, rng)  # odd sizes: ceil/floor splits
    H = plr.compress(M, rmax=6, eps=1e-8)
    X = rng.standard_normal((77, 3)) + 1j * rng.standard_normal((77, 3))
    a = plr.matvec(H, X)
    b = plr.sparse_factorized_matvec(H, X)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-12 * np.abs(a).max())
    assert np.allclose(a, plr.to_dense(H) @ X, rtol=1e-12, atol=1e-12 * np.abs(a).max())


def test_stored_entries_hand_counted_tree():
    # 8 x 8 block [[rank 1, rank 2], [0, full rank]] with r_max = 2: the whole block has rank > 2 and splits;
    # top-left: one low-rank leaf of rank 1 (4 + 4) * 1 = 8 entries; top-right: rank 2, (4 + 4) * 2 = 16;
    # bottom-left: rank 0 (no stored entries); bottom-right: full rank, splits into four 2 x 2 dense leaves
    # (min side 2 <= r_max), 4 * 4 = 16.  Hand count: 8 + 16 + 0 + 16 = 40 entries in 7 leaves.
    rng = np.random.default_rng(5)
    M = np.zeros((8, 8), dtype=np.complex128)
    M[:4, :4] = rand_lowrank(4, 4, 1, rng)
    M[:4, 4:] = rand_lowrank(4, 4, 2, rng)
    M[4:, 4:] = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    H = plr.compress(M, rmax=2, eps=1e-9)
    lv = plr.leaves(H)
    assert len(lv) == 7
    assert sorted((lf.kind, lf.m, lf.n) for lf in lv) == sorted(
        [("lr", 4, 4)] * 3 + [("dense", 2, 2)] * 4)
    assert plr.stored_entries(H) == 40
    # odd sides: 7 x 7 full rank, r_max = 2 -> quarters 4x4, 4x3, 3x4, 3x3 (all still full rank, min side > 2)
    # -> each splits again into 2x2 / 2x1 / 1x2 / 1x1 dense pieces covering it: 49 stored entries in 16 leaves
    N = rng.standard_normal((7, 7)) + 1j * rng.standard_normal((7, 7))
    H = plr.compress(N, rmax=2, eps=1e-9)
    assert plr.stored_entries(H) == 49 and len(plr.leaves(H)) == 16
    assert all(lf.kind == "dense" for lf in plr.leaves(H))
