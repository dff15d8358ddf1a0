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
