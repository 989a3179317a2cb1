"""Pins of the oracle's HODLR compression and SMW factor/solve (Sec. 2)."""
import numpy as np
import pytest

from oracle import hodlr
from oracle.symbolic import _bisect_tree


def _kernel_block(m, n, seed, gap=1.0):
    """Smooth interaction between two separated point clusters (numerically
    low rank, full rank in exact arithmetic)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, (m, 2)) + np.array([1.0 + gap, 0.0])
    y = rng.uniform(0, 1, (n, 2))
    d = np.linalg.norm(x[:, None, :] - y[None, :, :], axis=2)
    return -np.log(d)


def test_svd_truncation_eckart_young():
    B = _kernel_block(60, 45, 0)
    s = np.linalg.svd(B, compute_uv=False)
    for eps in (1e-2, 1e-5, 1e-9):
        lr = hodlr.svd_compress(B, eps)
        r = lr.rank
        err = np.linalg.norm(B - lr.U @ lr.V.T, 2)
        assert s[r - 1] >= eps * s[0] > (s[r] if r < s.shape[0] else 0)
        assert err == pytest.approx(s[r] if r < s.shape[0] else 0.0, rel=1e-8, abs=1e-14 * s[0])


def test_complete_pivot_lu_reconstructs_pivot_block():
    rng = np.random.default_rng(1)
    Bh = rng.standard_normal((12, 9))
    rows, cols, Lr, Ur = hodlr.complete_pivot_lu(Bh, 0.0)
    assert rows.shape[0] == 9
    assert np.allclose(np.diag(Lr), 1) and np.allclose(Lr, np.tril(Lr)) and np.allclose(Ur, np.triu(Ur))
    assert np.abs(Bh[np.ix_(rows, cols)] - Lr @ Ur).max() < 1e-12
    # complete pivoting: multipliers bounded by 1 (up to the tie tolerance)
    assert np.abs(Lr).max() <= 1 / (1 - hodlr.TIE_REL) + 1e-12
    # first pivot is the largest entry
    assert abs(Ur[0, 0]) == np.abs(Bh).max()


def test_skeleton_full_sets_max_norm_bound():
    """With all rows and columns, the LU residual is the Schur complement of
    the pivot block, whose entries are below the next (rejected) pivot."""
    for seed in range(3):
        B = _kernel_block(50, 70, seed, gap=0.5)
        I, J = np.arange(50), np.arange(70)
        for eps in (1e-2, 1e-4, 1e-7):
            lr = hodlr.skeleton(B, I, J, eps)
            E = B - lr.U @ lr.V.T
            assert np.abs(E).max() < eps * np.abs(B).max() / (1 - hodlr.TIE_REL)
            # the skeleton is exact on the pivot rows and columns
            assert np.abs(E[lr.piv_rows]).max() < 1e-10 * np.abs(B).max()
            assert np.abs(E[:, lr.piv_cols]).max() < 1e-10 * np.abs(B).max()


def test_skeleton_adaptive_recovers_from_poor_sets():
    B = _kernel_block(40, 40, 4, gap=0.3)
    I, J = np.array([0]), np.array([39])
    lr0 = hodlr.skeleton(B, I, J, 1e-6, adaptive=False)
    assert lr0.rank == 1
    lr = hodlr.skeleton(B, I, J, 1e-6, adaptive=True)
    E = B - lr.U @ lr.V.T
    assert np.abs(E).max() < 1e-6 * np.abs(B).max() / (1 - hodlr.TIE_REL)
    assert lr.rank > 1


def test_skeleton_eps0_exact():
    rng = np.random.default_rng(2)
    B = rng.standard_normal((20, 13))
    lr = hodlr.skeleton(B, np.arange(20), np.arange(13), 0.0)
    assert lr.rank == 13
    assert np.abs(B - lr.U @ lr.V.T).max() < 1e-12 * np.abs(B).max()


def _random_hodlr_dense(n, leaf, rank, seed):
    """Dense symmetric matrix whose off-diagonal blocks on the bisection
    cluster tree have exact rank ``rank``; diagonally dominant (SPD)."""
    rng = np.random.default_rng(seed)
    K = np.zeros((n, n))
    blocks = []
    tree = _bisect_tree(0, n, leaf, "pp", blocks)
    for b in blocks:
        U = rng.standard_normal((b.nr, rank))
        V = rng.standard_normal((b.nc, rank))
        K[b.r0:b.r0 + b.nr, b.c0:b.c0 + b.nc] = U @ V.T
    K = K + K.T
    K += np.diag(np.abs(K).sum(axis=1) + 1.0)
    for t in tree:
        if t.left < 0:
            D = rng.standard_normal((t.size, t.size)) * 0.1
            K[t.off:t.off + t.size, t.off:t.off + t.size] += D @ D.T
    return K, tree


@pytest.mark.parametrize("n,leaf,rank", [(64, 8, 3), (100, 12, 5), (37, 5, 2)])
def test_smw_solve_equals_dense(n, leaf, rank):
    K, tree = _random_hodlr_dense(n, leaf, rank, n)
    # eps well above rounding but far below the exact rank's singular values
    eps = 1e-11
    for comp in (lambda B, t: hodlr.svd_compress(B, eps),
                 lambda B, t: hodlr.skeleton(B, np.arange(B.shape[0]), np.arange(B.shape[1]), eps)):
        H = hodlr.build(K, tree, comp)
        Kd = hodlr.densify(H)
        assert np.abs(Kd - K).max() < 1e-9 * np.abs(K).max()
        x = np.random.default_rng(0).standard_normal((n, 3))
        assert np.abs(hodlr.matvec(H, x) - K @ x).max() < 1e-9 * np.abs(K @ x).max()
        hodlr.smw_factor(H)
        y = hodlr.smw_solve(H, x)
        yr = np.linalg.solve(K, x)
        assert np.abs(y - yr).max() < 1e-10 * np.abs(yr).max()
        # ranks were found exactly
        assert all(lr.rank == rank for lr in hodlr.blocks(H))


def test_skeleton_cross_meets_bound_on_the_cross():
    """Phase 2 on the sampled cross: every residual entry in the BDLR rows
    and columns meets the pivot-ratio rule, the rank lies between the
    one-phase and the whole-block ones, and the factors are the residual
    columns and rows of the pivots (U V^T reproduces B on them)."""
    B = _kernel_block(90, 70, 7, gap=0.15)
    rng = np.random.default_rng(3)
    I = np.sort(rng.choice(90, 6, replace=False))
    J = np.sort(rng.choice(70, 5, replace=False))
    eps = 1e-7
    lr0 = hodlr.skeleton(B, I, J, eps, adaptive=False)
    lrc = hodlr.skeleton(B, I, J, eps, adaptive="cross")
    lrw = hodlr.skeleton(B, I, J, eps, adaptive=True)
    assert lr0.rank < lrc.rank <= lrw.rank
    E = B - lrc.U @ lrc.V.T
    u11 = np.abs(B[np.ix_(I, J)]).max()
    bound = eps * u11 / (1 - hodlr.TIE_REL) * (1 + 1e-9)
    assert np.abs(E[I, :]).max() < bound and np.abs(E[:, J]).max() < bound
    # the pivots' rows and columns are reproduced (to rounding)
    assert np.abs(E[lrc.piv_rows, :]).max() < 1e-12 * np.abs(B).max()
    assert np.abs(E[:, lrc.piv_cols]).max() < 1e-12 * np.abs(B).max()
    # outside the cross the error is not bounded by the rule (it is what the
    # cross does not see), but it is no larger than the one-phase error
    assert np.abs(E).max() <= np.abs(B - lr0.U @ lr0.V.T).max() * (1 + 1e-9)


def test_skeleton_cross_with_full_sets_is_whole_block():
    B = _kernel_block(40, 33, 11, gap=0.3)
    I = np.arange(40)[::3]
    J = np.arange(33)
    lrc = hodlr.skeleton(B, np.arange(40), J, 1e-9, adaptive="cross")
    lrw = hodlr.skeleton(B, np.arange(40), J, 1e-9, adaptive=True)
    assert lrc.rank == lrw.rank
    assert np.array_equal(lrc.piv_rows, lrw.piv_rows) and np.array_equal(lrc.piv_cols, lrw.piv_cols)
    assert np.abs(lrc.U @ lrc.V.T - lrw.U @ lrw.V.T).max() == 0.0
    # all columns sampled: the cross is the whole block even with few rows
    lrc2 = hodlr.skeleton(B, I, J, 1e-9, adaptive="cross")
    lrw2 = hodlr.skeleton(B, I, J, 1e-9, adaptive=True)
    assert lrc2.rank == lrw2.rank and np.array_equal(lrc2.piv_cols, lrw2.piv_cols)
