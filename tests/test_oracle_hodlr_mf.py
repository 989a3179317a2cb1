"""Pins of the oracle's HODLR-accelerated multifrontal method (Sec. 4.2)."""
import numpy as np
import pytest

from mfinputs import q1_grid, p1_kuhn_cube, rhs
from oracle import symbolic, dense_mf, hodlr_mf, gmres, hodlr


CASES = [
    (lambda: q1_grid(14, 2), 8),
    (lambda: q1_grid(7, 3), 16),
    (lambda: p1_kuhn_cube(6, 0.2, 2), 16),
]


@pytest.mark.parametrize("maker,leaf", CASES)
@pytest.mark.parametrize("compress", ["skeleton", "svd"])
@pytest.mark.parametrize("n_c", [0, 40])
def test_eps0_reproduces_dense(maker, leaf, compress, n_c):
    p = maker()
    sym = symbolic.analyze(p.A, p.coords, leaf)
    opts = hodlr_mf.Options(eps=0.0, depth=-1, cap=10 ** 6, n_c=n_c, compress=compress)
    hf = hodlr_mf.factor(sym, p.A.vals, opts)
    df = dense_mf.factor(sym, p.A.vals)
    b = rhs(p.A.n, 2, "normal", 3)
    xh = hodlr_mf.solve(hf, b)
    xd = dense_mf.solve(df, b)
    assert np.abs(xh - xd).max() <= 1e-12 * np.abs(xd).max() * 10
    assert hf.updates_symmetric < 1e-12


@pytest.mark.parametrize("maker,leaf", CASES)
@pytest.mark.parametrize("depth", [1, 3, -1])
def test_block_error_bound_and_gmres(maker, leaf, depth):
    p = maker()
    sym = symbolic.analyze(p.A, p.coords, leaf)
    eps = 1e-4
    hf = hodlr_mf.factor(sym, p.A.vals, hodlr_mf.Options(eps=eps, depth=depth, cap=64, record_errors=True))
    errs = [e for ff in hf.fronts if ff.errors for e in ff.errors if e is not None]
    assert errs
    # max-norm contract of the adaptive skeleton, per block
    assert max(e[0] for e in errs) < eps / (1 - hodlr.TIE_REL)
    assert hf.updates_symmetric < 1e-10
    S = p.A.to_scipy()
    b = rhs(p.A.n, 1, "normal", 4)[:, 0]
    x, info = gmres.fgmres(lambda v: S @ v, lambda v: hodlr_mf.solve(hf, v), b, 1e-10)
    assert info.converged and info.iters <= 10
    xr = np.linalg.solve(p.A.to_dense(), b)
    assert np.linalg.norm(x - xr) <= 1e-8 * np.linalg.norm(xr)
    assert np.linalg.norm(b - S @ x) <= 1e-10 * np.linalg.norm(b)


def test_svd_mode_two_norm_bound():
    p = q1_grid(7, 3)
    sym = symbolic.analyze(p.A, p.coords, 16)
    eps = 1e-3
    hf = hodlr_mf.factor(sym, p.A.vals, hodlr_mf.Options(eps=eps, compress="svd", record_errors=True))
    errs = [e for ff in hf.fronts if ff.errors for e in ff.errors if e is not None]
    assert max(e[1] for e in errs) < eps


def test_compression_saves_memory_and_lowers_rank_with_eps():
    p = q1_grid(10, 3)
    sym = symbolic.analyze(p.A, p.coords, 32)
    ranks = []
    for eps in (1e-2, 1e-4, 1e-8):
        hf = hodlr_mf.factor(sym, p.A.vals, hodlr_mf.Options(eps=eps, depth=-1, cap=256))
        ranks.append(sum(sum(ff.ranks) for ff in hf.fronts if ff.ranks))
    assert ranks[0] < ranks[1] < ranks[2]
