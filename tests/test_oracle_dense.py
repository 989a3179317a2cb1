"""Pins of the oracle's conventional multifrontal factor/solve (Sec. 4.1)."""
import numpy as np
import pytest

from mfinputs import q1_grid, p1_kuhn_cube, q1_elasticity, q1_elasticity_lift, rhs
from mfinputs.fem import q1_dirichlet_lift
from oracle import symbolic, dense_mf


@pytest.mark.parametrize("maker,leaf", [
    (lambda: q1_grid(12, 2), 8),
    (lambda: q1_grid(6, 3), 16),
    (lambda: q1_grid(5, 3, k_elem=np.exp(np.random.default_rng(0).standard_normal((6, 6, 6)))), 10),
    (lambda: p1_kuhn_cube(5, 0.2, 1), 12),
    (lambda: q1_elasticity(4), 24),                    # 3 unknowns per node
])
def test_factor_is_the_cholesky_factor(maker, leaf):
    """The Cholesky factor of an SPD matrix is unique, so the multifrontal L
    must equal LAPACK's chol(P A P^T) entry by entry."""
    p = maker()
    sym = symbolic.analyze(p.A, p.coords, leaf)
    fac = dense_mf.factor(sym, p.A.vals)
    D = p.A.to_dense()
    L = np.linalg.cholesky(D[np.ix_(sym.perm, sym.perm)])
    Lm = dense_mf.global_L(fac)
    assert np.abs(L - Lm).max() <= 1e-12 * np.abs(L).max()
    b = rhs(p.A.n, 3, "normal", 1)
    x = dense_mf.solve(fac, b)
    xr = np.linalg.solve(D, b)
    assert np.abs(x - xr).max() <= 1e-11 * np.abs(xr).max()


def test_dst_spectral_solve_2d():
    """Constant-coefficient Q1 Poisson on the square is diagonalised by the
    DST-I basis; compare with the multifrontal solve."""
    n = 15
    h = 1.0 / (n + 1)
    p = q1_grid(n, 2)
    sym = symbolic.analyze(p.A, p.coords, 16)
    fac = dense_mf.factor(sym, p.A.vals)
    b = rhs(p.A.n, 1, "uniform", 0)[:, 0]
    k = np.arange(1, n + 1)
    S = np.sqrt(2 * h) * np.sin(np.outer(k, k) * np.pi * h)      # orthogonal, symmetric
    lam = (2.0 / h) * (1 - np.cos(k * np.pi * h))
    mu = (h / 3.0) * (2 + np.cos(k * np.pi * h))
    E = lam[:, None] * mu[None, :] + mu[:, None] * lam[None, :]   # E[kx, ky]
    Bg = b.reshape(n, n).T                                        # Bg[x, y]
    Xg = S @ ((S @ Bg @ S) / E) @ S
    x_ref = Xg.T.ravel()
    x = dense_mf.solve(fac, b)
    assert np.abs(x - x_ref).max() <= 1e-11 * np.abs(x_ref).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_multilinear_boundary_data_reproduced(dim):
    g = (lambda X: 1 + 2 * X[:, 0] - 3 * X[:, 1] + 0.5 * X[:, 0] * X[:, 1]) if dim == 2 else \
        (lambda X: 1 + X[:, 0] - 2 * X[:, 1] + 3 * X[:, 2] + X[:, 0] * X[:, 1] * X[:, 2])
    n = 9 if dim == 2 else 6
    p = q1_grid(n, dim)
    b, gI = q1_dirichlet_lift(n, dim, g)
    sym = symbolic.analyze(p.A, p.coords, 8)
    x = dense_mf.solve(dense_mf.factor(sym, p.A.vals), b)
    assert np.abs(x - gI).max() < 1e-12


def test_elasticity_patch_test_through_the_multifrontal_solve():
    """The constant-strain patch test of the vector problem, solved by the
    oracle's multifrontal factorisation (3 unknowns per node, the nested
    dissection sees repeated node coordinates)."""
    G = np.array([[0.2, 0.1, -0.3], [0.0, -0.1, 0.05], [0.4, 0.2, 0.1]])
    p = q1_elasticity(6)
    b, u = q1_elasticity_lift(6, G)
    sym = symbolic.analyze(p.A, p.coords, 48)
    x = dense_mf.solve(dense_mf.factor(sym, p.A.vals), b)
    assert np.abs(x - u).max() <= 1e-12 * np.abs(u).max()
