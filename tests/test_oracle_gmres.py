"""Pins of the oracle's right-preconditioned flexible GMRES (Sec. 3)."""
import numpy as np

from mfinputs import q1_grid, rhs
from oracle import gmres


def _spd(n=60, seed=0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return Q @ np.diag(np.linspace(1, 50, n)) @ Q.T


def test_exact_preconditioner_one_iteration():
    A = _spd()
    b = np.random.default_rng(1).standard_normal(60)
    Ainv = np.linalg.inv(A)
    x, info = gmres.fgmres(lambda v: A @ v, lambda v: Ainv @ v, b, 1e-10)
    assert info.converged and info.iters == 1
    assert np.linalg.norm(A @ x - b) <= 1e-10 * np.linalg.norm(b)


def test_unpreconditioned_matches_lapack_and_monotone():
    p = q1_grid(8, 2)
    A = p.A.to_dense()
    b = rhs(p.A.n, 1, "uniform", 0)[:, 0]
    x, info = gmres.fgmres(lambda v: A @ v, lambda v: v, b, 1e-12, m=30)
    xr = np.linalg.solve(A, b)
    assert info.converged
    assert np.linalg.norm(x - xr) <= 1e-9 * np.linalg.norm(xr)
    h = np.array(info.history[:30])
    assert np.all(np.diff(h) <= 1e-15)      # GMRES residual non-increasing within a cycle


def test_maxit_reports_not_converged():
    A = _spd(80, 3)
    b = np.ones(80)
    x, info = gmres.fgmres(lambda v: A @ v, lambda v: v, b, 1e-14, m=5, maxit=7)
    assert not info.converged and info.iters == 7
