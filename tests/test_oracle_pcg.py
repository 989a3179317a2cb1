"""Pins of the oracle's preconditioned CG (oracle/pcg.py) against facts
about conjugate gradients that do not depend on the oracle itself."""
import numpy as np
import scipy.sparse.linalg as spla

from mfinputs import q1_grid, rhs
from oracle import pcg


def _spd(n, eigs, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (Q * np.asarray(eigs)) @ Q.T


def test_exact_preconditioner_one_iteration():
    p = q1_grid(10, 2)
    A = p.A.to_dense()
    b = rhs(p.A.n, 1, "uniform", 0)[:, 0]
    x, info = pcg.pcg(lambda v: A @ v, lambda v: np.linalg.solve(A, v), b, 1e-12)
    assert info.converged and info.iters == 1
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-10 * np.linalg.norm(x)


def test_distinct_eigenvalues_bound_iterations():
    """Without preconditioning CG ends in at most as many iterations as A has
    distinct eigenvalues (in exact arithmetic; well separated values here)."""
    eigs = np.repeat([1.0, 3.0, 10.0], 20)
    A = _spd(60, eigs, 1)
    b = np.random.default_rng(2).standard_normal(60)
    x, info = pcg.pcg(lambda v: A @ v, lambda v: v, b, 1e-10)
    assert info.converged and info.iters <= 3


def test_energy_norm_error_never_grows_and_meets_tol():
    p = q1_grid(12, 2)
    A = p.A.to_scipy()
    b = rhs(p.A.n, 1, "normal", 4)[:, 0]
    xs = np.linalg.solve(p.A.to_dense(), b)
    d = 1.0 / A.diagonal()
    hist = []
    x, info = pcg.pcg(lambda v: A @ v, lambda v: d * v, b, 1e-10, x_hist=hist)
    errs = [float((xk - xs) @ (A @ (xk - xs))) for xk in hist]
    assert all(e1 <= e0 * (1 + 1e-9) for e0, e1 in zip(errs, errs[1:]))
    assert info.converged and np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)
    kappa = np.linalg.cond(p.A.to_dense())
    assert np.linalg.norm(x - xs) <= 2 * kappa * 1e-10 * np.linalg.norm(xs)


def test_unpreconditioned_agrees_with_scipy_cg():
    p = q1_grid(9, 2)
    A = p.A.to_scipy()
    b = rhs(p.A.n, 1, "uniform", 6)[:, 0]
    x, info = pcg.pcg(lambda v: A @ v, lambda v: v, b, 1e-11)
    xr, flag = spla.cg(A, b, rtol=1e-13, maxiter=5000)
    assert flag == 0 and info.converged
    assert np.linalg.norm(x - xr) <= 1e-8 * np.linalg.norm(xr)


def test_maxit_reports_not_converged():
    p = q1_grid(12, 2)
    A = p.A.to_scipy()
    b = rhs(p.A.n, 1, "normal", 8)[:, 0]
    x, info = pcg.pcg(lambda v: A @ v, lambda v: v, b, 1e-12, maxit=3)
    assert not info.converged and info.iters == 3
