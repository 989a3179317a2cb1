"""Oracle: preconditioned conjugate gradients (test infrastructure only;
float64).

The paper notes (Sec. 3) that its low-accuracy multifrontal factor can
precondition any iterative solver, conjugate gradients among them.  A is a
symmetric positive definite stiffness matrix and the multifrontal factor of
a symmetric HODLR approximation is symmetric, so CG applies.  Reading used:
x0 = 0; the flexible (Polak-Ribiere) update
    beta_k = <z_{k+1}, r_{k+1} - r_k> / <z_k, r_k>,
which equals the classical <z_{k+1}, r_{k+1}> / <z_k, r_k> when the
preconditioner is an exactly fixed linear operator (then <z_{k+1}, r_k> = 0)
and keeps the iteration stable when it is applied in reduced precision;
stop when the recursive residual meets tol, then check the true residual
||b - A x||_2 <= tol ||b||_2, and if it does not hold restart from x with the
true residual; at most ``maxit`` iterations.

Pins (tests/test_oracle_pcg.py): one iteration with the exact inverse as
preconditioner; at most k iterations without preconditioning when A has k
distinct eigenvalues (exact arithmetic property of CG); the A-norm of the
error never grows; the result meets tol on the true residual and agrees
with a LAPACK solve; without preconditioning it agrees with SciPy's CG.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class PcgInfo:
    iters: int
    relres: float
    converged: bool
    history: list          # recursive relative residual after each iteration


def pcg(matvec, precond, b: np.ndarray, tol: float = 1e-10, maxit: int = 4000, x_hist: list | None = None):
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros(b.shape[0])
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, PcgInfo(0, 0.0, True, [])
    iters = 0
    hist = []
    r = b.copy()
    while True:
        # (re)start from x with its true residual r
        z = precond(r)
        p = z.copy()
        rz = float(r @ z)
        while np.linalg.norm(r) > tol * bnorm and iters < maxit:
            q = matvec(p)
            alpha = rz / float(p @ q)
            x = x + alpha * p
            r_new = r - alpha * q
            iters += 1
            hist.append(np.linalg.norm(r_new) / bnorm)
            if x_hist is not None:
                x_hist.append(x.copy())
            if np.linalg.norm(r_new) <= tol * bnorm:
                r = r_new
                break
            z_new = precond(r_new)
            beta = float(z_new @ (r_new - r)) / rz
            rz = float(r_new @ z_new)
            p = z_new + beta * p
            r = r_new
        r = b - matvec(x)
        rel = np.linalg.norm(r) / bnorm
        if rel <= tol:
            return x, PcgInfo(iters, rel, True, hist)
        if iters >= maxit:
            return x, PcgInfo(iters, rel, False, hist)


def solve_multi(matvec, precond, B: np.ndarray, tol: float = 1e-10, maxit: int = 4000):
    """Column-by-column PCG for a block of right-hand sides."""
    X = np.zeros_like(B)
    infos = []
    for k in range(B.shape[1]):
        X[:, k], info = pcg(matvec, precond, B[:, k], tol, maxit)
        infos.append(info)
    return X, infos
