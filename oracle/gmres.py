"""Oracle: right-preconditioned flexible GMRES(m) (test infrastructure only;
float64).

The paper runs GMRES with the low-accuracy multifrontal factor as
preconditioner (Sec. 3, Sec. 6) but does not state the variant.  Reading
used: right preconditioning, x0 = 0, modified Gram-Schmidt Arnoldi, Givens
rotations, flexible form (the preconditioned vectors Z are stored, since a
reduced-precision preconditioner is not an exactly fixed operator), restart
m = 30, stop when the true residual ||b - A x||_2 <= tol ||b||_2 (checked
whenever the Arnoldi estimate says so, and at every restart), at most
``maxit`` total iterations.

Pins (tests/test_oracle_gmres.py): with an exact preconditioner one
iteration suffices; without preconditioning the result matches a LAPACK
solve; the Arnoldi residual estimate is non-increasing within a cycle; the
final true residual meets tol.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class GmresInfo:
    iters: int
    relres: float
    converged: bool
    history: list


def fgmres(matvec, precond, b: np.ndarray, tol: float = 1e-10, m: int = 30,
           maxit: int = 4000) -> tuple:
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    x = np.zeros(n)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, GmresInfo(0, 0.0, True, [])
    r = b.copy()
    beta = np.linalg.norm(r)
    iters = 0
    hist = []
    while True:
        if beta <= tol * bnorm:
            return x, GmresInfo(iters, beta / bnorm, True, hist)
        if iters >= maxit:
            return x, GmresInfo(iters, beta / bnorm, False, hist)
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            Z[j] = precond(V[j])
            w = matvec(Z[j])
            iters += 1
            for i in range(j + 1):                 # modified Gram-Schmidt
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):                     # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= tol * bnorm or iters >= maxit or H[j, j] == 0:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):             # back substitution
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + Z[:k].T @ y
        r = b - matvec(x)
        beta = np.linalg.norm(r)


def solve_multi(matvec, precond, B: np.ndarray, tol: float = 1e-10, m: int = 30, maxit: int = 4000):
    """Column-by-column FGMRES for a block of right-hand sides."""
    X = np.zeros_like(B)
    infos = []
    for k in range(B.shape[1]):
        X[:, k], info = fgmres(matvec, precond, B[:, k], tol, m, maxit)
        infos.append(info)
    return X, infos
