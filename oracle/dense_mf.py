"""Oracle: conventional multifrontal Cholesky and solve (test infrastructure
only; float64).

Follows Sec. 4.1 of the paper:

* F_bar_p: the entries of A on (I_p u I_p^f) x (I_p u I_p^f) with the
  I_p^f x I_p^f block set to zero (Eq. fbar).
* F_p = F_bar_p (+) U_c1 (+) ... : extend-add of the children's update
  matrices through their relative maps.
* F_p is split into [F_pp F_pf; F_fp F_ff]; F_pp is factored (Cholesky) and
  the update matrix U_p = F_ff - F_fp F_pp^{-1} F_pf is passed to the parent
  (Eq. update).
* Solve: upward pass b_f <- b_f - F_fp F_pp^{-1} b_p (Eq. upward) from the
  leaves to the root, then downward pass x_p = F_pp^{-1} (b_p - F_pf x_f)
  (Eq. downward) from the root to the leaves.

Pins (tests/test_oracle_dense.py): the global factor assembled from
L_pp = chol(F_pp) and L_fp = F_fp L_pp^{-T} equals the unique Cholesky factor
of P A P^T; the solve equals a LAPACK solve; constant-coefficient Poisson
equals a spectral (DST-I) solve; linear boundary data is reproduced nodally.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla

from .symbolic import Symbolic


def front_bar(sym: Symbolic, vals: np.ndarray, p: int) -> np.ndarray:
    """Dense F_bar_p (Eq. fbar): A's entries on the front, ff block zero."""
    f = sym.fronts[p]
    F = np.zeros((f.n, f.n))
    sel = np.flatnonzero(sym.asm_front == p)
    r = sym.asm_row[sel]
    c = sym.asm_col[sel]
    v = vals[sym.asm_src[sel]]
    F[r, c] = v
    F[c, r] = v
    return F


def extend_add(F: np.ndarray, U: np.ndarray, relmap: np.ndarray) -> None:
    """F <- F (+) U : add the child's update matrix at the positions given by
    its relative map."""
    F[np.ix_(relmap, relmap)] += U


@dataclasses.dataclass
class DenseFactor:
    sym: Symbolic
    chol: list       # cho_factor of F_pp per front
    Fpp_L: list      # lower Cholesky factor of F_pp
    Ffp: list        # F_fp per front (n_f x n_p)


def factor(sym: Symbolic, vals: np.ndarray) -> DenseFactor:
    upd = [None] * sym.nfronts
    chol, Ls, Ffp = [], [], []
    for p, f in enumerate(sym.fronts):
        F = front_bar(sym, vals, p)
        for c in f.children:
            extend_add(F, upd[c], sym.fronts[c].relmap)
            upd[c] = None
        npv = f.npiv
        Fpp = F[:npv, :npv]
        Fpf = F[:npv, npv:]
        Ffp_p = F[npv:, :npv]
        cf = sla.cho_factor(Fpp, lower=True)
        chol.append(cf)
        Ls.append(np.tril(cf[0]))
        Ffp.append(Ffp_p.copy())
        if f.nf > 0:
            # U_p = F_ff - F_fp F_pp^{-1} F_pf   (Eq. update)
            upd[p] = F[npv:, npv:] - Ffp_p @ sla.cho_solve(cf, Fpf)
    return DenseFactor(sym, chol, Ls, Ffp)


def global_L(fac: DenseFactor) -> np.ndarray:
    """Assemble the global Cholesky factor of P A P^T from the fronts:
    column block I_p holds L_pp on I_p and L_fp = F_fp L_pp^{-T} on I_p^f."""
    sym = fac.sym
    L = np.zeros((sym.n, sym.n))
    for p, f in enumerate(sym.fronts):
        s, m = f.start, f.npiv
        L[s:s + m, s:s + m] = fac.Fpp_L[p]
        if f.nf > 0:
            Lfp = sla.solve_triangular(fac.Fpp_L[p], fac.Ffp[p].T, lower=True).T
            L[np.ix_(f.upd, np.arange(s, s + m))] = Lfp
    return L


def solve(fac: DenseFactor, b: np.ndarray) -> np.ndarray:
    """Upward then downward pass (Eq. upward, Eq. downward).  ``b`` in the
    original ordering, shape (n,) or (n, k)."""
    sym = fac.sym
    squeeze = b.ndim == 1
    B = b.reshape(sym.n, -1)
    bn = B[sym.perm]                  # new ordering
    bu = [None] * sym.nfronts         # upward-pass front vectors
    contrib = [None] * sym.nfronts
    for p, f in enumerate(sym.fronts):
        t = np.zeros((f.n, B.shape[1]))
        t[:f.npiv] = bn[f.start:f.start + f.npiv]
        for c in f.children:
            t[sym.fronts[c].relmap] += contrib[c]
            contrib[c] = None
        # b_f <- b_f - F_fp F_pp^{-1} b_p
        if f.nf > 0:
            contrib[p] = t[f.npiv:] - fac.Ffp[p] @ sla.cho_solve(fac.chol[p], t[:f.npiv])
        bu[p] = t[:f.npiv]
    xn = np.zeros_like(bn)
    for p in range(sym.nfronts - 1, -1, -1):
        f = sym.fronts[p]
        rhs = bu[p]
        if f.nf > 0:
            rhs = rhs - fac.Ffp[p].T @ xn[f.upd]          # F_pf = F_fp^T
        xn[f.start:f.start + f.npiv] = sla.cho_solve(fac.chol[p], rhs)
    x = np.empty_like(xn)
    x[sym.perm] = xn
    return x[:, 0] if squeeze else x
