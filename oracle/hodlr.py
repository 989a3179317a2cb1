"""Oracle: HODLR matrices, low-rank compression and the recursive
Sherman-Morrison-Woodbury (SMW) factor/solve (test infrastructure only;
float64).

HODLR structure (Sec. 2.1, Eq. HODLR2): a symmetric matrix K on a binary
cluster tree; for an internal node with children (alpha, beta) the lower
off-diagonal block K(beta, alpha) is stored as U V^T (U: |beta| x r,
V: |alpha| x r) and the upper one is its transpose; leaves are dense.
Eq. HODLR2 as printed has two index typos (a transposed U_3 and a level-1
V_{4,3}); the structure meant is the regular one used here.

Compression (Sec. 2.2):
* ``skeleton``: the BDLR pseudo-skeleton.  B_hat = B(I, J) is factored by LU
  with complete pivoting, P B_hat Q = L U (Eq. Bhat), stopped at the first
  pivot with |u_{r+1,r+1} / u_11| < eps.  Then C~ = (B Q)(:, 1:r) U_r^{-1}
  and R~ = L_r^{-1} (P B)(1:r, :), and B ~= C~ R~; we store U = C~, V = R~^T.
  (The paper calls the U_r solve lower-triangular; U_r is upper-triangular.)
  Pivot choice: the entry of largest magnitude, with magnitudes compared
  after truncation to 20 mantissa bits (the float64 bit pattern of |v| with
  its low 32 bits cleared); entries equal after truncation are tied and the
  lowest column, then the lowest row (block positions) wins.  The chosen
  pivot is within a factor (1 - 2^-20) of the largest entry, and the choice
  is reproducible across implementations whose rounding differs.
* ``svd``: truncated SVD, rank r = number of singular values >= eps * s_1
  (so ||B - U V^T||_2 = s_{r+1} < eps s_1).

SMW factorisation of a HODLR node tau with children (alpha, beta):
  K_tau = D + Ubar C Ubar^T,  D = blockdiag(K_alpha, K_beta),
  Ubar = blockdiag(V, U),     C = [[0, I], [I, 0]]  (C^{-1} = C),
  K_tau^{-1} = D^{-1} - D^{-1} Ubar (C + Ubar^T D^{-1} Ubar)^{-1} Ubar^T D^{-1}.
So a node keeps Y_alpha = K_alpha^{-1} V, Y_beta = K_beta^{-1} U and the LU
of the 2r x 2r capacitance [[V^T Y_alpha, I], [I, U^T Y_beta]]; leaves keep a
Cholesky factor.  The factor is computed recursively straight from this
definition.

Pins (tests/test_oracle_hodlr.py): SVD truncation meets the Eckart-Young
bound exactly; skeleton with all rows/columns meets the max-norm bound
max|B - UV^T| <= eps max|B| / (1 - 2^-20) (the LU residual is the Schur
complement of the pivot block); skeleton at eps = 0 reproduces B; SMW solve
of random symmetric HODLR matrices equals a dense solve; densify/matvec
agree.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla

TIE_REL = 2.0 ** -20
# Pivots below 64 unit roundoffs (float64) of |u_11| are rounding noise: the
# pivot-ratio rule uses max(eps, NOISE_REL), so eps = 0 means "no truncation
# beyond the numerical rank" instead of pivoting on noise.
NOISE_REL = 64 * 2.0 ** -53


def _stop(piv: float, eps: float, u11: float) -> bool:
    return abs(piv) < max(eps, NOISE_REL) * u11


def _pick_pivot(W: np.ndarray, live_r: np.ndarray, live_c: np.ndarray, mask: np.ndarray = None):
    """(row, col) of the complete-pivoting choice among live entries (and
    within ``mask`` when given), or None when every such entry is zero."""
    q = np.abs(W).view(np.int64) & ~np.int64(0xFFFFFFFF)   # |v| truncated to 20 mantissa bits
    ok = live_r[:, None] & live_c[None, :]
    if mask is not None:
        ok = ok & mask
    q = np.where(ok, q, -1)
    qmax = q.max() if q.size else -1
    if qmax <= 0:
        return None
    cand = np.argwhere(q == qmax)
    k = np.lexsort((cand[:, 0], cand[:, 1]))[0]               # lowest column, then row
    return int(cand[k, 0]), int(cand[k, 1])


@dataclasses.dataclass
class LowRank:
    U: np.ndarray
    V: np.ndarray
    rank: int
    piv_rows: np.ndarray = None   # block-local pivot rows (skeleton only), pivot order
    piv_cols: np.ndarray = None


def complete_pivot_lu(Bh: np.ndarray, eps: float):
    """Truncated LU with complete pivoting of B_hat (Eq. Bhat).  Returns
    (rows, cols, Lr, Ur): pivot rows/cols of B_hat in pivot order, the unit
    lower r x r factor and the upper r x r factor, so that
    B_hat[rows][:, cols] = Lr @ Ur."""
    W = np.array(Bh, dtype=np.float64, copy=True)
    m, n = W.shape
    live_r = np.ones(m, dtype=bool)
    live_c = np.ones(n, dtype=bool)
    rows, cols, lcols, urows = [], [], [], []
    u11 = None
    for _ in range(min(m, n)):
        pick = _pick_pivot(W, live_r, live_c)
        if pick is None:
            break
        i, j = pick
        piv = W[i, j]
        if u11 is None:
            u11 = abs(piv)
        if _stop(piv, eps, u11):
            break
        l = W[:, j] / piv
        u = W[i, :].copy()
        l[~live_r] = 0.0
        l[i] = 1.0
        W -= np.outer(l, u)
        W[i, :] = 0.0
        W[:, j] = 0.0
        live_r[i] = False
        live_c[j] = False
        rows.append(i)
        cols.append(j)
        lcols.append(l)
        urows.append(u)
    r = len(rows)
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    Lr = np.zeros((r, r))
    Ur = np.zeros((r, r))
    for b in range(r):
        Lr[:, b] = lcols[b][rows]
        Ur[b, :] = urows[b][cols]
    Lr = np.tril(Lr)
    Ur = np.triu(Ur)
    return rows, cols, Lr, Ur


def skeleton(B: np.ndarray, I: np.ndarray, J: np.ndarray, eps: float,
             adaptive=True) -> LowRank:
    """BDLR pseudo-skeleton of block B from row set I and column set J
    (block-local indices), Eq. Bhat.

    Phase 1 is the paper's: complete-pivot LU of B_hat = B(I, J) stopped by
    the pivot ratio, then C~ = B(:, J_r) U_r^{-1}, R~ = L_r^{-1} B(I_r, :).

    Phase 2 (``adaptive``) makes the pivot-ratio rule hold over the whole
    block: the residual E = B - C~ R~ is exactly the Schur complement left by
    the phase-1 pivots, so complete pivoting simply continues on E (largest
    remaining entry of the full block, same tie rule) until the next pivot
    satisfies |u_{k+1,k+1}| < eps |u_11|; each extra pivot (i, j) appends
    column E(:, j) to C~ and row E(i, :) / E(i, j) to R~.  At exit
    max|B - C~ R~| < eps |u_11| / (1 - 2^-20) <= eps max|B| / (1 - 2^-20).
    u_11 is the first pivot taken (from B_hat, or from B when phase 1 takes
    none).

    ``adaptive="cross"`` runs phase 2 on the sampled cross only: the pivot
    is the largest live residual entry in the BDLR rows I or columns J
    (E(I, :) and E(:, J), the entries a front that is never assembled
    forms), and the stopping rule holds there; each pivot still appends the
    whole residual column and row, so a sampled front fetches one row and
    one column of B per extra pivot.  With I and J covering the block this
    is the whole-block phase 2."""
    m, n = B.shape
    Ct = np.zeros((m, 0))
    Rt = np.zeros((0, n))
    Ir = np.zeros(0, np.int64)
    Jr = np.zeros(0, np.int64)
    u11 = None
    if I.shape[0] > 0 and J.shape[0] > 0:
        Bh = B[np.ix_(I, J)]
        pr, pc, Lr, Ur = complete_pivot_lu(Bh, eps)
        if pr.shape[0] > 0:
            u11 = abs(Ur[0, 0])
            Ir = I[pr]
            Jr = J[pc]
            # C~ = B(:, J_r) U_r^{-1}
            Ct = sla.solve_triangular(Ur, B[:, Jr].T, trans="T", lower=False).T
            # R~ = L_r^{-1} B(I_r, :)
            Rt = sla.solve_triangular(Lr, B[Ir, :], lower=True, unit_diagonal=True)
    if adaptive and m > 0 and n > 0:
        E = B - Ct @ Rt
        live_r = np.ones(m, dtype=bool)
        live_c = np.ones(n, dtype=bool)
        live_r[Ir] = False
        live_c[Jr] = False
        mask = None
        if adaptive == "cross":
            in_i = np.zeros(m, dtype=bool)
            in_j = np.zeros(n, dtype=bool)
            in_i[I] = True
            in_j[J] = True
            mask = in_i[:, None] | in_j[None, :]
        cols_add, rows_add, ir_add, jc_add = [], [], [], []
        while live_r.any() and live_c.any():
            pick = _pick_pivot(E, live_r, live_c, mask)
            if pick is None:
                break
            i, j = pick
            piv = E[i, j]
            if u11 is None:
                u11 = abs(piv)
            if _stop(piv, eps, u11):
                break
            c = E[:, j].copy()
            r = E[i, :] / piv
            E -= np.outer(c, r)
            live_r[i] = False
            live_c[j] = False
            cols_add.append(c)
            rows_add.append(r)
            ir_add.append(i)
            jc_add.append(j)
        if cols_add:
            Ct = np.concatenate([Ct, np.stack(cols_add, axis=1)], axis=1)
            Rt = np.concatenate([Rt, np.stack(rows_add, axis=0)], axis=0)
            Ir = np.concatenate([Ir, np.asarray(ir_add, np.int64)])
            Jr = np.concatenate([Jr, np.asarray(jc_add, np.int64)])
    return LowRank(Ct, Rt.T.copy(), Ct.shape[1], Ir, Jr)


def svd_compress(B: np.ndarray, eps: float) -> LowRank:
    m, n = B.shape
    if m == 0 or n == 0:
        return LowRank(np.zeros((m, 0)), np.zeros((n, 0)), 0)
    U, s, Vt = np.linalg.svd(B, full_matrices=False)
    if s.shape[0] == 0 or s[0] == 0.0:
        return LowRank(np.zeros((m, 0)), np.zeros((n, 0)), 0)
    r = int(np.sum(s >= eps * s[0])) if eps > 0 else int(np.sum(s > 0))
    return LowRank(U[:, :r] * s[:r], Vt[:r].T.copy(), r)


@dataclasses.dataclass
class HNode:
    off: int
    size: int
    left: "HNode" = None
    right: "HNode" = None
    D: np.ndarray = None       # dense leaf block
    lr: LowRank = None         # lower off-diagonal block K(beta, alpha) = U V^T
    # factorisation
    chol: tuple = None
    Ya: np.ndarray = None
    Yb: np.ndarray = None
    cap_lu: tuple = None

    @property
    def is_leaf(self) -> bool:
        return self.left is None


def build(F: np.ndarray, tree: list, compress, base: int = None) -> HNode:
    """HODLR of the dense symmetric matrix F over a cluster tree (TreeNode
    list over positions; ``base`` is the position of F[0, 0]).  ``compress``
    maps (block B, tree node) to a LowRank."""
    base = tree[0].off if base is None else base

    def rec(i: int) -> HNode:
        t = tree[i]
        h = HNode(t.off - base, t.size)
        if t.left < 0:
            o = t.off - base
            h.D = F[o:o + t.size, o:o + t.size].copy()
            return h
        h.left = rec(t.left)
        h.right = rec(t.right)
        a, b = tree[t.left], tree[t.right]
        B = F[b.off - base:b.off - base + b.size, a.off - base:a.off - base + a.size]
        h.lr = compress(B, t)
        return h

    return rec(0)


def densify(h: HNode) -> np.ndarray:
    if h.is_leaf:
        return h.D.copy()
    A = densify(h.left)
    Bd = densify(h.right)
    na = A.shape[0]
    K = np.zeros((h.size, h.size))
    K[:na, :na] = A
    K[na:, na:] = Bd
    low = h.lr.U @ h.lr.V.T
    K[na:, :na] = low
    K[:na, na:] = low.T
    return K


def matvec(h: HNode, x: np.ndarray) -> np.ndarray:
    if h.is_leaf:
        return h.D @ x
    na = h.left.size
    ya = matvec(h.left, x[:na]) + h.lr.V @ (h.lr.U.T @ x[na:])
    yb = matvec(h.right, x[na:]) + h.lr.U @ (h.lr.V.T @ x[:na])
    return np.concatenate([ya, yb], axis=0)


def smw_factor(h: HNode) -> None:
    if h.is_leaf:
        h.chol = sla.cho_factor(h.D, lower=True)
        return
    smw_factor(h.left)
    smw_factor(h.right)
    U, V = h.lr.U, h.lr.V
    r = h.lr.rank
    if r == 0:
        return
    h.Ya = smw_solve(h.left, V)         # K_alpha^{-1} V
    h.Yb = smw_solve(h.right, U)        # K_beta^{-1} U
    I = np.eye(r)
    cap = np.block([[V.T @ h.Ya, I], [I, U.T @ h.Yb]])
    h.cap_lu = sla.lu_factor(cap)


def smw_solve(h: HNode, b: np.ndarray) -> np.ndarray:
    """x = K^{-1} b using the SMW factorisation."""
    if h.is_leaf:
        return sla.cho_solve(h.chol, b)
    na = h.left.size
    ya = smw_solve(h.left, b[:na])
    yb = smw_solve(h.right, b[na:])
    r = h.lr.rank
    if r == 0:
        return np.concatenate([ya, yb], axis=0)
    q = np.concatenate([h.lr.V.T @ ya, h.lr.U.T @ yb], axis=0)   # Ubar^T D^{-1} b
    q = sla.lu_solve(h.cap_lu, q)
    return np.concatenate([ya - h.Ya @ q[:r], yb - h.Yb @ q[r:]], axis=0)


def blocks(h: HNode) -> list:
    """Low-rank blocks in level order (root first, left to right)."""
    out, q = [], [h]
    while q:
        nxt = []
        for x in q:
            if not x.is_leaf:
                out.append(x.lr)
                nxt += [x.left, x.right]
        q = nxt
    return out

