"""Oracle: HODLR-accelerated multifrontal factorisation and solve (test
infrastructure only; float64).

Follows Sec. 4.2 of the paper:

* The front F_p = F_bar_p (+) U_c1^HODLR (+) ... is formed from A's entries
  and the children's *compressed* updates U_c = F_ff,c^HODLR - W_c V_c^T
  (Eq. update_HODLR, Eq. HODLR_EA_Expand).  The oracle forms it densely: the
  method's fast extend-add only extracts the BDLR rows/columns and dense
  leaves of that same matrix, so the values the compression sees are the
  same.
* F_p^HODLR: the top split is [I_p | I_p^f]; F_fp ~= W V^T; F_pp and F_ff are
  HODLR on their cluster trees (Eq. frontalMatrix_HODLR, whose figure is
  missing from the source; reconstructed from the text).
* F_pp^HODLR is factored by the recursive SMW solver (the paper defers to a
  HODLR solver; see oracle.hodlr).
* U_p^HODLR = F_ff^HODLR - W S W^T with S = V^T (F_pp^HODLR)^{-1} V
  (Eq. update_HODLR_Parent; the printed equation has F_ff^{-1} and
  W_cp/V_cp where F_pp^{-1} and the F_fp/F_pf factors are meant).
* Fronts with n_p + n_f < n_c are factored densely (Sec. 4.2: small dense
  updates enter the parent's extend-add as they are).
* Solve (Sec. 4.2.2): the conventional upward/downward passes with F_pp^{-1}
  replaced by the HODLR solve and F_fp, F_pf applied as W V^T, V W^T.

Pins (tests/test_oracle_hodlr_mf.py): eps = 0 with all rows/columns
reproduces the dense multifrontal solve to 1e-12; every update matrix is
symmetric; every truncated block meets its error bound; as a preconditioner
inside GMRES the final x matches the dense solve.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla

from . import hodlr
from .dense_mf import front_bar, extend_add
from .symbolic import Symbolic, bdlr_sets


@dataclasses.dataclass
class Options:
    eps: float = 1e-4
    depth: int = -1        # BDLR depth d; < 0: all rows/columns
    cap: int = 192         # BDLR set size cap
    n_c: int = 0           # fronts with n_p + n_f < n_c stay dense
    compress: str = "skeleton"   # "skeleton" (BDLR, Sec. 2.2) or "svd"
    adaptive: object = True  # phase 2: True whole block, "cross" the sampled rows and columns, False none
    record_errors: bool = False


@dataclasses.dataclass
class FrontFactor:
    dense: bool
    chol: tuple = None            # dense: cho_factor(F_pp)
    Ffp: np.ndarray = None        # dense: F_fp
    Hpp: hodlr.HNode = None       # HODLR: factored F_pp^HODLR
    W: np.ndarray = None          # HODLR: F_fp ~= W V^T
    V: np.ndarray = None
    X: np.ndarray = None          # (F_pp^HODLR)^{-1} V
    ranks: list = None            # block ranks in the front's block order
    errors: list = None           # per block (max-norm rel, 2-norm rel) if recorded


@dataclasses.dataclass
class HodlrFactor:
    sym: Symbolic
    opts: Options
    fronts: list
    updates_symmetric: float      # max relative asymmetry seen over all U_p


def _compressor(sym, front, opts, block_lookup, errors):
    def comp(B, blk_index):
        blk = front.blocks[blk_index]
        if opts.compress == "svd":
            lr = hodlr.svd_compress(B, opts.eps)
        else:
            I, J = bdlr_sets(sym, front, blk, opts.depth, opts.cap)
            lr = hodlr.skeleton(B, I - blk.r0, J - blk.c0, opts.eps, opts.adaptive)
        if errors is not None:
            E = B - lr.U @ lr.V.T
            bmax = np.abs(B).max() if B.size else 0.0
            bn2 = np.linalg.norm(B, 2) if B.size else 0.0
            errors[blk_index] = (
                float(np.abs(E).max() / bmax) if bmax > 0 else 0.0,
                float(np.linalg.norm(E, 2) / bn2) if bn2 > 0 else 0.0,
            )
        return lr
    return comp


def factor(sym: Symbolic, vals: np.ndarray, opts: Options) -> HodlrFactor:
    upd = [None] * sym.nfronts
    out = []
    asym = 0.0
    for p, f in enumerate(sym.fronts):
        F = front_bar(sym, vals, p)
        for c in f.children:
            extend_add(F, upd[c], sym.fronts[c].relmap)
            upd[c] = None
        npv = f.npiv
        if f.n < opts.n_c:
            cf = sla.cho_factor(F[:npv, :npv], lower=True)
            ff = FrontFactor(True, chol=cf, Ffp=F[npv:, :npv].copy())
            if f.nf > 0:
                upd[p] = F[npv:, npv:] - ff.Ffp @ sla.cho_solve(cf, F[:npv, npv:])
            out.append(ff)
        else:
            errors = {} if opts.record_errors else None
            comp = _compressor(sym, f, opts, None, errors)
            ranks = [0] * len(f.blocks)

            def comp_tree(B, t, comp=comp, ranks=ranks):
                lr = comp(B, t.block)
                ranks[t.block] = lr.rank
                return lr

            Hpp = hodlr.build(F, f.pp_tree, comp_tree, base=0)
            hodlr.smw_factor(Hpp)
            ff = FrontFactor(False, Hpp=Hpp, ranks=ranks)
            if f.nf > 0:
                top = comp(F[npv:, :npv], 0)
                ranks[0] = top.rank
                W, V = top.U, top.V
                X = hodlr.smw_solve(Hpp, V) if top.rank > 0 else np.zeros((npv, 0))
                S = V.T @ X
                S = 0.5 * (S + S.T)
                Hff = hodlr.build(F[npv:, npv:], f.ff_tree, comp_tree, base=npv)
                U = hodlr.densify(Hff) - W @ S @ W.T
                nrm = np.abs(U).max()
                if nrm > 0:
                    asym = max(asym, float(np.abs(U - U.T).max() / nrm))
                upd[p] = 0.5 * (U + U.T)
                ff.W, ff.V, ff.X = W, V, X
            ff.errors = [errors.get(i) for i in range(len(f.blocks))] if errors is not None else None
            out.append(ff)
    return HodlrFactor(sym, opts, out, asym)


def _pp_solve(ff: FrontFactor, t: np.ndarray) -> np.ndarray:
    if ff.dense:
        return sla.cho_solve(ff.chol, t)
    return hodlr.smw_solve(ff.Hpp, t)


def solve(fac: HodlrFactor, b: np.ndarray) -> np.ndarray:
    """Apply the HODLR-multifrontal approximate inverse to b (original
    ordering, shape (n,) or (n, k))."""
    sym = fac.sym
    squeeze = b.ndim == 1
    B = b.reshape(sym.n, -1)
    bn = B[sym.perm]
    bu = [None] * sym.nfronts
    contrib = [None] * sym.nfronts
    for p, f in enumerate(sym.fronts):
        ff = fac.fronts[p]
        t = np.zeros((f.n, B.shape[1]))
        t[:f.npiv] = bn[f.start:f.start + f.npiv]
        for c in f.children:
            t[sym.fronts[c].relmap] += contrib[c]
            contrib[c] = None
        if f.nf > 0:
            z = _pp_solve(ff, t[:f.npiv])
            if ff.dense:
                contrib[p] = t[f.npiv:] - ff.Ffp @ z
            else:
                contrib[p] = t[f.npiv:] - ff.W @ (ff.V.T @ z)     # F_fp = W V^T
        bu[p] = t[:f.npiv]
    xn = np.zeros_like(bn)
    for p in range(sym.nfronts - 1, -1, -1):
        f = sym.fronts[p]
        ff = fac.fronts[p]
        rhs = bu[p]
        if f.nf > 0:
            xf = xn[f.upd]
            if ff.dense:
                rhs = rhs - ff.Ffp.T @ xf
            else:
                rhs = rhs - ff.V @ (ff.W.T @ xf)                # F_pf = V W^T
        xn[f.start:f.start + f.npiv] = _pp_solve(ff, rhs)
    x = np.empty_like(xn)
    x[sym.perm] = xn
    return x[:, 0] if squeeze else x
