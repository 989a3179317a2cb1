"""Oracle symbolic analysis (test infrastructure only).

What it computes, following Sec. 4.1.1 of the paper:

* a nested-dissection elimination order and elimination tree.  The paper
  relies on nested dissection but gives no ordering rule; the reading used
  here is a coordinate-median vertex separator:
    - a node set S with |S| <= leaf is a tree leaf;
    - otherwise choose the axis of largest coordinate extent (ties -> lowest
      axis), sort S by (coordinate, original id), let c be the coordinate of
      element floor(|S|/2); L = {coord < c}, R = {coord >= c};
      Sep = {v in R : v has a graph neighbour in L}; R' = R \\ Sep;
    - if L or Sep is empty, S is a leaf; else recurse on L, then R', and
      number L's subtree, then R''s subtree, then Sep (postorder).
  Inside a leaf or a separator, nodes are numbered in kd order: ascending
  original id when |S| <= leaf, else split at floor(|S|/2) of the
  (coordinate, id) order along the largest-extent axis and concatenate.
* per tree node p (a front): the pivot set I_p (a contiguous range of new
  indices), the coupling set S_p (Eq. couplingSet: higher-numbered unknowns
  structurally coupled to I_p), and the frontal index set
  I_p^f = (S_p U union of children's update sets) \\ I_p.  The front's index
  list is I_p followed by I_p^f in ascending new index.
* the relative (extend-add) map of every child's update set into its parent's
  front, and the map of each lower-triangle entry of P A P^T to (front, row
  position, column position).
* per front: the HODLR cluster trees (top split [I_p | I_p^f]; each part
  bisected at floor(m/2) until it has at most ``leaf`` indices) and their
  off-diagonal blocks.
* BDLR row/column sets of each off-diagonal block (Sec. 2.2, Sec. 4.2.1): in
  the graph of A restricted to the front's whole index set, rows of the block
  within graph distance <= d of the block's column cluster and vice versa.  At most
  ``cap`` indices are kept, closest first (ties -> lower position).
  ``d < 0`` means every index (unreachable ones last).

Everything here is integer work and must agree bit for bit with the C++
analysis of the library.

Pins (tests/test_oracle_symbolic.py): perm is a permutation; I_p contiguous;
parents numbered after children; fill of chol(P A P^T) lies inside the front
blocks (dense Cholesky on tiny grids); each lower entry mapped exactly once;
structured closed forms of the root separator and front counts.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class Block:
    """Lower off-diagonal block of a front: rows [r0, r0+nr), cols [c0, c0+nc)
    in front positions.  ``kind`` is 'top' (F_fp), 'pp' or 'ff'."""
    kind: str
    r0: int
    nr: int
    c0: int
    nc: int
    level: int           # depth in its cluster tree (top block: -1)


@dataclasses.dataclass
class TreeNode:
    off: int
    size: int
    level: int
    left: int = -1
    right: int = -1
    block: int = -1      # index into Front.blocks when internal


@dataclasses.dataclass
class Front:
    start: int           # first new index of I_p
    npiv: int            # n_p
    upd: np.ndarray      # I_p^f, ascending new indices (int64)
    parent: int
    children: list
    height: int
    relmap: np.ndarray = None   # positions of upd in the parent's front list
    blocks: list = None
    pp_tree: list = None        # TreeNode list, root first
    ff_tree: list = None

    @property
    def nf(self) -> int:
        return int(self.upd.shape[0])

    @property
    def n(self) -> int:
        return self.npiv + self.nf

    def index_list(self) -> np.ndarray:
        return np.concatenate([np.arange(self.start, self.start + self.npiv, dtype=np.int64), self.upd])


@dataclasses.dataclass
class Symbolic:
    n: int
    leaf: int
    perm: np.ndarray      # perm[new] = old
    iperm: np.ndarray     # iperm[old] = new
    fronts: list          # in postorder
    levels: list          # levels[h] = front ids of height h
    pattern_new: sp.csr_matrix  # structural pattern of P A P^T (bool)
    # assembly map of lower entries of P A P^T
    asm_front: np.ndarray
    asm_row: np.ndarray
    asm_col: np.ndarray
    asm_src: np.ndarray   # index into A's CSR value array

    @property
    def nfronts(self) -> int:
        return len(self.fronts)


def _extent_axis(c: np.ndarray) -> int:
    ext = c.max(axis=0) - c.min(axis=0)
    return int(np.argmax(ext))          # first maximum: ties go to the lowest axis


def kd_order(ids: np.ndarray, coords: np.ndarray, leaf: int) -> np.ndarray:
    """kd order of a node set (see module docstring)."""
    ids = np.asarray(ids, dtype=np.int64)
    if ids.shape[0] <= leaf:
        return np.sort(ids)
    ax = _extent_axis(coords[ids])
    order = np.lexsort((ids, coords[ids, ax]))
    s = ids[order]
    m = s.shape[0] // 2
    return np.concatenate([kd_order(s[:m], coords, leaf), kd_order(s[m:], coords, leaf)])


def nested_dissection(rowptr, colind, coords, leaf):
    """Returns (perm, tree) where tree is a list of (start, size, children)
    in postorder."""
    n = rowptr.shape[0] - 1
    coords = np.asarray(coords, dtype=np.float64)
    if coords.ndim == 1:
        coords = coords[:, None]
    perm = []
    tree = []
    inL = np.zeros(n, dtype=bool)

    def has_nb_in(R: np.ndarray, mask: np.ndarray) -> np.ndarray:
        deg = rowptr[R + 1] - rowptr[R]
        out = np.zeros(R.shape[0], dtype=bool)
        nz = deg > 0
        if not nz.any():
            return out
        Rn = R[nz]
        starts = rowptr[Rn].astype(np.int64)
        lens = (rowptr[Rn + 1] - rowptr[Rn]).astype(np.int64)
        idx = np.repeat(starts - np.cumsum(np.r_[0, lens[:-1]]), lens) + np.arange(lens.sum())
        hits = mask[colind[idx]]
        seg = np.cumsum(np.r_[0, lens[:-1]])
        out[nz] = np.logical_or.reduceat(hits, seg)
        return out

    def rec(S: np.ndarray) -> int:
        if S.shape[0] <= leaf:
            return make_leaf(S)
        ax = _extent_axis(coords[S])
        cs = coords[S, ax]
        order = np.lexsort((S, cs))
        c = cs[order[S.shape[0] // 2]]
        L = S[cs < c]
        R = S[cs >= c]
        if L.shape[0] == 0:
            return make_leaf(S)
        inL[L] = True
        sep_mask = has_nb_in(R, inL)
        inL[L] = False
        Sep = R[sep_mask]
        if Sep.shape[0] == 0:
            return make_leaf(S)
        Rp = R[~sep_mask]
        kids = [rec(L)]
        if Rp.shape[0] > 0:
            kids.append(rec(Rp))
        start = len(perm)
        perm.extend(kd_order(Sep, coords, leaf).tolist())
        tree.append((start, Sep.shape[0], kids))
        return len(tree) - 1

    def make_leaf(S):
        start = len(perm)
        perm.extend(kd_order(S, coords, leaf).tolist())
        tree.append((start, S.shape[0], []))
        return len(tree) - 1

    rec(np.arange(n, dtype=np.int64))
    return np.asarray(perm, dtype=np.int64), tree


def _bisect_tree(off: int, size: int, leaf: int, kind: str, blocks: list) -> list:
    """Cluster tree over positions [off, off+size): nodes in level order
    (root first).  Internal nodes register their lower off-diagonal block."""
    nodes = [TreeNode(off, size, 0)]
    i = 0
    while i < len(nodes):
        t = nodes[i]
        if t.size > leaf:
            m = t.size // 2
            t.left = len(nodes)
            nodes.append(TreeNode(t.off, m, t.level + 1))
            t.right = len(nodes)
            nodes.append(TreeNode(t.off + m, t.size - m, t.level + 1))
        i += 1
    for t in nodes:
        if t.left >= 0:
            l, r = nodes[t.left], nodes[t.right]
            t.block = len(blocks)
            blocks.append(Block(kind, r.off, r.size, l.off, l.size, t.level))
    return nodes


def analyze(A, coords, leaf: int) -> Symbolic:
    """Symbolic analysis of an SPD matrix given in full-pattern CSR."""
    rowptr = np.asarray(A.rowptr, dtype=np.int64)
    colind = np.asarray(A.colind, dtype=np.int64)
    n = rowptr.shape[0] - 1
    perm, tree = nested_dissection(rowptr, colind, coords, leaf)
    assert perm.shape[0] == n
    iperm = np.empty(n, dtype=np.int64)
    iperm[perm] = np.arange(n)

    # pattern of P A P^T (structural)
    rows_old = np.repeat(np.arange(n), np.diff(rowptr))
    rn = iperm[rows_old]
    cn = iperm[colind]
    pat = sp.csr_matrix((np.ones(rn.shape[0], dtype=bool), (rn, cn)), shape=(n, n))
    pat.sort_indices()

    nf = len(tree)
    parent = np.full(nf, -1, dtype=np.int64)
    for p, (_, _, kids) in enumerate(tree):
        for c in kids:
            parent[c] = p
    owner = np.empty(n, dtype=np.int64)
    for p, (s, m, _) in enumerate(tree):
        owner[s:s + m] = p

    fronts = []
    height = np.zeros(nf, dtype=np.int64)
    for p, (s, m, kids) in enumerate(tree):
        e = s + m
        # S_p (Eq. couplingSet): new indices j > last(I_p) coupled to I_p
        nb = pat.indices[pat.indptr[s]:pat.indptr[e]]
        Sp = np.unique(nb[nb >= e])
        parts = [Sp] + [fronts[c].upd for c in kids]
        U = np.unique(np.concatenate(parts)) if parts else np.zeros(0, dtype=np.int64)
        U = U[(U < s) | (U >= e)]
        assert U.shape[0] == 0 or U[0] >= e
        h = 0 if not kids else 1 + max(int(height[c]) for c in kids)
        height[p] = h
        fronts.append(Front(s, m, U.astype(np.int64), int(parent[p]), list(kids), h))

    # relative maps
    for p, f in enumerate(fronts):
        lst = f.index_list()
        for c in f.children:
            fc = fronts[c]
            pos = np.searchsorted(lst, fc.upd)
            assert np.all(lst[pos] == fc.upd)
            fc.relmap = pos.astype(np.int64)

    # cluster trees and blocks
    for f in fronts:
        f.blocks = []
        if f.nf > 0 and f.npiv > 0:
            f.blocks.append(Block("top", f.npiv, f.nf, 0, f.npiv, -1))
        f.pp_tree = _bisect_tree(0, f.npiv, leaf, "pp", f.blocks)
        f.ff_tree = _bisect_tree(f.npiv, f.nf, leaf, "ff", f.blocks) if f.nf > 0 else []

    # assembly map: lower entries (i >= j) of P A P^T go to the front owning j
    keep = rn >= cn
    src = np.flatnonzero(keep)
    i_new = rn[keep]
    j_new = cn[keep]
    fr = owner[j_new]
    col = j_new - np.array([fronts[p].start for p in range(nf)])[fr]
    row = np.empty_like(col)
    for p in range(nf):
        sel = np.flatnonzero(fr == p)
        if sel.shape[0] == 0:
            continue
        row[sel] = np.searchsorted(fronts[p].index_list(), i_new[sel])
        assert np.all(fronts[p].index_list()[row[sel]] == i_new[sel])

    levels = [[] for _ in range(int(height.max()) + 1)]
    for p in range(nf):
        levels[int(height[p])].append(p)
    return Symbolic(n, leaf, perm, iperm, fronts, levels, pat, fr, row, col, src)


def bdlr_sets(sym: Symbolic, front: Front, blk: Block, depth: int, cap: int):
    """BDLR row set I (subset of the block's rows) and column set J (subset of
    its columns), in ascending front position (Sec. 2.2, Sec. 4.2.1).

    The interaction graph is the graph of A restricted to the front's whole
    index set I_p u I_p^f (Sec. 4.2.1).  Rows of the block are ranked by
    their graph distance to the block's column cluster (multi-source BFS from
    the columns, through any node of the front), columns by their distance to
    the row cluster.  Kept: distance 1..d (every index when d < 0, unreachable
    ones last), at most ``cap`` of them, closest first, ties to the lower
    position."""
    lst = front.index_list()
    sub = sym.pattern_new[lst][:, lst].astype(np.int8).tocsr()
    nloc = lst.shape[0]
    rows = np.arange(blk.r0, blk.r0 + blk.nr)
    cols = np.arange(blk.c0, blk.c0 + blk.nc)

    def bfs(src: np.ndarray) -> np.ndarray:
        dist = np.full(nloc, -1, dtype=np.int64)
        dist[src] = 0
        frontier = np.zeros(nloc, dtype=np.int8)
        frontier[src] = 1
        k = 0
        while True:
            k += 1
            if depth >= 0 and k > depth:
                break
            reach = (sub @ frontier) > 0
            new = reach & (dist < 0)
            if not new.any():
                break
            dist[new] = k
            frontier = new.astype(np.int8)
        return dist

    def pick(dist_part: np.ndarray, positions: np.ndarray) -> np.ndarray:
        if depth >= 0:
            ok = (dist_part >= 1) & (dist_part <= depth)
        else:
            ok = np.ones(dist_part.shape[0], dtype=bool)
        d = np.where(dist_part < 0, np.iinfo(np.int64).max, dist_part)[ok]
        p = positions[ok]
        order = np.lexsort((p, d))
        return np.sort(p[order[:cap]])

    I = pick(bfs(cols)[rows], rows)
    J = pick(bfs(rows)[cols], cols)
    return I.astype(np.int64), J.astype(np.int64)
