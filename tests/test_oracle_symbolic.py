"""Pins of the oracle's symbolic analysis (Sec. 4.1.1) against invariants and
closed forms of nested dissection on structured grids."""
import numpy as np
import pytest

from mfinputs import q1_grid, p1_kuhn_cube
from oracle import symbolic


def _check_invariants(p, sym):
    n = p.A.n
    assert np.array_equal(np.sort(sym.perm), np.arange(n))
    assert np.array_equal(sym.iperm[sym.perm], np.arange(n))
    # I_p contiguous ranges partitioning [0, n), postorder: parent after child
    covered = np.zeros(n, dtype=int)
    for q, f in enumerate(sym.fronts):
        covered[f.start:f.start + f.npiv] += 1
        for c in f.children:
            assert c < q and sym.fronts[c].parent == q
            assert sym.fronts[c].height < f.height
        # I_p^f lies in ancestors' pivot sets
        anc = set()
        a = f.parent
        while a >= 0:
            fa = sym.fronts[a]
            anc.update(range(fa.start, fa.start + fa.npiv))
            a = fa.parent
        assert set(f.upd.tolist()) <= anc
        # relative map: child's update set inside the front, increasing
        for c in f.children:
            rm = sym.fronts[c].relmap
            assert np.all(np.diff(rm) > 0)
            assert np.array_equal(f.index_list()[rm], sym.fronts[c].upd)
    assert np.all(covered == 1)
    # each lower entry of P A P^T mapped exactly once
    rows = np.repeat(np.arange(n), np.diff(p.A.rowptr))
    nlow = int(np.sum(sym.iperm[rows] >= sym.iperm[p.A.colind]))
    assert sym.asm_src.shape[0] == nlow
    assert np.unique(sym.asm_src).shape[0] == nlow
    key = sym.asm_front * (n + 1) ** 2 + sym.asm_row * (n + 1) + sym.asm_col
    assert np.unique(key).shape[0] == nlow
    assert np.all(sym.asm_row >= sym.asm_col)


@pytest.mark.parametrize("maker,leaf", [
    (lambda: q1_grid(12, 2), 8),
    (lambda: q1_grid(7, 3), 16),
    (lambda: p1_kuhn_cube(5, 0.2, 1), 12),
])
def test_invariants_and_fill_containment(maker, leaf):
    p = maker()
    sym = symbolic.analyze(p.A, p.coords, leaf)
    _check_invariants(p, sym)
    # fill of chol(P A P^T) lies inside the union of front blocks: every
    # structurally nonzero L[i, j] has i in the front list of j's front
    D = p.A.to_dense()
    L = np.linalg.cholesky(D[np.ix_(sym.perm, sym.perm)])
    owner = np.empty(p.A.n, dtype=int)
    for q, f in enumerate(sym.fronts):
        owner[f.start:f.start + f.npiv] = q
    ii, jj = np.nonzero(np.abs(L) > 1e-300)
    allowed = [set(f.index_list().tolist()) for f in sym.fronts]
    bad = [(i, j) for i, j in zip(ii, jj) if i not in allowed[owner[j]]]
    assert not bad


def test_structured_closed_forms_2d():
    n = 64
    p = q1_grid(n, 2)
    sym = symbolic.analyze(p.A, p.coords, 64)
    assert sym.nfronts == 127 and len(sym.levels) == 7
    root = sym.fronts[-1]
    sep = sym.perm[root.start:root.start + root.npiv]
    # root separator: the grid line x = floor(64/2) = 32, all 64 nodes
    assert root.npiv == 64 and root.nf == 0
    assert np.all(p.coords[sep, 0] == 32)
    # children: x < 32 (32 lines) and x > 32 (31 lines)
    sizes = sorted(sym.fronts[c].npiv + 0 for c in root.children)
    left, right = root.children
    def subtree_nodes(q):
        f = sym.fronts[q]
        out = list(range(f.start, f.start + f.npiv))
        for c in f.children:
            out += subtree_nodes(c)
        return out
    ln = sym.perm[subtree_nodes(left)]
    rn = sym.perm[subtree_nodes(right)]
    assert ln.shape[0] == 32 * 64 and np.all(p.coords[ln, 0] < 32)
    assert rn.shape[0] == 31 * 64 and np.all(p.coords[rn, 0] > 32)
    assert max(f.n for f in sym.fronts) == 97


def test_structured_closed_forms_3d():
    n = 16
    p = q1_grid(n, 3)
    sym = symbolic.analyze(p.A, p.coords, 128)
    root = sym.fronts[-1]
    sep = sym.perm[root.start:root.start + root.npiv]
    assert root.npiv == n * n and np.all(p.coords[sep, 0] == n // 2)
    # kd order inside the root separator: first half is y < 8 (extents tie in
    # y and z, so the lower axis y splits first)
    assert np.all(p.coords[sep[:128], 1] < 8) and np.all(p.coords[sep[128:], 1] >= 8)
    assert sym.nfronts == 63 and max(f.n for f in sym.fronts) == 384


def test_cluster_trees():
    p = q1_grid(16, 3)
    sym = symbolic.analyze(p.A, p.coords, 32)
    for f in sym.fronts:
        for tree, base, size in ((f.pp_tree, 0, f.npiv), (f.ff_tree, f.npiv, f.nf)):
            if size == 0:
                continue
            assert tree[0].off == base and tree[0].size == size
            for t in tree:
                if t.left >= 0:
                    l, r = tree[t.left], tree[t.right]
                    assert l.size == t.size // 2 and l.off == t.off and r.off == t.off + l.size
                    b = f.blocks[t.block]
                    assert (b.r0, b.nr, b.c0, b.nc) == (r.off, r.size, l.off, l.size)
                else:
                    assert t.size <= 32


def test_bdlr_sets_definition():
    p = q1_grid(10, 2)
    sym = symbolic.analyze(p.A, p.coords, 8)
    D = p.A.to_dense() != 0
    Pn = D[np.ix_(sym.perm, sym.perm)]
    f = max(sym.fronts, key=lambda f: f.n)
    lst = f.index_list()
    G = Pn[np.ix_(lst, lst)]
    for blk in f.blocks:
        rows = np.arange(blk.r0, blk.r0 + blk.nr)
        cols = np.arange(blk.c0, blk.c0 + blk.nc)
        # brute-force graph distances inside the front
        dist = np.full(lst.shape[0], -1)
        dist[cols] = 0
        frontier = set(cols.tolist())
        k = 0
        while frontier:
            k += 1
            nxt = set()
            for v in frontier:
                for w in np.flatnonzero(G[v]):
                    if dist[w] < 0:
                        dist[w] = k
                        nxt.add(int(w))
            frontier = nxt
        for d in (1, 2, 3):
            I, J = symbolic.bdlr_sets(sym, f, blk, d, 10 ** 6)
            want = rows[(dist[rows] >= 1) & (dist[rows] <= d)]
            assert np.array_equal(I, want)
            assert np.all(np.diff(J) > 0) and set(J.tolist()) <= set(cols.tolist())
        I, J = symbolic.bdlr_sets(sym, f, blk, -1, 10 ** 6)
        assert np.array_equal(I, rows) and np.array_equal(J, cols)
        I, J = symbolic.bdlr_sets(sym, f, blk, -1, 3)
        assert I.shape[0] == min(3, blk.nr)
        d_in = np.where(dist[rows] < 0, 10 ** 9, dist[rows])
        kth = np.sort(d_in)[I.shape[0] - 1]
        assert np.all(d_in[I - blk.r0] <= kth)
