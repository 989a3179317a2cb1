// Host-side symbolic analysis of the multifrontal method (Sec. 4.1.1):
// nested-dissection order, elimination tree, I_p / S_p / I_p^f, relative
// maps, assembly map, HODLR cluster trees and BDLR sets (Sec. 2.2).
//
// Ordering rule (the paper uses nested dissection without fixing a rule):
// coordinate-median vertex separators.  For a node set S with |S| > leaf:
// axis = largest coordinate extent (ties -> lowest axis); sort S by
// (coordinate, original id); c = coordinate of element floor(|S|/2);
// L = {coord < c}, R = {coord >= c}, Sep = {v in R with a neighbour in L},
// R' = R \ Sep.  Empty L or Sep -> leaf.  Postorder numbering: L subtree,
// R' subtree, Sep.  Leaves and separators are numbered in kd order.
#include "symbolic.h"
#include "hostpool.h"

#include <algorithm>
#include <utility>
#include <atomic>
#include <cstring>
#include <limits>
#include <mutex>
#include <numeric>
#include <thread>
#include <tuple>

namespace mfh {
namespace {



// Output of one subtree of the dissection: its vertices in postorder and its
// tree nodes (indices local to this output).
struct NDOut {
  struct TNode { int start, size; std::vector<int> kids; };
  std::vector<int> perm;
  std::vector<TNode> tree;
  // appends a subtree's output; returns the subtree root's new index
  int append(NDOut& o, int root) {
    const int tb = (int)tree.size(), pb = (int)perm.size();
    perm.insert(perm.end(), o.perm.begin(), o.perm.end());
    for (auto& t : o.tree) {
      for (int& k : t.kids) k += tb;
      tree.push_back({t.start + pb, t.size, std::move(t.kids)});
    }
    return root + tb;
  }
};

struct NDCtx {
  int n, dim, leaf;
  const int32_t* rowptr;
  const int32_t* colind;
  const double* coords;

  double co(int v, int a) const { return coords[(int64_t)v * dim + a]; }

  // coordinate range of ids along every axis (large sets: per-chunk ranges, combined)
  void extents(const std::vector<int>& ids, double* mn, double* mx) const {
    for (int a = 0; a < dim; ++a) {
      mn[a] = std::numeric_limits<double>::infinity();
      mx[a] = -mn[a];
    }
    const int n_s = (int)ids.size();
    if (n_s < kParallelSplit) {
      for (int v : ids)
        for (int a = 0; a < dim; ++a) {
          const double c = co(v, a);
          mn[a] = std::min(mn[a], c);
          mx[a] = std::max(mx[a], c);
        }
      return;
    }
    std::mutex mu;
    parallel_for(n_s, 4096, [&](int i0, int i1, int) {
      double lo[3], hi[3];
      for (int a = 0; a < dim; ++a) {
        lo[a] = std::numeric_limits<double>::infinity();
        hi[a] = -lo[a];
      }
      for (int i = i0; i < i1; ++i)
        for (int a = 0; a < dim; ++a) {
          const double c = co(ids[i], a);
          lo[a] = std::min(lo[a], c);
          hi[a] = std::max(hi[a], c);
        }
      std::lock_guard<std::mutex> g(mu);
      for (int a = 0; a < dim; ++a) {
        mn[a] = std::min(mn[a], lo[a]);
        mx[a] = std::max(mx[a], hi[a]);
      }
    });
  }

  // axis of largest coordinate extent over ids (one pass for all axes)
  int extent_axis(const std::vector<int>& ids) const {
    double mn[3], mx[3];
    extents(ids, mn, mx);
    int best = 0;
    double bext = -1.0;
    for (int a = 0; a < dim; ++a) {
      const double ext = mx[a] - mn[a];
      if (a == 0 || ext > bext) { bext = ext; best = a; }   // first maximum wins
    }
    return best;
  }

  // places the element of rank m in (coordinate, id) order at ids[m], smaller
  // ones before it, larger ones after (the order inside each part is free);
  // the selection runs on (coordinate, id) pairs held contiguously
  void select_by_axis(std::vector<int>& ids, size_t m, int ax) const {
    std::vector<std::pair<double, int>> key(ids.size());
    for (size_t i = 0; i < ids.size(); ++i) key[i] = {co(ids[i], ax), ids[i]};
    std::nth_element(key.begin(), key.begin() + (std::ptrdiff_t)m, key.end());
    for (size_t i = 0; i < ids.size(); ++i) ids[i] = key[i].second;
  }
  // coordinate of the element of rank m in (coordinate, id) order: the
  // m-th smallest coordinate (ids only order equal coordinates)
  double median_coord(const std::vector<int>& ids, size_t m, int ax) const {
    const int n_s = (int)ids.size();
    if (n_s < kParallelMedian) {
      std::vector<double> key(ids.size());
      for (size_t i = 0; i < ids.size(); ++i) key[i] = co(ids[i], ax);
      std::nth_element(key.begin(), key.begin() + (std::ptrdiff_t)m, key.end());
      return key[m];
    }
    // large sets: a histogram of the coordinates over value bins (per
    // chunk, summed) finds the bin holding rank m; the selection then runs
    // on that bin's values alone.  The bin index is non-decreasing in the
    // value, so every value of an earlier bin is smaller: the result is the
    // exact m-th smallest coordinate.
    double mn[3], mx[3];
    extents(ids, mn, mx);
    const double lo = mn[ax], hi = mx[ax];
    if (!(hi > lo)) return lo;
    constexpr int NBIN = 4096;
    const double scale = NBIN / (hi - lo);
    auto bin = [&](double x) { return std::min(NBIN - 1, std::max(0, (int)((x - lo) * scale))); };
    const int nch = std::min(max_workers() * 4, n_s / 4096 + 1), per = (n_s + nch - 1) / nch;
    std::vector<std::vector<int>> hist(nch, std::vector<int>(NBIN, 0));
    parallel_for(nch, 1, [&](int c0, int c1, int) {
      for (int c = c0; c < c1; ++c)
        for (int i = c * per; i < std::min(n_s, (c + 1) * per); ++i) ++hist[c][bin(co(ids[i], ax))];
    });
    int64_t below = 0;
    int b = 0;
    for (;; ++b) {
      int64_t cnt = 0;
      for (int c = 0; c < nch; ++c) cnt += hist[c][b];
      if (below + cnt > (int64_t)m || b == NBIN - 1) break;
      below += cnt;
    }
    std::vector<std::vector<double>> part(nch);
    parallel_for(nch, 1, [&](int c0, int c1, int) {
      for (int c = c0; c < c1; ++c)
        for (int i = c * per; i < std::min(n_s, (c + 1) * per); ++i) {
          const double x = co(ids[i], ax);
          if (bin(x) == b) part[c].push_back(x);
        }
    });
    std::vector<double> key;
    for (auto& v : part) key.insert(key.end(), v.begin(), v.end());
    const size_t mm = m - (size_t)below;
    std::nth_element(key.begin(), key.begin() + (std::ptrdiff_t)mm, key.end());
    return key[mm];
  }
  // S split by keep(v) into (yes, no), both in S's order; large sets in
  // parallel chunks whose outputs are joined in chunk order
  template <typename F>
  void split(const std::vector<int>& S, F keep, std::vector<int>& yes, std::vector<int>& no) const {
    const int n_s = (int)S.size();
    if (n_s < kParallelSplit) {
      for (int v : S) (keep(v) ? yes : no).push_back(v);
      return;
    }
    const int nch = std::min(max_workers() * 4, n_s / 4096 + 1);
    std::vector<std::vector<int>> cy(nch), cn(nch);
    const int per = (n_s + nch - 1) / nch;
    parallel_for(nch, 1, [&](int c0, int c1, int) {
      for (int c = c0; c < c1; ++c)
        for (int i = c * per; i < std::min(n_s, (c + 1) * per); ++i) {
          const int v = S[i];
          (keep(v) ? cy[c] : cn[c]).push_back(v);
        }
    });
    for (int c = 0; c < nch; ++c) {
      yes.insert(yes.end(), cy[c].begin(), cy[c].end());
      no.insert(no.end(), cn[c].begin(), cn[c].end());
    }
  }
  static constexpr int kParallelSplit = 32768;
  static constexpr int kParallelMedian = 100000;

  void kd_order(std::vector<int> ids, std::vector<int>& out) const {
    if ((int)ids.size() <= leaf) {
      std::sort(ids.begin(), ids.end());
      out.insert(out.end(), ids.begin(), ids.end());
      return;
    }
    int ax = extent_axis(ids);
    size_t m = ids.size() / 2;
    select_by_axis(ids, m, ax);   // first half = the m smallest in (coordinate, id) order
    kd_order(std::vector<int>(ids.begin(), ids.begin() + m), out);
    kd_order(std::vector<int>(ids.begin() + m, ids.end()), out);
  }

  int make_leaf(const std::vector<int>& S, NDOut& out) const {
    int start = (int)out.perm.size();
    kd_order(S, out.perm);
    out.tree.push_back({start, (int)S.size(), {}});
    return (int)out.tree.size() - 1;
  }

  // Large sets near the root run their two halves as two host tasks (each
  // with its own marker array); the merged output equals the sequential one.
  int rec(const std::vector<int>& S, NDOut& out, std::vector<char>& inL, int spawn) const {
    if ((int)S.size() <= leaf) return make_leaf(S, out);
    int ax = extent_axis(S);
    const double c = median_coord(S, S.size() / 2, ax);
    std::vector<int> L, R;
    split(S, [&](int v) { return co(v, ax) < c; }, L, R);
    if (L.empty()) return make_leaf(S, out);
    for (int v : L) inL[v] = 1;
    std::vector<int> Sep, Rp;
    split(R, [&](int v) {
      for (int k = rowptr[v]; k < rowptr[v + 1]; ++k)
        if (inL[colind[k]]) return true;
      return false;
    }, Sep, Rp);
    for (int v : L) inL[v] = 0;
    if (Sep.empty()) return make_leaf(S, out);
    std::vector<int> kids;
    if (spawn > 0 && !Rp.empty() && (int)S.size() > 16 * leaf) {
      NDOut oL, oR;
      int rL = -1;
      TaskGroup g;
      g.add();
      HostPool::get().submit([&]() {
        std::vector<char> mark(n, 0);
        rL = rec(L, oL, mark, spawn - 1);
        g.done();
      });
      const int rR = rec(Rp, oR, inL, spawn - 1);
      g.wait();
      kids.push_back(out.append(oL, rL));
      kids.push_back(out.append(oR, rR));
    } else {
      kids.push_back(rec(L, out, inL, 0));
      if (!Rp.empty()) kids.push_back(rec(Rp, out, inL, 0));
    }
    int start = (int)out.perm.size();
    kd_order(Sep, out.perm);
    out.tree.push_back({start, (int)Sep.size(), kids});
    return (int)out.tree.size() - 1;
  }
};

void bisect_tree(int off, int size, int leaf, int kind, std::vector<TreeNode>& nodes,
                 std::vector<Block>& blocks) {
  nodes.clear();
  nodes.push_back({off, size, 0});
  for (size_t i = 0; i < nodes.size(); ++i) {
    TreeNode t = nodes[i];
    if (t.size > leaf) {
      int m = t.size / 2;
      nodes[i].left = (int)nodes.size();
      nodes.push_back({t.off, m, t.level + 1});
      nodes[i].right = (int)nodes.size();
      nodes.push_back({t.off + m, t.size - m, t.level + 1});
    }
  }
  for (auto& t : nodes) {
    if (t.left >= 0) {
      const TreeNode& l = nodes[t.left];
      const TreeNode& r = nodes[t.right];
      t.block = (int)blocks.size();
      blocks.push_back({kind, r.off, r.size, l.off, l.size, t.level});
    }
  }
}

std::string validate(int n, const int32_t* rowptr, const int32_t* colind) {
  if (n < 1) return "n must be >= 1";
  if (rowptr[0] != 0) return "rowptr[0] must be 0";
  for (int i = 0; i < n; ++i)
    if (rowptr[i + 1] < rowptr[i]) return "rowptr not monotone";
  // per-row checks in parallel; the lowest failing row is reported
  std::atomic<int> bad_row{n};
  std::vector<int> code(max_workers(), 0);
  std::vector<int> where(max_workers(), n);
  parallel_for(n, 1024, [&](int r0, int r1, int t) {
    for (int i = r0; i < r1 && i < bad_row.load(std::memory_order_relaxed); ++i) {
      int c = 0;
      bool diag = false;
      for (int k = rowptr[i]; k < rowptr[i + 1] && c == 0; ++k) {
        const int j = colind[k];
        if (j < 0 || j >= n) c = 1;
        else if (k > rowptr[i] && colind[k - 1] >= j) c = 2;
        else if (j == i) diag = true;
      }
      if (c == 0 && !diag) c = 3;
      if (c != 0) {
        code[t] = c;
        where[t] = i;
        int cur = bad_row.load();
        while (i < cur && !bad_row.compare_exchange_weak(cur, i)) {}
        return;
      }
    }
  });
  int first = n, fc = 0;
  for (size_t t = 0; t < code.size(); ++t)
    if (code[t] != 0 && where[t] < first) { first = where[t]; fc = code[t]; }
  if (fc == 1) return "column index out of range";
  if (fc == 2) return "columns not strictly increasing within a row";
  if (fc == 3) return "missing diagonal entry in row " + std::to_string(first);
  // symmetry: every entry (i, j) above the diagonal has its mirror (j, i)
  // (rows are sorted: a binary search in row j, which starts at the mirror's
  // position at or after the diagonal), and there are as many entries below
  // the diagonal as above.  Distinct entries above have distinct mirrors, so
  // equal counts make the mirroring a bijection: the pattern is symmetric.
  std::atomic<bool> asym{false};
  std::atomic<int64_t> upper{0}, lower{0};
  parallel_for(n, 1024, [&](int r0, int r1, int) {
    int64_t up = 0, lo = 0;
    for (int i = r0; i < r1 && !asym.load(std::memory_order_relaxed); ++i)
      for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
        const int j = colind[k];
        if (j < i) {
          ++lo;
          continue;
        }
        if (j == i) continue;
        ++up;
        if (!std::binary_search(colind + rowptr[j], colind + rowptr[j + 1], i)) {
          asym.store(true, std::memory_order_relaxed);
          break;
        }
      }
    upper += up;
    lower += lo;
  });
  if (asym.load() || upper.load() != lower.load()) return "pattern is not symmetric";
  return "";
}

}  // namespace

std::string analyze(int n, const int32_t* rowptr, const int32_t* colind, const double* coords,
                    int dim, int leaf, Symbolic& s) {
  if (dim < 1 || dim > 3) return "dim must be 1..3";
  if (leaf < 1) return "leaf must be >= 1";
  std::string err = validate(n, rowptr, colind);
  if (!err.empty()) return err;
  s = Symbolic();
  s.n = n; s.leaf = leaf; s.dim = dim;
  s.nnz = rowptr[n];
  s.rowptr.assign(rowptr, rowptr + n + 1);
  s.colind.resize(s.nnz);
  parallel_for(n, 4096, [&](int r0, int r1, int) {
    std::copy(colind + rowptr[r0], colind + rowptr[r1], s.colind.begin() + rowptr[r0]);
  });

  NDCtx ctx{n, dim, leaf, rowptr, colind, coords};
  NDOut nd;
  nd.perm.reserve(n);
  {
    std::vector<int> all(n);
    std::iota(all.begin(), all.end(), 0);
    std::vector<char> inL(n, 0);
    int spawn = 0;
    for (int w = max_workers(); w > 1; w >>= 1) ++spawn;    // up to 2^spawn subtrees at once
    ctx.rec(all, nd, inL, spawn);
  }
  s.perm = std::move(nd.perm);
  s.iperm.assign(n, 0);
  for (int i = 0; i < n; ++i) s.iperm[s.perm[i]] = i;

  // pattern of P A P^T
  s.prow.assign(n + 1, 0);
  for (int r = 0; r < n; ++r) s.prow[s.iperm[r] + 1] = rowptr[r + 1] - rowptr[r];
  for (int i = 0; i < n; ++i) s.prow[i + 1] += s.prow[i];
  s.pcol.resize(s.nnz);             // every entry is written below
  parallel_for(n, 1024, [&](int r0, int r1, int) {
    for (int r = r0; r < r1; ++r) {
      const int nr = s.iperm[r];
      int o = s.prow[nr];
      for (int k = rowptr[r]; k < rowptr[r + 1]; ++k) s.pcol[o++] = s.iperm[colind[k]];
      std::sort(s.pcol.begin() + s.prow[nr], s.pcol.begin() + s.prow[nr + 1]);
    }
  });

  const int nfr = (int)nd.tree.size();
  s.fronts.resize(nfr);
  for (int p = 0; p < nfr; ++p) {
    Front& f = s.fronts[p];
    f.start = nd.tree[p].start;
    f.npiv = nd.tree[p].size;
    f.children = nd.tree[p].kids;
    for (int c : f.children) s.fronts[c].parent = p;
  }
  for (int p = 0; p < nfr; ++p) {     // children come first in postorder
    Front& f = s.fronts[p];
    int h = 0;
    for (int c : f.children) h = std::max(h, s.fronts[c].height + 1);
    f.height = h;
  }
  int hmax = 0;
  for (auto& f : s.fronts) hmax = std::max(hmax, f.height);
  s.levels.assign(hmax + 1, {});
  for (int p = 0; p < nfr; ++p) s.levels[s.fronts[p].height].push_back(p);
  // I_p^f = (S_p u children's I^f) \ I_p, level by level (a level's fronts
  // only read their children's sets); duplicates are dropped with a
  // per-worker stamp array before sorting
  {
    std::vector<std::vector<int>> stamp(max_workers(), std::vector<int>());
    for (int h = 0; h <= hmax; ++h) {
      const std::vector<int>& L = s.levels[h];
      parallel_for((int)L.size(), 1, [&](int b, int e, int t) {
        std::vector<int>& mark = stamp[t];
        if (mark.empty()) mark.assign(n, -1);
        for (int q = b; q < e; ++q) {
          const int p = L[q];
          Front& f = s.fronts[p];
          const int st = f.start, en = f.start + f.npiv;
          std::vector<int> U;
          for (int i = st; i < en; ++i)
            for (int k = s.prow[i]; k < s.prow[i + 1]; ++k) {
              const int g = s.pcol[k];
              if (g >= en && mark[g] != p) {                  // S_p (Eq. couplingSet)
                mark[g] = p;
                U.push_back(g);
              }
            }
          for (int c : f.children)
            for (int v : s.fronts[c].upd)
              if ((v < st || v >= en) && mark[v] != p) {
                mark[v] = p;
                U.push_back(v);
              }
          std::sort(U.begin(), U.end());
          f.upd = std::move(U);
        }
      });
    }
  }
  // relative maps (each child belongs to one parent: fronts are independent)
  parallel_for(nfr, 16, [&](int b, int e, int) {
    for (int p = b; p < e; ++p) {
      const Front& f = s.fronts[p];
      for (int c : f.children) {
        // both update sets are ascending: one merge scan places the child's
        // indices among the parent's pivots and update set
        Front& fc = s.fronts[c];
        fc.relmap.resize(fc.upd.size());
        size_t q = 0;
        for (size_t a = 0; a < fc.upd.size(); ++a) {
          const int g = fc.upd[a];
          if (g < f.start + f.npiv) {
            fc.relmap[a] = g - f.start;
          } else {
            while (q < f.upd.size() && f.upd[q] < g) ++q;
            fc.relmap[a] = f.npiv + (int)q;
          }
        }
      }
    }
  });
  // cluster trees and blocks
  int nb = 0;
  s.block_base.assign(nfr + 1, 0);
  for (int p = 0; p < nfr; ++p) {
    Front& f = s.fronts[p];
    f.blocks.clear();
    if (f.nf() > 0 && f.npiv > 0) f.blocks.push_back({0, f.npiv, f.nf(), 0, f.npiv, -1});
    bisect_tree(0, f.npiv, leaf, 1, f.pp_tree, f.blocks);
    if (f.nf() > 0) bisect_tree(f.npiv, f.nf(), leaf, 2, f.ff_tree, f.blocks);
    else f.ff_tree.clear();
    s.block_base[p] = nb;
    nb += (int)f.blocks.size();
  }
  s.block_base[nfr] = nb;
  s.nblocks = nb;
  return "";
}

// Analysis of the block-diagonal matrix diag(A_1, ..., A_k) from those of
// its blocks.  The nested dissection of a block-diagonal matrix may keep
// each block's own order: no entry couples two blocks, so the elimination
// forest is the disjoint union of the blocks' trees, each front keeps its
// frontal sets, relative maps and cluster trees, and only global indices
// shift (rows of block i by n_1 + ... + n_{i-1}, fronts by the number of
// fronts before it).  Levels are by height, so fronts of every block that
// sit at one height share a level (Sec. 4.1: the fronts of one level are
// independent).  BDLR caches are dropped: the factorisation forms its sets
// per front.
std::string merge(const std::vector<const Symbolic*>& parts, Symbolic& s) {
  if (parts.empty()) return "no analyses to merge";
  for (const Symbolic* q : parts) {
    if (!q) return "null analysis";
    if (q->leaf != parts[0]->leaf || q->dim != parts[0]->dim) return "analyses differ in leaf size or dimension";
  }
  int64_t n = 0, nnz = 0, nfr = 0, nb = 0;
  int hmax = 0;
  for (const Symbolic* q : parts) {
    n += q->n;
    nnz += q->nnz;
    nfr += (int64_t)q->fronts.size();
    nb += q->nblocks;
    hmax = std::max(hmax, (int)q->levels.size());
  }
  if (n > std::numeric_limits<int32_t>::max() || nnz > std::numeric_limits<int32_t>::max())
    return "merged analysis exceeds 32-bit indices";
  s = Symbolic();
  s.n = (int)n; s.leaf = parts[0]->leaf; s.dim = parts[0]->dim; s.nnz = nnz;
  s.rowptr.resize(n + 1);
  s.colind.resize(nnz);
  s.prow.resize(n + 1);
  s.pcol.resize(nnz);
  s.perm.resize(n);
  s.iperm.resize(n);
  s.fronts.reserve(nfr);
  s.levels.assign(hmax, {});
  s.block_base.reserve(nfr + 1);
  int no = 0, fo = 0, bo = 0;
  int64_t eo = 0;
  for (const Symbolic* q : parts) {
    for (int r = 0; r < q->n; ++r) {
      s.rowptr[no + r] = (int)(eo + q->rowptr[r]);
      s.prow[no + r] = (int)(eo + q->prow[r]);
      s.perm[no + r] = no + q->perm[r];
      s.iperm[no + r] = no + q->iperm[r];
    }
    for (int64_t k = 0; k < q->nnz; ++k) {
      s.colind[eo + k] = no + q->colind[k];
      s.pcol[eo + k] = no + q->pcol[k];
    }
    for (const Front& f : q->fronts) {
      Front g = f;
      g.start += no;
      for (int& v : g.upd) v += no;
      if (g.parent >= 0) g.parent += fo;
      for (int& c : g.children) c += fo;
      s.fronts.push_back(std::move(g));
    }
    for (size_t h = 0; h < q->levels.size(); ++h)
      for (int p : q->levels[h]) s.levels[h].push_back(fo + p);
    for (size_t p = 0; p < q->fronts.size(); ++p) s.block_base.push_back(bo + q->block_base[p]);
    no += q->n;
    eo += q->nnz;
    fo += (int)q->fronts.size();
    bo += q->nblocks;
  }
  s.rowptr[n] = (int)nnz;
  s.prow[n] = (int)nnz;
  s.block_base.push_back(bo);
  s.nblocks = bo;
  return "";
}

// Assembly map of A's lower entries (F_bar_p, Eq. fbar), in CSR order: the
// front, the row and column inside it, and the entry's index in A.  Rows are
// split over workers: one pass counts each row's lower entries, a second
// writes them at their offsets.  (The factorisation places the entries on
// the device from the same rule; this host form is for inspection.)
void assembly_map(const Symbolic& s, bigvec<int>& asm_front, bigvec<int>& asm_row, bigvec<int>& asm_col,
                  bigvec<int>& asm_src) {
  const int n = s.n;
  const int* rowptr = s.rowptr.data();
  const int* colind = s.colind.data();
  std::vector<int> owner(n);
  for (int p = 0; p < (int)s.fronts.size(); ++p)
    for (int i = 0; i < s.fronts[p].npiv; ++i) owner[s.fronts[p].start + i] = p;
  {
    std::vector<int64_t> off(n + 1, 0);
    parallel_for(n, 2048, [&](int r0, int r1, int) {
      for (int r = r0; r < r1; ++r) {
        const int i = s.iperm[r];
        int c = 0;
        for (int k = rowptr[r]; k < rowptr[r + 1]; ++k) c += i >= s.iperm[colind[k]];
        off[r + 1] = c;
      }
    });
    for (int r = 0; r < n; ++r) off[r + 1] += off[r];
    const size_t tot = (size_t)off[n];
    asm_front.resize(tot);
    asm_row.resize(tot);
    asm_col.resize(tot);
    asm_src.resize(tot);
    parallel_for(n, 2048, [&](int r0, int r1, int) {
      for (int r = r0; r < r1; ++r) {
        int64_t o = off[r];
        const int i = s.iperm[r];
        // a row's entries fall in few fronts: the last front's row position
        // is reused instead of searching its update set again
        int lp = -1, lrow = 0;
        for (int k = rowptr[r]; k < rowptr[r + 1]; ++k) {
          const int j = s.iperm[colind[k]];
          if (i < j) continue;
          const int p = owner[j];
          const Front& f = s.fronts[p];
          if (p != lp) {
            lp = p;
            lrow = i < f.start + f.npiv
                       ? i - f.start
                       : f.npiv + (int)(std::lower_bound(f.upd.begin(), f.upd.end(), i) - f.upd.begin());
          }
          asm_front[o] = p;
          asm_row[o] = lrow;
          asm_col[o] = j - f.start;
          asm_src[o] = k;
          ++o;
        }
      }
    });
  }
}

// BDLR sets (Sec. 2.2): interaction graph = A restricted to the front's
// index set I_p u I_p^f (Sec. 4.2.1).  Rows of a block ranked by BFS distance
// to the block's column cluster, columns by distance to the row cluster.
void compute_bdlr(Symbolic& s, int depth, int cap) {
  if (s.bdlr_depth == depth && s.bdlr_cap == cap) return;
  bdlr_sets(s, depth, cap, s.bdlr_I, s.bdlr_Iptr, s.bdlr_J, s.bdlr_Jptr);
  s.bdlr_depth = depth;
  s.bdlr_cap = cap;
}

// One front: appends the sets of each of its blocks to I/J and one offset
// per block to Iptr/Jptr.
void bdlr_front(const Symbolic& s, int p, int depth, int cap, BdlrScratch& w, std::vector<int>& outI,
                std::vector<int>& outIptr, std::vector<int>& outJ, std::vector<int>& outJptr) {
  const long long INF = std::numeric_limits<long long>::max();
  const Front& f = s.fronts[p];
  const int m = f.n();
  if ((int)w.pos_of.size() != s.n) w.pos_of.assign(s.n, -1);
  for (int a = 0; a < m; ++a) w.pos_of[f.global(a)] = a;
  w.adjp.assign(m + 1, 0);
  w.adj.clear();
  for (int a = 0; a < m; ++a) {
    int g = f.global(a);
    for (int k = s.prow[g]; k < s.prow[g + 1]; ++k) {
      int b = w.pos_of[s.pcol[k]];
      if (b >= 0) w.adj.push_back(b);
    }
    w.adjp[a + 1] = (int)w.adj.size();
  }
  // Multi-source BFS from [lo, lo+cnt).  Once `cap` nodes of the target
  // range [tlo, tlo+tcnt) are settled, the selection (cap smallest
  // (distance, position)) can no longer change: stop after that layer.
  auto bfs = [&](int lo, int cnt, int tlo, int tcnt) {
    w.dist.assign(m, -1);
    w.frontier.clear();
    for (int a = lo; a < lo + cnt; ++a) { w.dist[a] = 0; w.frontier.push_back(a); }
    int settled = 0;
    for (int k = 1;; ++k) {
      if (depth >= 0 && k > depth) break;
      w.nxt.clear();
      for (int v : w.frontier)
        for (int e = w.adjp[v]; e < w.adjp[v + 1]; ++e) {
          int u = w.adj[e];
          if (w.dist[u] < 0) {
            w.dist[u] = k;
            w.nxt.push_back(u);
            if (u >= tlo && u < tlo + tcnt) ++settled;
          }
        }
      if (w.nxt.empty() || settled >= cap) break;
      w.frontier.swap(w.nxt);
    }
  };
  auto pick = [&](int lo, int cnt, std::vector<int>& out) {
    std::vector<std::pair<long long, int>> cand;
    for (int a = lo; a < lo + cnt; ++a) {
      int d = w.dist[a];
      if (depth >= 0) { if (d >= 1 && d <= depth) cand.push_back({d, a}); }
      else cand.push_back({d < 0 ? INF : (long long)d, a});
    }
    size_t k = std::min(cand.size(), (size_t)cap);
    std::partial_sort(cand.begin(), cand.begin() + k, cand.end());
    std::vector<int> sel;
    for (size_t i = 0; i < k; ++i) sel.push_back(cand[i].second);
    std::sort(sel.begin(), sel.end());
    out.insert(out.end(), sel.begin(), sel.end());
  };
  for (const Block& b : f.blocks) {
    bfs(b.c0, b.nc, b.r0, b.nr);
    pick(b.r0, b.nr, outI);
    outIptr.push_back((int)outI.size());
    bfs(b.r0, b.nr, b.c0, b.nc);
    pick(b.c0, b.nc, outJ);
    outJptr.push_back((int)outJ.size());
  }
  for (int a = 0; a < m; ++a) w.pos_of[f.global(a)] = -1;
}

void bdlr_sets(const Symbolic& s, int depth, int cap, std::vector<int>& outI, std::vector<int>& outIptr,
               std::vector<int>& outJ, std::vector<int>& outJptr) {
  outI.clear(); outJ.clear();
  outIptr.assign(1, 0); outJptr.assign(1, 0);
  BdlrScratch w;
  for (int p = 0; p < (int)s.fronts.size(); ++p) bdlr_front(s, p, depth, cap, w, outI, outIptr, outJ, outJptr);
}

}  // namespace mfh
