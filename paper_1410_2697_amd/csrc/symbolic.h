// Internal symbolic-analysis structures (host only).
#pragma once
#include <cstdint>
#include <string>
#include <memory>
#include <utility>
#include <vector>

namespace mfh {

// Allocator whose resize() leaves new elements of trivial types unwritten:
// large index arrays are then first written by the worker threads that fill
// them, instead of being zeroed by one thread beforehand.
template <typename T>
struct NoInitAlloc : std::allocator<T> {
  template <typename U>
  struct rebind { using other = NoInitAlloc<U>; };
  NoInitAlloc() = default;
  template <typename U>
  NoInitAlloc(const NoInitAlloc<U>&) noexcept {}
  template <typename U, typename... A>
  void construct(U* p, A&&... a) {
    if constexpr (sizeof...(A) == 0) ::new ((void*)p) U;
    else ::new ((void*)p) U(std::forward<A>(a)...);
  }
};
template <typename T>
using bigvec = std::vector<T, NoInitAlloc<T>>;


struct Block {            // lower off-diagonal block of a front, in front positions
  int kind;               // 0 top (F_fp), 1 pp, 2 ff
  int r0, nr, c0, nc;
  int level;              // depth in its cluster tree (-1: top)
};

struct TreeNode {         // cluster-tree node over front positions
  int off, size, level;
  int left = -1, right = -1;
  int block = -1;         // index into Front::blocks when internal
};

struct Front {
  int start = 0, npiv = 0;          // I_p = [start, start+npiv) in the new order
  std::vector<int> upd;             // I_p^f, ascending new indices
  int parent = -1;
  std::vector<int> children;
  int height = 0;
  std::vector<int> relmap;          // positions of upd in the parent's front list
  std::vector<Block> blocks;        // top block first, then pp tree, then ff tree (level order)
  std::vector<TreeNode> pp_tree;    // level order, root first
  std::vector<TreeNode> ff_tree;
  int nf() const { return (int)upd.size(); }
  int n() const { return npiv + nf(); }
  int global(int pos) const { return pos < npiv ? start + pos : upd[pos - npiv]; }
};

struct Symbolic {
  int n = 0, leaf = 0, dim = 0;
  int64_t nnz = 0;
  bigvec<int> rowptr, colind;       // copy of A's pattern (original order)
  std::vector<int> perm, iperm;     // perm[new] = old
  bigvec<int> prow, pcol;           // pattern of P A P^T (CSR, sorted)
  std::vector<Front> fronts;        // postorder
  std::vector<std::vector<int>> levels;  // by height
  // BDLR cache
  int bdlr_depth = -2, bdlr_cap = -1;
  std::vector<int> bdlr_I, bdlr_Iptr, bdlr_J, bdlr_Jptr;   // over all blocks in front order
  std::vector<int> block_base;      // first global block id of each front
  int nblocks = 0;
};

// Assembly map of A's lower entries into the fronts (F_bar_p, Eq. fbar), in
// CSR order: front, row and column inside it, index of the entry in A.
void assembly_map(const Symbolic& s, bigvec<int>& front, bigvec<int>& row, bigvec<int>& col, bigvec<int>& src);

// Returns "" on success or an error message.
std::string analyze(int n, const int32_t* rowptr, const int32_t* colind, const double* coords,
                    int dim, int leaf, Symbolic& out);
// Analysis of diag(A_1, ..., A_k) from the analyses of A_1, ..., A_k (equal
// leaf size and dimension).  Returns "" on success or an error message.
std::string merge(const std::vector<const Symbolic*>& parts, Symbolic& out);
// Reusable buffers for BDLR set construction.
struct BdlrScratch {
  std::vector<int> pos_of, adjp, adj, dist, frontier, nxt;
};
// BDLR sets of the blocks of front p (appended; one Iptr/Jptr entry per block).
void bdlr_front(const Symbolic& s, int p, int depth, int cap, BdlrScratch& w, std::vector<int>& I,
                std::vector<int>& Iptr, std::vector<int>& J, std::vector<int>& Jptr);
// BDLR sets of every block (front order, then block order), front positions.
void bdlr_sets(const Symbolic& s, int depth, int cap, std::vector<int>& I, std::vector<int>& Iptr,
               std::vector<int>& J, std::vector<int>& Jptr);
// Same, cached in the handle (for export).
void compute_bdlr(Symbolic& s, int depth, int cap);

}  // namespace mfh
