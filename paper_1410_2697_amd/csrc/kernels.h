// Device kernels of the multifrontal path and their launch descriptors.
// All matrices are column-major.  Every launch processes a list of
// independent problems ("grouped"/batched), so one launch covers all fronts
// of an elimination-tree level.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mfh {

constexpr int kTile = 64;            // GEMM output tile (rows and columns)
constexpr int kTileNarrow = 16;   // output tile width for right-hand-side blocks
template <typename T>
constexpr int kGemmBK = sizeof(T) == 4 ? 64 : 32;   // GEMM k step (LDS-staged)
constexpr int kFoldSlices = 8;      // most partial slices a product reads in place of a reduction
constexpr int kGemmSplitAlign = 64;  // split-K ranges are multiples of this (and of every k step)
constexpr double kTieRel = 1.0 / 1048576.0;   // 2^-20: near-ties in complete pivoting

enum GemmFlags : int {
  GF_LOWER_C = 1,   // write only C(i, j) with i >= j (symmetric updates)
  GF_A_LOWER = 2,   // op(A)(i, kk) == 0 for kk > i
  GF_A_UPPER = 4,   // op(A)(i, kk) == 0 for kk < i
  GF_B_LOWER = 8,   // op(B)(kk, j) == 0 for kk < j
  GF_B_UPPER = 16,  // op(B)(kk, j) == 0 for kk > j
  GF_A_BF16 = 32,   // A holds bfloat16 bit patterns (T = float only)
  GF_B_BF16 = 64,   // B holds bfloat16 bit patterns (T = float only)
};

// C = alpha * op(A) * op(B) + beta * C ; op(A) m x k, op(B) k x n.
// If kdev != nullptr the inner dimension is *kdev (a rank produced on the
// device); k is then an upper bound used only for validation.
// Split K (ksplit > 1, kchunk a multiple of kGemmSplitAlign): workgroup split
// s sums k in [s*kchunk, (s+1)*kchunk)
// into part + s*m*n (m x n, ld m); a reduction launch then forms
// C = alpha * sum_s part_s + beta * C in a fixed order (deterministic).
// Row maps (nullptr: none): a stored row index s of the array A (B) is
// read as row arow[s] (brow[s]); the stored rows are the rows of op(A) when
// opA == 0, its columns when opA == 1 (the same for B).  They gather
// through an index map, e.g. x(I_p^f), or the sampled rows of a basis.
template <typename T>
struct GemmDesc {
  const T* A;
  const T* B;
  T* C;
  const int* kdev;
  T* part;
  const int* arow;
  const int* brow;
  int m, n, k;
  int lda, ldb, ldc;
  int opA, opB;      // 0: N, 1: T
  int flags;
  int tile0;         // first launch tile of this problem
  int tiles_m, tiles_n;
  int ksplit, kchunk;
  double alpha, beta;
};

// Folded split K, one per GemmDesc of a launch_gemm_fold batch: B (op N, no
// row maps, n <= kTileNarrow) is the output of earlier split products whose
// reduction launch was left out.  Rows [0, split) of B come from source 0,
// rows [split, k) from source 1.  A source with `slices` > 0 (at most
// kFoldSlices) reads element (i, j) as
//   alpha * sum_s part[i + j*ld + s*ld*n] + beta * B(i, j)
// summed in slice order (the reduction's own order); a source with no
// slices reads B itself, and a descriptor with no sliced source runs as
// in launch_gemm.
template <typename T>
struct FoldDesc {
  const T* part[2];
  int slices[2], ld[2];
  int split, pad;
  double alpha[2], beta[2];
};

// In-place Cholesky of an n x n diagonal block (n <= 128) and, if Inv is
// set, its explicit lower-triangular inverse (full square written, zeros
// above the diagonal).
template <typename T>
struct PotrfDesc {
  T* A;
  T* Inv;
  int lda, ldi, n, pad;
};

// Register-resident skeleton (one 1024-thread workgroup per block).
//  whole-block mode: the block F(r0:r0+nr, c0:c0+nc) lives in registers;
//    complete pivoting is first confined to the BDLR rows/columns I x J
//    (phase 1), then, if `adaptive`, runs over the whole block (phase 2);
//    every pivot appends a column to U and V (phase 1: U = E(:,b)/piv,
//    V = E(a,:)^T; phase 2: U = E(:,b), V = E(a,:)^T/piv).
//  submatrix mode: the block is B_hat = F(I, J); phase 1 only; outputs the
//    in-place LU in pivot order (M) and the pivots, for SkelFacDesc.
template <typename T>
struct SkRegDesc {
  const T* F;
  const int* I;
  const int* J;
  int* piv_r;        // front positions, capacity cap
  int* piv_c;
  T* M;              // submatrix mode: r x r LU, ld = ldm
  T* U;              // whole-block mode: nr x cap, ld ldu
  T* V;              // whole-block mode: nc x cap, ld ldv
  int* rank1;        // phase-1 rank
  int* rank;         // final rank
  double* u11;
  int ld, r0, nr, c0, nc, nI, nJ, ldm, ldu, ldv, cap, pad;
};

// C~ = B(:, J_r) U_r^{-1} (rows of U) and R~^T = (L_r^{-1} B(I_r, :))^T
// (rows of V) for a block B = F(r0 : r0+nr, c0 : c0+nc).  The pivot
// columns are read from F (ld), the pivot rows from FR (ldr): the same front
// when it is staged densely, else the block's column and row samples (then
// r0 = c0 = 0 and the pivots index the samples).
template <typename T>
struct SkelFacDesc {
  const T* F;
  const T* FR;
  int ldr, pad;
  const int* piv_r;
  const int* piv_c;
  const T* M;
  const int* rank;
  T* U;
  T* V;
  int ld, r0, nr, c0, nc, ldm, ldu, ldv;
  int wg0;           // first launch workgroup of this block
  int wgU;           // workgroups for the U rows (the rest do V rows)
};

// Phase 2: continue complete pivoting on E = B - U V^T (held in place in
// the front) until the pivot-ratio rule holds over the whole block.
template <typename T>
struct Phase2Desc {
  T* F;
  const int* piv_r;
  const int* piv_c;
  const int* rank1;
  const double* u11;
  T* U;
  T* V;
  int* rank;         // out: final rank
  int ld, r0, nr, c0, nc, ldu, ldv, cap;
};

// rows of a block the multi-workgroup phase 2 takes (one bit per row and lane)
constexpr int kPhase2CoopMaxRows = 8192;

// Phase 2 spread over workgroups: workgroup j of a block keeps the residual
// columns [j*wcols, min(nc, (j+1)*wcols)) in LDS for the whole pivot loop.
// After each step every workgroup publishes its best pivot key and the
// updated column it belongs to (double-buffered by step parity), then waits
// at the block's barrier counter; all workgroups then pick the same pivot.
// Pivots, arithmetic and outputs are those of Phase2Desc.
template <typename T>
struct Phase2CoopDesc {
  T* F;      
  const int* piv_r;
  const int* piv_c;
  const int* rank1;
  const double* u11;
  T* U;
  T* V;
  int* rank;
  unsigned long long* keys;      // 2 x nwg tagged key slots, all 1 << 63 before the launch
  T* cand;                       // 2 x nwg x nr
  int ld, r0, nr, c0, nc, ldu, ldv, cap;
  int wg0, nwg, wcols;
  int slice_lds;                 // host bookkeeping: slices in LDS (1) or in place (0)
};

// child update (front positions [npc, npc+nfc) of the child buffer) scatter
// added into the parent front through the relative map.
template <typename T>
struct ExtAddDesc {
  const T* child;
  T* parent;
  const int* relmap;
  int ldc, npc, nfc, ldp;
  int tile0, tiles_r;
};

template <typename S, typename D>
struct CopyDesc {   // dst(i, j) = alpha * src(i, j) (+ dst if accumulate)
  const S* src;
  D* dst;
  int rows, cols, lds, ldd;
  int accumulate;
  int tile0, tiles_r;
  int bf16;          // D = float only: 1 round the value to bfloat16 precision,
                     // 2 store bfloat16 bit patterns (dst holds 16-bit entries)
  double alpha;
};

// SMW capacitance K = [[A, I], [I, B]] with A = P(0:r, c:c+r) (V^T Y_alpha)
// and B = P(r:2r, c:c+r) (U^T Y_beta).  Its inverse is formed from the r x r
// matrix M = (I - A B)^{-1}:  K^{-1} = [[-B M, I + B M A], [M, -M A]].
// This kernel writes A and B in float64 (r x r each, ld r), the identity into
// Kinv(r:2r, 0:r) (to become I - A B) and Kinv(0:r, r:2r) (to become
// I + B M A), and Pa = float64 copy of P(:, 0:c) (ld 2r).
template <typename T>
struct CapDesc {
  const T* P;
  double* Kinv;      // 2r x 2r, ld 2r
  double* A;
  double* B;
  double* Pa;
  int r, c, ldp, pad;
};

struct InvDesc {      // in-place Gauss-Jordan inverse with partial pivoting, float64
  double* A;          // n x n, leading dimension ld
  int n, ld;
};
constexpr int kInvMax = 1024;   // largest n of InvDesc

// upward-pass front vector: t(0:npiv) = xn(start:start+npiv), t(npiv:) = 0,
// then t(relmap_c) += child's t_c(npiv_c:) for each child in order.
template <typename T>
struct VecAsmDesc {
  T* t;
  const T* xs;            // xn + start
  const T* ct[2];
  const int* crel[2];
  int nhat, npiv, ldt, ldx;
  int nchild;
  int cnp[2], cnf[2], cld[2];
};


// ---- sampled extend-add (Sec. 4.2.1, Eq. HODLR_EA_Expand, Fig. HODLR_EA) ----
// A HODLR front is not staged densely: only the entries its compression and
// factorisation read are formed, each as F_bar_p (A's entries in the pivot
// rows and columns) plus every child's update at the mapped position.
//
// Node of a HODLR child's F_ff^HODLR cluster tree: positions in the child's
// update set; an internal node holds its lower off-diagonal block (rows in
// the right child, columns in the left) as U V^T, a leaf its dense block.
struct FfNode {
  int off, size, left, right;   // left < 0: leaf
  int rank;
  const void* U;    // internal: right.size x rank (ld right.size); leaf: size x size (ld size)
  const void* V;    // internal: left.size x rank (ld left.size)
};
// A child's update U_c (nf x nf, symmetric) as a parent's gather sees it:
// dense staging (lower triangle at rows / columns npc..), or compressed,
// U_c = F_ff^HODLR - Wt W^T with Wt = W S (Eq. update_HODLR).
template <typename T>
struct ChildUpd {
  const int* inv;   // parent position -> index in the child's update set (-1: none)
  int dense;
  const T* F;       // dense child
  int ld, npc;
  const FfNode* nodes;   // compressed child: ff cluster tree, root first
  const T* W;       // nf x rtop (bfloat16 bit patterns when wbf)
  const T* Wt;      // nf x rtop
  int nf, rtop, wbf;
};
template <typename T>
struct GatherFront {
  int start, npiv, nhat;
  const int* upd;   // I_p^f as new indices
  int nchild;
  ChildUpd<T> ch[2];
};
// out(r, c) = F_p(rows[r], cols[c]), r < nr, c < nc (front positions; a null
// list is the range r0.. / c0..); one workgroup per 256 entries from tile0
template <typename T>
struct GatherDesc {
  const int* rows;
  const int* cols;
  T* out;
  int r0, c0, nr, nc, ldo;
  int front;
  int tile0;
};
// dense parent, compressed child: parent(relmap[a], relmap[b]) += U_c(a, b)
// for a >= b (lower triangle; one workgroup per 64 x 64 tile)
template <typename T>
struct ExtAddCDesc {
  ChildUpd<T> c;
  T* parent;
  const int* relmap;
  int ldp, nfc;
  int tile0, tiles_r;
};

// Phase 2 on the sampled cross of a block of a front that is never assembled
// (skeleton adaptive mode 2; one workgroup of kCrossThreads per block):
// complete pivoting over the live residual entries in the BDLR rows I and
// columns J until the pivot-ratio rule holds there.  A pivot (i, j) appends
// the residual column E(:, j) to U and the residual row E(i, :) / E(i, j) to
// V; a column outside J or a row outside I is formed from the front's
// entries (front_value) minus U V^T.  EJ and EI hold E(:, J) and E(I, :)
// (set to B(:, J) - U V(J, :)^T and B(I, :) - U(I, :) V^T before the
// launch) and take every pivot's rank-1 update.
template <typename T>
struct CrossDesc {
  T* EJ;                 // nr x nJ, ld nr
  T* EI;                 // nI x nc, ld nI
  const int* Il;         // block-local rows of I, ascending
  const int* Jl;         // block-local columns of J, ascending
  const int* piv_r;      // phase-1 pivots, as indices into Il and Jl
  const int* piv_c;
  const int* rank1;      // phase-1 rank
  const double* u11;     // |first phase-1 pivot| (0: none)
  T* U;                  // nr x cap, ld nr (phase-1 columns first)
  T* V;                  // nc x cap, ld nc
  int* rank;             // final rank
  const GatherFront<T>* front;
  int r0, c0, nr, nc, nI, nJ, cap, pad;
};
constexpr int kCrossThreads = 1024;

// ---- launchers (all asynchronous on `st`; descriptor arrays are device) ----
// MFMA accumulator layout probe (one wave, 64 x 4 entries per output)
template <typename T>
void launch_mfma_probe(int* rows, int* cols, int* assumed, hipStream_t st);
template <typename T>
// tn = kTile: 64 x 64 output tiles; tn = kTileNarrow: 64 x 16 tiles, for
// problems of at most 16 columns (tiles_n of the descriptors counts tn-wide tiles)
void launch_gemm(const GemmDesc<T>* d, int ndesc, int tiles, hipStream_t st, int tn = kTile);
// reduction of split-K partial sums: d lists only split problems, with
// tile0/tiles_m describing this launch's 64 x 64 output tiles
template <typename T>
void launch_gemm_reduce(const GemmDesc<T>* d, int ndesc, int tiles, hipStream_t st);
// 64 x 16 tiles with folded split-K sources for B (f[i] belongs to d[i])
template <typename T>
void launch_gemm_fold(const GemmDesc<T>* d, const FoldDesc<T>* f, int ndesc, int tiles, hipStream_t st);
template <typename T>
void launch_potrf(const PotrfDesc<T>* d, int ndesc, int nmax, int* status, hipStream_t st);
// whole-block register skeleton: blocks up to skreg_full_rows<T>() x skreg_full_cols<T>()
template <typename T>
void launch_skreg_full(const SkRegDesc<T>* d, int ndesc, double eps, int adaptive, int* status, hipStream_t st);
// submatrix register skeleton (phase 1 on B_hat): |I|, |J| up to skreg_hat_max<T>()
template <typename T>
void launch_skreg_hat(const SkRegDesc<T>* d, int ndesc, double eps, int* status, hipStream_t st);
template <typename T>
constexpr int skreg_full_rows() { return sizeof(T) == 8 ? 128 : 256; }
template <typename T>
constexpr int skreg_full_cols() { return 256; }
template <typename T>
constexpr int skreg_hat_max() { return sizeof(T) == 8 ? 128 : 192; }
// skeleton factors: one workgroup of kSkelFacThreads per 64 rows of C~ or of
// R~ (its waves share each row's update sums); LDS holds the solved values
// (rmax x 64), one column block of the factor and the waves' partial sums
constexpr int kSkelFacRows = 64;
constexpr int kSkelFacBlock = 16;
constexpr int kSkelFacThreads = 256;
template <typename T>
constexpr size_t skelfac_lds(int rmax) {
  return ((size_t)rmax * (kSkelFacRows + kSkelFacBlock) +
          (size_t)(kSkelFacThreads / 64 - 1) * kSkelFacBlock * kSkelFacRows) * sizeof(T);
}
template <typename T>
void launch_skelfac(const SkelFacDesc<T>* d, int ndesc, int wgs, int rmax, hipStream_t st);
template <typename T>
void launch_phase2(const Phase2Desc<T>* d, int ndesc, int maxrc, double eps, int* status, hipStream_t st);
// Multi-workgroup phase 2.  phase2_coop_wcols: columns per workgroup whose
// slice (nr x wcols) fits a workgroup's LDS (0 when not even one column
// does); phase2_coop_lds: dynamic LDS bytes of a workgroup, with the slice in
// LDS or (slice_lds false) updated in place in the front; phase2_coop_capacity:
// workgroups that can be resident at once with that LDS (a launch must not
// exceed it).  A launch waits on the host for the device's previous one
// unless both are on one stream; a barrier wait longer than wait_ticks
// ticks of the device's constant-rate clock sets status bit 8 and ends the
// loop (wait_ticks < 0: every workgroup gives up at its first barrier, a
// test hook).  Returns the launch or wait error.
constexpr int kPhase2CoopLds = 78 * 1024;   // two workgroups fill a CU's 160 KB of LDS
// threads of a multi-workgroup phase-2 workgroup (more waves make the
// per-step barriers slower than they make the update faster), and the
// fewest columns per workgroup the host gives a block (one per wave)
constexpr int kCoopThreads = 256;
constexpr int kCoopMinCols = kCoopThreads / 64;
template <typename T>
int phase2_coop_wcols(int nr);
template <typename T>
size_t phase2_coop_lds(int nr, int wcols, bool slice_lds);
template <typename T>
int phase2_coop_capacity(size_t lds, bool slice_lds);
template <typename T>
hipError_t launch_phase2_coop(const Phase2CoopDesc<T>* d, int ndesc, int wgs, size_t lds, bool slice_lds,
                              double eps, int* status, long long wait_ticks, hipStream_t st);
template <typename T>
void launch_extadd(const ExtAddDesc<T>* d, int ndesc, int tiles, hipStream_t st);
// sampled extend-add: every GatherDesc entry; rowptr/colind/vals are A in
// the original order and perm maps new indices to original ones
template <typename T>
void launch_gather(const GatherDesc<T>* d, int ndesc, int tiles, const GatherFront<T>* fronts, const int* rowptr,
                   const int* colind, const double* vals, const int* perm, hipStream_t st);
template <typename T>
void launch_extadd_c(const ExtAddCDesc<T>* d, int ndesc, int tiles, hipStream_t st);
// status bits: 2 capacity, 16 non-finite pivot; LDS nr + nc bytes of the largest block
template <typename T>
void launch_cross(const CrossDesc<T>* d, int ndesc, int maxrc, double eps, const int* rowptr, const int* colind,
                  const double* vals, const int* perm, int* status, hipStream_t st);
template <typename S, typename D>
void launch_copy(const CopyDesc<S, D>* d, int ndesc, int tiles, hipStream_t st);
template <typename T>
void launch_cap(const CapDesc<T>* d, int ndesc, hipStream_t st);
// kernel variant (a prof.h kind) for matrices up to nmax
int gj_kind(int nmax);
void launch_gj_inverse(const InvDesc* d, int ndesc, int nmax, int* status, hipStream_t st);
template <typename T>
void launch_fill(T* p, int64_t n, T v, hipStream_t st);
// out[i] = max |p_i(r, c)| over the rows x cols matrix p_i (ld), one
// workgroup per matrix
struct MaxAbsDesc {
  const double* p;
  int rows, cols, ld, pad;
};
void launch_maxabs(const MaxAbsDesc* d, int ndesc, double* out, hipStream_t st);
// out[0..na+nb] = a[0..na), b[0..nb), *c; out may be pinned host memory
// (its device address)
void launch_readback(const int* a, int na, const int* b, int nb, const int* c, int* out, hipStream_t st);
// One front for the assembly of A's entries (F_bar_p, Eq. fbar): element
// offset of its buffer in the workspace, pivot range, leading dimension,
// height, and its update set upd[upd0 .. upd0 + nupd), sorted.
struct AsmFront {
  int64_t off;
  int start, npiv, ld, height, upd0, nupd;
};
// Destination of each entry k of A: dest[k] (element offset in the
// workspace) and lvl[k] (height of the front, -1 for upper entries).
// rowptr/colind: A's pattern (original order); iperm: new index of each
// original index; owner: front of each new index.
void launch_asm_map(const int* rowptr, const int* colind, const int* iperm, const int* owner, const AsmFront* fr,
                    const int* upd, int n, int64_t* dest, signed char* lvl, hipStream_t st);
// ws[dest[k]] = vals[k] for every entry with lvl[k] == h
template <typename T>
void launch_assemble(T* ws, const int64_t* dest, const signed char* lvl, const double* vals, int64_t nnz, int h,
                     hipStream_t st);
template <typename T>
void launch_vec_asm(const VecAsmDesc<T>* d, int ndesc, int nrhs, hipStream_t st);
template <typename T>
void launch_perm_in(const double* r, T* xn, const int* perm, int N, int nrhs, hipStream_t st);
template <typename T>
void launch_perm_out(const T* xn, double* z, const int* iperm, int N, int nrhs, hipStream_t st);

// Per-column row windows (`win`, device int32[2 * nrhs] or null for all
// rows): column k of an n x nrhs block uses rows [win[2k], win[2k+1]) only.
// Independent systems solved together keep each system's right-hand sides in
// their own columns, zero outside its rows; the kernels below then read and
// write only those rows of each column (rows outside a window are left as
// they are and never read for that column's results).
// float64 CSR SpMV, column-major n x nrhs; y = alpha*A*x + beta*y
void launch_spmv(const int* rowptr, const int* colind, const double* vals, const double* x,
                 double* y, int n, int nrhs, double alpha, double beta, hipStream_t st,
                 const int* win = nullptr);
// dots[i*nrhs + k] (+)= <X_i(:,k), w(:,k)> for i < nv; X_i = X + i*ld*nrhs...
// `partial` holds mdot_chunks(nrhs) * nv * nrhs doubles: the row range is cut
// into that many chunks per right-hand side (more for few right-hand sides,
// so that one launch still spreads over the whole chip)
inline int mdot_chunks(int nrhs) { return nrhs >= 16 ? 64 : nrhs >= 2 ? 1024 / nrhs : 512; }
void launch_mdot(const double* X, int64_t xstride, int nv, const double* w, int n, int nrhs,
                 double* partial, double* out, int accumulate, hipStream_t st, const int* win = nullptr);
void launch_maxpy(const double* X, int64_t xstride, int nv, const double* coef, double* w, int n,
                  int nrhs, double sign, hipStream_t st, const int* win = nullptr);
void launch_scale_cols(const double* w, double* v, const double* norms, int n, int nrhs,
                       hipStream_t st, const int* win = nullptr);
void launch_xupdate(const double* Z, int64_t zstride, int nv, const double* y, double* x, int n,
                    int nrhs, hipStream_t st, const int* win = nullptr);
void launch_axpby(const double* a, const double* b, double* c, double alpha, double beta, int64_t n,
                  hipStream_t st);
// conjugate-gradient updates per column k (act[k] == 0: zero step):
// x += alpha p, rprev = r, r -= alpha q with alpha_k = rz_k / pq_k
void launch_cg_xr(double* x, double* r, double* rprev, const double* p, const double* q, const double* rz,
                  const double* pq, const int* act, int n, int nrhs, hipStream_t st);
// p = z + beta p with beta_k = (rzn_k - rzo_k) / rz_k
void launch_cg_p(double* p, const double* z, const double* rzn, const double* rzo, const double* rz, const int* act,
                 int n, int nrhs, hipStream_t st);

}  // namespace mfh
