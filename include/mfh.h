/*
 * mfh.h -- C ABI of the HODLR-accelerated multifrontal solver (gfx950).
 *
 * Solves A x = b for a sparse symmetric positive definite finite-element
 * stiffness matrix A (Sec. 1 of Aminfar & Darve, "A Fast and Memory Efficient
 * Sparse Solver with Applications to Finite-Element Matrices"): a
 * low-accuracy multifrontal factorisation whose large frontal matrices are
 * HODLR-compressed (Sec. 4.2) is used as the preconditioner of GMRES
 * (Sec. 3).  A plain dense-front multifrontal factorisation (Sec. 4.1) is
 * available through the same calls for comparison.
 *
 * Conventions
 *  - No torch types cross this boundary: plain host or device pointers and
 *    sizes.  "host" pointers are read during the call and may be freed after
 *    it returns; "device" pointers are borrowed, must stay valid until the
 *    work enqueued on the given stream has finished, and are never freed by
 *    the library.
 *  - Handles are owned by the library and released by the matching *_free.
 *    A numeric handle keeps a reference to the data it needs from its
 *    symbolic handle; the symbolic handle must outlive it.
 *  - Every call returns an mf_status; on a non-OK status mf_last_error()
 *    returns a message for the calling thread.  No exception crosses the ABI.
 *  - One handle is used from one thread/stream at a time; distinct handles
 *    may be used concurrently.
 *  - Multi right-hand-side vectors are column-major n x nrhs float64 arrays
 *    (column k starts at k*n), in the caller's original unknown ordering.
 *  - Streams: a hipStream_t passed as void*; NULL means the null stream.
 *    Streams are used at their default priority.
 */
#ifndef MFH_H
#define MFH_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MF_OK = 0,
  MF_EINVAL = 1,      /* malformed argument (CSR, sizes, options)            */
  MF_ENOMEM = 2,      /* device or host allocation failed                    */
  MF_EBUDGET = 3,     /* a request's estimated bytes exceed the whole device  */
  MF_ENOTSPD = 4,     /* a Cholesky pivot was not positive                   */
  MF_ENOCONV = 5,     /* GMRES hit maxit before reaching tol                 */
  MF_ECAPACITY = 6,   /* a block rank exceeded the configured rank capacity  */
  MF_EHIP = 7,        /* a HIP runtime call failed                           */
  MF_ESTATE = 8       /* call not valid for this handle (e.g. no GPU)        */
} mf_status;

typedef struct mf_symbolic_s mf_symbolic_t;   /* opaque */
typedef struct mf_numeric_s mf_numeric_t;     /* opaque */

/* arithmetic of the factor and of the preconditioner apply */
enum { MF_FP64 = 0, MF_FP32 = 1 };
/* factorisation method */
enum { MF_METHOD_HODLR = 0, MF_METHOD_DENSE = 1 };

typedef struct {
  int32_t method;       /* MF_METHOD_HODLR (Sec. 4.2) or MF_METHOD_DENSE (Sec. 4.1) */
  int32_t precision;    /* MF_FP64 or MF_FP32 (factors and apply)                   */
  int32_t n_c;          /* HODLR only: fronts with n_p + n_f < n_c are dense (Table 1 "n_c") */
  int32_t bdlr_depth;   /* BDLR depth d (Sec. 2.2, Table 1 "d"); < 0: every row/column    */
  int32_t bdlr_cap;     /* at most this many BDLR rows (and columns) per block; 0: the most */
                        /* the pivot kernel takes (128 float64, 192 float32)                */
  int32_t adaptive;     /* phase 2 of the skeleton (Sec. 2.2), after the pivoting on B(I, J):
                           0: none (the paper's scheme);
                           1: complete pivoting continues over the whole block until the
                              pivot-ratio rule holds there (max-norm error < eps*|u_11|);
                           2 (sampled = 1 only): it continues over the sampled cross, the
                              residual rows I and columns J, until the rule holds there;
                              each extra pivot forms one more row and column of the front */
  int32_t rank_cap;     /* capacity per block rank (a block's capacity is the larger of this
                           and its phase-1 bound min(|I|, |J|)); exceeding it -> MF_ECAPACITY */
  int32_t uv_bf16;      /* HODLR + FP32 only: round the compressed bases U, V (and the F_fp
                           basis W) to bfloat16 right after compression and keep them in
                           bfloat16; the factorisation and the apply both use the rounded
                           values, so the preconditioner is that of the rounded matrix     */
  int32_t apply_graph;  /* k >= 1 (default 4): the k-th preconditioner apply (Sec. 4.1.2)
                           with a given right-hand-side count records its kernel sequence
                           as a HIP graph, and it and every later apply with that count
                           replay it; earlier applies launch each kernel (recording costs
                           about as much as a few applies).  0: never record.  At most
                           2^20.  A timing session (mf_prof_start) times the direct
                           applies' launches; the graph is recorded untimed, so its
                           replays run as they would without the session.             */
  int32_t sampled;      /* HODLR only, 1: the sampled extend-add of Sec. 4.2.1 (Eq. HODLR_EA_Expand):
                           compressed fronts are never staged densely; only the BDLR rows
                           and columns of each block and the diagonal leaves are formed, from
                           A's entries, dense children's updates and compressed children's
                           F_ff^HODLR - Wt W^T, and compression uses those samples alone, so
                           it needs adaptive 0 (the paper's scheme) or 2.  0: every front is
                           staged densely and children's updates are scatter-added whole   */
  int32_t apply_split_chunk;   /* launch shape of the apply's GEMMs (Sec. 4.1.2), tuned per
                                  workload: the smallest k range one split-K workgroup sums, a
                                  multiple of 64 in [64, 4096]; 0: 128                        */
  int32_t apply_split_target;  /* workgroups one such launch aims for by splitting k, in
                                  [1, 65536]; 0: 1024 for right-hand-side tiles (at most 16
                                  right-hand sides), 512 for wider ones.  Both change only the
                                  order of the partial sums                                   */
  double eps;           /* low-rank tolerance (Sec. 2.2: stop when |u_r+1,r+1/u_11| < eps) */
  void* stream;         /* hipStream_t, borrowed; NULL = null stream                      */
} mf_opts;

typedef struct {
  int32_t restart;      /* Krylov dimension m of GMRES(m); default 30      */
  int32_t maxit;        /* total iterations per right-hand side; default 4000 */
  void* stream;         /* hipStream_t, borrowed; NULL = null stream       */
} mf_gmres_opts;

typedef struct {
  int32_t iters;        /* GMRES iterations spent on this right-hand side   */
  int32_t converged;    /* 1 if ||b - A x||_2 <= tol ||b||_2                 */
  double relres;        /* final true relative residual                      */
} mf_gmres_info;

typedef struct {
  int64_t n, nnz, nfronts, nlevels, max_front, max_npiv;
} mf_symbolic_info;

typedef struct {
  int64_t persistent_bytes;   /* factor bytes kept for the apply (all device arrays of the factor) */
  int64_t peak_bytes;         /* peak device bytes held by the library during mf_factor             */
  int64_t workspace_bytes;    /* front workspace (dense staging) part of the peak                   */
  int64_t nblocks;            /* compressed off-diagonal blocks                                      */
  int64_t rank_sum;           /* sum of block ranks                                                  */
  int32_t rank_max;
  int32_t dense_fronts;       /* fronts factored densely                                             */
  int32_t hodlr_fronts;
  int32_t status_bits;        /* device status word (1: non-positive pivot, 2: rank capacity,
                                 4: singular capacitance, 16: non-finite block entry)                */
  double factor_seconds;      /* wall time of mf_factor (host clock, synchronised)                   */
  int64_t resident_bytes;     /* device bytes the handle holds now: factor, copy of A, apply and
                                 GMRES workspaces                                                    */
} mf_factor_info;

/* Fill *o with defaults: HODLR, FP32, n_c 0, d -1 (no depth limit), cap 0
 * (the pivot kernel's maximum), adaptive 1, rank_cap 512, eps 1e-4, null
 * stream. */
mf_status mf_opts_default(mf_opts* o);
mf_status mf_gmres_opts_default(mf_gmres_opts* o);

/*
 * Symbolic analysis (Sec. 4.1.1): nested-dissection ordering by coordinate
 * median vertex separators, elimination tree, pivot sets I_p (contiguous in
 * the new order), coupling sets S_p (Eq. couplingSet), frontal sets I_p^f,
 * relative extend-add maps, the map of A's lower entries into fronts, HODLR
 * cluster trees of every front.  Host-only integer work: needs no GPU.
 *   n        number of unknowns (>= 1)
 *   rowptr   host int32[n+1], colind host int32[rowptr[n]]: full symmetric
 *            pattern of A, columns sorted and unique within each row,
 *            diagonal present.  Explicit zeros count as structure.
 *   coords   host float64[n*dim] (row-major: node i at coords[i*dim..]),
 *            positions used by the separator rule; dim in 1..3
 *   leaf     nested-dissection leaf size, also the HODLR leaf size (>= 1)
 * Errors: MF_EINVAL for a malformed pattern (unsorted, out of range,
 * duplicate, missing diagonal, asymmetric), MF_ENOMEM.
 */
mf_status mf_analyze(int32_t n, const int32_t* rowptr, const int32_t* colind,
                     const double* coords, int32_t dim, int32_t leaf,
                     mf_symbolic_t** out);
mf_status mf_symbolic_get_info(const mf_symbolic_t* s, mf_symbolic_info* info);

/*
 * Analysis of the block-diagonal matrix diag(A_1, ..., A_k) from the
 * analyses of A_1, ..., A_k, for factoring independent systems together:
 * the elimination forest is the disjoint union of the parts' trees and the
 * fronts of every part at one height share an etree level, so one
 * factorisation and one apply process all parts' fronts of a level in the
 * same launches (Sec. 4.1: fronts of one level are independent).
 *   parts    host array of `count` (>= 1) analysis handles, all with the
 *            same leaf size and dimension; read only, still owned by the
 *            caller (they may be freed after the call)
 *   out      receives a new handle (free with mf_symbolic_free)
 * Layout of the merged system: rows of part i follow those of parts
 * 0..i-1 (offset n_0 + ... + n_{i-1}); its CSR pattern is the parts'
 * patterns in that order, so its values for mf_factor are the parts' value
 * arrays concatenated.  Fronts and blocks are numbered part by part (the
 * exports and mf_factor_ranks list part 0's first).  The merged order and
 * fronts are the parts' own, shifted: factoring the merged system gives
 * every part the ranks it gets alone.
 * Errors: MF_EINVAL for count < 1, a null handle, differing leaf size or
 * dimension, or more than 2^31 - 1 unknowns or entries in total.
 */
mf_status mf_symbolic_merge(const mf_symbolic_t* const* parts, int32_t count, mf_symbolic_t** out);

/*
 * Read-only export of the analysis, for bit-exact comparison.  `what`
 * selects an int32 array (codes below); if buf is NULL or cap is too small,
 * only *len is set.  BDLR sets (Sec. 2.2) need mf_symbolic_bdlr first.
 */
enum {
  MF_EXP_PERM = 0,        /* perm[new] = old                                   */
  MF_EXP_FRONT = 1,       /* per front: start, npiv, nf, parent, height, nchild */
  MF_EXP_UPD = 2,         /* concatenated I_p^f lists (new indices)            */
  MF_EXP_UPD_PTR = 3,     /* nfronts+1 offsets into MF_EXP_UPD                  */
  MF_EXP_RELMAP = 4,      /* concatenated relative maps (same offsets as UPD)  */
  MF_EXP_ASM = 5,         /* per lower entry: front, row, col, csr index       */
  MF_EXP_BLOCKS = 6,      /* per block: front, kind(0 top,1 pp,2 ff), r0, nr, c0, nc, level */
  MF_EXP_BDLR_I = 7,      /* concatenated BDLR row sets (front positions)       */
  MF_EXP_BDLR_IPTR = 8,   /* nblocks+1 offsets                                  */
  MF_EXP_BDLR_J = 9,
  MF_EXP_BDLR_JPTR = 10
};
mf_status mf_symbolic_export(const mf_symbolic_t* s, int32_t what, int32_t* buf,
                             int64_t cap, int64_t* len);
/* Compute (and cache in the handle) the BDLR sets of every block for depth d
 * (< 0: all) and set-size cap (>= 1).  Host-only. */
mf_status mf_symbolic_bdlr(mf_symbolic_t* s, int32_t depth, int32_t cap);
void mf_symbolic_free(mf_symbolic_t* s);

/*
 * Numeric factorisation on the current HIP device.
 *   vals   host float64[nnz]: A's values in the CSR order given to mf_analyze
 *   eps    low-rank tolerance (overrides opts->eps); ignored for DENSE
 *   leaf   HODLR leaf size; 0 or the analysis leaf (one value serves both)
 *   opts   nullable (defaults)
 * HODLR (Sec. 4.2): each front F_p = F_bar_p (+) children's updates is
 * staged in device memory; fronts with n_p + n_f >= n_c are compressed
 * (F_fp ~= W V^T, F_pp and F_ff HODLR, Sec. 2.1) by the BDLR skeleton
 * (Sec. 2.2, Eq. Bhat), F_pp is factored by recursive Sherman-Morrison-
 * Woodbury, and U_p = F_ff^HODLR - W S W^T with S = V^T F_pp^{-1} V
 * (Eq. update_HODLR_Parent) goes to the parent.  DENSE (Sec. 4.1): Cholesky
 * of F_pp and U_p = F_ff - F_fp F_pp^{-1} F_pf (Eq. update).
 * Synchronous: returns after the factor is complete.
 * Errors: MF_EINVAL, MF_ENOMEM, MF_ENOTSPD, MF_ECAPACITY, MF_EHIP,
 * MF_ESTATE (no GPU).
 */
mf_status mf_factor(const mf_symbolic_t* s, const double* vals, double eps,
                    int32_t leaf, const mf_opts* opts, mf_numeric_t** out);
mf_status mf_factor_get_info(const mf_numeric_t* f, mf_factor_info* info);
/* Per-block ranks of the factor in MF_EXP_BLOCKS order (-1 for blocks of
 * dense fronts); buf NULL -> only *len. */
mf_status mf_factor_ranks(const mf_numeric_t* f, int32_t* buf, int64_t cap, int64_t* len);
void mf_factor_free(mf_numeric_t* f);

/*
 * Preconditioner apply z = M^{-1} r: the multifrontal upward pass
 * (Eq. upward) and downward pass (Eq. downward) with F_pp^{-1} replaced by
 * the HODLR solve for compressed fronts (Sec. 4.2.2).
 *   r, z   device float64[n*nrhs], column-major, original ordering; may not alias
 *   stream hipStream_t or NULL; asynchronous
 */
mf_status mf_apply(mf_numeric_t* f, int32_t nrhs, const double* r, double* z, void* stream);

/*
 * Preconditioner apply that allocates nothing, for callers that cannot
 * allocate device memory (serving loops, harnesses that forbid hipMalloc,
 * code recorded into a HIP graph once the handle and nrhs have been used
 * before capture).  Same z = M^{-1} r, same kernels, same split-K choices as
 * mf_apply (the results are equal bit for bit); its workspace, split-K
 * partial sums and step descriptors live in one static device array of
 * MF_APPLY_SCRATCH_BYTES that each GPU the library runs on keeps until the
 * process ends.  No hipMalloc, hipFree or allocating library call is made.
 *   r, z    device float64[n*nrhs], column-major, original ordering; may not alias
 *   stream  hipStream_t or NULL; asynchronous once the descriptors are in place
 * Every call on a GPU shares that GPU's array, which keeps the last call's
 * contents: when it last held another handle's plan or another nrhs, the
 * call uploads the descriptors again (host planning and a copy that waits on
 * `stream`).  Nothing in the array needs clearing: every entry a call reads
 * it has written first.  Calls that overlap on one GPU (two streams or
 * threads without synchronisation between them) race: order them.  The
 * call does not register its stream with the handle: synchronise the stream
 * before mf_factor_free.
 * Errors: MF_EINVAL when the workspace for nrhs columns plus the split-K
 * area and descriptors exceed MF_APPLY_SCRATCH_BYTES (use mf_apply, or fewer
 * right-hand sides per call); MF_ESTATE when the factor's device is not the
 * current device.
 */
#define MF_APPLY_SCRATCH_BYTES (64ull << 20)
mf_status mf_apply_noalloc(mf_numeric_t* f, int32_t nrhs, const double* r, double* z, void* stream);

/*
 * Right-preconditioned flexible GMRES(m) with M = the factor (Sec. 3):
 * x0 = 0, classical Gram-Schmidt with reorthogonalisation in float64, stop
 * when ||b - A x||_2 <= tol ||b||_2 (true residual, float64 SpMV with A) for
 * every right-hand side.
 *   b, x   device float64[n*nrhs], column-major, original ordering
 *   info   host array of nrhs entries (may be NULL)
 * Synchronous.  Returns MF_ENOCONV (x = last iterate, info filled) when a
 * right-hand side does not converge within maxit.
 */
mf_status gmres_solve(mf_numeric_t* f, int32_t nrhs, const double* b, double* x,
                      double tol, const mf_gmres_opts* opts, mf_gmres_info* info);

/*
 * Preconditioned conjugate gradients with M = the factor (Sec. 3: the
 * multifrontal preconditioner serves any Krylov solver, conjugate gradients
 * among them).  A is SPD and the factor is a symmetric approximation of it;
 * CG needs that approximation positive definite, which a loose eps may not
 * give (gmres_solve has no such need).  x0 = 0; flexible beta
 * <z_k+1, r_k+1 - r_k> / <z_k, r_k>, since the reduced-precision apply is
 * not an exactly fixed linear operator; per right-hand side: stop when the
 * recursive residual meets tol, then check the true residual
 * ||b - A x||_2 <= tol ||b||_2 (float64 SpMV with A) and start again from x
 * when it misses.  No Krylov basis is stored: five n x nrhs float64 vectors.
 *   b, x   device float64[n*nrhs], column-major, original ordering
 *   info   host array of nrhs entries (may be NULL): iterations, converged,
 *          final true relative residual
 * Synchronous.  Returns MF_ENOCONV (x = last iterate, info filled) when a
 * right-hand side does not converge within maxit.
 */
typedef struct {
  int32_t maxit;        /* iterations per right-hand side; default 4000 */
  int32_t reserved;     /* must be 0 */
  void* stream;         /* hipStream_t, borrowed; NULL = null stream */
} mf_pcg_opts;
mf_status mf_pcg_opts_default(mf_pcg_opts* o);
mf_status pcg_solve(mf_numeric_t* f, int32_t nrhs, const double* b, double* x, double tol,
                    const mf_pcg_opts* opts, mf_gmres_info* info);

/*
 * Direct solve with the factor (Conclusion: at high accuracy the solver is a
 * standalone direct solver, not only a preconditioner): x = M^{-1} b, then
 * `refine` steps of iterative refinement x += M^{-1} (b - A x), the residual
 * in float64.  Build the factor with a small eps (and MF_FP64) for this use.
 *   b, x    device float64[n*nrhs], column-major, original ordering; may not alias
 *   refine  refinement steps, 0..64
 *   info    host array of nrhs entries (may be NULL): iters = refine,
 *           converged = 1, relres = final ||b - A x||_2 / ||b||_2
 * Synchronous.
 */
mf_status mf_direct_solve(mf_numeric_t* f, int32_t nrhs, const double* b, double* x, int32_t refine,
                          void* stream, mf_gmres_info* info);

/* y = A x with the factor's device copy of A (float64 CSR), column-major
 * n x nrhs device arrays; asynchronous on stream. */
mf_status mf_spmv(mf_numeric_t* f, int32_t nrhs, const double* x, double* y, void* stream);

/*
 * Device bytes of a factorisation with these options, before running it:
 * *peak = most held during mf_factor, *persistent = what the handle then
 * keeps, including apply and GMRES(restart) workspaces for nrhs right-hand
 * sides.  Exact for the front workspace, dense fronts and fixed buffers; the
 * HODLR part bounds each block rank by min(rows, cols, rank_cap,
 * 8 sqrt(max(rows, cols))) (ranks grow like sqrt(n), Sec. 1).  Host only.
 */
mf_status mf_estimate_bytes(const mf_symbolic_t* sym, const mf_opts* opts, int32_t nrhs, int32_t restart,
                            int64_t* persistent, int64_t* peak);

/*
 * Serving: a request server that factors and solves independent systems as
 * they arrive, several at once on the device (continuous batching).
 *  - mf_server_submit analyses the request on the caller's thread (copying
 *    every input) and queues it with its mf_estimate_bytes peak.
 *  - `slots` worker threads, each with its own HIP stream (default
 *    priority), take queued requests in arrival order as soon as the head
 *    request's estimated peak fits the memory budget next to the requests
 *    running and the factors kept resident; their factorisations and solves
 *    overlap on the device.  A request larger than the whole budget runs
 *    when nothing else holds memory; one whose estimate exceeds the device's
 *    total memory is refused at submit with MF_EBUDGET.  A factor serves one
 *    solve at a time: a resolve waits while another solve of the same factor
 *    runs, and requests queued behind it may start first.  Resident factors that no request is
 *    using are dropped, least recently used first, when memory is needed.
 *  - With merge > 1 (and no keep_factors), a slot that admits a request
 *    also takes the requests queued right behind it, in arrival order, up to
 *    `merge` requests and 16 right-hand sides in all, while their summed
 *    estimates (plus the merged solve's vectors) fit the budget.  It factors
 *    them as one block-diagonal system (mf_symbolic_merge: fronts of every
 *    request at one etree level share the level's launches) and solves them
 *    with one GMRES call in which each request's right-hand sides are their
 *    own columns, zero outside its rows: every column's iteration is the one
 *    it has alone, and each request gets its own x, status and iteration
 *    counts (the factor and solve times are the group's).  If the merged
 *    factorisation fails for a reason one request can cause (MF_ENOTSPD,
 *    MF_ECAPACITY, MF_EINVAL), each request of the group is factored and
 *    solved alone instead, so only the faulty one reports the error.
 *  - With keep_factors, a request's factor stays on the device after its
 *    solve; mf_server_resolve queues another solve with it (repeated
 *    right-hand sides) until mf_server_release.
 *  - mf_server_wait blocks until a request is done, copies x (host,
 *    n x nrhs column-major, original ordering) and fills its timings.
 * Handles of one server may be used from any thread.
 */
typedef struct mf_server_s mf_server_t;
typedef struct {
  int32_t slots;          /* requests on the device at once                                   */
  int32_t leaf;           /* nested-dissection and HODLR leaf size                            */
  int64_t mem_budget;     /* device bytes for running requests and resident factors;
                             0 = 80% of the free device memory when the server starts       */
  double tol;             /* GMRES tolerance (relative residual)                              */
  mf_opts factor;         /* factorisation options (stream ignored)                           */
  mf_gmres_opts gmres;    /* GMRES options (stream ignored)                                   */
  int32_t keep_factors;   /* 1: keep each factor resident for mf_server_resolve               */
  int32_t merge;          /* 1..16: most queued requests a slot factors and solves together
                             (1: one at a time; ignored with keep_factors)                   */
} mf_server_opts;

typedef struct {
  int32_t status;         /* mf_status of the request                                          */
  int32_t iters_max;      /* largest GMRES iteration count over its right-hand sides           */
  double relres_max;      /* largest final relative residual                                   */
  double t_queue;         /* seconds from submit to admission                                  */
  double t_analyze;       /* symbolic analysis (at submit)                                     */
  double t_factor;        /* numeric factorisation (0 for a resolve)                           */
  double t_solve;         /* GMRES, including copies of b and x                                */
  double t_total;         /* submit to done                                                    */
  int64_t est_bytes;      /* estimated peak used for admission                                 */
  int64_t peak_bytes;     /* peak device bytes of its factorisation                            */
  int64_t resident_bytes; /* device bytes its factor keeps (if resident)                       */
  int32_t group_size;     /* requests factored and solved together with it (itself included)   */
  int32_t reserved;
} mf_request_info;

mf_status mf_server_opts_default(mf_server_opts* o);
mf_status mf_server_create(const mf_server_opts* o, mf_server_t** out);
mf_status mf_server_submit(mf_server_t* sv, int32_t n, const int32_t* rowptr, const int32_t* colind,
                           const double* vals, const double* coords, int32_t dim, int32_t nrhs,
                           const double* b, int64_t* ticket);
mf_status mf_server_resolve(mf_server_t* sv, int64_t factor_ticket, int32_t nrhs, const double* b,
                            int64_t* ticket);
mf_status mf_server_wait(mf_server_t* sv, int64_t ticket, double* x, mf_request_info* info);
mf_status mf_server_release(mf_server_t* sv, int64_t factor_ticket);
/* Bytes the server accounts now (running estimates + resident factors) and its budget. */
mf_status mf_server_memory(mf_server_t* sv, int64_t* in_use, int64_t* budget);
void mf_server_destroy(mf_server_t* sv);

/*
 * Kernel timing for roofline reports (process-wide, all handles).
 * mf_prof_start(names): from now on, every launch of the named device
 * kernels (semicolon-separated trace names such as "gemm_kernel<float>" or
 * "skreg_kernel<float, 3, 24, false, 512>"; NULL or "" = all timed kernels)
 * is timed and the host adds up the launch's algorithmic work (flops; bytes
 * that the operation must move at least once).  Each timed launch gets start
 * and end events stamped by the runtime at the kernel's own start and end
 * (the dispatch interval a kernel trace reports); the events cost launch
 * throughput, so time throughput outside a session.  mf_prof_stop waits for the
 * work, writes one mf_kstat per kernel that ran (at most cap; *n = count)
 * and stops timing.
 */
typedef struct {
  char name[64];        /* device kernel name as it appears in a kernel trace */
  int64_t launches;
  double seconds;       /* sum of event-measured launch durations */
  double flops;         /* algorithmic floating-point operations, all launches */
  double bytes;         /* algorithmic bytes moved, all launches */
} mf_kstat;
mf_status mf_prof_start(const char* names);
mf_status mf_prof_stop(mf_kstat* out, int32_t cap, int32_t* n);

const char* mf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MFH_H */
