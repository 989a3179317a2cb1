/*
 * mfh_testing.h -- kernel-level test hooks of libmfh (not part of the
 * solver API).  Each hook runs one batched kernel of the library on a single
 * problem so that tests can compare it with a plain reference.  All pointers
 * are device pointers; `precision` is MF_FP64 (double data) or MF_FP32
 * (float data); calls are synchronous and return an mf_status.
 */
#ifndef MFH_TESTING_H
#define MFH_TESTING_H

#include "mfh.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Lane layout of the 16x16x4 MFMA accumulator: for lane l and value v,
 * rows[4l+v] / cols[4l+v] are the output row / column that value holds and
 * assumed[4l+v] the row the GEMM epilogue assumes (host int32[256] each). */
mf_status mfh_test_mfma_layout(int32_t precision, int32_t* rows, int32_t* cols, int32_t* assumed);

/* C = alpha * op(A) * op(B) + beta * C through the grouped MFMA GEMM;
 * flags as the library's GemmFlags (1 lower-only C, 2/4 op(A) lower/upper,
 * 8/16 op(B) lower/upper triangular).  kchunk > 0 splits k into ranges of
 * kchunk (a multiple of 64; MF_EINVAL otherwise), summed by the separate
 * reduction kernel; 0 runs one workgroup per output tile. */
mf_status mfh_test_gemm(int32_t precision, int32_t m, int32_t n, int32_t k, const void* A, int32_t lda,
                        int32_t opA, const void* B, int32_t ldb, int32_t opB, void* C, int32_t ldc,
                        double alpha, double beta, int32_t flags, int32_t kchunk);

/* The same product with row maps on the stored arrays (device int32, or
 * NULL): stored row s of A is read as row arow[s] (rows of op(A) when
 * opA == 0, its columns when opA == 1), likewise brow for B.  The apply
 * reads x(I_p^f) through brow; the sampled skeleton reads the sampled rows
 * of its bases through them. */
mf_status mfh_test_gemm_rows(int32_t precision, int32_t m, int32_t n, int32_t k, const void* A, int32_t lda,
                             int32_t opA, const int32_t* arow, const void* B, int32_t ldb, int32_t opB,
                             const int32_t* brow, void* C, int32_t ldc, double alpha, double beta, int32_t kchunk);

/* C = alpha * op(A) * Bf + beta * C (n <= 16, slices[s] <= 8) where Bf
 * is B as a product that folds a split-K reduction reads it: rows [0, bsplit) of Bf from
 * source 0, rows [bsplit, k) from source 1.  Source s with slices[s] > 0
 * gives Bf(i, j) = coef[2s] * sum_q part_s[i' + j*ld[s] + q*ld[s]*n]
 * + coef[2s+1] * B(i, j), with i' the row inside the source and the slices
 * summed in order q = 0, 1, ...; a source with slices[s] == 0 reads B.
 * part0/part1 are device arrays of slices[s] * ld[s] * n elements (ld[s] at
 * least the source's row count); slices, ld and coef are host arrays of 2,
 * 2 and 4 entries.  kchunk as for mfh_test_gemm.  The apply reads the
 * split outputs of h_p, q and z this way. */
mf_status mfh_test_gemm_fold(int32_t precision, int32_t m, int32_t n, int32_t k, const void* A, int32_t lda,
                             int32_t opA, const void* B, int32_t ldb, void* C, int32_t ldc, double alpha,
                             double beta, int32_t kchunk, int32_t bsplit, const void* part0, const void* part1,
                             const int32_t* slices, const int32_t* ld, const double* coef);

/* In-place Cholesky of the n x n lower triangle of A (n <= 128) and the
 * explicit inverse of the factor into Inv (full square, zeros above).
 * *status_out receives the kernel's status word (1: non-positive pivot). */
mf_status mfh_test_potrf(int32_t precision, int32_t n, void* A, int32_t lda, void* Inv, int32_t ldi,
                         int32_t* status_out);

/* Skeleton compression (Sec. 2.2, Eq. Bhat) of the block
 * F(r0:r0+nr, c0:c0+nc) of an ld-strided matrix F from BDLR row/column
 * sets I, J (device int32, positions in F; at most 128 (FP64) / 192 (FP32)
 * entries each).  U (nr x cap) and V (nc x cap) receive C~ and R~^T.
 * adaptive: 0 = pivoting on B(I, J) only; 1 = then continue over the whole
 * block, with the block spread over several workgroups when it is larger
 * than one workgroup's registers and a column slice fits LDS; 2 = as 1 but
 * with one workgroup streaming the block; 3 = as 1 with workgroups of at
 * most 4 columns updating the block in place.  The block of F may be
 * overwritten by a residual.  *rank_out receives the final rank.  Returns
 * MF_ENOTSPD when a chosen pivot is not finite (the kernels stop there). */
mf_status mfh_test_skeleton(int32_t precision, void* F, int32_t ld, int32_t r0, int32_t nr, int32_t c0,
                            int32_t nc, const int32_t* I, int32_t nI, const int32_t* J, int32_t nJ, double eps,
                            int32_t adaptive, int32_t cap, void* U, void* V, int32_t* rank_out);

/* In-place inverse of the n x n float64 matrix A (column-major, leading
 * dimension lda >= n, 1 <= n <= 1024) by Gauss-Jordan elimination with
 * partial pivoting: the kernel the capacitance inverse M = (I - A B)^{-1}
 * of the SMW factorization (Sec. 2.1) runs on.  *status_out receives the
 * kernel's status word (4: a zero pivot column). */
mf_status mfh_test_inverse(int32_t n, double* A, int32_t lda, int32_t* status_out);

/* Truncation error of every compressed block (Sec. 2.2: the pivot-ratio
 * rule at eps).  While on, factorisations with assembled fronts keep a
 * float64 copy of each block before compression and, once its rank is
 * known, measure max|B| and max|B - U V^T| in float64 with the bases as
 * computed (before any bfloat16 rounding).  Debug cost: one float64 copy of
 * a level's blocks and a device synchronisation per level. */
mf_status mfh_test_record_block_errors(int32_t on);
/* The recorded errors of a factor, 6 doubles per block in level order:
 * front, block (index in the front's block list), rank, max|B|, |u_11|
 * (the first pivot), max|B - U V^T|.  *count receives the number of blocks;
 * at most cap are written. */
mf_status mfh_test_block_errors(const mf_numeric_t* f, double* out, int64_t cap, int64_t* count);

/* Barrier wait of the multi-workgroup phase 2 (Sec. 2.2 compression spread
 * over workgroups) for every later factorisation in the process, in ticks
 * of the device's constant-rate clock: 0 restores the default (two
 * seconds); a negative value makes every workgroup give up at its first
 * barrier, so mf_factor must end with MF_EHIP while every kernel exits
 * normally.  Host only; takes effect at the next phase-2 launch. */
mf_status mfh_test_phase2_wait(int64_t ticks);

#ifdef __cplusplus
}
#endif
#endif /* MFH_TESTING_H */
