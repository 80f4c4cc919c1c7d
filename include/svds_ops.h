/*
 * svds_ops.h -- single steps of the truncated-SVD hot path, exposed through
 * the same C ABI conventions as svds.h (device pointers, caller-owned
 * buffers, integer return codes, synchronous on `stream`).  They run the very
 * kernels the solver runs, so each step can be checked and timed alone.
 */
#ifndef SVDS_OPS_H
#define SVDS_OPS_H

#include <stdint.h>
#include "svds.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Mat-vec of Alg. 1 steps 2/5/7 with the fused Lanczos term:
 *   y = x_scale * (A x) - coef * yprev
 * x (A->n), yprev and y (A->m) are device vectors of `basis_dtype`
 * (SVDS_F64 or SVDS_F32; A's values F64 or F32 are widened to it).
 * x_scale and coef are DEVICE pointers to one double each, or NULL
 * (x_scale NULL = 1, coef NULL = no yprev term).  For A^T x pass the CSR of
 * A^T (see svds_op_csc_build).  EINVAL on null pointers or bad row_ptr. */
int svds_op_spmv_csr(const svds_csr *A, const void *x, const double *x_scale, const double *coef,
                     const void *yprev, void *y, int32_t basis_dtype, void *stream);

/* The sparse mat-vec as the solver runs it (Alg. 1 steps 2/5/7):
 *   y = x_scale * op(A) x - coef * yprev, op(A) = A or A^T (transpose != 0),
 * through a plan of A that is created, used once and destroyed: A^T x uses
 * the plan's device transpose and, when x is long (more than 2 MiB of FP64
 * entries) and A^T has enough entries per row, the column-panel form
 * (sum over row panels A_g of A of A_g^T x_g, each XCD gathering from one
 * slice of x; partial sums added in panel order).  x has op(A)'s column
 * count, yprev and y its row count; device vectors of `basis_dtype`.  With
 * FP32 vectors the plan is a mixed-precision one, so FP64 values are read
 * from its FP32 copies (rounded to nearest), as in the FP32 cycles of a
 * mixed solve.
 * x_scale, coef: DEVICE pointers to one double each, or NULL as in
 * svds_op_spmv_csr.  *panels (host, may be NULL) receives the number of
 * column panels used (1 = the plain product).  A needs m >= 2, n >= 3
 * (a plan's smallest Lanczos dimension); EINVAL otherwise or on null
 * pointers; ENOMEM if the plan does not fit. */
int svds_op_csr_matvec(const svds_csr *A, int32_t transpose, const void *x, const double *x_scale,
                       const double *coef, const void *yprev, void *y, int32_t basis_dtype,
                       int32_t *panels, void *stream);

/* Dense mat-vec (column-major A, F64/F32/BF16 storage widened exactly):
 *   y = x_scale * op(A) x - coef * yprev, op(A) = A or A^T (transpose != 0). */
int svds_op_dense_matvec(const svds_dense *A, int32_t transpose, const void *x, const double *x_scale,
                         const double *coef, const void *yprev, void *y, int32_t basis_dtype,
                         void *stream);

/* CSR of A^T (n rows): t_row_ptr (n+1), t_col_idx (nnz, the row index of A,
 * increasing within each row of A^T), t_val (nnz, A's value type).
 * Bit-exact and deterministic (stable radix sort of the column keys). */
int svds_op_csc_build(const svds_csr *A, int32_t *t_row_ptr, int32_t *t_col_idx, void *t_val,
                      void *stream);

/* Full re-orthogonalization (Sec. 2.1, after Alg. 1) as CGS2:
 *   out = (I - Q Q^T)(I - Q Q^T) w, *norm_out = |out|_2 (host double),
 * Q (L x j, column-major, ld ldq >= L), w, out of length L, all `dtype`
 * (SVDS_F64 / SVDS_F32).  j = 0 gives out = w.  j <= 1024. */
int svds_op_cgs2(int64_t L, int32_t j, const void *Q, int64_t ldq, const void *w, void *out,
                 double *norm_out, int32_t dtype, void *stream);

/* svds_op_cgs2 for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, kernels and results as svds_op_cgs2 (bit-identical), but
 * no allocation of any kind: the call's scratch (column partials, the two
 * coefficient vectors, the intermediate vector of L entries, norm partials)
 * lives in one static device array of the library, about 24 MiB, that each
 * GPU holds from the first call on it until the process ends.
 *   - Limit: L * sizeof(element) <= SVDS_CGS2_NOALLOC_MAX_VECTOR_BYTES
 *     (2^21 FP64 or 2^22 FP32 entries), j <= 1024; EINVAL beyond.
 *   - Every call on one GPU shares that array, and a call leaves its
 *     contents behind: calls that overlap on one GPU (from several host
 *     threads or on several streams) race and give undefined results.
 *     Serialize them.  No word of the array has to start at zero: each call
 *     writes every word it reads before reading it.
 *   - Synchronous on `stream` (the norm is read back to the host). */
enum { SVDS_CGS2_NOALLOC_MAX_VECTOR_BYTES = 16 << 20 };
int svds_op_cgs2_noalloc(int64_t L, int32_t j, const void *Q, int64_t ldq, const void *w, void *out,
                         double *norm_out, int32_t dtype, void *stream);

/* Alg. 2 steps 4-9 on the device: T is the (p+1) x (p+1) row-major FP64
 * matrix of the Lanczos process (T(i,i) = alpha, T(i,i+1) = beta); its
 * leading p x p block is decomposed by the one-sided Jacobi SVD.  Outputs:
 * Uk (p x k, ld p), Vext ((p+1) x (k+1), ld p+1: leading right vectors,
 * zero last row, last column e_{p+1}), sig (k, descending), res (k, eq. (4)
 * estimates |beta_p Uh(p,j)| / sigma_j), rho (k, beta_p Uh(p,j), eq. (6)),
 * flags_host[0..2] = {all res < tol, leading count < tol, Jacobi sweeps}.
 * T is overwritten by the restarted matrix [diag(sig), rho] (step 9). */
int svds_op_small_svd(int32_t p, int32_t k, double tol, double *T, double *Uk, double *Vext,
                      double *sig, double *res, double *rho, int32_t *flags_host, void *stream);

/* The harmonic-Ritz restart coefficients of SVDS_FLAG_HARMONIC (the
 * augmented restart for the smallest values that Sec. 1 cites): T is the
 * (p+1) x (p+1) row-major FP64 Lanczos matrix (B = [T(1:p,1:p), beta e_p] =
 * its first p rows; row p+1 is read as zero), only read.  Outputs (device,
 * FP64, column-major unless stated): QC ((p+1) x (k+1), ld p+1: [y_1..y_k,
 * y_0] H, y_j the right singular vectors of the k smallest singular values
 * of B, y_0 its null vector, H the Householder reflection that zeroes
 * QC(p+1, 1:k); QC(p+1, k+1) > 0), QM (p x k, ld p: the matching left
 * singular vectors), R (k x k, row-major: QM^T B QC(:, 1:k)).  Each y_j
 * (with x_j) is determined up to sign, and within a repeated value up to
 * rotation.  EINVAL unless 1 <= k < p <= 1022 and all pointers are set. */
int svds_op_harmonic_basis(int32_t p, int32_t k, const double *T, double *QC, double *QM, double *R,
                           void *stream);

/* Restart rotation (Alg. 2 steps 8 and 16): out(:, 0:kc) = B(:, 0:pc) Y,
 * B L x pc of `btype` (F64/F32, ld ldb), Y pc x kc FP64 (ld ldy),
 * out L x kc FP64 (ld ldo).  Runs on the matrix cores (FP64 or FP32
 * MFMA, as the solver does); btype | SVDS_ROTATE_VECTOR selects the vector
 * FMA kernel instead (same arithmetic type, another summation order). */
enum { SVDS_ROTATE_VECTOR = 256 };
int svds_op_rotate(int64_t L, int32_t pc, int32_t kc, const void *B, int64_t ldb, int32_t btype,
                   const double *Y, int64_t ldy, double *out, int64_t ldo, void *stream);

/* Philox4x32-10 normal vector (the start vector of Alg. 1 step 1 when none
 * is given): block b of stream q gives out[2b], out[2b+1] by Box-Muller from
 * counter (b_lo, b_hi, q, 0) and key (seed_lo, seed_hi). */
int svds_op_philox_normal(int64_t L, uint64_t seed, uint32_t stream_id, double *out, void *stream);

/* Gather copy out[i] = x[idx[i]], i < L (idx int32, x and out FP64,
 * device): the gather-rate reference for the sparse products.  Per entry it
 * streams what the CSR product streams (a 4-byte index in, an 8-byte value:
 * here out instead of A's value) plus the gather of x, without the product's
 * row sums.  seg (HOST, nseg + 1 offsets from 0 to L, non-decreasing; NULL =
 * nseg equal parts) cuts the entries into nseg <= 64 segments; workgroup b
 * takes chunk b / nseg (2048 entries) of segment b % nseg, so with nseg = 8
 * the workgroups of one XCD gather one segment only, as those of the
 * column-panel product A^T y do.  Every idx[i] must index x: not checked.
 * The kernel runs reps >= 1 times back to back; *ms_per_launch (host, may
 * be NULL) receives their average duration from events around the
 * launches.  Synchronous on `stream`; EINVAL on bad arguments. */
int svds_op_gather_copy(int64_t L, const int32_t *idx, const double *x, double *out, int32_t nseg,
                        const int64_t *seg, int32_t reps, double *ms_per_launch, void *stream);

/* Plain device copy dst = src (L doubles): the bandwidth reference used to
 * calibrate hardware traffic counters. */
int svds_op_copy_f64(int64_t L, const double *src, double *dst, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SVDS_OPS_H */
