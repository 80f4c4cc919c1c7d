/*
 * svds.h -- C ABI of the MI355X (gfx950) truncated-SVD library.
 *
 * The library computes the k largest singular triplets of a sparse (CSR) or
 * dense m x n matrix A by the augmented, restarted Lanczos bidiagonalization
 * with full re-orthogonalization that the svds-C paper (Feng, Yu, Xie,
 * arXiv 2405.18966) re-implements from Matlab's svds:
 *   - Alg. 1 (Lanczos bidiagonalization, LBP) builds orthonormal bases
 *     U (m x t), V (n x (t+1)) and the projected matrix T with
 *     T(i,i) = alpha_i, T(i,i+1) = beta_i; every new basis vector is
 *     re-orthogonalized against the previous ones (Sec. 2.1, after Alg. 1;
 *     done here as classical Gram-Schmidt applied twice);
 *   - Proposition 1 / eq. (4) gives the residual estimate
 *     |beta_t Uh(t,j)| / sigma_j used as the stopping test (Alg. 2 step 5);
 *   - the augmented restart (eqs. (5)-(7), Alg. 2 steps 8-12) keeps the k
 *     Ritz vectors and the arrow column rho_j = beta_t Uh(t,j).
 * The paper's Lanczos dimension t is called p here.
 *
 * Conventions for every entry point:
 *   - All matrix/vector pointers are DEVICE pointers (hipMalloc'd or torch
 *     CUDA tensors) on the device that is current when the call is made.
 *     Work is enqueued on opts->stream (a hipStream_t; NULL = default stream)
 *     and the call returns after the stream has finished the solve.
 *   - Dense matrices and the U, V outputs are column-major (the paper's `mat`,
 *     Sec. 2.3), leading dimension = number of rows unless stated.
 *   - CSR is 0-based, three arrays: row i holds entries
 *     [row_ptr[i], row_ptr[i+1]) of col_idx/val, column indices strictly
 *     increasing within a row (the paper's `mat_csr` is the 1-based,
 *     pointerB/pointerE form of the same thing).
 *   - The caller owns every input and output buffer.  The library owns the
 *     device workspace of a plan (bases, transposed copies of A, FP32 value
 *     copies of a mixed plan, T, scratch), allocated at plan creation (as the
 *     paper allocates all buffers at the start, Sec. 2.2.2) and freed by
 *     svds_plan_destroy, and process-wide caches of timing events and of the
 *     pinned host buffers that plan creation reads row pointers into, kept
 *     until the process ends (at most 512 MiB of pinned memory).
 *   - Return codes: 0 = success, 1 = SVDS_NOT_CONVERGED (outputs hold the
 *     current Ritz triplets; info->nconv of the leading ones meet tol),
 *     negative = error, outputs untouched.  Nothing is thrown across the ABI.
 */
#ifndef SVDS_H
#define SVDS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SVDS_OK = 0,
  SVDS_NOT_CONVERGED = 1,
  SVDS_EINVAL = -1,      /* bad sizes, null pointers, k/p out of range      */
  SVDS_ENOMEM = -2,      /* device workspace allocation failed              */
  SVDS_EDEVICE = -3,     /* a HIP runtime call failed                       */
  SVDS_EUNSUPPORTED = -4 /* valid request the library does not implement    */
};

/* Storage type of A's values. */
enum { SVDS_F64 = 0, SVDS_F32 = 1, SVDS_BF16 = 2 };

/* Arithmetic of the solve.
 * SVDS_PREC_FP64 : bases, mat-vecs, re-orthogonalization in FP64.
 * SVDS_PREC_MIXED: FP32 cycles (bases, mat-vecs, re-orthogonalization in
 *                  FP32) until the eq. (4) estimate reaches max(tol, 1e-5),
 *                  then FP64 cycles restarted from the FP32 Ritz vectors.
 * The small SVD of T, T itself and the final residuals are FP64 always.
 * A stored in FP32/BF16 is widened exactly; that widened matrix is the
 * matrix whose SVD is computed.  A sparse A stored in FP64 is read, in the
 * FP32 cycles, from FP32 copies of its values that the plan makes (4 bytes
 * per nonzero and per copy of the values the plan holds, counted in
 * workspace_bytes); the FP64 cycles and the residuals read the FP64 values. */
enum { SVDS_PREC_FP64 = 0, SVDS_PREC_MIXED = 1 };

/* Option flags. */
enum {
  SVDS_FLAG_TIMING = 1,       /* record per-kernel-class device time in info   */
  SVDS_FLAG_NO_RESIDUALS = 2, /* skip the explicit FP64 residuals at the end   */
  SVDS_FLAG_NO_SIGNFIX = 4,   /* leave the signs of (u_j, v_j) as computed     */
  SVDS_FLAG_GRAPH = 8,        /* replay each restart cycle as a captured HIP graph */
  SVDS_FLAG_AUTOTUNE = 16,    /* pick launch shapes by timing them at plan time */
  /* Fixed launch shapes of the CSR products (the tuner's candidates; with
   * SVDS_FLAG_AUTOTUNE the tuner's choice replaces the first two, and
   * SVDS_FLAG_NO_PANELS keeps panels out of its candidates): */
  SVDS_FLAG_ITEMS_1K = 32,    /* work items of at most 1024 nonzeros, not 2048  */
  SVDS_FLAG_UNSORTED = 64,    /* no column-sorted copy of the work items        */
  SVDS_FLAG_NO_PANELS = 128,  /* A^T y over the plain CSR of A^T, no panels     */
  SVDS_FLAG_SMALLEST = 256,   /* the k smallest triplets instead (see below)    */
  SVDS_FLAG_SELECTIVE_REORTH = 512, /* second CGS pass only when needed (below) */
  SVDS_FLAG_PARTIAL_REORTH = 1024,  /* omega-recurrence partial re-orth. (below) */
  SVDS_FLAG_EARLY_STOP = 2048,      /* eq. (4) test inside a cycle (below)        */
  SVDS_FLAG_HARMONIC = 4096,        /* harmonic-Ritz restarts, smallest (below)   */
  SVDS_FLAG_EXPECT_BREAKDOWNS = 8192 /* wide breakdown repairs from step 1 (below) */
};

/* SVDS_FLAG_HARMONIC (with SVDS_FLAG_SMALLEST): restarts keep harmonic Ritz
 * vectors instead of Ritz vectors (the augmented restart of Baglama and
 * Reichel that Sec. 1 cites for the smallest values).  With A V = U T and
 * A^T U = V T^T + beta v e^T, the harmonic Ritz values of A^T A on span(V)
 * are the squared singular values of B = [T, beta e] (p x (p+1)); the
 * harmonic Ritz vectors of the k smallest and the common direction of their
 * residuals span [V v_{p+1}] span{y_1..y_k, y_0} (y_j B's right singular
 * vectors, y_0 its null vector).  Each cycle runs one more one-sided Jacobi
 * SVD, of the stored (p+1) x (p+1) matrix [B; 0], then: V_{k+1} = [V v_{p+1}]
 * Q_C (Q_C = [y_1..y_k, y_0] times the Householder reflection that zeroes
 * the last row of its first k columns), U_k = U Q_M (B's matching left
 * singular vectors), T(1:k,1:k) = Q_M^T B Q_C(:,1:k), and u_{k+1} = A v_{k+1}
 * re-orthogonalized against U_k with its two CGS coefficient vectors as
 * T(1:k, k+1).  The test of eq. (4) and the outputs stay those of the Ritz
 * triplets of T.  Converges in fewer cycles than plain Ritz augmentation on
 * some spectra (clustered small values), in more on others.  EINVAL without
 * SVDS_FLAG_SMALLEST or with SVDS_FLAG_SELECTIVE_REORTH /
 * SVDS_FLAG_PARTIAL_REORTH; EUNSUPPORTED for p > 1022 and in the batched
 * solver. */

/* SVDS_FLAG_EXPECT_BREAKDOWNS: a breakdown (Alg. 1 steps 6 and 8 meet an
 * invariant subspace: the re-orthogonalized vector's norm is at most 2^-40
 * times the largest value seen) replaces the vector by a Philox normal
 * vector taken twice against the whole basis.  With a basis of more than
 * 2^21 entries (rows x columns) that repair runs over up to 128 workgroups of
 * a cooperative launch instead of one workgroup: 575 -> 48 ms for the twenty
 * breakdowns of a rank-30 1,000,000 x 500,000 matrix at p = 40 on MI355X.
 * A cooperative dispatch costs ~17 us more than a plain one, paid at every
 * Lanczos step whether or not it breaks down (+7 % at 1,000,000 x 500,000,
 * p = 150), so the wide form is the default only from the cycle after one
 * that saw a breakdown (the count is read back with the cycle's small-SVD
 * flags; cycles ended by SVDS_FLAG_EARLY_STOP, whose small SVD runs on a
 * side stream, do not switch it on); this flag turns it on from the first
 * step, for matrices known to be rank-deficient.  Never inside captured cycles
 * (SVDS_FLAG_GRAPH keeps the one-workgroup repair there); ignored by the
 * batched solver. */

/* SVDS_FLAG_EARLY_STOP: Proposition 1 holds for the leading block T(1:j,1:j)
 * of a cycle at every Lanczos dimension j, so the test of eq. (4) can pass
 * before the cycle reaches p.  While the Lanczos steps go on, the library
 * copies T(1:j,1:j) and beta_j and runs the small SVD and the test on a
 * second stream of its own from a host thread of its own (checks start at
 * j = k + 1 + max(2, (p - k)/8); after a failed check the next one is placed
 * by the decrease of the largest estimate between the last two checks).  A
 * passing check at j ends the cycle: the outputs are the Ritz triplets of
 * T(1:j,1:j) with the first j basis vectors, so every estimate is below tol
 * exactly as at a full cycle's end.  The host enqueues at most 4 Lanczos
 * steps ahead of the device, so the steps run after j are few.
 * info->early_checks counts the checks, info->lanczos_dim_last is the Lanczos
 * dimension of the small SVD the outputs come from (p without an early stop).
 * Single and mixed solves; ignored with SVDS_FLAG_GRAPH (a captured cycle is
 * a fixed sequence) and by the batched solver. */

/* SVDS_FLAG_PARTIAL_REORTH: partial re-orthogonalization in the manner of
 * PROPACK (the alternative to full re-orthogonalization that Sec. 1 names).
 * The loss of orthogonality of each new vector against every earlier one of
 * its basis is estimated on the device from the two Lanczos relations
 * A V = U T and A^T U = V T^T (a recurrence over T and the estimates of the
 * previous vectors, plus a local rounding term eps * sigma_est / |w|).  Only
 * when an estimate exceeds sqrt(eps) is the vector re-orthogonalized (CGS2),
 * and then only against the columns whose estimate exceeds eps^(3/4), plus
 * the same columns for the next vector of that basis.  The restart vector of
 * eq. (7) is still taken against all k kept vectors.  Singular values come
 * out as accurate as with full re-orthogonalization; the bases, and so U and
 * V, are only semi-orthogonal (|U^T U - I|, |V^T V - I| up to ~sqrt(eps)),
 * and the explicit residuals |A^T u_j - s_j v_j| can exceed tol * s_j by up
 * to ~sqrt(eps) * s_1 / s_j.  info->partial_steps, partial_columns and
 * partial_possible count the vectors re-orthogonalized, the columns taken
 * and the columns full re-orthogonalization would take.  FP64 single solves
 * only (EUNSUPPORTED with SVDS_PREC_MIXED and in the batched solver); EINVAL
 * together with SVDS_FLAG_SELECTIVE_REORTH. */

/* SVDS_FLAG_SELECTIVE_REORTH: the re-orthogonalization of each new vector w
 * against its basis Q does the second classical Gram-Schmidt pass only when
 * the first removed more than 1/sqrt(2) of w's norm, i.e. when
 * |w - Q Q^T w|^2 < |w|^2 / 2 (the test of Daniel, Gragg, Kaufman and
 * Stewart, 1976).  The paper's operation count for a Lanczos step (eq. (8))
 * counts one projection per vector; the default (flag off) always does two.
 * The decision is taken on the device in the basis precision from norms
 * accumulated by the first two passes, so the passes over Q drop from three
 * to two whenever it skips.  info->reorth_tests and
 * info->reorth_second_passes count the tests and the second passes run.
 * FP64 and mixed single solves; EUNSUPPORTED in the batched solver. */

/* SVDS_FLAG_SMALLEST: the bidiagonalization approximates the smallest
 * singular values as well as the largest (Sec. 1).  Each cycle keeps the k
 * smallest Ritz triplets of T instead of the k largest; the restart of eqs.
 * (5)-(7) and the test of eq. (4) hold for any k Ritz triplets.  S is then
 * ascending (U, V in the same order).  The test's sigma floor stays
 * 2^-52 times the largest Ritz value, so exactly zero singular values never
 * pass it.  This is plain Ritz augmentation unless SVDS_FLAG_HARMONIC is
 * set, so convergence is fast only when the wanted values are well
 * separated relative to sigma_1.  FP64 path only: EUNSUPPORTED with
 * SVDS_PREC_MIXED and in the batched solver. */

/* SVDS_FLAG_AUTOTUNE: plan creation times candidate launch shapes on the
 * plan's own matrix and keeps the fastest (svds_tuning reports the choice).
 *   - CSR products A x and A^T y: nonzeros per work item (2048 or 1024; rows
 *     longer than that are split into pieces), column-sorted items on or
 *     off, and for A^T y the column-panel form on or off.
 *   - CGS2 (not for the batched solver, whose passes are segmented): the
 *     first pass's row-slab count (x 1/2, 1, 2) and the fused pass's columns
 *     per wave (8 or 10), timed at basis widths p/4, p/2 and p.
 * The choice depends on measured times; without the flag the built-in rules
 * apply.  Choices are cached for the process, keyed by the device, the
 * sizes, the value type, k, p, the precision and a hash of the row pointers
 * of A and A^T: a later plan with the same key takes the stored choice
 * without timing (svds_tuning.tuned = 2 instead of 1), so two tuned plans of
 * one matrix run the same launch shapes and give bit-identical results.  If
 * the environment variable SVDS_AUTOTUNE_CACHE names a file, the cache also
 * persists there: entries are read from it at the first tuned plan and each
 * new choice is appended as one text line. */

/* SVDS_FLAG_GRAPH: the launches of a restart cycle that follow the small SVD
 * (the restart vector of eq. (7) and the Lanczos steps k+1..p, Alg. 2 steps
 * 10-13) are captured once per plan into a HIP graph and replayed with one
 * hipGraphLaunch per cycle (the batched solver captures again when its set
 * of unconverged problems changes).  Results are bit-identical to the
 * ordinary launches.  The capture uses a private stream of the plan; the
 * graph runs on opts->stream.  With SVDS_FLAG_TIMING the captured launches
 * are counted but not timed. */

typedef struct {
  int64_t m, n, nnz;
  const int32_t *row_ptr; /* m+1 entries, row_ptr[0] = 0, row_ptr[m] = nnz   */
  const int32_t *col_idx; /* nnz entries in [0, n)                          */
  const void *val;        /* nnz values of type `dtype` (SVDS_F64/SVDS_F32) */
  int32_t dtype;
} svds_csr;

typedef struct {
  int64_t m, n, ld;       /* ld >= m                                        */
  const void *a;          /* column-major, type `dtype` (F64, F32 or BF16)  */
  int32_t dtype;
} svds_dense;

typedef struct {
  int32_t k;        /* number of triplets, 1 <= k                           */
  int32_t p;        /* Lanczos dimension t; 0 -> max(15, 3k) (Alg. 2 step 1)*/
  double tol;       /* eq. (4) tolerance; 0 -> 1e-10 (Sec. 3)               */
  int32_t maxit;    /* max Lanczos cycles (= max restarts + 1); 0 -> 10     */
  int32_t precision;/* SVDS_PREC_FP64 or SVDS_PREC_MIXED                    */
  uint64_t seed;    /* Philox4x32-10 seed of v1 (if v0 == NULL) and of
                       breakdown replacement vectors                         */
  const double *v0; /* optional device start vector, n entries (Alg. 1 step 1
                       draws randn(n,1)); need not be normalized, nonzero    */
  void *stream;     /* hipStream_t, NULL = default stream                    */
  int32_t flags;    /* SVDS_FLAG_*                                           */
} svds_opts;

/* With SVDS_FLAG_TIMING, one launch in each group of SVDS_TIMING_SAMPLE
 * consecutive launches of a kernel class is timed with HIP events on the
 * solve's stream (launch i is sampled when i mod 16 == (i / 16) mod 16).
 * The products and the three CGS2 passes carry the events on their own
 * dispatches (hipExtLaunchKernel), so the sampled time is the kernels' own;
 * the other classes are bracketed by event markers. */
enum { SVDS_TIMING_SAMPLE = 16 };

/* Kernel classes reported by SVDS_FLAG_TIMING. */
enum {
  SVDS_KC_SPMV = 0,      /* w = A x - beta u          (Alg. 1 step 7)       */
  SVDS_KC_SPMVT,         /* w = A^T y - alpha v       (Alg. 1 step 5)       */
  SVDS_KC_CGS_PROJ,      /* h1 = Q^T w                (first CGS pass)      */
  SVDS_KC_CGS_UPDPROJ,   /* w1 = w - Q h1, h2 = Q^T w1                      */
  SVDS_KC_CGS_UPDNORM,   /* w2 = w1 - Q h2, |w2|      (alpha/beta)          */
  SVDS_KC_CGS_REDUCE,    /* cross-block sums of the CGS passes, norm finish */
  SVDS_KC_SMALLSVD,      /* SVD of T, test, restart set-up (Alg. 2 4-9)     */
  SVDS_KC_ROTATE,        /* U Uh_k, V Vh_k            (Alg. 2 steps 8, 16)  */
  SVDS_KC_OTHER,         /* restart update, residuals, signs, casts         */
  SVDS_KC_COUNT
};

/* Launch shapes chosen by SVDS_FLAG_AUTOTUNE (all zero without it). */
typedef struct {
  int32_t tuned;                     /* 1 tuner ran, 2 choice from the cache     */
  int32_t fwd_nnz_cap, fwd_sorted;   /* A x: nonzeros per item, column-sorted    */
  int32_t bwd_nnz_cap, bwd_sorted;   /* A^T y: same                              */
  int32_t bwd_panels;                /* A^T y column panels (1 = none)           */
  int32_t cgs_slab_shift;            /* CGS2 pass-1 slabs x 2^shift              */
  int32_t cgs_cpw;                   /* fused-pass columns per wave (0 = rule)   */
  double fwd_us, fwd_default_us;     /* A x: chosen and built-in shape, us       */
  double bwd_us, bwd_default_us;     /* A^T y: same                              */
  double cgs_us, cgs_default_us;     /* CGS2 at widths p/4, p/2, p summed        */
  double ms_tune;                    /* wall time of the tuning                  */
} svds_tuning;

typedef struct {
  int32_t nconv;        /* leading triplets with eq. (4) estimate < tol     */
  int32_t cycles;       /* Lanczos cycles run (FP32 + FP64)                 */
  int32_t cycles_fp32, cycles_fp64;
  int32_t breakdowns;   /* invariant-subspace replacements                  */
  int32_t converged;    /* 1 if every estimate < tol at the end             */
  int64_t n_spmv, n_spmvT;    /* products A x and A^T y (excl. residuals)   */
  double max_res_est;   /* max_j eq. (4) estimate at the last small SVD     */
  double max_res_true;  /* max_j |A^T u_j - s_j v_j| / s_j, FP64 explicit   */
  double max_res_av;    /* max_j |A v_j - s_j u_j| / s_1,  FP64 explicit    */
  double ms_total;      /* wall time of the execute call                    */
  double bytes_alg;     /* algorithmic HBM bytes of SpMV + CGS kernels      */
  /* Per kernel class.  With SVDS_FLAG_TIMING every SVDS_TIMING_SAMPLE-th
   * launch of a class is timed with HIP events on the solve's stream:
   * kc_ms is the device time of those sampled launches, kc_sampled_* their
   * count and algorithmic bytes; kc_bytes/kc_flops/kc_launches cover all. */
  double kc_ms[SVDS_KC_COUNT];
  double kc_bytes[SVDS_KC_COUNT];
  double kc_flops[SVDS_KC_COUNT];
  int64_t kc_launches[SVDS_KC_COUNT];
  int64_t kc_sampled_launches[SVDS_KC_COUNT];
  double kc_sampled_bytes[SVDS_KC_COUNT];
  int64_t workspace_bytes;         /* device memory the plan holds          */
  int32_t graph_captures;          /* SVDS_FLAG_GRAPH: cycle graphs captured */
  int32_t graph_replays;           /* ... and cycles run by replaying one    */
  svds_tuning tuning;              /* SVDS_FLAG_AUTOTUNE choices of the plan */
  int32_t reorth_tests;            /* SVDS_FLAG_SELECTIVE_REORTH: tests made */
  int32_t reorth_second_passes;    /* ... and second passes run             */
  int64_t partial_steps;           /* SVDS_FLAG_PARTIAL_REORTH: vectors re-orthogonalized */
  int64_t partial_columns;         /* ... basis columns they were taken against */
  int64_t partial_possible;        /* ... columns full re-orthogonalization takes */
  int32_t early_checks;            /* SVDS_FLAG_EARLY_STOP: checks made       */
  int32_t lanczos_dim_last;        /* Lanczos dimension of the last small SVD */
} svds_info;

typedef struct svds_plan svds_plan;

/* Plan creation: validates the input (EINVAL when k < 1, p <= k, p > m,
 * p + 1 > n, a null pointer, or nnz != row_ptr[m] cannot be checked cheaply
 * and is trusted), allocates the device workspace once (Sec. 2.2.2: all
 * buffers are allocated at the start), and for CSR builds the transposed
 * copy A^T (CSR of A^T, entries of each column in increasing row order) on
 * the device.  `A` and the buffers it points to must stay alive and
 * unchanged until svds_plan_destroy.  `opts` is copied.  Without room for
 * the column-panel copy of A^T (or its work items) the plan falls back to
 * the plain transpose product; the environment variable SVDS_TEST_NO_ROOM
 * ("arena" or "panel_items") forces those fallbacks for tests. */
int svds_plan_create_csr(const svds_csr *A, const svds_opts *opts, svds_plan **plan);
int svds_plan_create_dense(const svds_dense *A, const svds_opts *opts, svds_plan **plan);

/* Runs Alg. 2 to convergence or opts->maxit cycles and writes
 * U (m x k, ld = m), S (k, descending; ascending with SVDS_FLAG_SMALLEST), V (n x k, ld = n), all FP64 device
 * buffers owned by the caller (Alg. 2 steps 15-16).  `info` may be NULL. */
int svds_plan_execute(svds_plan *plan, double *U, double *S, double *V, svds_info *info);

void svds_plan_destroy(svds_plan *plan);

/* create + execute + destroy. */
int svds_csr_solve(const svds_csr *A, const svds_opts *opts,
                   double *U, double *S, double *V, svds_info *info);
int svds_dense_solve(const svds_dense *A, const svds_opts *opts,
                     double *U, double *S, double *V, svds_info *info);

/* Many independent CSR problems with the same options (k, p, tol, maxit,
 * precision, flags), solved in lockstep: the problems are stacked as one
 * block-diagonal matrix (each padded to a multiple of 256 rows and columns)
 * and every kernel launch serves all of them; projections, norms and
 * residuals are reduced per problem, the small SVDs run one workgroup per
 * problem.  A problem whose eq. (4) test passes is frozen at the next
 * restart: its Ritz vectors stay in the leading basis columns and every
 * later launch skips it, while the others go on until they converge or
 * maxit cycles ran.  Each problem reports its own estimates, breakdowns,
 * residuals and cycle counts (the cycles it ran before it froze, per
 * precision phase).
 *   - U[i] (m_i x k, ld m_i), S[i] (k), V[i] (n_i x k, ld n_i): per-problem
 *     FP64 device outputs; infos (count entries) may be NULL.
 *   - All problems must share the value type (F64 or F32).
 *   - Start vectors: opts->v0, if given, is the concatenation of the
 *     problems' start vectors (sum of n_i doubles, unpadded); otherwise
 *     problem i draws Philox stream 0 of seed opts->seed + i.
 *   - Limits: p <= 62 (one-workgroup small SVD) and k + 1 <= 64, else
 *     SVDS_EUNSUPPORTED; sums of padded rows, columns and nnz < 2^31.
 * Returns SVDS_NOT_CONVERGED if any problem did not converge. */
int svds_csr_solve_batched(int32_t count, const svds_csr *As, const svds_opts *opts,
                           double *const *U, double *const *S, double *const *V,
                           svds_info *infos);

/* Explicit FP64 residuals of given triplets (Proposition 1, eq. (2)):
 * res_av[j] = |A v_j - s_j u_j|_2 and res_atu[j] = |A^T u_j - s_j v_j|_2,
 * j < k, for device U (m x k), S (k), V (n x k); outputs are device arrays
 * of k doubles.  Synchronous on `stream`. */
int svds_residuals_csr(const svds_csr *A, int32_t k, const double *U, const double *S,
                       const double *V, double *res_av, double *res_atu, void *stream);

/* The same for a dense A (column-major, F64/F32/BF16 storage widened
 * exactly): both sides are FP64 block products over all k triplets at once
 * (one pass over the stored A per side, FP64 matrix cores), with the
 * partial sums added in a fixed order.  k + 1 <= m and k + 2 <= n, else
 * EINVAL.  Synchronous on `stream`. */
int svds_residuals_dense(const svds_dense *A, int32_t k, const double *U, const double *S,
                         const double *V, double *res_av, double *res_atu, void *stream);

const char *svds_strerror(int code);

/* Library version string. */
const char *svds_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SVDS_H */
