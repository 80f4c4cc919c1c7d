// Host-side plan: device workspace arena, operator (A and A^T), per-kernel
// timing, and the Lanczos cycle driver of Alg. 2.
#pragma once
#include <new>
#include <vector>
#include <string>
#include <chrono>

#include "../../include/svds.h"
#include "common.hpp"
#include "kernels_spmv.hpp"

// Around the body of every C entry point: no exception (a failed host
// allocation) crosses the C ABI; it becomes an error code.
#define SVDS_ABI_TRY try {
#define SVDS_ABI_CATCH                                                        \
  }                                                                           \
  catch (const std::bad_alloc &) {                                            \
    return SVDS_ENOMEM;                                                       \
  }                                                                           \
  catch (...) {                                                               \
    return SVDS_EDEVICE;                                                      \
  }

namespace svds {

constexpr int GMAX = 1024;  // largest grid of the reduction kernels

// ---------------------------------------------------------------------------
// Device arena: one hipMalloc, carved in 256-byte aligned pieces.
// ---------------------------------------------------------------------------
struct Arena {
  char *base = nullptr;
  size_t size = 0, used = 0;
  bool counting = true;
  template <typename T> T *take(size_t count) {
    const size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    T *p = counting ? nullptr : reinterpret_cast<T *>(base + used);
    used += bytes;
    return p;
  }
};

constexpr int SPMV_TUNE_MIN_CAP = 1024;  // smallest item nnz cap a plan uses (SVDS_FLAG_ITEMS_1K, tuner)

// Work decomposition of one CSR product (see kernels_spmv.hpp).
struct SpmvPlan {
  int nitems = 0, nlong = 0, npieces = 0;
  int4 *items = nullptr;
  LongRow *longrows = nullptr;
  double *partials = nullptr;  // npieces (TB <= 8 bytes)
  std::vector<int4> h_items;
  std::vector<LongRow> h_long;
  // column-sorted nonzeros of the items (sort_items_kernel), or null: the
  // product then reads the matrix's own arrays in row order
  int32_t *scol = nullptr;
  void *sval = nullptr;
  uint16_t *spos = nullptr;
  const int32_t *x_tile_inst = nullptr;  // problem of each 256-entry tile of x (batched), or null
  const int32_t *active = nullptr;       // per-problem work mask (batched), or null
  const int32_t *side_tiles = nullptr;   // tiles of x the side task covers (batched), or null: all
  int side_ntiles = 0;
  bool sorted = true;  // use the column-sorted copy when it exists (the tuner may turn it off)
  int cap_items = 0, cap_long = 0, cap_pieces = 0;  // sizes of the device item buffers
};

// Work items of a CSR product.  With seg_end (nseg consecutive row ranges
// ending at seg_end[g], one per problem of a batch) items never cross a range
// and carry the range index g; without it there is one range, index 0.
// nnz_cap (<= SPMV_NNZ_BLK): largest nonzero count of a MULTI item; longer
// rows become PIECE items.
void build_spmv_items(const int32_t *rp, int64_t m, SpmvPlan &sp, const int64_t *seg_end = nullptr,
                      int nseg = 1, int nnz_cap = SPMV_NNZ_BLK);

// ---------------------------------------------------------------------------
// Per-kernel-class accounting and optional device timing with event pairs.
// ---------------------------------------------------------------------------
struct Accounting {
  bool timing = false;
  hipStream_t stream = nullptr;
  std::vector<hipEvent_t> pool;
  size_t next = 0;
  std::vector<int> cls;  // class of each recorded pair
  double ms[SVDS_KC_COUNT] = {};
  double bytes[SVDS_KC_COUNT] = {};
  double flops[SVDS_KC_COUNT] = {};
  int64_t launches[SVDS_KC_COUNT] = {};
  int64_t sampled[SVDS_KC_COUNT] = {};
  double sampled_bytes[SVDS_KC_COUNT] = {};
  bool sampling = false;  // the launch between before() and after() is timed
  // Attached timing: the sampled bracket's first launch carries att_start and
  // its last launch att_stop as dispatch events (hipExtLaunchKernel), so the
  // time is the kernels' own, without marker packets between launches.
  bool attach = false;
  hipEvent_t att_start = nullptr, att_stop = nullptr;
  bool att_started = false, att_stopped = false;

  void reset() {
    for (int i = 0; i < SVDS_KC_COUNT; ++i)
      ms[i] = bytes[i] = flops[i] = sampled_bytes[i] = 0, launches[i] = sampled[i] = 0;
    next = 0;
    cls.clear();
    sampling = attach = false;
  }
  int harvest();
  int before(int kc, bool attached = false);
  int after(int kc, double b, double f);
  int device = 0;  // device the events belong to
  int grow();      // adds events to the pool
  void destroy();  // returns the pool's events to the process-wide cache
};

// ---------------------------------------------------------------------------
// Captured Lanczos cycles (SVDS_FLAG_GRAPH).  The launches of one cycle after
// the small SVD (restart vector, Lanczos steps k+1..p) are captured once into
// an executable HIP graph and replayed on every later cycle that starts from
// the same ping-pong buffer: one graph per (basis type, buffer).  A graph is
// valid for one work-list version (the batched solver changes its launch
// grids when problems freeze; a single problem has one version for the
// plan's lifetime).  The accounting and mat-vec counters a captured body adds
// are recorded at capture and added again on every replay.
// ---------------------------------------------------------------------------
struct CycleGraphs {
  hipStream_t cap = nullptr;       // capture stream (default priority)
  hipGraphExec_t exec[2][2] = {};  // [basis is FP64][buffer the cycle starts from]
  uint64_t ver[2][2] = {};         // work-list version captured (0: none)
  int next_cur[2][2] = {};         // buffer after the body
  double dbytes[2][2][SVDS_KC_COUNT] = {}, dflops[2][2][SVDS_KC_COUNT] = {};
  int64_t dlaunch[2][2][SVDS_KC_COUNT] = {}, dspmv[2][2] = {}, dspmvT[2][2] = {}, dreorth[2][2] = {};
  int64_t captures = 0, replays = 0;
  void drop(int t, int c) {
    if (exec[t][c]) (void)hipGraphExecDestroy(exec[t][c]);
    exec[t][c] = nullptr;
    ver[t][c] = 0;
  }
  void destroy() {
    for (int t = 0; t < 2; ++t)
      for (int c = 0; c < 2; ++c) drop(t, c);
    if (cap) (void)hipStreamDestroy(cap);
    cap = nullptr;
  }
};

// ---------------------------------------------------------------------------
// The matrix operator: y = xs * A x - coef * yprev and the transpose.
// ---------------------------------------------------------------------------
struct Operator {
  bool dense = false;
  int64_t m = 0, n = 0, nnz = 0;
  int vt = SVDS_F64;  // stored value type
  // CSR of A (caller's) and of A^T (plan-owned)
  const int32_t *rp = nullptr, *ci = nullptr;
  const void *val = nullptr;
  int32_t *trp = nullptr, *tci = nullptr;
  void *tval = nullptr;
  SpmvPlan fwd, bwd;
  // A^T u by column panels (see spmv_panel_sum_kernel): npanel > 1 for a
  // single problem whose u is large; stacked CSR (npanel n rows) and partial
  // products (npanel n) in the arena, work items in their own allocation
  // (their count is known only once they are built)
  int npanel = 1;
  int32_t *prp = nullptr, *pci = nullptr;
  void *pval = nullptr;
  double *ypart = nullptr;
  SpmvPlan bwdp;
  void *pbuf_items = nullptr;
  size_t pbuf_bytes = 0;  // bytes of pbuf_items
  // FP32 copies of the values of an FP64-stored CSR matrix for the FP32 phase
  // of a mixed solve (A, A^T, the column-sorted copies, the panel copy; null
  // where that array does not exist); one allocation, v32buf
  float *val32 = nullptr, *tval32 = nullptr, *fsval32 = nullptr, *bsval32 = nullptr, *pval32 = nullptr;
  void *v32buf = nullptr;
  size_t v32_bytes = 0;
  // dense
  const void *a = nullptr;
  int64_t lda = 0;
  double *dpart = nullptr;        // slab partials of A x
};

}  // namespace svds

// Internal entry points (C++ linkage) used by the single-step operations.
int svds_plan_residuals(svds_plan *P, int k, const double *U, const double *S, const double *V,
                        double *res_av, double *res_atu);
int svds_plan_matvec(svds_plan *P, int trans, const void *x, const double *xs, const double *coef,
                     const void *yprev, void *y, int basis_dtype);
int svds_plan_panels(const svds_plan *P);
int svds_plan_transpose_copy(svds_plan *P, int32_t *t_row_ptr, int32_t *t_col_idx, void *t_val);
int svds_cgs2_op(int64_t L, int32_t j, const void *Q, int64_t ldq, const void *w, void *out,
                 double *norm_out, int32_t dtype, void *stream);
// Small SVD of T (p x p block of the (p+1) x (p+1) row-major T) and restart
// set-up, enqueued on `st` (smallest != 0: keep the k smallest Ritz triplets); `work` holds jacobi_work_bytes(p) bytes of device
// memory, `h_counts` JAC_MAX_SWEEPS host ints (pinned or not).  The
// multi-workgroup schedule reads its sweep counters back between chunks of
// sweeps (stream synchronizations).
int svds_small_svd_run(hipStream_t st, double *T, int p, int k, double tol, double *work, double *Uk,
                       double *Vext, double *sig, double *res, double *rho, int *flags, double *sigma_est,
                       int *h_counts, int smallest = 0);
// Harmonic-Ritz restart coefficients from the stored (p+1) x (p+1) T (see
// harm_finish): QC ((p+1) x (k+1)), QM (p x k), R (k x k row-major); `work`
// holds jacobi_work_bytes(p + 1) bytes.  T is only read.
int svds_harmonic_basis_run(hipStream_t st, const double *T, int p, int k, double *work, double *QC, double *QM,
                            double *R, int *h_counts);
