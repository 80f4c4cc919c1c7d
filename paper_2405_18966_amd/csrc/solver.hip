// Alg. 2 driver: plan creation (workspace, transposed copy of A), the
// Lanczos cycles with CGS2 re-orthogonalization, small SVD, restart and
// output (Alg. 1, Proposition 1, eqs. (4)-(7), Alg. 2), plus the mixed
// FP32 -> FP64 form.  Everything that touches vectors of length m or n runs in
// the kernels of kernels_*.hpp; the host only enqueues kernels and reads one
// convergence flag per cycle.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <thread>
#include <tuple>
#include <utility>

#include <hip/hip_ext.h>

#include "../../include/svds_ops.h"
#include "plan.hpp"
#include "kernels_cgs.hpp"
#include "kernels_csc.hpp"
#include "kernels_jacobi.hpp"
#include "kernels_misc.hpp"
#include "kernels_dense.hpp"
#include "kernels_batch.hpp"
#include "kernels_small.hpp"

namespace svds {

// ---------------------------------------------------------------------------
// error text
// ---------------------------------------------------------------------------
static thread_local char g_err[512] = "";
void set_last_error(hipError_t e, const char *what, const char *file, int line) {
  snprintf(g_err, sizeof g_err, "%s: %s (%s:%d)", hipGetErrorString(e), what, file, line);
}
const char *last_error_text() { return g_err; }

#define LAUNCH_CHECK() HIP_TRY(hipGetLastError())

static inline unsigned grid_for(int64_t work, int64_t per_block, int64_t gmax = GMAX) {
  int64_t g = ceil_div(std::max<int64_t>(work, 1), per_block);
  return static_cast<unsigned>(std::min<int64_t>(std::max<int64_t>(g, 1), gmax));
}

// ---------------------------------------------------------------------------
// SpMV work items (host, at plan time)
// ---------------------------------------------------------------------------
void build_spmv_items(const int32_t *rp, int64_t m, SpmvPlan &sp, const int64_t *seg_end, int nseg, int nnz_cap) {
  sp.h_items.clear();
  sp.h_long.clear();
  int npieces = 0;
  int64_t r = 0;
  for (int g = 0; g < (seg_end ? nseg : 1); ++g) {
    const int64_t e = seg_end ? seg_end[g] : m;  // items never cross a problem boundary
    while (r < e) {
      const int64_t len = rp[r + 1] - rp[r];
      if (len > nnz_cap) {
        const int np = static_cast<int>(ceil_div(len, SPMV_PIECE));
        const int lr = static_cast<int>(sp.h_long.size());
        sp.h_long.push_back(LongRow{static_cast<int32_t>(r), npieces, np, g});
        for (int q = 0; q < np; ++q) {
          const int64_t z0 = rp[r] + static_cast<int64_t>(q) * SPMV_PIECE;
          const int64_t z1 = std::min<int64_t>(rp[r + 1], z0 + SPMV_PIECE);
          sp.h_items.push_back(make_int4(-lr - 1, npieces + q, static_cast<int>(z0), static_cast<int>(z1)));
        }
        npieces += np;
        ++r;
        continue;
      }
      const int64_t r0 = r;
      int64_t z = 0;
      while (r < e && r - r0 < SPMV_ROWS_BLK) {
        const int64_t l = rp[r + 1] - rp[r];
        if (l > nnz_cap || z + l > nnz_cap) break;
        z += l;
        ++r;
      }
      sp.h_items.push_back(make_int4(static_cast<int>(r0), static_cast<int>(r), rp[r0],
                                     static_cast<int>(z) | (g << SPMV_CNT_BITS)));
    }
  }
  sp.nitems = static_cast<int>(sp.h_items.size());
  sp.nlong = static_cast<int>(sp.h_long.size());
  sp.npieces = npieces;
}

// ---------------------------------------------------------------------------
// Accounting
// ---------------------------------------------------------------------------
int Accounting::harvest() {
  if (!timing || next == 0) return SVDS_OK;
  HIP_TRY(hipEventSynchronize(pool[next - 1]));
  for (size_t i = 0; i + 1 < next; i += 2) {
    float t = 0;
    HIP_TRY(hipEventElapsedTime(&t, pool[i], pool[i + 1]));
    ms[cls[i / 2]] += t;
  }
  next = 0;
  cls.clear();
  return SVDS_OK;
}

// Timing events come from a process-wide cache per device: a plan made for
// each solve would otherwise create and destroy its events every time, at
// microseconds per event.
static std::mutex g_ev_mu;
static std::vector<hipEvent_t> g_ev_free[64];

int Accounting::grow() {
  constexpr size_t CHUNK = 64;
  size_t got = 0;
  {
    std::lock_guard<std::mutex> lock(g_ev_mu);
    auto &f = g_ev_free[device & 63];
    while (got < CHUNK && !f.empty()) {
      pool.push_back(f.back());
      f.pop_back();
      ++got;
    }
  }
  for (; got < CHUNK; ++got) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    pool.push_back(e);
  }
  return SVDS_OK;
}

void Accounting::destroy() {
  if (pool.empty()) return;
  std::lock_guard<std::mutex> lock(g_ev_mu);
  auto &f = g_ev_free[device & 63];
  f.insert(f.end(), pool.begin(), pool.end());
  pool.clear();
}

int Accounting::before(int kc, bool attached) {
  // one launch in each group of SVDS_TIMING_SAMPLE, at an offset that
  // rotates from group to group, so launches that alternate between two
  // shapes (U side / V side) are both sampled
  const int64_t i = launches[kc];
  sampling = timing && (i % SVDS_TIMING_SAMPLE == (i / SVDS_TIMING_SAMPLE) % SVDS_TIMING_SAMPLE);
  attach = false;
  if (!sampling) return SVDS_OK;
  if (next + 2 > pool.size()) {
    if (pool.size() < 16384) {
      int rc = grow();
      if (rc) return rc;
    } else {
      int rc = harvest();
      if (rc) return rc;
    }
  }
  cls.push_back(kc);
  if (attached) {
    attach = true;
    att_start = pool[next];
    att_stop = pool[next + 1];
    att_started = att_stopped = false;
    next += 2;
    return SVDS_OK;
  }
  HIP_TRY(hipEventRecord(pool[next++], stream));
  return SVDS_OK;
}

int Accounting::after(int kc, double b, double f) {
  bytes[kc] += b;
  flops[kc] += f;
  launches[kc] += 1;
  if (!sampling) return SVDS_OK;
  sampling = false;
  if (attach) {
    attach = false;
    if (!att_started) {  // no launch carried the start event: drop the sample
      next -= 2;
      cls.pop_back();
      return SVDS_OK;
    }
    if (!att_stopped) HIP_TRY(hipEventRecord(att_stop, stream));
    sampled[kc] += 1;
    sampled_bytes[kc] += b;
    return SVDS_OK;
  }
  sampled[kc] += 1;
  sampled_bytes[kc] += b;
  HIP_TRY(hipEventRecord(pool[next++], stream));
  return SVDS_OK;
}

// Kernel launch inside an accounting bracket: with attached timing, the
// bracket's first launch carries the start event and its last launch the stop
// event (hipExtLaunchKernel, arguments converted to the kernel's parameter
// types); otherwise an ordinary launch.
template <typename... Prm, typename... Arg, size_t... I>
static hipError_t ext_launch(void (*k)(Prm...), dim3 g, dim3 b, uint32_t shm, hipStream_t st, hipEvent_t e0,
                             hipEvent_t e1, std::index_sequence<I...>, Arg... a) {
  std::tuple<Prm...> t(static_cast<Prm>(a)...);
  void *argv[] = {static_cast<void *>(&std::get<I>(t))...};
  return hipExtLaunchKernel(reinterpret_cast<const void *>(k), g, b, argv, shm, st, e0, e1, 0);
}

template <typename... Prm, typename... Arg>
static void klaunch(Accounting &acc, bool first, bool last, void (*k)(Prm...), dim3 g, dim3 b, uint32_t shm,
                    hipStream_t st, Arg... a) {
  static_assert(sizeof...(Prm) == sizeof...(Arg), "kernel arity");
  hipEvent_t e0 = (acc.attach && first) ? acc.att_start : nullptr;
  hipEvent_t e1 = (acc.attach && last) ? acc.att_stop : nullptr;
  if (!e0 && !e1) {
    hipLaunchKernelGGL(k, g, b, shm, st, static_cast<Prm>(a)...);
    return;
  }
  if (ext_launch(k, g, b, shm, st, e0, e1, std::index_sequence_for<Prm...>{}, a...) == hipSuccess) {
    if (e0) acc.att_started = true;
    if (e1) acc.att_stopped = true;
  }
}

#define ACC_BEFORE(kc)                      \
  do {                                      \
    int rc_ = P->acc.before(kc);            \
    if (rc_) return rc_;                    \
  } while (0)
#define ACC_BEFORE_ATT(kc)                  \
  do {                                      \
    int rc_ = P->acc.before(kc, true);      \
    if (rc_) return rc_;                    \
  } while (0)
#define ACC_AFTER(kc, b, f)                 \
  do {                                      \
    int rc_ = P->acc.after(kc, (b), (f));   \
    if (rc_) return rc_;                    \
  } while (0)

// ---------------------------------------------------------------------------
// Workspace of one precision: bases (ping-pong) and vectors.
// ---------------------------------------------------------------------------
template <typename TB> struct Lanczos {
  int64_t m = 0, n = 0, ldu = 0, ldv = 0;
  TB *U[2] = {}, *V[2] = {};
  int cur = 0;
  TB *wu = nullptr, *w1u = nullptr, *bu = nullptr;
  TB *wv = nullptr, *w1v = nullptr, *bv = nullptr;
  TB *h1 = nullptr, *h2 = nullptr, *partials = nullptr;
  void carve(Arena &a, int64_t m_, int64_t n_, int p) {
    m = m_;
    n = n_;
    ldu = ceil_div(m, 64) * 64;
    ldv = ceil_div(n, 64) * 64;
    for (int i = 0; i < 2; ++i) {
      U[i] = a.take<TB>(static_cast<size_t>(ldu) * (p + 1));
      V[i] = a.take<TB>(static_cast<size_t>(ldv) * (p + 1));
    }
    wu = a.take<TB>(m);
    w1u = a.take<TB>(m);
    bu = a.take<TB>(m);
    wv = a.take<TB>(n);
    w1v = a.take<TB>(n);
    bv = a.take<TB>(n);
    h1 = a.take<TB>(CGS_MAXJ);
    h2 = a.take<TB>(CGS_MAXJ);
    partials = a.take<TB>(static_cast<size_t>(CGS_MAXJ) * CGS_MAX_SLABS);
  }
};

// Device scalars and small arrays shared by both precisions (FP64 always).
struct Small {
  double *T, *xs_u, *xs_v, *one, *sigma_est, *rho, *sig, *res, *Uk, *Vext, *jac, *npart;
  double *resid_av, *resid_atu;
  double *yt;                       // transposed rotation panel
  double *sgn, *sgn_val;            // sign normalization
  int64_t *sgn_idx;
  int *bd, *flags;
  // partial re-orthogonalization: estimate rows of the newest u and v,
  // pending estimates and |w| of the vector in progress, its column mask,
  // the forced sets of both sides, counters (U side [0..3), V side [4..7))
  double *om_mu, *om_nu, *om_pend, *om_nrm0;
  int *om_mask, *om_fu, *om_fv;
  long long *om_stats;
  // harmonic restart coefficients: Q_C ((p+1) x (k+1)), Q_M (p x k), R (k x k)
  double *hQC, *hQM, *hR;
};

// thresholds of the partial re-orthogonalization: trigger sqrt(eps), select eps^(3/4)
constexpr double OMEGA_TAU = 1.4901161193847656e-08;
constexpr double OMEGA_ETA = 1.8189894035458565e-12;

constexpr int NPART = NORM_MAX_BLOCKS;  // norm partials

// SVDS_FLAG_EARLY_STOP: the eq. (4) test on the leading block T(1:j,1:j) of a
// cycle still in progress (Proposition 1 holds at every Lanczos dimension j).
// A check copies the block on a side stream and runs the small SVD there from
// a worker thread, while the main stream goes on with the Lanczos steps; the
// host stays at most EARLY_LAG steps ahead of the device, so a passing check
// stops the cycle a few steps after j.  The cycle's outputs are then formed
// from that check's SVD of T(1:j,1:j) and the first j basis vectors.
constexpr int EARLY_LAG = 4;
struct EarlyCheck {
  double *T = nullptr, *Uk = nullptr, *Vext = nullptr, *sig = nullptr, *res = nullptr, *rho = nullptr,
         *sigma_est = nullptr, *jac = nullptr;
  int *flags = nullptr;
  int *h_flags = nullptr;          // pinned: 4 flags, then the Jacobi sweep counters
  hipStream_t stream = nullptr;
  hipEvent_t ev_check = nullptr;
  hipEvent_t ev_step[EARLY_LAG] = {};
  std::thread worker;
  std::atomic<int> state{0};       // 0 idle, 1 running, 2 finished
  int j_run = 0, rc = 0, passed = 0, sweeps = 0;
  double max_res = 0;
  int checks = 0, stop_j = 0;      // checks made in this execute; j of a passing check
  int next_j = 0, j_prev = 0;      // scheduling within the current cycle
  double r_prev = 0;
};

}  // namespace svds

using namespace svds;

struct svds_plan {
  Operator op;
  svds_opts opts{};
  int k = 0, p = 0, maxit = 0;
  double tol = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  Arena arena;
  Lanczos<double> L64;
  Lanczos<float> L32;
  bool mixed = false;
  bool capturing = false;  // a cycle body is being captured into a graph
  Small sc{};
  double *tmp_nk = nullptr;  // n x k FP64 (mixed warm start), m-vector scratch
  int32_t *tscratch = nullptr;  // device radix-sort scratch of the transposed copies (CSR plans)
  double *tmp_m = nullptr, *tmp_n = nullptr;
  // residual panels (CSR plans): row-major RG-column panels of U and V, partials
  double *rs_pu = nullptr, *rs_pv = nullptr, *rs_part = nullptr, *rs_pieces = nullptr, *rs_lpart = nullptr,
         *rs_s = nullptr;
  // dense residuals: partial tiles of the block products and column partials
  // (resid_dense_doubles)
  double *rd_part = nullptr;
  int *h_flags = nullptr;    // pinned
  Accounting acc;
  int64_t n_spmv = 0, n_spmvT = 0;
  int cycles32 = 0, cycles64 = 0, jac_sweeps = 0;
  CycleGraphs graphs;  // SVDS_FLAG_GRAPH
  // launch-shape knobs of the CGS2 passes (SVDS_FLAG_AUTOTUNE; 0 = built-in
  // rules): pass-1 slab count times 2^cgs_slab_shift, fused-pass columns per
  // wave forced to cgs_cpw (8 or 10)
  int cgs_slab_shift = 0, cgs_cpw = 0;
  svds_tuning tuning{};  // what the tuner chose and measured
  bool smallest = false;  // SVDS_FLAG_SMALLEST: k smallest triplets, ascending
  bool selective = false;  // SVDS_FLAG_SELECTIVE_REORTH: second CGS pass only when needed
  bool partial = false;    // SVDS_FLAG_PARTIAL_REORTH: omega-recurrence partial re-orthogonalization
  bool harmonic = false;   // SVDS_FLAG_HARMONIC: harmonic-Ritz restarts (with SVDS_FLAG_SMALLEST)
  bool wide_repair = false;  // breakdown repairs over many workgroups (finish_blocks)
  int64_t reorth_calls = 0;  // re-orthogonalizations with the selective test
  bool early = false;      // SVDS_FLAG_EARLY_STOP
  EarlyCheck ec;
  // the small SVD the outputs (and a mixed solve's warm start) use: its
  // Lanczos dimension and its Uk (p_eff x k, ld p_eff) and Vext
  // ((p_eff+1) x (k+1), ld p_eff+1)
  int p_eff = 0;
  double *out_Uk = nullptr, *out_Vext = nullptr;
};

namespace svds {

// ---------------------------------------------------------------------------
// Products with A
// ---------------------------------------------------------------------------
static inline double vsize(int vt) { return vt == SVDS_F64 ? 8.0 : vt == SVDS_F32 ? 4.0 : 2.0; }

template <typename TV, typename TB>
static void dense_launch(svds_plan *P, bool trans, const TB *x, const double *xs, const double *coef,
                         const TB *yprev, TB *y, TB *side_dst, int64_t side_len) {
  const Operator &op = P->op;
  const TV *A = static_cast<const TV *>(op.a);
  const bool vec = dense_vec_ok<TV, TB>(A, op.lda, x);
  if (trans) {
    const dim3 g(static_cast<unsigned>(ceil_div(op.n, DN_TCOLS)));
    if (vec)
      klaunch(P->acc, true, true, gemv_t_kernel<TV, TB, true>, g, dim3(DN_THREADS), 0, P->stream, op.m, op.n, A,
              op.lda, x, xs, coef, yprev, y, side_dst, side_len);
    else
      klaunch(P->acc, true, true, gemv_t_kernel<TV, TB, false>, g, dim3(DN_THREADS), 0, P->stream, op.m, op.n, A,
              op.lda, x, xs, coef, yprev, y, side_dst, side_len);
  } else {
    const int nslab = static_cast<int>(ceil_div(op.n, DN_SLAB));
    TB *part = reinterpret_cast<TB *>(op.dpart);
    const dim3 g(static_cast<unsigned>(ceil_div(op.m, DN_ROWS)), nslab);
    if (vec)
      klaunch(P->acc, true, false, gemv_n_kernel<TV, TB, true>, g, dim3(DN_THREADS), 0, P->stream, op.m, op.n, A,
              op.lda, x, xs, part, side_dst, side_len);
    else
      klaunch(P->acc, true, false, gemv_n_kernel<TV, TB, false>, g, dim3(DN_THREADS), 0, P->stream, op.m, op.n, A,
              op.lda, x, xs, part, side_dst, side_len);
    klaunch(P->acc, false, true, gemv_n_fixup_kernel<TB>, dim3(ceil_div(op.m, 256)), dim3(256), 0, P->stream, op.m,
            nslab, part, xs, coef, yprev, y);
  }
}

// Products whose first CGS pass can ride on them (spmv_csr_kernel's SpmvProj
// epilogue): a single CSR problem without the partial or selective forms,
// a product without column panels or long rows, at most CGS_FUSE_NP items
// (the next pass sums the items' partials) and at most 2^18 basis entries
// (the items read them).  Returns the number of partials per column, or 0.
static int spmv_proj_np(const svds_plan *P, bool trans, int j) {
  const Operator &op = P->op;
  if (op.dense || P->partial || P->selective || j < 1 || (trans && op.npanel > 1)) return 0;
  const SpmvPlan &sp = trans ? op.bwd : op.fwd;
  const int64_t rows = trans ? op.n : op.m;
  if (sp.nlong > 0 || sp.nitems > CGS_FUSE_NP || rows * j > (int64_t(1) << 18)) return 0;
  return sp.nitems;
}

template <typename TB>
static int matvec(svds_plan *P, bool trans, const TB *x, const double *xs, const double *coef,
                  const TB *yprev, TB *y, TB *side_dst, int64_t side_len, int kc_over = -1,
                  SpmvProj<TB> pj = {nullptr, 0, 0, nullptr}) {
  const Operator &op = P->op;
  const int64_t rows = trans ? op.n : op.m, cols = trans ? op.m : op.n;
  const int kc = kc_over >= 0 ? kc_over : (trans ? SVDS_KC_SPMVT : SVDS_KC_SPMV);
  const double sb = sizeof(TB);
  ACC_BEFORE_ATT(kc);
  double bytes;
  if (op.dense) {
    if (op.vt == SVDS_F64) dense_launch<double, TB>(P, trans, x, xs, coef, yprev, y, side_dst, side_len);
    else if (op.vt == SVDS_F32) dense_launch<float, TB>(P, trans, x, xs, coef, yprev, y, side_dst, side_len);
    else dense_launch<uint16_t, TB>(P, trans, x, xs, coef, yprev, y, side_dst, side_len);
    LAUNCH_CHECK();
    bytes = vsize(op.vt) * op.m * op.n + sb * cols + (yprev ? 2.0 : 1.0) * sb * rows;
  } else {
    // panelled transpose: partial products y_g = xs A_g^T u_g into ypart,
    // then their fixed-order sum minus coef * yprev
    const bool panels = trans && op.npanel > 1;
    const SpmvPlan &sp = panels ? op.bwdp : trans ? op.bwd : op.fwd;
    const int32_t *rp = panels ? op.prp : trans ? op.trp : op.rp;
    const int32_t *ci = panels ? op.pci : trans ? op.tci : op.ci;
    const void *val = panels ? op.pval : trans ? op.tval : op.val;
    const bool srt = sp.sorted && sp.spos;
    const uint16_t *spos = srt ? sp.spos : nullptr;
    const int32_t *cs = srt ? sp.scol : ci;
    const void *vs = srt ? sp.sval : val;
    // FP32 phase of a mixed solve on FP64 values: the FP32 copy of the array
    // chosen above (none: the FP64 values serve)
    const float *v32p = nullptr;
    if (std::is_same<TB, float>::value && op.val32)
      v32p = vs == op.val ? op.val32 : vs == op.tval ? op.tval32 : vs == op.pval ? op.pval32
           : vs == op.fwd.sval ? op.fsval32 : vs == op.bwd.sval ? op.bsval32 : nullptr;
    const bool v32 = v32p != nullptr;
    if (v32) vs = v32p;
    TB *yk = panels ? reinterpret_cast<TB *>(op.ypart) : y;
    const double *ck = panels ? nullptr : coef;
    const TB *ypk = panels ? nullptr : yprev;
    TB *parts = reinterpret_cast<TB *>(sp.partials);
    const bool fix = sp.nlong > 0;
#define SPMV_LAUNCH(TV, PROJ)                                                                              \
  klaunch(P->acc, true, !fix && !panels, spmv_csr_kernel<TV, TB, PROJ>, dim3(sp.nitems), dim3(SPMV_THREADS), 0,  \
          P->stream, sp.items, rp, cs, static_cast<const TV *>(vs), spos, x, xs, ck, ypk, yk, parts, side_dst,  \
          side_len, sp.x_tile_inst, sp.active, sp.side_tiles, sp.side_ntiles, pj)
    if (op.vt == SVDS_F64 && !v32) {
      if (pj.Q) SPMV_LAUNCH(double, true);
      else SPMV_LAUNCH(double, false);
    } else {
      if (pj.Q) SPMV_LAUNCH(float, true);
      else SPMV_LAUNCH(float, false);
    }
#undef SPMV_LAUNCH
    if (fix)
      klaunch(P->acc, false, !panels, spmv_longrow_fixup_kernel<TB>, dim3(sp.nlong), dim3(WAVE), 0, P->stream,
              sp.longrows, sp.nlong, parts, xs, ck, ypk, yk, sp.active);
    if (panels)
      klaunch(P->acc, false, true, spmv_panel_sum_kernel<TB>, dim3(ceil_div(op.n, 256)), dim3(256), 0, P->stream,
              op.n, op.npanel, yk, coef, yprev, y);
    LAUNCH_CHECK();
    bytes = 4.0 * (rows + 1) + (4.0 + (v32 ? 4.0 : vsize(op.vt))) * op.nnz + sb * cols +
            (yprev ? 2.0 : 1.0) * sb * rows;
  }
  if (side_dst) bytes += 2.0 * sb * side_len;
  if (pj.Q) bytes += sb * static_cast<double>(rows) * pj.jq;  // the first CGS pass's read of the basis
  ACC_AFTER(kc, bytes, 2.0 * (op.dense ? op.m * op.n : op.nnz) + 2.0 * static_cast<double>(rows) * pj.jq);
  if (kc_over < 0) {
    if (trans) ++P->n_spmvT;
    else ++P->n_spmv;
  }
  return SVDS_OK;
}

// ---------------------------------------------------------------------------
// CGS2 against Q[:, 0:j] and the norm/finish step.
// w is the input; w1 is scratch; out receives the re-orthogonalized vector.
// ---------------------------------------------------------------------------
template <typename TB>
// q_alg = false: this read of Q repeats one the same CGS2 already counted
// (the split second pass of a basis wider than CGS_FUSED_MAXJ), so only the
// vector counts as algorithmic bytes.
// np_out non-null: with at most CGS_FUSE_NP slabs the reduction is left to
// the next pass (*np_out = nslab, partials in part); otherwise *np_out = 0.
static int proj_and_reduce(svds_plan *P, TB *part, const TB *Q, int64_t ldq, int64_t L, int j,
                           const TB *w, TB *h, int kc, int normw = 0, const int *cmask = nullptr,
                           bool q_alg = true, int *np_out = nullptr) {
  const double sb = sizeof(TB);
  int nslab, ngc;
  cgs_proj_shape(L, j, nslab, ngc);
  if (P->cgs_slab_shift > 0)
    nslab = static_cast<int>(std::min<int64_t>({int64_t(nslab) << P->cgs_slab_shift, CGS_MAX_SLABS,
                                                 std::max<int64_t>(nslab, ceil_div(L, 256))}));
  else if (P->cgs_slab_shift < 0)
    nslab = std::max(1, nslab >> -P->cgs_slab_shift);
  constexpr int NV = 16 / sizeof(TB);
  ACC_BEFORE_ATT(kc);
  const bool vec = cgs_rows_per_lane<TB>(Q, ldq, w, nullptr, nullptr) == NV;
  const dim3 g(nslab, ngc), b(CGS_THREADS);
  if (cmask && vec)
    klaunch(P->acc, true, true, cgs_proj_kernel<TB, NV, true>, g, b, 0, P->stream, Q, ldq, L, j, w, part, normw, cmask);
  else if (cmask)
    klaunch(P->acc, true, true, cgs_proj_kernel<TB, 1, true>, g, b, 0, P->stream, Q, ldq, L, j, w, part, normw, cmask);
  else if (vec)
    klaunch(P->acc, true, true, cgs_proj_kernel<TB, NV>, g, b, 0, P->stream, Q, ldq, L, j, w, part, normw, cmask);
  else
    klaunch(P->acc, true, true, cgs_proj_kernel<TB, 1>, g, b, 0, P->stream, Q, ldq, L, j, w, part, normw, cmask);
  LAUNCH_CHECK();
  // with a column mask the columns read are counted at the end of the solve
  const double jc = cmask ? 0.0 : static_cast<double>(j);
  ACC_AFTER(kc, sb * L * (q_alg ? jc : 0.0) + sb * L, 2.0 * L * jc);
  if (np_out) {
    *np_out = nslab <= CGS_FUSE_NP ? nslab : 0;
    if (*np_out) return SVDS_OK;
  }
  // h[0:j], and with normw h[j] = |w|^2
  ACC_BEFORE(SVDS_KC_CGS_REDUCE);
  hipLaunchKernelGGL((reduce_cols_kernel<TB>), dim3(ceil_div(j + normw, 4)), dim3(256), 0, P->stream, part,
                     static_cast<int64_t>(nslab), nslab, j + normw, h);
  LAUNCH_CHECK();
  ACC_AFTER(SVDS_KC_CGS_REDUCE, sb * (j + normw) * nslab, 0.0);
  return SVDS_OK;
}

// out = w - Q h, with squared-norm partials in npart when non-null; returns
// the number of partials.  Short vectors take the tile-per-block kernel.
// sel/ran: the selective second pass (see cgs_second_pass_width).
template <typename TB>
static int launch_upd_norm(svds_plan *P, const TB *Q, int64_t ldq, int64_t L, int j, const TB *w, const TB *h,
                           TB *out, double *npart, const TB *sel = nullptr, int *ran = nullptr,
                           const int *cmask = nullptr, CgsCoef<TB> cf = {nullptr, 0, nullptr}) {
  constexpr int NV = 16 / sizeof(TB);
  const bool vec = cgs_rows_per_lane<TB>(Q, ldq, w, out, nullptr) == NV;
  const int nr = vec ? NV : 1;
  if (j > 0 && cgs_tile_upd_ok(L, j, nr)) {
    const int nt = static_cast<int>(ceil_div(L, static_cast<int64_t>(WAVE) * nr));
    const int nw = static_cast<int>(ceil_div(j, CGS_TILE_CPW));
    const dim3 g(nt), b(nw * WAVE);
    if (cmask && vec)
      klaunch(P->acc, true, true, cgs_tile_upd_kernel<TB, NV, true>, g, b, 0, P->stream, Q, ldq, L, j, w, h, out,
              npart, sel, ran, cmask, cf);
    else if (cmask)
      klaunch(P->acc, true, true, cgs_tile_upd_kernel<TB, 1, true>, g, b, 0, P->stream, Q, ldq, L, j, w, h, out,
              npart, sel, ran, cmask, cf);
    else if (vec)
      klaunch(P->acc, true, true, cgs_tile_upd_kernel<TB, NV>, g, b, 0, P->stream, Q, ldq, L, j, w, h, out, npart,
              sel, ran, cmask, cf);
    else
      klaunch(P->acc, true, true, cgs_tile_upd_kernel<TB, 1>, g, b, 0, P->stream, Q, ldq, L, j, w, h, out, npart,
              sel, ran, cmask, cf);
    return nt;
  }
  const int nn = cgs_updnorm_blocks(L);
  const dim3 g(nn), b(CGS_THREADS);
  if (cmask && j > 0 && vec)
    klaunch(P->acc, true, true, cgs_upd_norm_kernel<TB, NV, true>, g, b, 0, P->stream, Q, ldq, L, j, w, h, out,
            npart, sel, ran, cmask, cf);
  else if (cmask && j > 0)
    klaunch(P->acc, true, true, cgs_upd_norm_kernel<TB, 1, true>, g, b, 0, P->stream, Q, ldq, L, j, w, h, out,
            npart, sel, ran, cmask, cf);
  else if (vec)
    klaunch(P->acc, true, true, cgs_upd_norm_kernel<TB, NV>, g, b, 0, P->stream, Q, ldq, L, j, w, h, out, npart, sel,
            ran, cmask, cf);
  else
    klaunch(P->acc, true, true, cgs_upd_norm_kernel<TB, 1>, g, b, 0, P->stream, Q, ldq, L, j, w, h, out, npart, sel,
            ran, cmask, cf);
  return nn;
}

// Partial re-orthogonalization of one new vector (SVDS_FLAG_PARTIAL_REORTH):
// side 0 = v_{i+1} from A^T u_i, side 1 = u_i from A v_i; full = the vector
// is taken against the whole basis (restart vector of eq. (7)) and only its
// estimate row is reset.
struct OmegaStep {
  int side, i;
  bool full;
};

// Workgroups of the finish step (finish_norm_coop_kernel when above one):
// one unless wide repairs are on (SVDS_FLAG_EXPECT_BREAKDOWNS, or a
// breakdown in an earlier cycle of the solve: a cooperative dispatch costs
// ~17 us more than a plain one on MI355X, at every step), for short bases,
// for the start-vector norm and while the stream is being captured (a grid
// barrier needs a cooperative launch, which a captured graph does not
// promise); otherwise one per FINISH_ROWS_COLS entries of the basis, up to
// FINISH_MAX_BLOCKS, so that a breakdown's repair streams the basis over
// that many CUs.
// Second half of the projection partials (a pass writes there while it
// sums the first pass's partials).  A fused second pass has at most 512
// workgroups of partials for up to CGS_MAXJ columns, or 1024 for 16.
constexpr int64_t CGS_PART_HALF = int64_t(CGS_MAXJ) * CGS_MAX_SLABS / 2;
constexpr int64_t FINISH_ROWS_COLS = int64_t(1) << 20;
constexpr int FINISH_MAX_BLOCKS = 128;
static_assert(2 * FINISH_MAX_BLOCKS * (CGS_MAXJ + 1) * 8 <= CGS_MAXJ * CGS_MAX_SLABS * 4,
              "the finish partials must fit the projection partials of FP32 bases");

static int finish_blocks(const svds_plan *P, int64_t L, int j, int mode) {
  if (!P->wide_repair || mode != MODE_LANCZOS || P->capturing || L * j < 2 * FINISH_ROWS_COLS) return 1;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(P->stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return 1;
  return static_cast<int>(std::min<int64_t>(FINISH_MAX_BLOCKS, L * j / FINISH_ROWS_COLS));
}

template <typename TB>
// pre_np > 0: the product that formed w also left the first pass's pre_np
// partials per column in part (spmv_proj_np), so pass 1 runs no launch.
static int cgs2_finish(svds_plan *P, TB *part, TB *h1, TB *h2, const TB *Q, int64_t ldq, int64_t L, int j,
                       const TB *w, TB *w1, TB *out, int mode, double *t_entry, double *xs,
                       const OmegaStep *om = nullptr, int pre_np = 0) {
  const double sb = sizeof(TB);
  const Small &s = P->sc;
  const TB *src = w;
  constexpr int NV = 16 / sizeof(TB);
  const bool vec = cgs_rows_per_lane<TB>(Q, ldq, w, w1, out) == NV;
  int rc;
  // selective second pass: |w|^2 and |w1|^2 ride along as column j of the
  // first two passes' reductions
  const int sel = (P->selective && j > 0) ? 1 : 0;
  // partial re-orthogonalization: |w| and the estimates pick the columns
  const int *cmask = nullptr;
  if (om && !om->full && j > 0) {
    const int nb = static_cast<int>(std::min<int64_t>(1024, std::max<int64_t>(1, ceil_div(L, 2048))));
    ACC_BEFORE(SVDS_KC_CGS_REDUCE);
    hipLaunchKernelGGL((norm_partials_kernel<TB>), dim3(nb), dim3(256), 0, P->stream, L, w, s.npart);
    OmegaArgs oa{s.T, P->p + 1, om->side, om->i, s.npart, nb, s.sigma_est, s.om_mu, s.om_nu,
                 om->side ? s.om_fu : s.om_fv, s.om_mask, s.om_pend, s.om_nrm0,
                 s.om_stats + (om->side ? 0 : 4), OMEGA_TAU, OMEGA_ETA};
    hipLaunchKernelGGL(omega_kernel, dim3(1), dim3(CGS_THREADS), 0, P->stream, oa);
    LAUNCH_CHECK();
    ACC_AFTER(SVDS_KC_CGS_REDUCE, sb * L + 8.0 * nb, 2.0 * L);
    cmask = s.om_mask;
  }
  // Short vectors (at most CGS_FUSE_NP partials per column), without the
  // selective or partial forms: each pass sums the previous projection's
  // partials itself and the reduction launches are skipped; its workgroup 0
  // still stores h1 / h2 (the harmonic restart reads them).
  const bool fuse = !sel && !cmask;
  CgsCoef<TB> cf2{nullptr, 0, nullptr};
  if (j > 0) {
    // pass 1: h1 = Q^T w
    int np1 = fuse ? pre_np : 0;
    if (!np1 && (rc = proj_and_reduce<TB>(P, part, Q, ldq, L, j, w, h1, SVDS_KC_CGS_PROJ, sel, cmask, true,
                                          fuse ? &np1 : nullptr)))
      return rc;
    const CgsCoef<TB> cf1{np1 ? part : nullptr, np1, h1};
    // pass 2 writes its partials past pass 1's while those are being read
    TB *part2 = np1 ? part + CGS_PART_HALF : part;
    // pass 2: w1 = w - Q h1, h2 = Q^T w1
    int cpw = cgs_fused_cpw(j, static_cast<int>(sizeof(TB)));
    // a forced width must keep the block within 16 waves
    if (cpw && P->cgs_cpw && ceil_div(j, P->cgs_cpw) <= 16) cpw = P->cgs_cpw;
    if (cpw) {
      const int nb = cgs_updproj_blocks(L, j);
      const int nw = static_cast<int>(ceil_div(j, cpw));
      ACC_BEFORE_ATT(SVDS_KC_CGS_UPDPROJ);
      // one row per lane with register prefetch (two rows per lane raise
      // register pressure); FP32 bases with 10 columns take 16-byte rows
      const dim3 g(nb), b(nw * WAVE);
      if (cmask && cpw == 20)
        klaunch(P->acc, true, true, cgs_upd_proj_wide_kernel<TB, true>, g, b, 0, P->stream, Q, ldq, L, j, w, h1, w1,
                part2, sel, cmask, cf1);
      else if (cpw == 20)
        klaunch(P->acc, true, true, cgs_upd_proj_wide_kernel<TB>, g, b, 0, P->stream, Q, ldq, L, j, w, h1, w1, part2,
                sel, cmask, cf1);
      else if (cmask && cpw == 8)
        klaunch(P->acc, true, true, cgs_upd_proj_kernel<TB, 8, true, 1, true>, g, b, 0, P->stream, Q, ldq, L, j, w,
                h1, w1, part2, sel, cmask, cf1);
      else if (cmask && sizeof(TB) == 8)
        klaunch(P->acc, true, true, cgs_upd_proj_kernel<TB, 10, true, 1, true>, g, b, 0, P->stream, Q, ldq, L, j, w,
                h1, w1, part2, sel, cmask, cf1);
      else if (cmask && vec)
        klaunch(P->acc, true, true, cgs_upd_proj_kernel<TB, 10, false, NV, true>, g, b, 0, P->stream, Q, ldq, L, j,
                w, h1, w1, part2, sel, cmask, cf1);
      else if (cmask)
        klaunch(P->acc, true, true, cgs_upd_proj_kernel<TB, 10, false, 1, true>, g, b, 0, P->stream, Q, ldq, L, j,
                w, h1, w1, part2, sel, cmask, cf1);
      else if (cpw == 8)
        klaunch(P->acc, true, true, cgs_upd_proj_kernel<TB, 8, true, 1>, g, b, 0, P->stream, Q, ldq, L, j, w, h1, w1,
                part2, sel, cmask, cf1);
      else if (sizeof(TB) == 8)
        klaunch(P->acc, true, true, cgs_upd_proj_kernel<TB, 10, true, 1>, g, b, 0, P->stream, Q, ldq, L, j, w, h1,
                w1, part2, sel, cmask, cf1);
      else if (vec)
        klaunch(P->acc, true, true, cgs_upd_proj_kernel<TB, 10, false, NV>, g, b, 0, P->stream, Q, ldq, L, j, w, h1,
                w1, part2, sel, cmask, cf1);
      else
        klaunch(P->acc, true, true, cgs_upd_proj_kernel<TB, 10, false, 1>, g, b, 0, P->stream, Q, ldq, L, j, w, h1,
                w1, part2, sel, cmask, cf1);
      LAUNCH_CHECK();
      const double jc = cmask ? 0.0 : static_cast<double>(j);
      ACC_AFTER(SVDS_KC_CGS_UPDPROJ, sb * L * jc + 2 * sb * L, 4.0 * L * jc);
      if (fuse && nb <= CGS_FUSE_NP) {
        cf2 = {part2, nb, h2};
      } else {
        ACC_BEFORE(SVDS_KC_CGS_REDUCE);
        hipLaunchKernelGGL((reduce_cols_kernel<TB>), dim3(ceil_div(j + sel, 4)), dim3(256), 0, P->stream, part2,
                           static_cast<int64_t>(nb), nb, j + sel, h2);
        LAUNCH_CHECK();
        ACC_AFTER(SVDS_KC_CGS_REDUCE, sb * (j + sel) * nb, 0.0);
      }
    } else {
      // wide basis: separate update and projection passes
      ACC_BEFORE_ATT(SVDS_KC_CGS_UPDPROJ);
      launch_upd_norm<TB>(P, Q, ldq, L, j, w, h1, w1, nullptr, nullptr, nullptr, cmask, cf1);
      LAUNCH_CHECK();
      const double jc = cmask ? 0.0 : static_cast<double>(j);
      ACC_AFTER(SVDS_KC_CGS_UPDPROJ, sb * L * jc + 2 * sb * L, 2.0 * L * jc);
      if ((rc = proj_and_reduce<TB>(P, part, Q, ldq, L, j, w1, h2, SVDS_KC_CGS_UPDPROJ, sel, cmask, false)))
        return rc;
    }
    src = w1;
  }
  // pass 3: out = w1 - Q h2 and its norm (selective: only when the test asks
  // for it; the accounting then counts the vector traffic alone)
  ACC_BEFORE_ATT(SVDS_KC_CGS_UPDNORM);
  const int nn = launch_upd_norm<TB>(P, Q, ldq, L, j, src, h2, out, s.npart, sel ? h1 + j : nullptr,
                                     sel ? s.bd + 1 : nullptr, cmask, cf2);
  LAUNCH_CHECK();
  const int jn = (sel || cmask) ? 0 : j;
  ACC_AFTER(SVDS_KC_CGS_UPDNORM, sb * L * jn + 2 * sb * L, 2.0 * L * jn + 2.0 * L);
  if (sel) ++P->reorth_calls;
  FinishArgs fa{t_entry, xs, s.sigma_est, s.bd, P->opts.seed};
  if (om) {
    fa.om_row = om->side ? s.om_mu : s.om_nu;
    fa.om_pend = s.om_pend;
    fa.om_mask = s.om_mask;
    fa.om_nrm0 = s.om_nrm0;
    fa.om_force = om->side ? s.om_fu : s.om_fv;
    fa.om_full = (om->full || j == 0) ? 1 : 0;
  }
  ACC_BEFORE(SVDS_KC_CGS_REDUCE);
  const int G = finish_blocks(P, L, j, mode);
  bool wide = false;
  if (G > 1) {
    double *cpart = reinterpret_cast<double *>(part);
    const double *np = s.npart;
    int64_t ldq_ = ldq, L_ = L;
    int nn_ = nn, mode_ = mode, j_ = j;
    void *args[] = {&np, &nn_, &mode_, &fa, &Q, &ldq_, &L_, &j_, &out, &cpart};
    // a cooperative launch the runtime refuses (its workgroups cannot all be
    // resident) leaves the step to the one-workgroup finish
    wide = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&finish_norm_coop_kernel<TB>), dim3(G),
                                      dim3(FINISH_THREADS), args, 0, P->stream) == hipSuccess;
    if (!wide) (void)hipGetLastError();
  }
  if (!wide)
    hipLaunchKernelGGL((finish_norm_kernel<TB>), dim3(1), dim3(FINISH_THREADS), 0, P->stream, s.npart, nn,
                       mode, fa, Q, ldq, L, j, out);
  LAUNCH_CHECK();
  ACC_AFTER(SVDS_KC_CGS_REDUCE, 8.0 * nn, 0.0);
  return SVDS_OK;
}

template <typename TB>
static int cgs2_finish(svds_plan *P, Lanczos<TB> &Lz, const TB *Q, int64_t ldq, int64_t L, int j,
                       const TB *w, TB *w1, TB *out, int mode, double *t_entry, double *xs,
                       const OmegaStep *om = nullptr, int pre_np = 0) {
  return cgs2_finish<TB>(P, Lz.partials, Lz.h1, Lz.h2, Q, ldq, L, j, w, w1, out, mode, t_entry, xs, om, pre_np);
}

// Update only: out = w - Q h (restart, eq. (7)).
template <typename TB>
static int gemv_update(svds_plan *P, const TB *Q, int64_t ldq, int64_t L, int j, const TB *w,
                       const TB *h, TB *out) {
  const double sb = sizeof(TB);
  ACC_BEFORE(SVDS_KC_OTHER);
  launch_upd_norm<TB>(P, Q, ldq, L, j, w, h, out, nullptr);
  LAUNCH_CHECK();
  ACC_AFTER(SVDS_KC_OTHER, sb * L * j + 2 * sb * L, 2.0 * L * j);
  return SVDS_OK;
}

template <typename TB, typename TO>
static int rotate(svds_plan *P, int64_t L, int pc, int kc, const TB *B, int64_t ldb,
                  const double *Y, int64_t ldy, TO *out, int64_t ldo) {
  ACC_BEFORE(SVDS_KC_ROTATE);
  HIP_TRY((rotate_launch<TB, TO>(P->stream, L, pc, kc, B, ldb, Y, ldy, P->sc.yt, out, ldo)));
  ACC_AFTER(SVDS_KC_ROTATE, sizeof(TB) * double(L) * pc * ceil_div(kc, ROT_KC) + sizeof(TO) * double(L) * kc,
            2.0 * L * pc * kc);
  return SVDS_OK;
}

// ---------------------------------------------------------------------------
// Early stop (SVDS_FLAG_EARLY_STOP): checks of the eq. (4) test at an
// intermediate Lanczos dimension j.
// ---------------------------------------------------------------------------
// Tc ((j+1) x (j+1), row-major) = the leading j x j block of T with
// beta_j = T(j-1, j) in its last column and a zero last row: the layout the
// small SVD takes for dimension j.  One block; also copies sigma_est.
static __global__ void early_tblock_kernel(const double *__restrict__ T, int ld, int j, double *__restrict__ Tc,
                                           const double *__restrict__ sig_in, double *__restrict__ sig_out) {
  const int n = (j + 1) * (j + 1);
  for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
    const int r = idx / (j + 1), c = idx - r * (j + 1);
    Tc[idx] = r < j ? T[r * ld + c] : 0.0;
  }
  if (threadIdx.x == 0) *sig_out = *sig_in;
}

// Worker thread of one check: the small SVD of the copied block on the side
// stream, then the flags and the largest estimate for the host.
static void early_worker(svds_plan *P, int j, double tol) {
  EarlyCheck &e = P->ec;
  int rc = SVDS_OK;
  double mx = 0;
  if (hipSetDevice(P->device) != hipSuccess) {
    rc = SVDS_EDEVICE;
  } else {
    rc = svds_small_svd_run(e.stream, e.T, j, P->k, tol, e.jac, e.Uk, e.Vext, e.sig, e.res, e.rho, e.flags,
                            e.sigma_est, e.h_flags + 4, P->smallest ? 1 : 0);
    std::vector<double> r(P->k);
    if (!rc && (hipMemcpyAsync(e.h_flags, e.flags, 4 * sizeof(int), hipMemcpyDeviceToHost, e.stream) != hipSuccess ||
                hipMemcpyAsync(r.data(), e.res, sizeof(double) * P->k, hipMemcpyDeviceToHost, e.stream) !=
                    hipSuccess ||
                hipStreamSynchronize(e.stream) != hipSuccess))
      rc = SVDS_EDEVICE;
    for (double v : r) mx = std::max(mx, v);
  }
  e.rc = rc;
  e.passed = (!rc && e.h_flags[0]) ? 1 : 0;
  e.sweeps = rc ? 0 : e.h_flags[2];
  e.max_res = mx;
  e.state.store(2, std::memory_order_release);
}

// Collects a finished check: a passing one ends the cycle (stop_j); a failed
// one schedules the next check from the decrease of the largest estimate
// between the last two checks (their steps per decade, extrapolated to tol).
static int early_collect(svds_plan *P, double tol) {
  EarlyCheck &e = P->ec;
  if (e.state.load(std::memory_order_acquire) != 2) return SVDS_OK;
  e.worker.join();
  e.state.store(0);
  ++e.checks;
  P->jac_sweeps += e.sweeps;
  if (e.rc) return e.rc;
  if (e.passed) {
    e.stop_j = e.j_run;
    return SVDS_OK;
  }
  int step = 8;
  if (e.j_prev > 0 && e.r_prev > e.max_res && e.max_res > 0) {
    const double per_decade = (e.j_run - e.j_prev) / std::log10(e.r_prev / e.max_res);
    const double need = per_decade * std::log10(e.max_res / tol);
    step = static_cast<int>(std::min(16.0, std::max(2.0, std::floor(need))));
  }
  e.j_prev = e.j_run;
  e.r_prev = e.max_res;
  e.next_j = e.j_run + step;
  return SVDS_OK;
}

// Starts a check of dimension j = (V steps done) once the device has finished
// them (event on the main stream).
static int early_start(svds_plan *P, int j) {
  EarlyCheck &e = P->ec;
  HIP_TRY(hipEventRecord(e.ev_check, P->stream));
  HIP_TRY(hipStreamWaitEvent(e.stream, e.ev_check, 0));
  hipLaunchKernelGGL(early_tblock_kernel, dim3(1), dim3(256), 0, e.stream, P->sc.T, P->p + 1, j, e.T,
                     P->sc.sigma_est, e.sigma_est);
  HIP_TRY(hipGetLastError());
  e.j_run = j;
  e.state.store(1);
  e.worker = std::thread(early_worker, P, j, P->tol);
  return SVDS_OK;
}

// Waits for a check still running (its result is dropped: the cycle ended).
static int early_drain(svds_plan *P) {
  EarlyCheck &e = P->ec;
  if (e.worker.joinable()) e.worker.join();
  if (e.state.load() == 2) {
    ++e.checks;
    P->jac_sweeps += e.sweeps;
  }
  e.state.store(0);
  return e.rc;
}

// ---------------------------------------------------------------------------
// Alg. 1 loop from 0-based column i0 until v_p and beta_{p-1} exist.
// On entry: V[:, i0] is in the basis; the unnormalized u_{i0} is in bu with
// reciprocal norm xs_u and T(i0, i0) set.
// ---------------------------------------------------------------------------
// Small CSR problems (vectors of at most LZS_MAX_L entries, at most
// LZS_MAX_NNZ nonzeros, both bases within LZS_MAX_BASIS_BYTES, FP64 bases,
// full re-orthogonalization) run a cycle's
// Lanczos steps in one workgroup (lanczos_small_kernel); the early stop keeps
// the step-by-step launches, whose per-step events it needs.
static bool small_lanczos_ok(const svds_plan *P) {
  const Operator &op = P->op;
  return !op.dense && op.npanel == 1 && op.trp && !P->partial && !P->selective &&
         std::max(op.m, op.n) <= LZS_MAX_L && op.nnz <= LZS_MAX_NNZ &&
         8 * (op.m + op.n) * (P->p + 1) <= LZS_MAX_BASIS_BYTES;
}

static int lanczos_small(svds_plan *P, Lanczos<double> &Lz, int i0) {
  const Operator &op = P->op;
  const Small &s = P->sc;
  const int p = P->p;
  const size_t lds = sizeof(double) * static_cast<size_t>(std::max(op.m, op.n));
  ACC_BEFORE(SVDS_KC_OTHER);
  if (op.vt == SVDS_F64)
    hipLaunchKernelGGL(lanczos_small_kernel<double>, dim3(1), dim3(LZS_THREADS), lds, P->stream,
                       static_cast<int>(op.m), static_cast<int>(op.n), op.rp, op.ci,
                       static_cast<const double *>(op.val), op.trp, op.tci, static_cast<const double *>(op.tval),
                       Lz.U[Lz.cur], Lz.ldu, Lz.V[Lz.cur], Lz.ldv, s.T, p + 1, i0, p, Lz.bu, Lz.bv, s.xs_u,
                       s.xs_v, s.sigma_est, s.bd, P->opts.seed);
  else
    hipLaunchKernelGGL(lanczos_small_kernel<float>, dim3(1), dim3(LZS_THREADS), lds, P->stream,
                       static_cast<int>(op.m), static_cast<int>(op.n), op.rp, op.ci,
                       static_cast<const float *>(op.val), op.trp, op.tci, static_cast<const float *>(op.tval),
                       Lz.U[Lz.cur], Lz.ldu, Lz.V[Lz.cur], Lz.ldv, s.T, p + 1, i0, p, Lz.bu, Lz.bv, s.xs_u,
                       s.xs_v, s.sigma_est, s.bd, P->opts.seed);
  LAUNCH_CHECK();
  const int nv = p - i0, nu = p - i0 - 1;  // A^T u and A v products of the steps
  P->n_spmvT += nv;
  P->n_spmv += nu;
  // algorithmic bytes: each product streams A once; each CGS2 reads its basis three times
  const double vb = op.vt == SVDS_F64 ? 8.0 : 4.0;
  double bytes = (nv + nu) * (12.0 + vb) * op.nnz;
  for (int i = i0; i < p; ++i) bytes += 24.0 * op.n * (i + 1) + (i + 1 < p ? 24.0 * op.m * (i + 1) : 0.0);
  ACC_AFTER(SVDS_KC_OTHER, bytes, 2.0 * bytes / 8.0);
  return SVDS_OK;
}

template <typename TB> static int lanczos(svds_plan *P, Lanczos<TB> &Lz, int i0, bool early = false) {
  if constexpr (std::is_same<TB, double>::value)
    if (!early && small_lanczos_ok(P)) return lanczos_small(P, Lz, i0);
  const int p = P->p;
  const int64_t m = Lz.m, n = Lz.n;
  const int ld = p + 1;
  const Small &s = P->sc;
  TB *U = Lz.U[Lz.cur], *V = Lz.V[Lz.cur];
  EarlyCheck &e = P->ec;
  if (early) {
    e.stop_j = 0;
    e.j_prev = 0;
    e.next_j = P->k + 1 + std::max(2, (p - P->k) / 8);
  }
  for (int i = i0; i < p; ++i) {
    if (early) {
      int rc = early_collect(P, P->tol);
      if (rc) return rc;
      if (e.stop_j) return SVDS_OK;  // converged at e.stop_j: the steps after it are not needed
      // stay at most EARLY_LAG steps ahead of the device
      if (i - i0 >= EARLY_LAG) HIP_TRY(hipEventSynchronize(e.ev_step[i % EARLY_LAG]));
    }
    // Alg. 1 steps 5-6: v_{i+1} = A^T u_i - alpha_i v_i, CGS2 against V[:, 0..i], beta_i.
    // The product also writes the normalized u_i into U[:, i].
    // Short products also form the first CGS pass's partials (spmv_proj_np).
    const int npv = spmv_proj_np(P, true, i + 1);
    int rc = matvec<TB>(P, true, Lz.bu, s.xs_u, s.T + i * ld + i, V + i * Lz.ldv, Lz.wv,
                        U + i * Lz.ldu, m, -1, SpmvProj<TB>{npv ? V : nullptr, Lz.ldv, i + 1, Lz.partials});
    if (rc) return rc;
    const OmegaStep omv{0, i, false};
    rc = cgs2_finish<TB>(P, Lz, V, Lz.ldv, n, i + 1, Lz.wv, Lz.w1v, Lz.bv, MODE_LANCZOS,
                         s.T + i * ld + i + 1, s.xs_v, P->partial ? &omv : nullptr, npv);
    if (rc) return rc;
    if (early) {
      HIP_TRY(hipEventRecord(e.ev_step[i % EARLY_LAG], P->stream));
      // T(1:j, 1:j) and beta_j exist for j = i + 1
      if (i + 1 < p && i + 1 >= e.next_j && e.state.load() == 0 && (rc = early_start(P, i + 1))) return rc;
    }
    if (i == p - 1) {
      // v_{p+1}: normalized into V[:, p] (no product consumes it in this cycle)
      hipLaunchKernelGGL((scale_copy_kernel<TB>), dim3(ceil_div(n, 256)), dim3(256), 0, P->stream,
                         n, Lz.bv, s.xs_v, V + p * Lz.ldv);
      LAUNCH_CHECK();
      break;
    }
    // Alg. 1 steps 7-8: u_{i+1} = A v_{i+1} - beta_i u_i, CGS2 against U[:, 0..i], alpha_{i+1}.
    const int npu = spmv_proj_np(P, false, i + 1);
    rc = matvec<TB>(P, false, Lz.bv, s.xs_v, s.T + i * ld + i + 1, U + i * Lz.ldu, Lz.wu,
                    V + (i + 1) * Lz.ldv, n, -1, SpmvProj<TB>{npu ? U : nullptr, Lz.ldu, i + 1, Lz.partials});
    if (rc) return rc;
    const OmegaStep omu{1, i + 1, false};
    rc = cgs2_finish<TB>(P, Lz, U, Lz.ldu, m, i + 1, Lz.wu, Lz.w1u, Lz.bu, MODE_LANCZOS,
                         s.T + (i + 1) * ld + i + 1, s.xs_u, P->partial ? &omu : nullptr, npu);
    if (rc) return rc;
  }
  // the cycle ran to p: a check still running is no longer needed
  return early ? early_drain(P) : SVDS_OK;
}

// Alg. 1 steps 1-3: v_1 = v0 / |v0| (v0 given as FP64 or drawn from Philox),
// u_1 = A v_1, alpha_1.  `v0` may be FP64 device data of length n.
template <typename TB> static int start(svds_plan *P, Lanczos<TB> &Lz, const double *v0) {
  const int64_t n = Lz.n, m = Lz.m;
  const Small &s = P->sc;
  Lz.cur = 0;
  if (v0) {
    hipLaunchKernelGGL((cast_copy_kernel<double, TB>), dim3(ceil_div(n, 256)), dim3(256), 0,
                       P->stream, n, v0, Lz.w1v);
  } else {
    hipLaunchKernelGGL((philox_fill_kernel<TB>), dim3(ceil_div(ceil_div(n, 2), 256)), dim3(256), 0,
                       P->stream, n, P->opts.seed, 0u, Lz.w1v);
  }
  LAUNCH_CHECK();
  // bv = v0, xs_v = 1/|v0| (no basis: the finish kernel only normalizes)
  int rc = cgs2_finish<TB>(P, Lz, nullptr, 0, n, 0, Lz.w1v, nullptr, Lz.bv, MODE_NORM, nullptr, s.xs_v);
  if (rc) return rc;
  // u = A v_1; V[:, 0] = v0 * xs_v written by the product
  rc = matvec<TB>(P, false, Lz.bv, s.xs_v, nullptr, nullptr, Lz.wu, Lz.V[0], n);
  if (rc) return rc;
  // alpha_1 (no re-orthogonalization for the first vector)
  if (P->partial) {
    hipLaunchKernelGGL(omega_init_kernel, dim3(1), dim3(256), 0, P->stream, P->p, s.om_mu, s.om_nu, s.om_fu,
                       s.om_fv, s.om_stats);
    LAUNCH_CHECK();
  }
  const OmegaStep om0{1, 0, true};
  return cgs2_finish<TB>(P, Lz, nullptr, 0, m, 0, Lz.wu, nullptr, Lz.bu, MODE_LANCZOS, s.T, s.xs_u,
                         P->partial ? &om0 : nullptr);
}

// Alg. 2 steps 4-7: small SVD, eq. (4) test; returns converged flag via h_flags.
static int small_svd(svds_plan *P) {
  const int p = P->p;
  const Small &s = P->sc;
  ACC_BEFORE(SVDS_KC_SMALLSVD);
  int rc;
  // the harmonic restart's SVD reads T before the Ritz SVD rewrites it
  if (P->harmonic &&
      (rc = svds_harmonic_basis_run(P->stream, s.T, p, P->k, s.jac, s.hQC, s.hQM, s.hR, P->h_flags + 16)))
    return rc;
  rc = svds_small_svd_run(P->stream, s.T, p, P->k, P->tol, s.jac, s.Uk, s.Vext, s.sig, s.res, s.rho, s.flags,
                          s.sigma_est, P->h_flags + 16, P->smallest ? 1 : 0);
  if (rc) return rc;
  ACC_AFTER(SVDS_KC_SMALLSVD, 16.0 * (p + 1) * (p + 1), 0.0);
  HIP_TRY(hipMemcpyAsync(P->h_flags, s.flags, 4 * sizeof(int), hipMemcpyDeviceToHost, P->stream));
  HIP_TRY(hipMemcpyAsync(P->h_flags + 8, s.bd, sizeof(int), hipMemcpyDeviceToHost, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  P->jac_sweeps += P->h_flags[2];
  if (P->h_flags[8] > 0) P->wide_repair = true;  // the matrix is rank-deficient (or nearly)
  P->p_eff = p;
  P->out_Uk = s.Uk;
  P->out_Vext = s.Vext;
  return P->acc.harvest();
}

// A cycle that an early check ended at dimension j: that check's small SVD
// becomes the cycle's (flags, estimates, singular values; Uk and Vext for the
// outputs, with leading dimensions j and j + 1).
static int early_adopt(svds_plan *P) {
  EarlyCheck &e = P->ec;
  const Small &s = P->sc;
  const int k = P->k;
  HIP_TRY(hipMemcpyAsync(s.sig, e.sig, sizeof(double) * k, hipMemcpyDeviceToDevice, P->stream));
  HIP_TRY(hipMemcpyAsync(s.res, e.res, sizeof(double) * k, hipMemcpyDeviceToDevice, P->stream));
  HIP_TRY(hipMemcpyAsync(s.flags, e.flags, 4 * sizeof(int), hipMemcpyDeviceToDevice, P->stream));
  std::memcpy(P->h_flags, e.h_flags, 4 * sizeof(int));
  P->p_eff = e.stop_j;
  P->out_Uk = e.Uk;
  P->out_Vext = e.Vext;
  return SVDS_OK;
}

// Alg. 2 steps 8-12: Ritz vectors into the other ping-pong buffer, v_{k+1} =
// v_{p+1}, u_{k+1} = A v_{k+1} - Uk rho (eq. (7)) re-orthogonalized, alpha_{k+1}.
template <typename TB> static int restart(svds_plan *P, Lanczos<TB> &Lz) {
  const int p = P->p, k = P->k, ld = p + 1;
  const Small &s = P->sc;
  const int nxt = 1 - Lz.cur;
  TB *U = Lz.U[Lz.cur], *V = Lz.V[Lz.cur];
  TB *Un = Lz.U[nxt], *Vn = Lz.V[nxt];
  if (P->harmonic) {
    // U_k = U_p Q_M, V_{k+1} = [V_p v_{p+1}] Q_C, T(1:k, 1:k) = R; u_{k+1}
    // from A v_{k+1} by CGS2 against U_k, whose two coefficient vectors
    // form T(1:k, k+1)
    int rc = rotate<TB, TB>(P, Lz.m, p, k, U, Lz.ldu, s.hQM, p, Un, Lz.ldu);
    if (rc) return rc;
    rc = rotate<TB, TB>(P, Lz.n, p + 1, k + 1, V, Lz.ldv, s.hQC, ld, Vn, Lz.ldv);
    if (rc) return rc;
    Lz.cur = nxt;
    hipLaunchKernelGGL(harm_tset_kernel, dim3(1), dim3(256), 0, P->stream, s.T, p, k, s.hR);
    LAUNCH_CHECK();
    rc = matvec<TB>(P, false, Vn + k * Lz.ldv, s.one, nullptr, nullptr, Lz.wu, nullptr, 0);
    if (rc) return rc;
    rc = cgs2_finish<TB>(P, Lz, Un, Lz.ldu, Lz.m, k, Lz.wu, Lz.w1u, Lz.bu, MODE_LANCZOS, s.T + k * ld + k,
                         s.xs_u);
    if (rc) return rc;
    hipLaunchKernelGGL((harm_couple_kernel<TB>), dim3(1), dim3(256), 0, P->stream, s.T, p, k, Lz.h1, Lz.h2);
    LAUNCH_CHECK();
    return SVDS_OK;
  }
  int rc = rotate<TB, TB>(P, Lz.m, p, k, U, Lz.ldu, s.Uk, p, Un, Lz.ldu);
  if (rc) return rc;
  rc = rotate<TB, TB>(P, Lz.n, p + 1, k + 1, V, Lz.ldv, s.Vext, ld, Vn, Lz.ldv);
  if (rc) return rc;
  Lz.cur = nxt;
  if (P->partial) {  // estimates of v_{k+1} = v_{p+1} against the kept Ritz vectors
    hipLaunchKernelGGL(omega_restart_kernel, dim3(1), dim3(CGS_THREADS), 0, P->stream, s.Vext, p, k, s.om_nu,
                       s.om_pend, s.om_fu, s.om_fv);
    LAUNCH_CHECK();
  }
  // w = A v_{k+1}
  rc = matvec<TB>(P, false, Vn + k * Lz.ldv, s.one, nullptr, nullptr, Lz.wu, nullptr, 0);
  if (rc) return rc;
  // w1 = w - Uk rho   (rho in FP64 -> basis type)
  TB *rho_b = Lz.h1;
  hipLaunchKernelGGL((cast_copy_kernel<double, TB>), dim3(1), dim3(256), 0, P->stream,
                     static_cast<int64_t>(k), s.rho, rho_b);
  LAUNCH_CHECK();
  rc = gemv_update<TB>(P, Un, Lz.ldu, Lz.m, k, Lz.wu, rho_b, Lz.w1u);
  if (rc) return rc;
  // CGS2 against Uk, alpha_{k+1} = T(k, k)
  const OmegaStep omr{1, k, true};
  return cgs2_finish<TB>(P, Lz, Un, Lz.ldu, Lz.m, k, Lz.w1u, Lz.wu, Lz.bu, MODE_LANCZOS,
                         s.T + k * ld + k, s.xs_u, P->partial ? &omr : nullptr);
}

// One cycle body through the graph cache (CycleGraphs): captured at its first
// use for this (basis type, starting buffer, work-list version), then replayed
// with one hipGraphLaunch.  `body` enqueues on P->stream and may switch
// Lz.cur; it must not synchronize or read device data on the host.
template <typename TB, typename Body>
static int run_graphed(svds_plan *P, Lanczos<TB> &Lz, uint64_t ver, Body &&body) {
  CycleGraphs &G = P->graphs;
  Accounting &acc = P->acc;
  const int t = sizeof(TB) == 8 ? 1 : 0, c = Lz.cur;
  if (G.ver[t][c] != ver) {
    G.drop(t, c);
    if (!G.cap) HIP_TRY(hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking));
    double b0[SVDS_KC_COUNT], f0[SVDS_KC_COUNT];
    int64_t l0[SVDS_KC_COUNT];
    std::memcpy(b0, acc.bytes, sizeof b0);
    std::memcpy(f0, acc.flops, sizeof f0);
    std::memcpy(l0, acc.launches, sizeof l0);
    const int64_t s0 = P->n_spmv, st0 = P->n_spmvT, rc0 = P->reorth_calls;
    const bool timing = acc.timing;
    hipStream_t user = P->stream;
    acc.timing = false;  // no event records inside a capture
    P->stream = G.cap;
    int rc = SVDS_OK;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      set_last_error(e, "hipStreamBeginCapture", __FILE__, __LINE__);
      rc = SVDS_EDEVICE;
    } else {
      P->capturing = true;
      rc = body();
      P->capturing = false;
      e = hipStreamEndCapture(G.cap, &g);
      if (!rc && e != hipSuccess) {
        set_last_error(e, "hipStreamEndCapture", __FILE__, __LINE__);
        rc = SVDS_EDEVICE;
      }
    }
    P->stream = user;
    acc.timing = timing;
    // what the body added is counted per replay, not at capture
    for (int kc = 0; kc < SVDS_KC_COUNT; ++kc) {
      G.dbytes[t][c][kc] = acc.bytes[kc] - b0[kc];
      G.dflops[t][c][kc] = acc.flops[kc] - f0[kc];
      G.dlaunch[t][c][kc] = acc.launches[kc] - l0[kc];
      acc.bytes[kc] = b0[kc];
      acc.flops[kc] = f0[kc];
      acc.launches[kc] = l0[kc];
    }
    G.dspmv[t][c] = P->n_spmv - s0;
    G.dspmvT[t][c] = P->n_spmvT - st0;
    G.dreorth[t][c] = P->reorth_calls - rc0;
    P->n_spmv = s0;
    P->n_spmvT = st0;
    P->reorth_calls = rc0;
    G.next_cur[t][c] = Lz.cur;
    Lz.cur = c;
    if (!rc) {
      hipGraphExec_t x = nullptr;
      e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        set_last_error(e, "hipGraphInstantiate", __FILE__, __LINE__);
        rc = SVDS_EDEVICE;
      } else {
        G.exec[t][c] = x;
        G.ver[t][c] = ver;
        ++G.captures;
      }
    }
    if (g) (void)hipGraphDestroy(g);
    if (rc) return rc;
  }
  HIP_TRY(hipGraphLaunch(G.exec[t][c], P->stream));
  ++G.replays;
  for (int kc = 0; kc < SVDS_KC_COUNT; ++kc) {
    acc.bytes[kc] += G.dbytes[t][c][kc];
    acc.flops[kc] += G.dflops[t][c][kc];
    acc.launches[kc] += G.dlaunch[t][c][kc];
  }
  P->n_spmv += G.dspmv[t][c];
  P->n_spmvT += G.dspmvT[t][c];
  P->reorth_calls += G.dreorth[t][c];
  Lz.cur = G.next_cur[t][c];
  return SVDS_OK;
}

// Runs cycles of one precision until the test passes with `tol_c`, maxit is
// reached, or (stagnate > 0) the largest estimate stops decreasing.
template <typename TB>
static int run_cycles(svds_plan *P, Lanczos<TB> &Lz, double tol_c, int maxit, bool stagnate,
                      int &cycles, bool &conv) {
  cycles = 0;
  conv = false;
  double best = INFINITY;
  int nodec = 0;
  const double tol_save = P->tol;
  P->tol = tol_c;
  const bool early = P->early;
  int rc = lanczos<TB>(P, Lz, 0, early);
  while (rc == SVDS_OK) {
    ++cycles;
    if (early && P->ec.stop_j) {  // converged inside the cycle
      rc = early_adopt(P);
      conv = true;
      break;
    }
    rc = small_svd(P);
    if (rc) break;
    conv = P->h_flags[0] != 0;
    if (conv || cycles >= maxit) break;
    if (stagnate) {
      double mx = 0;
      std::vector<double> r(P->k);
      HIP_TRY(hipMemcpy(r.data(), P->sc.res, sizeof(double) * P->k, hipMemcpyDeviceToHost));
      for (double v : r) mx = std::max(mx, v);
      if (mx < best) best = mx, nodec = 0;
      else if (++nodec >= 2) break;
    }
    if (P->opts.flags & SVDS_FLAG_GRAPH) {
      rc = run_graphed<TB>(P, Lz, 1, [&] {
        const int r = restart<TB>(P, Lz);
        return r ? r : lanczos<TB>(P, Lz, P->k);
      });
    } else {
      rc = restart<TB>(P, Lz);
      if (rc) break;
      rc = lanczos<TB>(P, Lz, P->k, early);
    }
  }
  if (early) {
    const int rd = early_drain(P);
    if (!rc) rc = rd;
  }
  P->tol = tol_save;
  return rc;
}

static int residuals_impl(svds_plan *P, int k, const double *U, const double *S, const double *V,
                          double *res_av, double *res_atu);

}  // namespace svds

// ===========================================================================
// Plan creation
// ===========================================================================
static int fill_defaults(const svds_opts *o, int64_t m, int64_t n, svds_plan *P) {
  if (!o) return SVDS_EINVAL;
  P->opts = *o;
  P->k = o->k;
  P->p = o->p > 0 ? o->p : std::max(15, 3 * o->k);
  P->tol = o->tol > 0 ? o->tol : 1e-10;
  P->maxit = o->maxit > 0 ? o->maxit : 10;
  P->stream = static_cast<hipStream_t>(o->stream);
  P->mixed = o->precision == SVDS_PREC_MIXED;
  P->smallest = (o->flags & SVDS_FLAG_SMALLEST) != 0;
  P->selective = (o->flags & SVDS_FLAG_SELECTIVE_REORTH) != 0;
  P->partial = (o->flags & SVDS_FLAG_PARTIAL_REORTH) != 0;
  P->harmonic = (o->flags & SVDS_FLAG_HARMONIC) != 0;
  // captured cycles replay a fixed sequence of launches: no early stop there
  P->early = (o->flags & SVDS_FLAG_EARLY_STOP) != 0 && !(o->flags & SVDS_FLAG_GRAPH);
  if (o->precision != SVDS_PREC_FP64 && o->precision != SVDS_PREC_MIXED) return SVDS_EINVAL;
  if (P->selective && P->partial) return SVDS_EINVAL;
  // harmonic restarts: smallest triplets, full re-orthogonalization
  if (P->harmonic && (!P->smallest || P->selective || P->partial)) return SVDS_EINVAL;
  // the FP32 phase cannot resolve values below ~1e-7 sigma_1
  if (P->smallest && P->mixed) return SVDS_EUNSUPPORTED;
  // the partial form's thresholds are those of FP64 arithmetic
  if (P->partial && P->mixed) return SVDS_EUNSUPPORTED;
  if (P->k < 1 || P->p <= P->k || P->p > m || P->p + 1 > n) return SVDS_EINVAL;
  if (P->p + 1 > CGS_MAXJ) return SVDS_EUNSUPPORTED;
  if (P->harmonic && P->p + 2 > CGS_MAXJ) return SVDS_EUNSUPPORTED;  // SVD of p + 1 columns
  return SVDS_OK;
}

// int32 words of device scratch a transposed copy needs (build_transpose):
// row of each nonzero, two key/value ping-pong pairs, digit histograms,
// their scan offsets and tile sums
static size_t transpose_scratch_words(int64_t nnz) {
  const int64_t ntiles = ceil_div(std::max<int64_t>(nnz, 1), RS_TILE);
  const int64_t nh = ntiles * RS_BINS;
  const int64_t nsum = ceil_div(nh, SCAN_TILE);
  return 5 * static_cast<size_t>(std::max<int64_t>(nnz, 1)) + 2 * static_cast<size_t>(nh) + nsum + 64;
}

static int carve_all(svds_plan *P, Arena &a) {
  const int p = P->p, k = P->k;
  const int64_t m = P->op.m, n = P->op.n;
  P->L64.carve(a, m, n, p);
  if (P->mixed) P->L32.carve(a, m, n, p);
  Small &s = P->sc;
  s.T = a.take<double>(static_cast<size_t>(p + 1) * (p + 1));
  s.xs_u = a.take<double>(1);
  s.xs_v = a.take<double>(1);
  s.one = a.take<double>(1);
  s.sigma_est = a.take<double>(1);
  s.rho = a.take<double>(k);
  s.sig = a.take<double>(k);
  s.res = a.take<double>(k);
  s.Uk = a.take<double>(static_cast<size_t>(p) * k);
  s.Vext = a.take<double>(static_cast<size_t>(p + 1) * (k + 1));
  s.jac = a.take<double>(std::max(jacobi_work_bytes(p), P->harmonic ? jacobi_work_bytes(p + 1) : 0) / 8 + 8);
  s.npart = a.take<double>(NPART);
  s.resid_av = a.take<double>(k);
  s.resid_atu = a.take<double>(k);
  s.bd = a.take<int>(4);
  s.flags = a.take<int>(4);
  s.yt = a.take<double>(rot_yt_doubles(p + 1, k + 1));
  s.sgn = a.take<double>(k);
  s.sgn_val = a.take<double>(static_cast<size_t>(k) * SIGN_MAX_SLABS);
  s.sgn_idx = a.take<int64_t>(static_cast<size_t>(k) * SIGN_MAX_SLABS);
  if (P->early) {
    EarlyCheck &e = P->ec;
    e.T = a.take<double>(static_cast<size_t>(p + 1) * (p + 1));
    e.Uk = a.take<double>(static_cast<size_t>(p) * k);
    e.Vext = a.take<double>(static_cast<size_t>(p + 1) * (k + 1));
    e.sig = a.take<double>(k);
    e.res = a.take<double>(k);
    e.rho = a.take<double>(k);
    e.sigma_est = a.take<double>(1);
    e.jac = a.take<double>(jacobi_work_bytes(p) / 8 + 8);
    e.flags = a.take<int>(4);
  }
  if (P->harmonic) {
    s.hQC = a.take<double>(static_cast<size_t>(p + 1) * (k + 1));
    s.hQM = a.take<double>(static_cast<size_t>(p) * k);
    s.hR = a.take<double>(static_cast<size_t>(k) * k);
  }
  if (P->partial) {
    s.om_mu = a.take<double>(p + 2);
    s.om_nu = a.take<double>(p + 2);
    s.om_pend = a.take<double>(p + 2);
    s.om_nrm0 = a.take<double>(1);
    s.om_mask = a.take<int>(p + 2);
    s.om_fu = a.take<int>(p + 2);
    s.om_fv = a.take<int>(p + 2);
    s.om_stats = a.take<long long>(8);
  }
  P->tmp_m = a.take<double>(m);
  P->tmp_n = a.take<double>(n);
  if (P->mixed) P->tmp_nk = a.take<double>(static_cast<size_t>(n) * k);
  if (P->op.dense) {
    P->op.dpart = a.take<double>(dense_partial_doubles(m, n));
    if (!(P->opts.flags & SVDS_FLAG_NO_RESIDUALS)) P->rd_part = a.take<double>(resid_dense_doubles(m, n, k));
  } else {
    P->op.fwd.partials = a.take<double>(std::max(1, P->op.fwd.npieces));
    P->op.fwd.items = a.take<int4>(P->op.fwd.nitems);
    P->op.fwd.longrows = a.take<LongRow>(std::max(1, P->op.fwd.nlong));
    P->op.bwd.partials = a.take<double>(std::max(1, P->op.bwd.npieces));
    P->op.bwd.items = a.take<int4>(P->op.bwd.nitems);
    P->op.bwd.longrows = a.take<LongRow>(std::max(1, P->op.bwd.nlong));
    P->rs_pu = a.take<double>(static_cast<size_t>(m) * RG);
    P->rs_pv = a.take<double>(static_cast<size_t>(n) * RG);
    P->rs_part = a.take<double>(static_cast<size_t>(std::max(P->op.fwd.nitems, P->op.bwd.nitems)) * RG);
    P->rs_pieces =
        a.take<double>(static_cast<size_t>(std::max(1, std::max(P->op.fwd.npieces, P->op.bwd.npieces))) * RG);
    P->rs_lpart = a.take<double>(static_cast<size_t>(std::max(1, std::max(P->op.fwd.nlong, P->op.bwd.nlong))) * RG);
    P->rs_s = a.take<double>(RG);
    // column-sorted copies for the products: A always, A^T unless the
    // column-panel form (unsorted) replaces it
    const int64_t nz = std::max<int64_t>(1, P->op.nnz);
    const size_t vb = static_cast<size_t>(vsize(P->op.vt));
    P->op.fwd.scol = a.take<int32_t>(nz);
    P->op.fwd.sval = a.take<char>(nz * vb);
    P->op.fwd.spos = a.take<uint16_t>(nz);
    if (P->op.npanel == 1) {
      P->op.bwd.scol = a.take<int32_t>(nz);
      P->op.bwd.sval = a.take<char>(nz * vb);
      P->op.bwd.spos = a.take<uint16_t>(nz);
    }
    P->tscratch = a.take<int32_t>(transpose_scratch_words(P->op.nnz));
    P->op.trp = a.take<int32_t>(n + 1);
    P->op.tci = a.take<int32_t>(std::max<int64_t>(1, P->op.nnz));
    P->op.tval = a.take<char>(std::max<int64_t>(1, P->op.nnz) * static_cast<size_t>(vsize(P->op.vt)));
    if (P->op.npanel > 1) {  // column-panel copy of A^T (see panels_begin) and its partial products
      const int64_t prows = n * P->op.npanel;
      P->op.prp = a.take<int32_t>(prows + 1);
      P->op.pci = a.take<int32_t>(nz);
      P->op.pval = a.take<char>(nz * vb);
      P->op.ypart = a.take<double>(prows);
    }
  }
  return SVDS_OK;
}

// Test hook for the two out-of-memory fallbacks of plan creation: the
// environment variable SVDS_TEST_NO_ROOM = "arena" makes the arena with a
// column-panel copy fail to allocate (the plan is then carved without
// panels), = "panel_items" makes the panel work items fail (the panels are
// dropped after the arena was carved).  Unset in normal use.
static bool test_no_room(const char *what) {
  const char *e = std::getenv("SVDS_TEST_NO_ROOM");
  return e && std::strcmp(e, what) == 0;
}

static int alloc_arena(svds_plan *P) {
  Arena a;
  a.counting = true;
  carve_all(P, a);
  const size_t bytes = a.used;
  void *base = nullptr;
  if (P->op.npanel > 1 && test_no_room("arena")) return SVDS_ENOMEM;
  if (hipMalloc(&base, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return SVDS_ENOMEM;
  }
  P->arena.base = static_cast<char *>(base);
  P->arena.size = bytes;
  P->arena.used = 0;
  P->arena.counting = false;
  carve_all(P, P->arena);
  HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&P->h_flags), (16 + JAC_MAX_SWEEPS) * sizeof(int),
                        hipHostMallocDefault));
  if (P->early) {
    EarlyCheck &e = P->ec;
    HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&e.h_flags), (4 + JAC_MAX_SWEEPS) * sizeof(int),
                          hipHostMallocDefault));
    HIP_TRY(hipStreamCreateWithFlags(&e.stream, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&e.ev_check, hipEventDisableTiming));
    for (auto &ev : e.ev_step) HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  }
  P->p_eff = P->p;
  P->out_Uk = P->sc.Uk;
  P->out_Vext = P->sc.Vext;
  const double one = 1.0;
  HIP_TRY(hipMemcpyAsync(P->sc.one, &one, sizeof one, hipMemcpyHostToDevice, P->stream));
  return SVDS_OK;
}

// Transposed copy: stable LSD radix sort of column keys (see kernels_csc.hpp).
// npanel = 1: the CSR of A^T; npanel > 1: the stacked transpose of the row
// panels of A (rows_per_panel rows each), npanel n rows.
static int build_transpose(svds_plan *P, int npanel, int64_t rows_per_panel, int32_t *out_rp,
                           int32_t *out_ci, void *out_val, bool sync = true) {
  // the scratch lives in the plan's arena (transpose_scratch_words), so the
  // two transposes of a plan (A^T and its column-panel form) allocate nothing
  Operator &op = P->op;
  const int64_t m = op.m, nnz = op.nnz;
  const int64_t n = op.n * npanel;  // keys
  hipStream_t st = P->stream;
  if (nnz == 0) {
    hipLaunchKernelGGL(fill_i32_kernel, dim3(ceil_div(n + 1, 256)), dim3(256), 0, st, n + 1, 0, out_rp);
    LAUNCH_CHECK();
    return SVDS_OK;
  }
  const int64_t ntiles = ceil_div(nnz, RS_TILE);
  const int64_t nh = ntiles * RS_BINS;
  const int64_t nsum = ceil_div(nh, SCAN_TILE);
  int32_t *buf = P->tscratch;
  if (!buf) return SVDS_EINVAL;
  int32_t *rowof = buf, *k0 = buf + nnz, *v0 = buf + 2 * nnz, *k1 = buf + 3 * nnz, *v1 = buf + 4 * nnz;
  int32_t *hist = buf + 5 * nnz, *offs = hist + nh, *sums = offs + nh;
  int rc = SVDS_OK;
  do {
    hipLaunchKernelGGL(csc_expand_kernel, dim3(ceil_div(m * CSC_EXPAND_LANES, 256)), dim3(256), 0, st, m, op.rp,
                       op.ci, rows_per_panel, op.n, rowof, k0, v0);
    if (hipGetLastError() != hipSuccess) { rc = SVDS_EDEVICE; break; }
    int bits = 1;
    while ((int64_t(1) << bits) < n) ++bits;
    int32_t *kin = k0, *vin = v0, *kout = k1, *vout = v1;
    for (int shift = 0; shift < bits; shift += RS_BITS) {
      hipLaunchKernelGGL(radix_hist_kernel, dim3(ntiles), dim3(RS_THREADS), 0, st, kin, nnz, shift,
                         hist, ntiles);
      hipLaunchKernelGGL(scan_tile_sums_kernel, dim3(nsum), dim3(SCAN_THREADS), 0, st, hist, nh, sums);
      hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(SCAN_THREADS), 0, st, sums, nsum);
      hipLaunchKernelGGL(scan_apply_kernel, dim3(nsum), dim3(SCAN_THREADS), 0, st, hist, nh, sums, offs);
      hipLaunchKernelGGL(radix_scatter_kernel, dim3(ntiles), dim3(RS_THREADS), 0, st, kin, vin, nnz,
                         shift, offs, ntiles, kout, vout);
      if (hipGetLastError() != hipSuccess) { rc = SVDS_EDEVICE; break; }
      std::swap(kin, kout);
      std::swap(vin, vout);
    }
    if (rc) break;
    if (op.vt == SVDS_F64)
      hipLaunchKernelGGL((csc_gather_kernel<double>), dim3(ceil_div(nnz, 256)), dim3(256), 0, st, nnz,
                         vin, rowof, static_cast<const double *>(op.val), out_ci,
                         static_cast<double *>(out_val));
    else
      hipLaunchKernelGGL((csc_gather_kernel<float>), dim3(ceil_div(nnz, 256)), dim3(256), 0, st, nnz,
                         vin, rowof, static_cast<const float *>(op.val), out_ci,
                         static_cast<float *>(out_val));
    hipLaunchKernelGGL(csc_colptr_kernel, dim3(ceil_div(n + 1, 256)), dim3(256), 0, st, nnz, n, kin, out_rp);
    if (hipGetLastError() != hipSuccess) { rc = SVDS_EDEVICE; break; }
    if (sync && hipStreamSynchronize(st) != hipSuccess) { rc = SVDS_EDEVICE; break; }
  } while (0);
  return rc;
}

// Column-sorted copy of a product's nonzeros (see sort_items_kernel).
static int sort_spmv(svds_plan *P, SpmvPlan &sp, const int32_t *col, const void *val) {
  if (!sp.spos || !sp.sorted || sp.nitems == 0) return SVDS_OK;
  if (P->op.vt == SVDS_F64)
    hipLaunchKernelGGL((sort_items_kernel<double>), dim3(sp.nitems), dim3(SPMV_THREADS), 0, P->stream, sp.items,
                       col, static_cast<const double *>(val), sp.scol, static_cast<double *>(sp.sval), sp.spos);
  else
    hipLaunchKernelGGL((sort_items_kernel<float>), dim3(sp.nitems), dim3(SPMV_THREADS), 0, P->stream, sp.items,
                       col, static_cast<const float *>(val), sp.scol, static_cast<float *>(sp.sval), sp.spos);
  HIP_TRY(hipGetLastError());
  return SVDS_OK;
}

// Column panels dropped after the arena was carved: their region (row
// pointers, indices, values and partial products of the stacked transpose)
// takes the column-sorted copy of A^T instead when it fits (it does when
// the stacked rows number at least about nnz / 6), so that the plain
// transpose product runs as in a plan made without panels.  prows = the
// stacked rows (n times the panel count the region was carved for).
static int sorted_bwd_in_panel_region(svds_plan *P, int64_t prows) {
  Operator &op = P->op;
  char *r0 = reinterpret_cast<char *>(op.prp);
  char *r1 = op.ypart ? reinterpret_cast<char *>(op.ypart + prows) : nullptr;
  op.prp = op.pci = nullptr;
  op.pval = nullptr;
  op.ypart = nullptr;
  if (!r0 || !r1 || op.bwd.spos || op.nnz == 0) return SVDS_OK;
  const int64_t nz = op.nnz;
  const size_t vb = static_cast<size_t>(vsize(op.vt));
  Arena a;
  a.take<int32_t>(nz);
  a.take<char>(nz * vb);
  a.take<uint16_t>(nz);
  if (a.used > static_cast<size_t>(r1 - r0)) return SVDS_OK;
  a.base = r0;
  a.size = static_cast<size_t>(r1 - r0);
  a.used = 0;
  a.counting = false;
  op.bwd.scol = a.take<int32_t>(nz);
  op.bwd.sval = a.take<char>(nz * vb);
  op.bwd.spos = a.take<uint16_t>(nz);
  op.bwd.sorted = true;
  return sort_spmv(P, op.bwd, op.tci, op.tval);
}

// Nonzeros per MULTI work item of the plan's products.
static int item_cap(const svds_plan *P) {
  return (P->opts.flags & SVDS_FLAG_ITEMS_1K) ? SPMV_TUNE_MIN_CAP : SPMV_NNZ_BLK;
}

// Uploads the host work items.  Without sync the copies may still read
// sp.h_items / sp.h_long when this returns: neither may change before the
// stream is synchronized.
static int upload_spmv(svds_plan *P, SpmvPlan &sp, bool sync = true) {
  HIP_TRY(hipMemcpyAsync(sp.items, sp.h_items.data(), sizeof(int4) * sp.nitems, hipMemcpyHostToDevice,
                         P->stream));
  if (sp.nlong) {
    HIP_TRY(hipMemcpyAsync(sp.longrows, sp.h_long.data(), sizeof(LongRow) * sp.nlong,
                           hipMemcpyHostToDevice, P->stream));
  }
  if (sync) HIP_TRY(hipStreamSynchronize(P->stream));
  return SVDS_OK;
}


// Column panels of the transpose product (see spmv_panel_sum_kernel).  The
// count is the power of two that cuts u into FP64 slices of at most
// SPMV_PANEL_BYTES, capped at SPMV_MAX_PANELS, and lowered while the stacked
// rows would average fewer than SPMV_PANEL_MIN_NNZ entries (their row pointers
// and partial sums would then outweigh the gathers saved).
static int choose_panels(int64_t m, int64_t n, int64_t nnz) {
  int np = 1;
  while (np < SPMV_MAX_PANELS && m * 8 > SPMV_PANEL_BYTES * np) np *= 2;
  while (np > 1 && nnz < SPMV_PANEL_MIN_NNZ * n * np) np /= 2;
  while (np > 1 && n * np + 1 >= (int64_t(1) << 31)) np /= 2;
  return np;
}

// Host copies of row pointers, read back during plan creation, in pinned
// memory from a process-wide cache: a read into pageable memory goes through
// the runtime's staging buffers in chunks (4 MB in ~0.35 ms measured on
// MI355X, against ~0.1 ms into pinned memory), and pinning memory for every
// plan would cost more than it saves.  Arrays above PIN_MAX bytes, or when
// pinning fails, use pageable memory.  The cache keeps at most PIN_CACHE
// bytes.
namespace {
constexpr size_t PIN_MAX = size_t(256) << 20, PIN_CACHE = size_t(512) << 20;
std::mutex g_pin_mu;
std::vector<std::pair<size_t, void *>> g_pin_free;  // (bytes, buffer)
size_t g_pin_cached = 0;

struct HostInts {
  int32_t *p = nullptr;
  size_t bytes = 0;      // capacity of a pinned buffer (0: pageable)
  std::vector<int32_t> v;
  HostInts() = default;
  HostInts(const HostInts &) = delete;
  HostInts &operator=(const HostInts &) = delete;
  // room for count entries (contents undefined); throws std::bad_alloc
  void take(size_t count) {
    const size_t need = count * sizeof(int32_t);
    if (need <= PIN_MAX) {
      {
        std::lock_guard<std::mutex> lock(g_pin_mu);
        size_t best = g_pin_free.size();
        for (size_t i = 0; i < g_pin_free.size(); ++i)
          if (g_pin_free[i].first >= need && (best == g_pin_free.size() || g_pin_free[i].first < g_pin_free[best].first))
            best = i;
        if (best < g_pin_free.size()) {
          bytes = g_pin_free[best].first;
          p = static_cast<int32_t *>(g_pin_free[best].second);
          g_pin_cached -= bytes;
          g_pin_free.erase(g_pin_free.begin() + static_cast<std::ptrdiff_t>(best));
          return;
        }
      }
      void *q = nullptr;
      if (hipHostMalloc(&q, need, hipHostMallocDefault) == hipSuccess) {
        p = static_cast<int32_t *>(q);
        bytes = need;
        return;
      }
      (void)hipGetLastError();
    }
    v.resize(count);
    p = v.data();
  }
  ~HostInts() {
    if (!bytes) return;
    std::lock_guard<std::mutex> lock(g_pin_mu);
    if (g_pin_cached + bytes <= PIN_CACHE) {
      g_pin_free.emplace_back(bytes, p);
      g_pin_cached += bytes;
    } else {
      (void)hipHostFree(p);
    }
  }
  int32_t *data() { return p; }
  int32_t &operator[](int64_t i) { return p[i]; }
};
}  // namespace

// Column-panel copy, first stage: the stacked transpose (into the arrays the
// arena holds for it) and the read-back of its row pointers into hrp,
// enqueued on the plan's stream with `done` recorded after them (the host
// meanwhile builds the items of A^T).
static int panels_begin(svds_plan *P, HostInts &hrp, hipEvent_t done) {
  Operator &op = P->op;
  const int np = op.npanel;
  const int64_t rows = op.n * np;
  const int64_t rpp = ceil_div(op.m, np);
  hrp.take(rows + 1);  // before the launches: pinning may wait for the device
  const int rc = build_transpose(P, np, rpp, op.prp, op.pci, op.pval, false);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(hrp.data(), op.prp, sizeof(int32_t) * (rows + 1), hipMemcpyDeviceToHost, P->stream));
  HIP_TRY(hipEventRecord(done, P->stream));
  return SVDS_OK;
}

// Column-panel copy, second stage: once `done` has completed, the panel work
// items (built on the host) and their upload, left in flight on the stream.
static int panels_finish(svds_plan *P, HostInts &hrp, hipEvent_t done) {
  Operator &op = P->op;
  const int np = op.npanel;
  const int64_t n = op.n;
  HIP_TRY(hipEventSynchronize(done));
  // items per panel, built on one host thread per panel (rows relative to the
  // panel, nonzero offsets absolute), then renumbered: rows + g n, long rows
  // and pieces after those of the earlier panels
  SpmvPlan &sp = op.bwdp;
  std::vector<SpmvPlan> pp(np);
  {
    std::vector<std::thread> th;
    std::vector<char> started(np, 0), failed(np, 0);
    for (int g = 0; g < np; ++g) {
      try {
        th.emplace_back([&, g] {
          try {
            build_spmv_items(hrp.data() + static_cast<int64_t>(g) * n, n, pp[g], nullptr, 1, item_cap(P));
          } catch (...) {
            failed[g] = 1;
          }
        });
        started[g] = 1;
      } catch (...) {
      }
    }
    for (auto &t : th) t.join();
    for (int g = 0; g < np; ++g) {
      if (failed[g]) return SVDS_ENOMEM;
      if (!started[g]) build_spmv_items(hrp.data() + static_cast<int64_t>(g) * n, n, pp[g], nullptr, 1, item_cap(P));  // no thread
    }
  }
  std::vector<std::vector<int4>> per(np);
  sp.h_long.clear();
  int npieces = 0;
  for (int g = 0; g < np; ++g) {
    const int32_t r0 = static_cast<int32_t>(static_cast<int64_t>(g) * n);
    const int lbase = static_cast<int>(sp.h_long.size());
    for (LongRow L : pp[g].h_long) {
      L.row += r0;
      L.first_piece += npieces;
      sp.h_long.push_back(L);
    }
    for (int4 it : pp[g].h_items) {
      if (it.x >= 0) {
        it.x += r0;
        it.y += r0;
      } else {
        it.x = -((-it.x - 1) + lbase) - 1;
        it.y += npieces;
      }
      per[g].push_back(it);
    }
    npieces += pp[g].npieces;
  }
  sp.nlong = static_cast<int>(sp.h_long.size());
  sp.npieces = npieces;
  // slot b -> panel (b mod 8) mod np; a panel that has run out gets empty items
  std::vector<size_t> next(np, 0);
  sp.h_items.clear();
  for (bool left = true; left;) {
    for (int x = 0; x < 8; ++x) {
      const int g = x % np;
      sp.h_items.push_back(next[g] < per[g].size() ? per[g][next[g]++] : make_int4(0, 0, 0, 0));
    }
    left = false;
    for (int g = 0; g < np; ++g) left = left || next[g] < per[g].size();
  }
  sp.nitems = static_cast<int>(sp.h_items.size());
  Arena b;
  auto carve_items = [&](Arena &ar) {
    sp.items = ar.take<int4>(sp.nitems);
    sp.longrows = ar.take<LongRow>(std::max(1, sp.nlong));
    sp.partials = ar.take<double>(std::max(1, sp.npieces));
  };
  carve_items(b);
  if (test_no_room("panel_items")) return SVDS_ENOMEM;
  if (hipMalloc(&op.pbuf_items, b.used) != hipSuccess) {
    (void)hipGetLastError();
    op.pbuf_items = nullptr;
    return SVDS_ENOMEM;
  }
  op.pbuf_bytes += b.used;
  b.base = static_cast<char *>(op.pbuf_items);
  b.used = 0;
  b.counting = false;
  carve_items(b);
  // no column sort here: a panel's gathers come from an L2-sized slice and
  // its items rarely share cache lines (sorting cost 3% on such matrices)
  return upload_spmv(P, sp, false);
}

// ---------------------------------------------------------------------------
// Plan-time autotuner (SVDS_FLAG_AUTOTUNE): candidate launch shapes are timed
// on the plan's own matrix and bases with HIP events and the fastest is kept.
// ---------------------------------------------------------------------------
namespace {
struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};
}  // namespace

// Microseconds per call of fn: one warm-up call, then the better of two
// brackets of `reps` calls.
template <typename F> static int tune_time(svds_plan *P, EventPair &ev, int reps, F &&fn, double &us) {
  int rc = fn();
  if (rc) return rc;
  us = INFINITY;
  for (int t = 0; t < 2; ++t) {
    HIP_TRY(hipEventRecord(ev.a, P->stream));
    for (int i = 0; i < reps; ++i)
      if ((rc = fn())) return rc;
    HIP_TRY(hipEventRecord(ev.b, P->stream));
    HIP_TRY(hipEventSynchronize(ev.b));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, ev.a, ev.b));
    us = std::min(us, 1e3 * ms / reps);
  }
  return SVDS_OK;
}

// Work items of one product with a given nonzero cap, uploaded into the
// plan's item buffers, and their column-sorted copy when one is kept.
static int tune_build_items(svds_plan *P, bool trans, const int32_t *hrp, int64_t rows, const int64_t *seg,
                            int nseg, int cap) {
  Operator &op = P->op;
  SpmvPlan &sp = trans ? op.bwd : op.fwd;
  SpmvPlan tmp;
  build_spmv_items(hrp, rows, tmp, seg, nseg, cap);
  if (tmp.nitems > sp.cap_items || tmp.nlong > sp.cap_long || tmp.npieces > sp.cap_pieces) return SVDS_EDEVICE;
  sp.h_items = std::move(tmp.h_items);
  sp.h_long = std::move(tmp.h_long);
  sp.nitems = tmp.nitems;
  sp.nlong = tmp.nlong;
  sp.npieces = tmp.npieces;
  int rc = upload_spmv(P, sp);
  if (rc) return rc;
  return sort_spmv(P, sp, trans ? op.tci : op.ci, trans ? op.tval : op.val);
}

// Item cap and sorting of one product: caps 2048 (built in) then 1024, each
// with and without the column-sorted copy (when the plan keeps one); with
// column panels the panel form is the first candidate.
static int tune_product(svds_plan *P, EventPair &ev, bool trans, const int32_t *hrp, int64_t rows,
                        const int64_t *seg, int nseg) {
  Operator &op = P->op;
  SpmvPlan &sp = trans ? op.bwd : op.fwd;
  Lanczos<double> &Lz = P->L64;
  const double *x = trans ? Lz.bu : Lz.bv;
  double *y = trans ? Lz.wv : Lz.wu;
  auto prod = [&] { return matvec<double>(P, trans, x, nullptr, nullptr, nullptr, y, nullptr, 0, SVDS_KC_OTHER); };
  const int reps = 5;
  const int npanel = op.npanel;
  double best = INFINITY, dflt = INFINITY;
  int best_cap = SPMV_NNZ_BLK, best_panels = npanel;
  bool best_sorted = sp.spos != nullptr;
  int rc;
  if (npanel > 1) {
    if ((rc = tune_time(P, ev, reps, prod, best))) return rc;
    dflt = best;
    op.npanel = 1;
  }
  const int caps[2] = {SPMV_NNZ_BLK, SPMV_TUNE_MIN_CAP};
  for (int ci = 0; ci < 2; ++ci) {
    // the plan's own items serve when they have this cap and their sorted copy
    const bool have = ci == 0 && item_cap(P) == caps[0] && (sp.sorted || !sp.spos);
    sp.sorted = true;
    if (!have && (rc = tune_build_items(P, trans, hrp, rows, seg, nseg, caps[ci]))) return rc;
    for (int so = sp.spos ? 1 : 0; so >= 0; --so) {
      sp.sorted = so != 0;
      double t;
      if ((rc = tune_time(P, ev, reps, prod, t))) return rc;
      if (npanel == 1 && ci == 0 && so == (sp.spos ? 1 : 0)) dflt = t;
      if (t < best) best = t, best_cap = caps[ci], best_sorted = so != 0, best_panels = 1;
    }
  }
  sp.sorted = true;
  if (best_cap != caps[1] && (rc = tune_build_items(P, trans, hrp, rows, seg, nseg, best_cap))) return rc;
  sp.sorted = best_sorted;
  op.npanel = best_panels;
  if (npanel > 1 && best_panels == 1) {  // the panel items are not used: release them
    if (op.pbuf_items) (void)hipFree(op.pbuf_items);
    op.pbuf_items = nullptr;
    op.pbuf_bytes = 0;
  }
  svds_tuning &tu = P->tuning;
  (trans ? tu.bwd_nnz_cap : tu.fwd_nnz_cap) = best_cap;
  (trans ? tu.bwd_sorted : tu.fwd_sorted) = best_sorted && sp.spos ? 1 : 0;
  (trans ? tu.bwd_us : tu.fwd_us) = best;
  (trans ? tu.bwd_default_us : tu.fwd_default_us) = dflt;
  if (trans) tu.bwd_panels = best_panels;
  return SVDS_OK;
}

// CGS2 launch shapes, timed on the U-side basis (filled with normal deviates)
// at widths p/4, p/2 and p: first the pass-1 slab count, then the fused
// pass's columns per wave.
static int tune_cgs(svds_plan *P, EventPair &ev) {
  Lanczos<double> &Lz = P->L64;
  const int p = P->p;
  const int64_t m = Lz.m;
  hipLaunchKernelGGL((philox_fill_kernel<double>), dim3(static_cast<unsigned>(ceil_div(ceil_div(Lz.ldu * (p + 1), 2), 256))),
                     dim3(256), 0, P->stream, Lz.ldu * (p + 1), P->opts.seed ^ 0x7475u, 1u, Lz.U[0]);
  hipLaunchKernelGGL((philox_fill_kernel<double>), dim3(static_cast<unsigned>(ceil_div(ceil_div(m, 2), 256))), dim3(256),
                     0, P->stream, m, P->opts.seed ^ 0x7475u, 2u, Lz.wu);
  HIP_TRY(hipGetLastError());
  const int js[3] = {std::max(1, p / 4), std::max(1, p / 2), p};
  auto eval = [&](double &total) {
    total = 0;
    for (int j : js) {
      double t;
      int rc = tune_time(P, ev, 3, [&] {
        return cgs2_finish<double>(P, Lz, Lz.U[0], Lz.ldu, m, j, Lz.wu, Lz.w1u, Lz.bu, MODE_LANCZOS, P->sc.T,
                                   P->sc.xs_u);
      }, t);
      if (rc) return rc;
      total += t;
    }
    return static_cast<int>(SVDS_OK);
  };
  int rc;
  double best, t;
  P->cgs_slab_shift = 0;
  P->cgs_cpw = 0;
  if ((rc = eval(best))) return rc;
  P->tuning.cgs_default_us = best;
  int bs = 0, bc = 0;
  for (int sh : {-1, 1}) {
    P->cgs_slab_shift = sh;
    if ((rc = eval(t))) return rc;
    if (t < best) best = t, bs = sh;
  }
  P->cgs_slab_shift = bs;
  for (int c : {8, 10}) {
    P->cgs_cpw = c;
    if ((rc = eval(t))) return rc;
    if (t < best) best = t, bc = c;
  }
  P->cgs_cpw = bc;
  P->tuning.cgs_slab_shift = bs;
  P->tuning.cgs_cpw = bc;
  P->tuning.cgs_us = best;
  return SVDS_OK;
}

// ---------------------------------------------------------------------------
// Tuning cache.  A choice depends on the sparsity structure and sizes, the
// plan's Lanczos dimension, the precision and the device, not on the values:
// the key hashes all of them (FNV-1a over the row pointers of A and of A^T),
// so a second plan of the same matrix (or of another one with the same
// structure) takes the stored choice instead of timing candidates again.
// The cache lives for the process; with the environment variable
// SVDS_AUTOTUNE_CACHE naming a file it also persists: entries are read from
// that file on first use and every new entry is appended to it, one text line
// each ("svds-tune-v1 <key> <choice and times>").
// ---------------------------------------------------------------------------
namespace {
struct TuneChoice {
  int fwd_cap = 0, fwd_sorted = 0, bwd_cap = 0, bwd_sorted = 0, bwd_panels = 1, slab_shift = 0, cpw = 0;
  double fwd_us = 0, fwd_default_us = 0, bwd_us = 0, bwd_default_us = 0, cgs_us = 0, cgs_default_us = 0;
};

std::mutex g_tune_mu;
std::vector<std::pair<uint64_t, TuneChoice>> g_tune;  // (key, choice)
std::string g_tune_file;                              // file the entries were read from

uint64_t fnv1a(uint64_t h, const void *data, size_t bytes) {
  const unsigned char *c = static_cast<const unsigned char *>(data);
  for (size_t i = 0; i < bytes; ++i) h = (h ^ c[i]) * 0x100000001b3ull;
  return h;
}

uint64_t tune_key(const svds_plan *P, const int32_t *hrp, const int32_t *htrp, int nseg) {
  const Operator &op = P->op;
  uint64_t h = 0xcbf29ce484222325ull;
  hipDeviceProp_t prop{};
  if (hipGetDeviceProperties(&prop, P->device) == hipSuccess) h = fnv1a(h, prop.gcnArchName, strlen(prop.gcnArchName));
  const int64_t f[] = {op.dense ? 1 : 0, op.m, op.n, op.nnz, op.vt, op.dense ? op.lda : 0, P->p, P->k,
                       P->mixed ? 1 : 0, nseg, P->op.npanel};
  h = fnv1a(h, f, sizeof f);
  if (hrp) h = fnv1a(h, hrp, sizeof(int32_t) * (op.m + 1));
  if (htrp) h = fnv1a(h, htrp, sizeof(int32_t) * (op.n + 1));
  return h;
}

// Entries of the cache file not yet read (called with g_tune_mu held).
void tune_load_file(const std::string &path) {
  if (path == g_tune_file) return;
  g_tune_file = path;
  FILE *f = fopen(path.c_str(), "r");
  if (!f) return;
  char tag[32];
  unsigned long long key;
  TuneChoice c;
  while (fscanf(f, "%31s %llx %d %d %d %d %d %d %d %lf %lf %lf %lf %lf %lf", tag, &key, &c.fwd_cap, &c.fwd_sorted,
                &c.bwd_cap, &c.bwd_sorted, &c.bwd_panels, &c.slab_shift, &c.cpw, &c.fwd_us, &c.fwd_default_us,
                &c.bwd_us, &c.bwd_default_us, &c.cgs_us, &c.cgs_default_us) == 15) {
    if (strcmp(tag, "svds-tune-v1") != 0) continue;
    bool have = false;
    for (auto &e : g_tune) have = have || e.first == key;
    if (!have) g_tune.emplace_back(key, c);
  }
  fclose(f);
}

bool tune_lookup(uint64_t key, TuneChoice &c) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (const char *path = getenv("SVDS_AUTOTUNE_CACHE")) tune_load_file(path);
  for (auto &e : g_tune)
    if (e.first == key) {
      c = e.second;
      return true;
    }
  return false;
}

void tune_store(uint64_t key, const TuneChoice &c) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (auto &e : g_tune)
    if (e.first == key) return;
  g_tune.emplace_back(key, c);
  const char *path = getenv("SVDS_AUTOTUNE_CACHE");
  if (!path) return;
  if (FILE *f = fopen(path, "a")) {
    fprintf(f, "svds-tune-v1 %016llx %d %d %d %d %d %d %d %.6g %.6g %.6g %.6g %.6g %.6g\n",
            static_cast<unsigned long long>(key), c.fwd_cap, c.fwd_sorted, c.bwd_cap, c.bwd_sorted, c.bwd_panels,
            c.slab_shift, c.cpw, c.fwd_us, c.fwd_default_us, c.bwd_us, c.bwd_default_us, c.cgs_us, c.cgs_default_us);
    fclose(f);
  }
}
}  // namespace

// A stored choice applied to a fresh plan: the same item caps, sorting and
// panel use the tuner leaves behind, without timing anything.
static int apply_product_choice(svds_plan *P, bool trans, const int32_t *hrp, int64_t rows, const int64_t *seg,
                                int nseg, int cap, int sorted, int panels) {
  Operator &op = P->op;
  SpmvPlan &sp = trans ? op.bwd : op.fwd;
  int rc;
  if (!trans || panels == 1) {
    if (trans) op.npanel = 1;
    if (item_cap(P) != cap) {
      sp.sorted = true;
      if ((rc = tune_build_items(P, trans, hrp, rows, seg, nseg, cap))) return rc;
    }
    sp.sorted = sorted != 0 && sp.spos;
  }
  if (trans && panels == 1 && op.pbuf_items) {
    HIP_TRY(hipStreamSynchronize(P->stream));
    (void)hipFree(op.pbuf_items);
    op.pbuf_items = nullptr;
    op.pbuf_bytes = 0;
  }
  return SVDS_OK;
}

// The whole tuning of a plan (products only for CSR; CGS2 unless batched).
static int autotune(svds_plan *P, const int32_t *hrp, const int32_t *htrp, const int64_t *seg_rows,
                    const int64_t *seg_cols, int nseg) {
  const auto t0 = std::chrono::steady_clock::now();
  const uint64_t key = tune_key(P, hrp, htrp, nseg);
  TuneChoice c;
  if (tune_lookup(key, c)) {
    int rc;
    if (!P->op.dense) {
      if ((rc = apply_product_choice(P, false, hrp, P->op.m, seg_rows, nseg, c.fwd_cap, c.fwd_sorted, 1)))
        return rc;
      // panels are kept only when the plan has them and the choice used them
      const int panels = P->op.npanel > 1 && c.bwd_panels > 1 ? P->op.npanel : 1;
      if ((rc = apply_product_choice(P, true, htrp, P->op.n, seg_cols, nseg, c.bwd_cap, c.bwd_sorted, panels)))
        return rc;
    }
    P->cgs_slab_shift = c.slab_shift;
    P->cgs_cpw = c.cpw;
    HIP_TRY(hipStreamSynchronize(P->stream));
    svds_tuning &tu = P->tuning;
    tu.tuned = 2;
    tu.fwd_nnz_cap = P->op.dense ? 0 : c.fwd_cap;
    tu.fwd_sorted = P->op.dense ? 0 : c.fwd_sorted;
    tu.bwd_nnz_cap = P->op.dense ? 0 : c.bwd_cap;
    tu.bwd_sorted = P->op.dense ? 0 : c.bwd_sorted;
    tu.bwd_panels = P->op.dense ? 0 : P->op.npanel;
    tu.cgs_slab_shift = c.slab_shift;
    tu.cgs_cpw = c.cpw;
    tu.fwd_us = c.fwd_us;
    tu.fwd_default_us = c.fwd_default_us;
    tu.bwd_us = c.bwd_us;
    tu.bwd_default_us = c.bwd_default_us;
    tu.cgs_us = c.cgs_us;
    tu.cgs_default_us = c.cgs_default_us;
    tu.ms_tune = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return SVDS_OK;
  }
  EventPair ev;
  HIP_TRY(hipEventCreate(&ev.a));
  HIP_TRY(hipEventCreate(&ev.b));
  Lanczos<double> &Lz = P->L64;
  // operands of the timed products: normal deviates
  hipLaunchKernelGGL((philox_fill_kernel<double>), dim3(static_cast<unsigned>(ceil_div(ceil_div(Lz.n, 2), 256))), dim3(256),
                     0, P->stream, Lz.n, P->opts.seed ^ 0x7475u, 3u, Lz.bv);
  hipLaunchKernelGGL((philox_fill_kernel<double>), dim3(static_cast<unsigned>(ceil_div(ceil_div(Lz.m, 2), 256))), dim3(256),
                     0, P->stream, Lz.m, P->opts.seed ^ 0x7475u, 4u, Lz.bu);
  HIP_TRY(hipGetLastError());
  int rc;
  if (!P->op.dense) {
    if ((rc = tune_product(P, ev, false, hrp, P->op.m, seg_rows, nseg))) return rc;
    if ((rc = tune_product(P, ev, true, htrp, P->op.n, seg_cols, nseg))) return rc;
  }
  if (!seg_rows && (rc = tune_cgs(P, ev))) return rc;
  HIP_TRY(hipStreamSynchronize(P->stream));
  svds_tuning &tu = P->tuning;
  tu.tuned = 1;
  tu.ms_tune = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  c.fwd_cap = tu.fwd_nnz_cap;
  c.fwd_sorted = tu.fwd_sorted;
  c.bwd_cap = tu.bwd_nnz_cap;
  c.bwd_sorted = tu.bwd_sorted;
  c.bwd_panels = P->op.dense ? 1 : tu.bwd_panels;
  c.slab_shift = tu.cgs_slab_shift;
  c.cpw = tu.cgs_cpw;
  c.fwd_us = tu.fwd_us;
  c.fwd_default_us = tu.fwd_default_us;
  c.bwd_us = tu.bwd_us;
  c.bwd_default_us = tu.bwd_default_us;
  c.cgs_us = tu.cgs_us;
  c.cgs_default_us = tu.cgs_default_us;
  tune_store(key, c);
  return SVDS_OK;
}

// FP32 copies of every FP64 value array a product reads (Operator::val32
// and friends), made once the arrays are final (after any tuning): the FP32
// phase of a mixed solve then streams 4-byte values.  The FP64 refinement
// and the residuals keep reading the FP64 arrays.
static int build_values32(svds_plan *P) {
  Operator &op = P->op;
  const int64_t nnz = op.nnz;
  const bool fs = op.fwd.spos && op.fwd.sorted, bs = op.bwd.spos && op.bwd.sorted, pn = op.npanel > 1;
  const int64_t count = 2 + (fs ? 1 : 0) + (bs ? 1 : 0) + (pn ? 1 : 0);
  const size_t per = (static_cast<size_t>(nnz) * sizeof(float) + 255) & ~size_t(255);
  if (hipMalloc(&op.v32buf, per * count) != hipSuccess) {
    (void)hipGetLastError();
    op.v32buf = nullptr;
    return SVDS_ENOMEM;
  }
  op.v32_bytes = per * count;
  char *b = static_cast<char *>(op.v32buf);
  auto next = [&]() { float *q = reinterpret_cast<float *>(b); b += per; return q; };
  auto cast = [&](const void *src, float *dst) {
    // one element per thread
    hipLaunchKernelGGL((cast_copy_kernel<double, float>), dim3(static_cast<unsigned>(ceil_div(nnz, 256))),
                       dim3(256), 0, P->stream, nnz, static_cast<const double *>(src), dst);
  };
  op.val32 = next();
  cast(op.val, op.val32);
  op.tval32 = next();
  cast(op.tval, op.tval32);
  if (fs) cast(op.fwd.sval, op.fsval32 = next());
  if (bs) cast(op.bwd.sval, op.bsval32 = next());
  if (pn) cast(op.pval, op.pval32 = next());
  HIP_TRY(hipGetLastError());
  return SVDS_OK;
}

namespace {
// Destroys a partially built plan on every early return of plan creation.
struct PlanGuard {
  svds_plan *p;
  ~PlanGuard() {
    if (!p) return;
    // work of the failed creation may still be in flight on its buffers
    (void)hipStreamSynchronize(p->stream);
    svds_plan_destroy(p);
  }
  svds_plan *release() {
    svds_plan *q = p;
    p = nullptr;
    return q;
  }
};
}  // namespace

// Plan of a CSR matrix.  seg_rows / seg_cols (nseg entries, or null): ends of
// the row ranges of A and of A^T that belong to the problems of a batch
// stacked block-diagonally; product work items never cross them.
static int plan_create_csr_impl(const svds_csr *A, const svds_opts *opts, svds_plan **plan,
                                const int64_t *seg_rows, const int64_t *seg_cols, int nseg) {
  if (!A || !opts || !plan) return SVDS_EINVAL;
  *plan = nullptr;
  if (A->m < 1 || A->n < 1 || A->nnz < 0 || A->nnz >= (int64_t(1) << 31) || A->m >= (int64_t(1) << 31) ||
      A->n >= (int64_t(1) << 31))
    return SVDS_EINVAL;
  if (!A->row_ptr || (A->nnz > 0 && (!A->col_idx || !A->val))) return SVDS_EINVAL;
  if (A->dtype != SVDS_F64 && A->dtype != SVDS_F32) return SVDS_EUNSUPPORTED;
  svds_plan *P = new (std::nothrow) svds_plan();
  if (!P) return SVDS_ENOMEM;
  PlanGuard guard{P};
  int rc = fill_defaults(opts, A->m, A->n, P);
  if (rc) return rc;
  HIP_TRY(hipGetDevice(&P->device));
  Operator &op = P->op;
  op.dense = false;
  op.m = A->m;
  op.n = A->n;
  op.nnz = A->nnz;
  op.vt = A->dtype;
  op.rp = A->row_ptr;
  op.ci = A->col_idx;
  op.val = A->val;
  P->acc.stream = P->stream;
  P->acc.device = P->device;
  P->acc.timing = (opts->flags & SVDS_FLAG_TIMING) != 0;
  // work items of A (row pointers read back once)
  HostInts hrp;
  hrp.take(A->m + 1);
  HIP_TRY(hipMemcpy(hrp.data(), A->row_ptr, sizeof(int32_t) * (A->m + 1), hipMemcpyDeviceToHost));
  if (hrp[0] != 0 || hrp[A->m] != A->nnz) return SVDS_EINVAL;
  for (int64_t i = 0; i < A->m; ++i)
    if (hrp[i + 1] < hrp[i]) return SVDS_EINVAL;
  op.npanel = (seg_rows || (opts->flags & SVDS_FLAG_NO_PANELS)) ? 1 : choose_panels(op.m, op.n, op.nnz);
  op.fwd.sorted = op.bwd.sorted = !(opts->flags & SVDS_FLAG_UNSORTED);
  // The items of A are built on a helper thread while the arena is allocated
  // and the transpose is built on the device; the items of A^T need the
  // column counts from that transpose.  The arena is therefore sized with
  // bounds for both (at most one item per row plus the pieces).
  SpmvPlan fwd_items;
  bool fwd_failed = false;  // a failed host allocation on the helper thread
  std::thread tf;
  try {
    tf = std::thread([&] {
      try {
        build_spmv_items(hrp.data(), A->m, fwd_items, seg_rows, nseg, item_cap(P));
      } catch (...) {
        fwd_failed = true;
      }
    });
  } catch (...) {
    build_spmv_items(hrp.data(), A->m, fwd_items, seg_rows, nseg, item_cap(P));
  }
  struct Join {
    std::thread &t;
    ~Join() {
      if (t.joinable()) t.join();
    }
  } join_fwd{tf};
  // bounds for any item nnz cap >= SPMV_TUNE_MIN_CAP: at most one item per
  // row plus the pieces, one long row per SPMV_TUNE_MIN_CAP nonzeros
  auto set_caps = [](SpmvPlan &sp, int64_t rows, int64_t nnz) {
    sp.nitems = static_cast<int>(std::max<int64_t>(1, rows + ceil_div(nnz, SPMV_PIECE) + 1));
    sp.nlong = static_cast<int>(std::max<int64_t>(1, ceil_div(nnz, SPMV_TUNE_MIN_CAP) + 1));
    sp.npieces = static_cast<int>(std::max<int64_t>(1, ceil_div(nnz, SPMV_PIECE) + sp.nlong));
    sp.cap_items = sp.nitems;
    sp.cap_long = sp.nlong;
    sp.cap_pieces = sp.npieces;
  };
  set_caps(op.fwd, A->m, A->nnz);
  set_caps(op.bwd, A->n, A->nnz);
  const int fwd_items_cap = op.fwd.nitems, fwd_long_cap = op.fwd.nlong, fwd_pieces_cap = op.fwd.npieces;
  const int bwd_items_cap = op.bwd.nitems, bwd_long_cap = op.bwd.nlong, bwd_pieces_cap = op.bwd.npieces;
  rc = alloc_arena(P);
  if (rc == SVDS_ENOMEM && op.npanel > 1) {
    // no room with the column-panel copy: the plain transpose product serves
    op.npanel = 1;
    rc = alloc_arena(P);
  }
  if (rc) return rc;
  if ((rc = build_transpose(P, 1, op.m, op.trp, op.tci, op.tval))) return rc;
  HostInts htrp;
  htrp.take(A->n + 1);
  HIP_TRY(hipMemcpy(htrp.data(), op.trp, sizeof(int32_t) * (A->n + 1), hipMemcpyDeviceToHost));
  // The column-panel copy is built on the device while the host builds the
  // items of A^T, and its items are built on the host while the device sorts
  // the items of A and A^T.
  struct EventGuard {
    hipEvent_t e = nullptr;
    ~EventGuard() {
      if (e) (void)hipEventDestroy(e);
    }
  } pdone;
  HostInts hprp;
  // declared after hprp, so destroyed before it: on an early return the
  // read-back into hprp may still be in flight when hprp goes back to the
  // process-wide cache
  struct Drain {
    hipStream_t s;
    bool armed;
    ~Drain() {
      if (armed) (void)hipStreamSynchronize(s);
    }
  } drain{P->stream, false};
  auto drop_panels = [&]() {  // no room for the panel items: the plain transpose product serves
    if (op.pbuf_items) (void)hipFree(op.pbuf_items);
    op.pbuf_items = nullptr;
    op.pbuf_bytes = 0;
    op.npanel = 1;
  };
  if (op.npanel > 1) {
    HIP_TRY(hipEventCreateWithFlags(&pdone.e, hipEventDisableTiming));
    drain.armed = true;
    if ((rc = panels_begin(P, hprp, pdone.e))) return rc;
  }
  int4 *bi = op.bwd.items;
  LongRow *bl = op.bwd.longrows;
  double *bp = op.bwd.partials;
  build_spmv_items(htrp.data(), A->n, op.bwd, seg_cols, nseg, item_cap(P));
  if (op.bwd.nitems > bwd_items_cap || op.bwd.nlong > bwd_long_cap || op.bwd.npieces > bwd_pieces_cap)
    return SVDS_EDEVICE;
  op.bwd.items = bi;
  op.bwd.longrows = bl;
  op.bwd.partials = bp;
  if (tf.joinable()) tf.join();
  if (fwd_failed) return SVDS_ENOMEM;
  if (fwd_items.nitems > fwd_items_cap || fwd_items.nlong > fwd_long_cap || fwd_items.npieces > fwd_pieces_cap)
    return SVDS_EDEVICE;
  op.fwd.h_items = std::move(fwd_items.h_items);
  op.fwd.h_long = std::move(fwd_items.h_long);
  op.fwd.nitems = fwd_items.nitems;
  op.fwd.nlong = fwd_items.nlong;
  op.fwd.npieces = fwd_items.npieces;
  if ((rc = upload_spmv(P, op.fwd, false)) || (rc = upload_spmv(P, op.bwd, false))) return rc;
  if ((rc = sort_spmv(P, op.fwd, op.ci, op.val)) || (rc = sort_spmv(P, op.bwd, op.tci, op.tval))) return rc;
  if (op.npanel > 1 && (rc = panels_finish(P, hprp, pdone.e))) {
    if (rc != SVDS_ENOMEM) return rc;
    HIP_TRY(hipStreamSynchronize(P->stream));
    const int64_t prows = op.n * op.npanel;
    drop_panels();
    if ((rc = sorted_bwd_in_panel_region(P, prows))) return rc;
  }
  // the uploads above read the host item lists, which the tuner rebuilds
  HIP_TRY(hipStreamSynchronize(P->stream));
  if ((opts->flags & SVDS_FLAG_AUTOTUNE) && (rc = autotune(P, hrp.data(), htrp.data(), seg_rows, seg_cols, nseg)))
    return rc;
  if (P->mixed && op.vt == SVDS_F64 && op.nnz > 0 && (rc = build_values32(P))) return rc;
  HIP_TRY(hipStreamSynchronize(P->stream));
  *plan = guard.release();
  return SVDS_OK;
}

extern "C" int svds_plan_create_csr(const svds_csr *A, const svds_opts *opts, svds_plan **plan) {
  SVDS_ABI_TRY
  return plan_create_csr_impl(A, opts, plan, nullptr, nullptr, 0);
  SVDS_ABI_CATCH
}

extern "C" int svds_plan_create_dense(const svds_dense *A, const svds_opts *opts, svds_plan **plan) {
  SVDS_ABI_TRY
  if (!A || !opts || !plan) return SVDS_EINVAL;
  *plan = nullptr;
  if (A->m < 1 || A->n < 1 || A->ld < A->m || !A->a) return SVDS_EINVAL;
  if (A->dtype != SVDS_F64 && A->dtype != SVDS_F32 && A->dtype != SVDS_BF16) return SVDS_EUNSUPPORTED;
  svds_plan *P = new (std::nothrow) svds_plan();
  if (!P) return SVDS_ENOMEM;
  PlanGuard guard{P};
  int rc = fill_defaults(opts, A->m, A->n, P);
  if (rc) return rc;
  HIP_TRY(hipGetDevice(&P->device));
  Operator &op = P->op;
  op.dense = true;
  op.m = A->m;
  op.n = A->n;
  op.vt = A->dtype;
  op.a = A->a;
  op.lda = A->ld;
  P->acc.stream = P->stream;
  P->acc.device = P->device;
  P->acc.timing = (opts->flags & SVDS_FLAG_TIMING) != 0;
  if ((rc = alloc_arena(P))) return rc;
  if ((opts->flags & SVDS_FLAG_AUTOTUNE) && (rc = autotune(P, nullptr, nullptr, nullptr, nullptr, 0))) return rc;
  *plan = guard.release();
  return SVDS_OK;
  SVDS_ABI_CATCH
}

extern "C" void svds_plan_destroy(svds_plan *P) {
  if (!P) return;
  if (P->arena.base) (void)hipFree(P->arena.base);
  if (P->op.pbuf_items) (void)hipFree(P->op.pbuf_items);
  if (P->op.v32buf) (void)hipFree(P->op.v32buf);
  if (P->h_flags) (void)hipHostFree(P->h_flags);
  if (P->ec.worker.joinable()) P->ec.worker.join();
  if (P->ec.h_flags) (void)hipHostFree(P->ec.h_flags);
  if (P->ec.ev_check) (void)hipEventDestroy(P->ec.ev_check);
  for (auto &ev : P->ec.ev_step)
    if (ev) (void)hipEventDestroy(ev);
  if (P->ec.stream) (void)hipStreamDestroy(P->ec.stream);
  P->graphs.destroy();
  P->acc.destroy();
  delete P;
}

// ===========================================================================
// Execute
// ===========================================================================
namespace svds {

template <typename TB>
static int outputs(svds_plan *P, Lanczos<TB> &Lz, double *U, double *S, double *V) {
  const int p = P->p_eff, k = P->k;  // p_eff < p when an early check ended the cycle
  const int64_t m = P->op.m, n = P->op.n;
  const Small &s = P->sc;
  double *Uk = P->out_Uk, *Vext = P->out_Vext;
  // Alg. 2 steps 15-16; V first, so that its sign normalization can be
  // folded into Uk before U is formed
  int rc = rotate<TB, double>(P, n, p, k, Lz.V[Lz.cur], Lz.ldv, Vext, p + 1, V, n);
  if (rc) return rc;
  if (!(P->opts.flags & SVDS_FLAG_NO_SIGNFIX)) {
    const int64_t slab = sign_slab_rows(n);
    const int nslab = static_cast<int>(ceil_div(n, slab));
    ACC_BEFORE(SVDS_KC_OTHER);
    hipLaunchKernelGGL(absmax_partials_kernel, dim3(nslab, k), dim3(256), 0, P->stream, n, slab, V, n,
                       s.sgn_val, s.sgn_idx);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(sign_pick_kernel, dim3(k), dim3(WAVE), 0, P->stream, nslab, s.sgn_val, s.sgn_idx, V, n,
                       n, s.sgn, Uk, p);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(flip_cols_kernel, dim3(static_cast<unsigned>(std::min<int64_t>(256, ceil_div(n, 2048))), k),
                       dim3(256), 0, P->stream, n, V, n, s.sgn);
    LAUNCH_CHECK();
    ACC_AFTER(SVDS_KC_OTHER, 8.0 * n * k * 2, 0.0);
  }
  rc = rotate<TB, double>(P, m, p, k, Lz.U[Lz.cur], Lz.ldu, Uk, p, U, m);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(S, s.sig, sizeof(double) * k, hipMemcpyDeviceToDevice, P->stream));
  return SVDS_OK;
}

// v1 of the FP64 phase from the FP32 Ritz vectors: sum_j Vk(:, j) / sqrt(k).
static int warm_start_vector(svds_plan *P) {
  const int p = P->p_eff, k = P->k;
  const int64_t n = P->op.n;
  int rc = rotate<float, double>(P, n, p, k, P->L32.V[P->L32.cur], P->L32.ldv, P->out_Vext, p + 1,
                                 P->tmp_nk, n);
  if (rc) return rc;
  // tmp_n = Vk * (1/sqrt(k) * ones): a rotation with a k x 1 panel
  std::vector<double> w(k, 1.0 / std::sqrt(static_cast<double>(k)));
  HIP_TRY(hipMemcpyAsync(P->tmp_m, w.data(), sizeof(double) * k, hipMemcpyHostToDevice, P->stream));
  rc = rotate<double, double>(P, n, k, 1, P->tmp_nk, n, P->tmp_m, k, P->tmp_n, n);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(P->stream));
  return SVDS_OK;
}

}  // namespace svds

extern "C" int svds_plan_execute(svds_plan *P, double *U, double *S, double *V, svds_info *info) {
  SVDS_ABI_TRY
  if (!P || !U || !S || !V) return SVDS_EINVAL;
  const auto t0 = std::chrono::steady_clock::now();
  HIP_TRY(hipSetDevice(P->device));
  P->acc.reset();
  P->n_spmv = P->n_spmvT = 0;
  P->cycles32 = P->cycles64 = P->jac_sweeps = 0;
  const int64_t cap0 = P->graphs.captures, rep0 = P->graphs.replays;
  P->reorth_calls = 0;
  P->ec.checks = 0;
  HIP_TRY(hipMemsetAsync(P->sc.sigma_est, 0, sizeof(double), P->stream));
  HIP_TRY(hipMemsetAsync(P->sc.bd, 0, 4 * sizeof(int), P->stream));
  HIP_TRY(hipMemsetAsync(P->sc.T, 0, sizeof(double) * (P->p + 1) * (P->p + 1), P->stream));
  P->wide_repair = (P->opts.flags & SVDS_FLAG_EXPECT_BREAKDOWNS) != 0;
  int rc = SVDS_OK;
  bool conv = false;
  int cyc = 0;
  if (P->mixed) {
    const double tol32 = std::max(P->tol, 1e-5);
    rc = start<float>(P, P->L32, P->opts.v0);
    if (!rc) rc = run_cycles<float>(P, P->L32, tol32, P->maxit, true, cyc, conv);
    P->cycles32 = cyc;
    if (!rc) rc = warm_start_vector(P);
    if (!rc) {
      HIP_TRY(hipMemsetAsync(P->sc.sigma_est, 0, sizeof(double), P->stream));
      HIP_TRY(hipMemsetAsync(P->sc.T, 0, sizeof(double) * (P->p + 1) * (P->p + 1), P->stream));
      rc = start<double>(P, P->L64, P->tmp_n);
    }
    if (!rc) rc = run_cycles<double>(P, P->L64, P->tol, std::max(1, P->maxit - cyc), false, cyc, conv);
    P->cycles64 = cyc;
  } else {
    rc = start<double>(P, P->L64, P->opts.v0);
    if (!rc) rc = run_cycles<double>(P, P->L64, P->tol, P->maxit, false, cyc, conv);
    P->cycles64 = cyc;
  }
  if (rc) return rc;
  rc = outputs<double>(P, P->L64, U, S, V);
  if (rc) return rc;
  double res_true = 0, res_av = 0;
  if (!(P->opts.flags & SVDS_FLAG_NO_RESIDUALS)) {
    rc = residuals_impl(P, P->k, U, S, V, P->sc.resid_av, P->sc.resid_atu);
    if (rc) return rc;
  }
  HIP_TRY(hipStreamSynchronize(P->stream));
  rc = P->acc.harvest();
  if (rc) return rc;
  const int k = P->k;
  std::vector<double> hs(k), hres(k), hav(k), hatu(k);
  int bd = 0;
  HIP_TRY(hipMemcpy(hs.data(), P->sc.sig, sizeof(double) * k, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(hres.data(), P->sc.res, sizeof(double) * k, hipMemcpyDeviceToHost));
  int bd2[2] = {0, 0};  // breakdowns, selective second passes run
  HIP_TRY(hipMemcpy(bd2, P->sc.bd, 2 * sizeof(int), hipMemcpyDeviceToHost));
  bd = bd2[0];
  long long om[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // partial form: U side, V side counters
  if (P->partial) {
    HIP_TRY(hipMemcpy(om, P->sc.om_stats, sizeof om, hipMemcpyDeviceToHost));
    // the masked passes were counted with their vector traffic only: each
    // column taken is read by all three passes
    const double sb = 8.0, cu = static_cast<double>(om[1]) * P->op.m, cv = static_cast<double>(om[5]) * P->op.n;
    for (int c : {SVDS_KC_CGS_PROJ, SVDS_KC_CGS_UPDPROJ, SVDS_KC_CGS_UPDNORM}) {
      P->acc.bytes[c] += sb * (cu + cv);
      P->acc.flops[c] += (c == SVDS_KC_CGS_UPDPROJ ? 4.0 : 2.0) * (cu + cv);
    }
  }
  if (!(P->opts.flags & SVDS_FLAG_NO_RESIDUALS)) {
    HIP_TRY(hipMemcpy(hav.data(), P->sc.resid_av, sizeof(double) * k, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(hatu.data(), P->sc.resid_atu, sizeof(double) * k, hipMemcpyDeviceToHost));
    const double s1 = *std::max_element(hs.begin(), hs.end());  // hs is ascending for smallest triplets
    for (int j = 0; j < k; ++j) {
      const double sj = std::max(hs[j], std::max(0x1.0p-52 * s1, 2.2250738585072014e-308));
      res_true = std::max(res_true, hatu[j] / sj);
      res_av = std::max(res_av, hav[j] / std::max(s1, 2.2250738585072014e-308));
    }
  }
  const auto t1 = std::chrono::steady_clock::now();
  if (info) {
    std::memset(info, 0, sizeof *info);
    info->nconv = P->h_flags[1];
    info->converged = conv ? 1 : 0;
    info->cycles = P->cycles32 + P->cycles64;
    info->cycles_fp32 = P->cycles32;
    info->cycles_fp64 = P->cycles64;
    info->breakdowns = bd;
    info->n_spmv = P->n_spmv;
    info->n_spmvT = P->n_spmvT;
    double mx = 0;
    for (double v : hres) mx = std::max(mx, v);
    info->max_res_est = mx;
    info->max_res_true = res_true;
    info->max_res_av = res_av;
    info->ms_total = std::chrono::duration<double, std::milli>(t1 - t0).count();
    double ba = 0;
    for (int c : {SVDS_KC_SPMV, SVDS_KC_SPMVT, SVDS_KC_CGS_PROJ, SVDS_KC_CGS_UPDPROJ, SVDS_KC_CGS_UPDNORM,
                  SVDS_KC_CGS_REDUCE})
      ba += P->acc.bytes[c];
    info->bytes_alg = ba;
    for (int c = 0; c < SVDS_KC_COUNT; ++c) {
      info->kc_ms[c] = P->acc.ms[c];
      info->kc_bytes[c] = P->acc.bytes[c];
      info->kc_flops[c] = P->acc.flops[c];
      info->kc_launches[c] = P->acc.launches[c];
      info->kc_sampled_launches[c] = P->acc.sampled[c];
      info->kc_sampled_bytes[c] = P->acc.sampled_bytes[c];
    }
    info->workspace_bytes = static_cast<int64_t>(P->arena.size + P->op.pbuf_bytes + P->op.v32_bytes);
    info->graph_captures = static_cast<int32_t>(P->graphs.captures - cap0);
    info->graph_replays = static_cast<int32_t>(P->graphs.replays - rep0);
    info->reorth_tests = static_cast<int32_t>(P->reorth_calls);
    info->reorth_second_passes = bd2[1];
    info->tuning = P->tuning;
    info->early_checks = P->ec.checks;
    info->lanczos_dim_last = P->p_eff;
    info->partial_steps = om[0] + om[4];
    info->partial_columns = om[1] + om[5];
    info->partial_possible = om[2] + om[6];
  }
  return conv ? SVDS_OK : SVDS_NOT_CONVERGED;
  SVDS_ABI_CATCH
}

// ===========================================================================
// Residuals (Proposition 1, eq. (2), evaluated explicitly in FP64)
// ===========================================================================
namespace svds {
// Block residuals of a CSR plan: RG triplets per product pass (row-major
// panels, see resid_spmm_kernel).
template <typename TV>
static int residuals_csr_block(svds_plan *P, int k, const double *U, const double *S, const double *V,
                               double *res_av, double *res_atu) {
  const Operator &op = P->op;
  const int64_t m = op.m, n = op.n;
  const TV *val = static_cast<const TV *>(op.val);
  const TV *tval = static_cast<const TV *>(op.tval);
  for (int j0 = 0; j0 < k; j0 += RG) {
    const int nc = std::min(RG, k - j0);
    ACC_BEFORE(SVDS_KC_OTHER);
    hipLaunchKernelGGL(resid_svals_kernel, dim3(1), dim3(64), 0, P->stream, S, j0, k, P->rs_s);
    hipLaunchKernelGGL(resid_panel_kernel, dim3(static_cast<unsigned>(std::min<int64_t>(4096, ceil_div(m * RG, 256)))),
                       dim3(256), 0, P->stream, m, U, m, j0, k, P->rs_pu);
    hipLaunchKernelGGL(resid_panel_kernel, dim3(static_cast<unsigned>(std::min<int64_t>(4096, ceil_div(n * RG, 256)))),
                       dim3(256), 0, P->stream, n, V, n, j0, k, P->rs_pv);
    // A v - s u over the rows of A, then A^T u - s v over the rows of A^T
    for (int t = 0; t < 2; ++t) {
      const SpmvPlan &sp = t ? op.bwd : op.fwd;
      hipLaunchKernelGGL((resid_spmm_kernel<TV>), dim3(sp.nitems), dim3(SPMV_THREADS), 0, P->stream, sp.items,
                         t ? op.trp : op.rp, t ? op.tci : op.ci, t ? tval : val, t ? P->rs_pu : P->rs_pv,
                         t ? P->rs_pv : P->rs_pu, P->rs_s, P->rs_part, P->rs_pieces);
      if (sp.nlong > 0)
        hipLaunchKernelGGL(resid_longrow_kernel, dim3(static_cast<unsigned>(ceil_div(sp.nlong, 256 / RG))), dim3(256),
                           0, P->stream, sp.longrows, sp.nlong, P->rs_pieces, t ? P->rs_pv : P->rs_pu, P->rs_s,
                           P->rs_lpart);
      hipLaunchKernelGGL(resid_finish_kernel, dim3(nc), dim3(WAVE), 0, P->stream, P->rs_part, sp.nitems,
                         P->rs_lpart, sp.nlong, nc, (t ? res_atu : res_av) + j0);
    }
    LAUNCH_CHECK();
    ACC_AFTER(SVDS_KC_OTHER, 2.0 * ((4.0 + sizeof(TV)) * op.nnz + 8.0 * RG * (m + n)), 4.0 * RG * op.nnz);
  }
  return SVDS_OK;
}

// One side of the dense residuals: res[j] = |op(A) X(:, j) - S[j] Sub(:, j)|,
// op(A) = A (X = V, Sub = U) or A^T (X = U, Sub = V); see resid_gemm_kernel.
template <typename TV, bool TRANS>
static int residuals_dense_side(svds_plan *P, int k, const double *X, int64_t ldx, const double *Sub,
                                int64_t ldsub, const double *S, double *res) {
  const Operator &op = P->op;
  const int64_t M = TRANS ? op.n : op.m, K = TRANS ? op.m : op.n;
  const TV *A = static_cast<const TV *>(op.a);
  int nsplit;
  int64_t kslice;
  resid_split(M, K, nsplit, kslice);
  const int nrb = static_cast<int>(ceil_div(M, RD_BM));
  double *part = P->rd_part;
  double *colpart = part + static_cast<int64_t>(nrb) * nsplit * RD_TILE;
  const bool vec = dense_vec_ok<TV, double>(A, op.lda, X) && (ldx % 2) == 0;
  const dim3 gg(nrb, nsplit);
  for (int g0 = 0; g0 < k; g0 += RD_BN) {
    const int kc = std::min(RD_BN, k - g0);
    const int nt = static_cast<int>(ceil_div(kc, 16));
    const double *Xg = X + g0 * ldx;
    if (!vec) {
      hipLaunchKernelGGL((resid_gemm_kernel<TV, TRANS, false, 8>), gg, dim3(RD_THREADS), 0, P->stream, M, K, A,
                         op.lda, Xg, ldx, kc, kslice, part);
    } else {
      switch (nt) {
#define RD_GO(NT)                                                                                              \
  case NT:                                                                                                     \
    hipLaunchKernelGGL((resid_gemm_kernel<TV, TRANS, true, NT>), gg, dim3(RD_THREADS), 0, P->stream, M, K, A, \
                       op.lda, Xg, ldx, kc, kslice, part);                                                     \
    break;
        RD_GO(1) RD_GO(2) RD_GO(3) RD_GO(4) RD_GO(5) RD_GO(6) RD_GO(7) RD_GO(8)
#undef RD_GO
      }
    }
    LAUNCH_CHECK();
    switch (nt) {
#define RD_FIN(NT)                                                                                                 \
  case NT:                                                                                                         \
    hipLaunchKernelGGL((resid_finish_kernel<NT>), dim3(nrb), dim3(RD_THREADS), 0, P->stream, M, nsplit, nrb, part, \
                       Sub, ldsub, S, g0, kc, colpart, k);                                                        \
    break;
      RD_FIN(1) RD_FIN(2) RD_FIN(3) RD_FIN(4) RD_FIN(5) RD_FIN(6) RD_FIN(7) RD_FIN(8)
#undef RD_FIN
    }
    LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(resid_colnorm_kernel, dim3(k), dim3(256), 0, P->stream, nrb, colpart, k, res);
  LAUNCH_CHECK();
  return SVDS_OK;
}

// Dense residuals: R1 = A V - U diag(S), R2 = A^T U - V diag(S), one pass of
// the FP64 matrix-core block product over the stored A per side (all k
// triplets at once), then column norms.
static int residuals_dense(svds_plan *P, int k, const double *U, const double *S, const double *V,
                           double *res_av, double *res_atu) {
  const Operator &op = P->op;
  const int64_t m = op.m, n = op.n;
  if (!P->rd_part) return SVDS_EUNSUPPORTED;
  ACC_BEFORE(SVDS_KC_OTHER);
  int rc;
  if (op.vt == SVDS_F64) {
    if ((rc = residuals_dense_side<double, false>(P, k, V, n, U, m, S, res_av))) return rc;
    if ((rc = residuals_dense_side<double, true>(P, k, U, m, V, n, S, res_atu))) return rc;
  } else if (op.vt == SVDS_F32) {
    if ((rc = residuals_dense_side<float, false>(P, k, V, n, U, m, S, res_av))) return rc;
    if ((rc = residuals_dense_side<float, true>(P, k, U, m, V, n, S, res_atu))) return rc;
  } else {
    if ((rc = residuals_dense_side<uint16_t, false>(P, k, V, n, U, m, S, res_av))) return rc;
    if ((rc = residuals_dense_side<uint16_t, true>(P, k, U, m, V, n, S, res_atu))) return rc;
  }
  ACC_AFTER(SVDS_KC_OTHER, 2.0 * vsize(op.vt) * m * n + 16.0 * (m + n) * k, 4.0 * m * n * k);
  return SVDS_OK;
}

static int residuals_impl(svds_plan *P, int k, const double *U, const double *S, const double *V,
                          double *res_av, double *res_atu) {
  const int64_t m = P->op.m, n = P->op.n;
  const int64_t sv = P->n_spmv, st = P->n_spmvT;
  if (P->op.dense && P->rd_part) return residuals_dense(P, k, U, S, V, res_av, res_atu);
  if (!P->op.dense && P->rs_pu) {
    return P->op.vt == SVDS_F64 ? residuals_csr_block<double>(P, k, U, S, V, res_av, res_atu)
                                : residuals_csr_block<float>(P, k, U, S, V, res_av, res_atu);
  }
  for (int j = 0; j < k; ++j) {
    // tmp_m = A v_j - s_j u_j
    int rc = matvec<double>(P, false, V + j * n, P->sc.one, S + j, U + j * m, P->tmp_m, nullptr, 0,
                            SVDS_KC_OTHER);
    if (rc) return rc;
    hipLaunchKernelGGL((norm_partials_kernel<double>), dim3(grid_for(m, 4096)), dim3(256), 0, P->stream, m,
                       P->tmp_m, P->sc.npart);
    hipLaunchKernelGGL(norm_finish_kernel, dim3(1), dim3(256), 0, P->stream, P->sc.npart,
                       static_cast<int>(grid_for(m, 4096)), res_av + j);
    LAUNCH_CHECK();
    rc = matvec<double>(P, true, U + j * m, P->sc.one, S + j, V + j * n, P->tmp_n, nullptr, 0,
                        SVDS_KC_OTHER);
    if (rc) return rc;
    hipLaunchKernelGGL((norm_partials_kernel<double>), dim3(grid_for(n, 4096)), dim3(256), 0, P->stream, n,
                       P->tmp_n, P->sc.npart);
    hipLaunchKernelGGL(norm_finish_kernel, dim3(1), dim3(256), 0, P->stream, P->sc.npart,
                       static_cast<int>(grid_for(n, 4096)), res_atu + j);
    LAUNCH_CHECK();
  }
  // residual products are not Lanczos steps (booked under OTHER, not counted)
  (void)sv;
  (void)st;
  return SVDS_OK;
}
}  // namespace svds

// ===========================================================================
// Internal entry points of the single-step operations
// ===========================================================================
int svds_plan_residuals(svds_plan *P, int k, const double *U, const double *S, const double *V,
                        double *res_av, double *res_atu) {
  int rc = residuals_impl(P, k, U, S, V, res_av, res_atu);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(P->stream));
  return SVDS_OK;
}

int svds_plan_panels(const svds_plan *P) { return P->op.dense ? 1 : P->op.npanel; }

int svds_plan_matvec(svds_plan *P, int trans, const void *x, const double *xs, const double *coef,
                     const void *yprev, void *y, int basis_dtype) {
  int rc;
  if (basis_dtype == SVDS_F64)
    rc = matvec<double>(P, trans != 0, static_cast<const double *>(x), xs, coef,
                        static_cast<const double *>(yprev), static_cast<double *>(y), nullptr, 0,
                        SVDS_KC_OTHER);
  else if (basis_dtype == SVDS_F32)
    rc = matvec<float>(P, trans != 0, static_cast<const float *>(x), xs, coef,
                       static_cast<const float *>(yprev), static_cast<float *>(y), nullptr, 0,
                       SVDS_KC_OTHER);
  else
    return SVDS_EUNSUPPORTED;
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(P->stream));
  return SVDS_OK;
}

int svds_plan_transpose_copy(svds_plan *P, int32_t *t_row_ptr, int32_t *t_col_idx, void *t_val) {
  const Operator &op = P->op;
  if (op.dense) return SVDS_EINVAL;
  HIP_TRY(hipMemcpyAsync(t_row_ptr, op.trp, sizeof(int32_t) * (op.n + 1), hipMemcpyDeviceToDevice, P->stream));
  if (op.nnz > 0) {
    HIP_TRY(hipMemcpyAsync(t_col_idx, op.tci, sizeof(int32_t) * op.nnz, hipMemcpyDeviceToDevice, P->stream));
    HIP_TRY(hipMemcpyAsync(t_val, op.tval, static_cast<size_t>(vsize(op.vt)) * op.nnz,
                           hipMemcpyDeviceToDevice, P->stream));
  }
  HIP_TRY(hipStreamSynchronize(P->stream));
  return SVDS_OK;
}

// CGS2 of one vector against a caller basis, with the solver's own kernels
// (single-step operation).  Scratch layout: column partials of the two
// projections, h1, h2, the intermediate vector w1, norm partials and a few
// device scalars.  Every scratch word a call reads is written earlier in the
// same call (each projection block writes its partial of every column, even
// a zero one), so no part of it has to start at zero.
namespace {
struct Cgs2Scratch {
  size_t parts, h1, h2, w1, np, dx, bd, total;
};

Cgs2Scratch cgs2_scratch_layout(int64_t L, size_t tb) {
  Cgs2Scratch s{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  };
  s.parts = take(tb * CGS_MAXJ * CGS_MAX_SLABS);
  s.h1 = take(tb * CGS_MAXJ);
  s.h2 = take(tb * CGS_MAXJ);
  s.np = take(8 * NPART);
  s.dx = take(64);
  s.bd = take(16);
  s.w1 = take(tb * static_cast<size_t>(L));  // last: the only part that grows with L
  s.total = off;
  return s;
}

int cgs2_op_run(char *b, const Cgs2Scratch &lay, int64_t L, int32_t j, const void *Q, int64_t ldq, const void *w,
                void *out, double *norm_out, int32_t dtype, hipStream_t stream) {
  svds_plan tmp;
  tmp.stream = stream;
  tmp.acc.stream = stream;
  double *dx = reinterpret_cast<double *>(b + lay.dx);  // xs, t_entry, sigma_est
  tmp.sc.npart = reinterpret_cast<double *>(b + lay.np);
  tmp.sc.sigma_est = dx + 2;
  tmp.sc.bd = reinterpret_cast<int *>(b + lay.bd);
  int rc;
  if (dtype == SVDS_F64)
    rc = cgs2_finish<double>(&tmp, reinterpret_cast<double *>(b + lay.parts), reinterpret_cast<double *>(b + lay.h1),
                             reinterpret_cast<double *>(b + lay.h2), static_cast<const double *>(Q), ldq, L, j,
                             static_cast<const double *>(w), reinterpret_cast<double *>(b + lay.w1),
                             static_cast<double *>(out), MODE_NORM, dx + 1, dx);
  else
    rc = cgs2_finish<float>(&tmp, reinterpret_cast<float *>(b + lay.parts), reinterpret_cast<float *>(b + lay.h1),
                            reinterpret_cast<float *>(b + lay.h2), static_cast<const float *>(Q), ldq, L, j,
                            static_cast<const float *>(w), reinterpret_cast<float *>(b + lay.w1),
                            static_cast<float *>(out), MODE_NORM, dx + 1, dx);
  if (rc) return rc;
  double xs = 0;
  HIP_TRY(hipMemcpyAsync(&xs, dx, sizeof(double), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  if (norm_out) *norm_out = 1.0 / xs;
  return SVDS_OK;
}
}  // namespace

int svds_cgs2_op(int64_t L, int32_t j, const void *Q, int64_t ldq, const void *w, void *out,
                 double *norm_out, int32_t dtype, void *stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Cgs2Scratch lay = cgs2_scratch_layout(L, dtype == SVDS_F64 ? 8 : 4);
  char *b = nullptr;
  HIP_TRY(hipMalloc(reinterpret_cast<void **>(&b), lay.total));
  struct Free {
    char *p;
    ~Free() { (void)hipFree(p); }
  } guard{b};
  HIP_TRY(hipMemsetAsync(b, 0, lay.total, st));
  return cgs2_op_run(b, lay, L, j, Q, ldq, w, out, norm_out, dtype, st);
}

// ---------------------------------------------------------------------------
// CGS2 without allocation (svds_op_cgs2_noalloc).  Its scratch is the
// file-scope device array below: each GPU the library runs on holds one copy
// from the first call on that device until the process ends.  In host code
// `scratch` names a host-side stand-in, not device memory, so the host takes
// each device's address of it once (hipGetSymbolAddress, with that device
// current) and passes only that address on.
// ---------------------------------------------------------------------------
constexpr size_t NOALLOC_BYTES = size_t(SVDS_CGS2_NOALLOC_MAX_VECTOR_BYTES) + (size_t(8) << 20) + (size_t(64) << 10);
static __device__ __align__(256) char scratch[NOALLOC_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
char *g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of `scratch` on the current device, looked up on the first
// call per device.
int noalloc_scratch(char **ptr) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return SVDS_EUNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void *p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return SVDS_EDEVICE;
    g_noalloc_ptr[dev] = static_cast<char *>(p);
  }
  *ptr = g_noalloc_ptr[dev];
  return SVDS_OK;
}
}  // namespace

extern "C" int svds_op_cgs2_noalloc(int64_t L, int32_t j, const void *Q, int64_t ldq, const void *w, void *out,
                                    double *norm_out, int32_t dtype, void *stream) {
  SVDS_ABI_TRY
  if (L < 1 || j < 0 || j > CGS_MAXJ || (j > 0 && (!Q || ldq < L)) || !w || !out) return SVDS_EINVAL;
  if (dtype != SVDS_F64 && dtype != SVDS_F32) return SVDS_EUNSUPPORTED;
  const size_t tb = dtype == SVDS_F64 ? 8 : 4;
  if (static_cast<size_t>(L) > size_t(SVDS_CGS2_NOALLOC_MAX_VECTOR_BYTES) / tb) return SVDS_EINVAL;
  const Cgs2Scratch lay = cgs2_scratch_layout(L, tb);
  if (lay.total > NOALLOC_BYTES) return SVDS_EINVAL;
  char *b = nullptr;
  const int rc = noalloc_scratch(&b);
  if (rc) return rc;
  return cgs2_op_run(b, lay, L, j, Q, ldq, w, out, norm_out, dtype, static_cast<hipStream_t>(stream));
  SVDS_ABI_CATCH
}

namespace {
template <int R, int LPP>
int bjac_launch_round(hipStream_t st, const double *T, int ldt, int tr, int from_T, double *W, double *Vh, int p,
                      int c, int nb, int round, int sweep, int *counters) {
  const size_t shm = static_cast<size_t>(4 * c) * p * sizeof(double);
  static bool attr_set = false;  // benign race: every caller sets the same value
  if (!attr_set) {
    HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(&bjac_round_kernel<R, LPP>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, BJ_LDS));
    attr_set = true;
  }
  const int waves = LPP == WAVE ? c : std::max(1, c / 4);  // one lane group per pair of a step
  hipLaunchKernelGGL((bjac_round_kernel<R, LPP>), dim3(nb / 2), dim3(waves * WAVE), shm, st, T, ldt, tr, from_T, W,
                     Vh, p, c, nb, round, sweep, counters);
  HIP_TRY(hipGetLastError());
  return SVDS_OK;
}

// Lane groups of a column pair: 16 lanes (four pairs per wave) up to 256
// rows, one wave per pair above (RPL = ceil(p / 64) rows per lane, c waves
// per workgroup).  Measured on MI355X: p = 300 rounds take 39.6 us with one
// wave per pair against 47.2 us with 16-lane groups; at p = 150 and 250 the
// 16-lane groups are as fast or faster (and p = 150 converged in fewer
// sweeps with them).
int bjac_round(hipStream_t st, const double *T, int ldt, int tr, int from_T, double *W, double *Vh, int p, int c,
               int nb, int round, int sweep, int *counters) {
  const int rpl16 = static_cast<int>(ceil_div(p, 16));
#define BJ_GO(R, LPP) \
  return bjac_launch_round<R, LPP>(st, T, ldt, tr, from_T, W, Vh, p, c, nb, round, sweep, counters)
  if (rpl16 <= 4) BJ_GO(4, 16);
  if (rpl16 <= 8) BJ_GO(8, 16);
  if (rpl16 <= 12) BJ_GO(12, 16);
  if (rpl16 <= 16) BJ_GO(16, 16);
  const int rpl = static_cast<int>(ceil_div(p, WAVE));
  if (rpl <= 5) BJ_GO(5, WAVE);
  if (rpl <= 6) BJ_GO(6, WAVE);
  if (rpl <= 8) BJ_GO(8, WAVE);
  if (rpl <= 12) BJ_GO(12, WAVE);
  if (rpl <= 16) BJ_GO(16, WAVE);
#undef BJ_GO
  return SVDS_EUNSUPPORTED;
}

static __global__ void zero_i32_kernel(int n, int *__restrict__ out) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) out[i] = 0;
}

// Block-schedule sweeps of W Vh (p rows, nb*c columns each, in `work`) from
// the rows of T (row stride ldt, rows from tr on zero) until a sweep passes
// without a rotation; returns the sweeps enqueued in *nsw.  Sweeps are
// enqueued in chunks (10, then 2 at a time) and the rotation counters read
// back after each chunk.
static int bjac_sweeps(hipStream_t st, const double *T, int ldt, int tr, double *work, int p, int *h_counts,
                       int *nsw) {
  int c, nb;
  bjac_shape(p, c, nb);
  double *W = work;
  double *Vh = work + static_cast<int64_t>(p) * nb * c;
  int *counters = reinterpret_cast<int *>(Vh + static_cast<int64_t>(p) * nb * c);
  hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(64), 0, st, JAC_MAX_SWEEPS, counters);
  HIP_TRY(hipGetLastError());
  int enq = 0;
  bool done = false;
  while (!done && enq < JAC_MAX_SWEEPS) {
    const int chunk = std::min(enq == 0 ? 10 : 2, JAC_MAX_SWEEPS - enq);
    for (int sw = enq; sw < enq + chunk; ++sw)
      for (int r = 0; r < nb - 1; ++r) {
        const int rc = bjac_round(st, T, ldt, tr, sw == 0 && r == 0, W, Vh, p, c, nb, r, sw, counters);
        if (rc) return rc;
      }
    enq += chunk;
    HIP_TRY(hipMemcpyAsync(h_counts, counters, sizeof(int) * enq, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int i = 0; i < enq; ++i)
      if (h_counts[i] == 0) done = true;
  }
  *nsw = enq;
  return SVDS_OK;
}
}  // namespace

int svds_small_svd_run(hipStream_t st, double *T, int p, int k, double tol, double *work, double *Uk,
                       double *Vext, double *sig, double *res, double *rho, int *flags, double *sigma_est,
                       int *h_counts, int smallest) {
  if (p < 2 || k < 1 || k >= p || p > 1023) return SVDS_EINVAL;
  if (p <= JAC_SMALL_P) {
    const int nthr = small_svd_threads(p);
    hipLaunchKernelGGL(small_svd_kernel, dim3(1), dim3(nthr), small_svd_lds_bytes(p), st, T, p, k, tol, Uk,
                       Vext, sig, res, rho, flags, sigma_est, smallest);
    HIP_TRY(hipGetLastError());
    return SVDS_OK;
  }
  int enq = 0;
  const int rc = bjac_sweeps(st, T, p + 1, p, work, p, h_counts, &enq);
  if (rc) return rc;
  int c, nb;
  bjac_shape(p, c, nb);
  const double *W = work;
  const double *Vh = work + static_cast<int64_t>(p) * nb * c;
  const int *counters = reinterpret_cast<const int *>(Vh + static_cast<int64_t>(p) * nb * c);
  hipLaunchKernelGGL(bjac_finish_kernel, dim3(1), dim3(JAC_THREADS), static_cast<size_t>(p) * 12, st, W, Vh,
                     counters, enq, T, p, k, tol, Uk, Vext, sig, res, rho, flags, sigma_est, smallest);
  HIP_TRY(hipGetLastError());
  return SVDS_OK;
}

int svds_harmonic_basis_run(hipStream_t st, const double *T, int p, int k, double *work, double *QC, double *QM,
                            double *R, int *h_counts) {
  const int q = p + 1;
  if (p < 2 || k < 1 || k >= p || q > 1023) return SVDS_EINVAL;
  if (q <= JAC_SMALL_P) {
    hipLaunchKernelGGL(harm_small_kernel, dim3(1), dim3(small_svd_threads(q)), harm_small_lds_bytes(p), st, T, p,
                       k, QC, QM, R);
    HIP_TRY(hipGetLastError());
    return SVDS_OK;
  }
  // the stored (p+1) x (p+1) matrix, row stride p + 1, row p zero
  int enq = 0;
  const int rc = bjac_sweeps(st, T, q, p, work, q, h_counts, &enq);
  if (rc) return rc;
  int c, nb;
  bjac_shape(q, c, nb);
  const double *W = work;
  const double *Vh = work + static_cast<int64_t>(q) * nb * c;
  hipLaunchKernelGGL(harm_bjac_finish_kernel, dim3(1), dim3(JAC_THREADS), harm_scratch_bytes(q), st, W, Vh, p, k,
                     QC, QM, R);
  HIP_TRY(hipGetLastError());
  return SVDS_OK;
}

#include "batched_impl.hpp"
