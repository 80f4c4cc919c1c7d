// C ABI entry points that wrap plans (solve = create + execute + destroy),
// the batched form, explicit residuals, single-step operations (for parity
// tests and measurements of individual kernels) and error strings.
#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/svds.h"
#include "../../include/svds_ops.h"
#include "plan.hpp"
#include "kernels_cgs.hpp"
#include "kernels_csc.hpp"
#include "kernels_jacobi.hpp"
#include "kernels_misc.hpp"

using namespace svds;

extern "C" int svds_csr_solve(const svds_csr *A, const svds_opts *opts, double *U, double *S,
                              double *V, svds_info *info) {
  SVDS_ABI_TRY
  svds_plan *P = nullptr;
  int rc = svds_plan_create_csr(A, opts, &P);
  if (rc) return rc;
  rc = svds_plan_execute(P, U, S, V, info);
  svds_plan_destroy(P);
  return rc;
  SVDS_ABI_CATCH
}

extern "C" int svds_dense_solve(const svds_dense *A, const svds_opts *opts, double *U, double *S,
                                double *V, svds_info *info) {
  SVDS_ABI_TRY
  svds_plan *P = nullptr;
  int rc = svds_plan_create_dense(A, opts, &P);
  if (rc) return rc;
  rc = svds_plan_execute(P, U, S, V, info);
  svds_plan_destroy(P);
  return rc;
  SVDS_ABI_CATCH
}

extern "C" int svds_residuals_csr(const svds_csr *A, int32_t k, const double *U, const double *S,
                                  const double *V, double *res_av, double *res_atu, void *stream) {
  SVDS_ABI_TRY
  if (!A || k < 1 || !U || !S || !V || !res_av || !res_atu) return SVDS_EINVAL;
  svds_opts o{};
  o.k = 1;
  o.p = 2;
  o.stream = stream;
  if (A->m < 2 || A->n < 3) return SVDS_EINVAL;
  svds_plan *P = nullptr;
  int rc = svds_plan_create_csr(A, &o, &P);
  if (rc) return rc;
  rc = svds_plan_residuals(P, k, U, S, V, res_av, res_atu);
  svds_plan_destroy(P);
  return rc;
  SVDS_ABI_CATCH
}

extern "C" int svds_residuals_dense(const svds_dense *A, int32_t k, const double *U, const double *S,
                                    const double *V, double *res_av, double *res_atu, void *stream) {
  SVDS_ABI_TRY
  if (!A || k < 1 || !U || !S || !V || !res_av || !res_atu) return SVDS_EINVAL;
  if (A->m < k + 1 || A->n < k + 2) return SVDS_EINVAL;
  svds_opts o{};
  o.k = k;  // the plan's residual scratch is sized for k triplets
  o.p = k + 1;
  o.stream = stream;
  svds_plan *P = nullptr;
  int rc = svds_plan_create_dense(A, &o, &P);
  if (rc) return rc;
  rc = svds_plan_residuals(P, k, U, S, V, res_av, res_atu);
  svds_plan_destroy(P);
  return rc;
  SVDS_ABI_CATCH
}

extern "C" const char *svds_strerror(int code) {
  switch (code) {
    case SVDS_OK: return "ok";
    case SVDS_NOT_CONVERGED: return "not converged within maxit cycles (outputs hold current Ritz triplets)";
    case SVDS_EINVAL: return "invalid argument";
    case SVDS_ENOMEM: return "device workspace allocation failed";
    case SVDS_EDEVICE: {
      static thread_local char buf[600];
      snprintf(buf, sizeof buf, "HIP runtime error: %s", last_error_text());
      return buf;
    }
    case SVDS_EUNSUPPORTED: return "unsupported request";
    default: return "unknown error code";
  }
}

extern "C" const char *svds_version(void) { return "svds-mi355x 0.1 (gfx950)"; }

// ===========================================================================
// Single-step operations
// ===========================================================================
namespace {
struct Scratch {
  void *p = nullptr;
  ~Scratch() {
    if (p) (void)hipFree(p);
  }
};
}  // namespace

extern "C" int svds_op_spmv_csr(const svds_csr *A, const void *x, const double *x_scale,
                                const double *coef, const void *yprev, void *y, int32_t basis_dtype,
                                void *stream) {
  SVDS_ABI_TRY
  if (!A || !x || !y || A->m < 1 || A->n < 1) return SVDS_EINVAL;
  if (A->dtype != SVDS_F64 && A->dtype != SVDS_F32) return SVDS_EUNSUPPORTED;
  if (basis_dtype != SVDS_F64 && basis_dtype != SVDS_F32) return SVDS_EUNSUPPORTED;
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<int32_t> hrp(A->m + 1);
  HIP_TRY(hipMemcpy(hrp.data(), A->row_ptr, sizeof(int32_t) * (A->m + 1), hipMemcpyDeviceToHost));
  if (hrp[0] != 0 || hrp[A->m] != A->nnz) return SVDS_EINVAL;
  SpmvPlan sp;
  build_spmv_items(hrp.data(), A->m, sp);
  Scratch s;
  const size_t bi = sizeof(int4) * sp.nitems, bl = sizeof(LongRow) * std::max(1, sp.nlong),
               bp = sizeof(double) * std::max(1, sp.npieces);
  HIP_TRY(hipMalloc(&s.p, bi + bl + bp + 1024));
  char *b = static_cast<char *>(s.p);
  int4 *items = reinterpret_cast<int4 *>(b);
  LongRow *lr = reinterpret_cast<LongRow *>(b + ((bi + 255) & ~size_t(255)));
  double *parts = reinterpret_cast<double *>(reinterpret_cast<char *>(lr) + ((bl + 255) & ~size_t(255)));
  HIP_TRY(hipMemcpy(items, sp.h_items.data(), bi, hipMemcpyHostToDevice));
  if (sp.nlong) HIP_TRY(hipMemcpy(lr, sp.h_long.data(), sizeof(LongRow) * sp.nlong, hipMemcpyHostToDevice));
#define SPMV_GO(TV, TB)                                                                             \
  do {                                                                                              \
    hipLaunchKernelGGL((spmv_csr_kernel<TV, TB>), dim3(sp.nitems), dim3(SPMV_THREADS), 0, st, items, \
                       A->row_ptr, A->col_idx, static_cast<const TV *>(A->val), nullptr,            \
                       static_cast<const TB *>(x), x_scale, coef, static_cast<const TB *>(yprev),   \
                       static_cast<TB *>(y), reinterpret_cast<TB *>(parts), nullptr, 0, nullptr, nullptr, nullptr, 0, \
                       SpmvProj<TB>{nullptr, 0, 0, nullptr});                                       \
    if (sp.nlong)                                                                                   \
      hipLaunchKernelGGL((spmv_longrow_fixup_kernel<TB>), dim3(sp.nlong), dim3(WAVE), 0, \
                         st, lr, sp.nlong, reinterpret_cast<TB *>(parts), x_scale, coef,            \
                         static_cast<const TB *>(yprev), static_cast<TB *>(y), nullptr);            \
  } while (0)
  if (A->dtype == SVDS_F64 && basis_dtype == SVDS_F64) SPMV_GO(double, double);
  else if (A->dtype == SVDS_F32 && basis_dtype == SVDS_F64) SPMV_GO(float, double);
  else if (A->dtype == SVDS_F64 && basis_dtype == SVDS_F32) SPMV_GO(double, float);
  else SPMV_GO(float, float);
#undef SPMV_GO
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  return SVDS_OK;
  SVDS_ABI_CATCH
}

extern "C" int svds_op_dense_matvec(const svds_dense *A, int32_t transpose, const void *x,
                                    const double *x_scale, const double *coef, const void *yprev,
                                    void *y, int32_t basis_dtype, void *stream) {
  SVDS_ABI_TRY
  if (!A || !x || !y || A->m < 1 || A->n < 1 || A->ld < A->m) return SVDS_EINVAL;
  svds_opts o{};
  o.k = 1;
  o.p = 2;
  o.stream = stream;
  o.precision = basis_dtype == SVDS_F32 ? SVDS_PREC_MIXED : SVDS_PREC_FP64;
  o.flags = SVDS_FLAG_NO_RESIDUALS;  // no residual workspace for a single product
  if (A->m < 2 || A->n < 3) return SVDS_EINVAL;
  svds_plan *P = nullptr;
  int rc = svds_plan_create_dense(A, &o, &P);
  if (rc) return rc;
  rc = svds_plan_matvec(P, transpose, x, x_scale, coef, yprev, y, basis_dtype);
  svds_plan_destroy(P);
  return rc;
  SVDS_ABI_CATCH
}

extern "C" int svds_op_csr_matvec(const svds_csr *A, int32_t transpose, const void *x,
                                  const double *x_scale, const double *coef, const void *yprev,
                                  void *y, int32_t basis_dtype, int32_t *panels, void *stream) {
  SVDS_ABI_TRY
  if (!A || !x || !y) return SVDS_EINVAL;
  if (A->m < 2 || A->n < 3) return SVDS_EINVAL;
  if (basis_dtype != SVDS_F64 && basis_dtype != SVDS_F32) return SVDS_EUNSUPPORTED;
  svds_opts o{};
  o.k = 1;
  o.p = 2;
  o.stream = stream;
  o.precision = basis_dtype == SVDS_F32 ? SVDS_PREC_MIXED : SVDS_PREC_FP64;
  o.flags = SVDS_FLAG_NO_RESIDUALS;
  svds_plan *P = nullptr;
  int rc = svds_plan_create_csr(A, &o, &P);
  if (rc) return rc;
  if (panels) *panels = transpose ? svds_plan_panels(P) : 1;
  rc = svds_plan_matvec(P, transpose, x, x_scale, coef, yprev, y, basis_dtype);
  svds_plan_destroy(P);
  return rc;
  SVDS_ABI_CATCH
}

extern "C" int svds_op_csc_build(const svds_csr *A, int32_t *t_row_ptr, int32_t *t_col_idx,
                                 void *t_val, void *stream) {
  SVDS_ABI_TRY
  if (!A || !t_row_ptr || (A->nnz > 0 && (!t_col_idx || !t_val))) return SVDS_EINVAL;
  if (A->m < 2 || A->n < 3) return SVDS_EINVAL;
  svds_opts o{};
  o.k = 1;
  o.p = 2;
  o.stream = stream;
  svds_plan *P = nullptr;
  int rc = svds_plan_create_csr(A, &o, &P);
  if (rc) return rc;
  rc = svds_plan_transpose_copy(P, t_row_ptr, t_col_idx, t_val);
  svds_plan_destroy(P);
  return rc;
  SVDS_ABI_CATCH
}

extern "C" int svds_op_cgs2(int64_t L, int32_t j, const void *Q, int64_t ldq, const void *w, void *out,
                            double *norm_out, int32_t dtype, void *stream) {
  SVDS_ABI_TRY
  if (L < 1 || j < 0 || j > CGS_MAXJ || (j > 0 && (!Q || ldq < L)) || !w || !out) return SVDS_EINVAL;
  if (dtype != SVDS_F64 && dtype != SVDS_F32) return SVDS_EUNSUPPORTED;
  return svds_cgs2_op(L, j, Q, ldq, w, out, norm_out, dtype, stream);
  SVDS_ABI_CATCH
}

extern "C" int svds_op_small_svd(int32_t p, int32_t k, double tol, double *T, double *Uk, double *Vext,
                                 double *sig, double *res, double *rho, int32_t *flags_host,
                                 void *stream) {
  SVDS_ABI_TRY
  if (p < 2 || k < 1 || k >= p || !T || !Uk || !Vext || !sig || !res || !rho) return SVDS_EINVAL;
  if (p > 1023) return SVDS_EUNSUPPORTED;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t wb = jacobi_work_bytes(p);
  Scratch s;
  HIP_TRY(hipMalloc(&s.p, wb + 256));
  double *sigma_est = static_cast<double *>(s.p);
  int *flags = reinterpret_cast<int *>(sigma_est + 4);
  double *jac = sigma_est + 8;
  HIP_TRY(hipMemsetAsync(s.p, 0, 64, st));
  std::vector<int> counts(JAC_MAX_SWEEPS);
  int rc = svds_small_svd_run(st, T, p, k, tol, jac, Uk, Vext, sig, res, rho, flags, sigma_est, counts.data());
  if (rc) return rc;
  int hf[4] = {0, 0, 0, 0};
  HIP_TRY(hipMemcpyAsync(hf, flags, sizeof hf, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (flags_host) std::memcpy(flags_host, hf, 3 * sizeof(int));
  return SVDS_OK;
  SVDS_ABI_CATCH
}

extern "C" int svds_op_harmonic_basis(int32_t p, int32_t k, const double *T, double *QC, double *QM, double *R,
                                      void *stream) {
  SVDS_ABI_TRY
  if (p < 2 || k < 1 || k >= p || p > 1022 || !T || !QC || !QM || !R) return SVDS_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  Scratch s;
  HIP_TRY(hipMalloc(&s.p, jacobi_work_bytes(p + 1) + 256));
  std::vector<int> counts(JAC_MAX_SWEEPS);
  const int rc = svds_harmonic_basis_run(st, T, p, k, static_cast<double *>(s.p), QC, QM, R, counts.data());
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(st));
  return SVDS_OK;
  SVDS_ABI_CATCH
}

extern "C" int svds_op_rotate(int64_t L, int32_t pc, int32_t kc, const void *B, int64_t ldb,
                              int32_t btype, const double *Y, int64_t ldy, double *out, int64_t ldo,
                              void *stream) {
  SVDS_ABI_TRY
  if (L < 1 || pc < 1 || kc < 1 || !B || !Y || !out || ldb < L || ldy < pc || ldo < L) return SVDS_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool mfma = !(btype & SVDS_ROTATE_VECTOR);
  btype &= ~SVDS_ROTATE_VECTOR;
  if (btype != SVDS_F64 && btype != SVDS_F32) return SVDS_EUNSUPPORTED;
  Scratch yt;
  HIP_TRY(hipMalloc(&yt.p, sizeof(double) * rot_yt_doubles(pc, kc)));
  double *Yt = static_cast<double *>(yt.p);
  if (btype == SVDS_F64)
    HIP_TRY((rotate_launch<double, double>(st, L, pc, kc, static_cast<const double *>(B), ldb, Y, ldy, Yt,
                                           out, ldo, mfma)));
  else
    HIP_TRY((rotate_launch<float, double>(st, L, pc, kc, static_cast<const float *>(B), ldb, Y, ldy, Yt,
                                          out, ldo, mfma)));
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  return SVDS_OK;
  SVDS_ABI_CATCH
}

extern "C" int svds_op_philox_normal(int64_t L, uint64_t seed, uint32_t stream_id, double *out,
                                     void *stream) {
  SVDS_ABI_TRY
  if (L < 1 || !out) return SVDS_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL((philox_fill_kernel<double>), dim3(ceil_div(ceil_div(L, 2), 256)), dim3(256), 0, st,
                     L, seed, stream_id, out);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  return SVDS_OK;
  SVDS_ABI_CATCH
}

extern "C" int svds_op_gather_copy(int64_t L, const int32_t *idx, const double *x, double *out, int32_t nseg,
                                   const int64_t *seg, int32_t reps, double *ms_per_launch, void *stream) {
  SVDS_ABI_TRY
  if (L < 1 || !idx || !x || !out || nseg < 1 || nseg > 64 || reps < 1) return SVDS_EINVAL;
  std::vector<int64_t> hs(nseg + 1);
  if (seg) {
    for (int g = 0; g <= nseg; ++g) hs[g] = seg[g];
    if (hs[0] != 0 || hs[nseg] != L) return SVDS_EINVAL;
    for (int g = 0; g < nseg; ++g)
      if (hs[g + 1] < hs[g]) return SVDS_EINVAL;
  } else {
    for (int g = 0; g <= nseg; ++g) hs[g] = L * g / nseg;
  }
  int64_t chunks = 0;
  for (int g = 0; g < nseg; ++g) chunks = std::max<int64_t>(chunks, ceil_div(hs[g + 1] - hs[g], GATHER_CHUNK));
  if (chunks * nseg > INT32_MAX) return SVDS_EUNSUPPORTED;
  hipStream_t st = static_cast<hipStream_t>(stream);
  Scratch d;
  HIP_TRY(hipMalloc(&d.p, sizeof(int64_t) * (nseg + 1)));
  HIP_TRY(hipMemcpyAsync(d.p, hs.data(), sizeof(int64_t) * (nseg + 1), hipMemcpyHostToDevice, st));
  hipEvent_t ev[2] = {nullptr, nullptr};
  struct Ev {
    hipEvent_t *e;
    ~Ev() {
      for (int i = 0; i < 2; ++i)
        if (e[i]) (void)hipEventDestroy(e[i]);
    }
  } guard{ev};
  HIP_TRY(hipEventCreate(&ev[0]));
  HIP_TRY(hipEventCreate(&ev[1]));
  HIP_TRY(hipEventRecord(ev[0], st));
  for (int r = 0; r < reps && chunks > 0; ++r)
    hipLaunchKernelGGL(gather_copy_kernel, dim3(static_cast<unsigned>(chunks * nseg)), dim3(256), 0, st, idx, x,
                       out, nseg, static_cast<const int64_t *>(d.p));
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(ev[1], st));
  HIP_TRY(hipStreamSynchronize(st));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, ev[0], ev[1]));
  if (ms_per_launch) *ms_per_launch = static_cast<double>(ms) / reps;
  return SVDS_OK;
  SVDS_ABI_CATCH
}

extern "C" int svds_op_copy_f64(int64_t L, const double *src, double *dst, void *stream) {
  SVDS_ABI_TRY
  if (L < 1 || !src || !dst) return SVDS_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(copy_f64_kernel, dim3(ceil_div(L, 256)), dim3(256), 0, st, L, src, dst);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  return SVDS_OK;
  SVDS_ABI_CATCH
}
