// Lanczos steps of a small sparse problem in one workgroup (Alg. 1 steps
// 5-8 with the full re-orthogonalization by CGS2 that Sec. 2.1 asks for).
//
// For vectors of a few thousand entries a Lanczos half-step (one product,
// three CGS2 passes, the norm) costs four dependent launches of 3-10 us
// each while the work itself is a few hundred KB.  This kernel runs steps
// i0..p-1 of a cycle in one workgroup instead:
// the vector being orthogonalized stays in LDS, the bases (U m x (p+1),
// V n x (p+1), a few hundred KB) are read from L2, and the stages are
// separated by barriers, not launches.  It computes what the multi-launch
// path computes, step for step:
//   v-step i: U[:, i] = u_i = bu * xs_u; w = A^T u_i - T(i,i) v_i; CGS2
//             against V[:, 0..i]; beta_i = |w| -> T(i,i+1); v_{i+1}.
//   u-step:   V[:, i+1] = v_{i+1}; w = A v_{i+1} - beta_i u_i; CGS2 against
//             U[:, 0..i]; alpha_{i+1} = |w| -> T(i+1,i+1); u_{i+1}.
//   last v-step (i = p - 1): V[:, p] = v_p.
// with the same breakdown rule (|w| <= BREAKDOWN_REL * sigma_est: the same
// Philox replacement vector taken twice against the basis, 0 in T) and the
// same state left behind (bu, bv unnormalized with scales xs_u, xs_v,
// sigma_est, the breakdown counter); only the summation orders differ.
// One thread per row for the products (the eligible matrices have short
// rows), one wave per basis column for the projections.
#pragma once
#include "common.hpp"
#include "kernels_cgs.hpp"

namespace svds {

constexpr int LZS_THREADS = 1024;
constexpr int64_t LZS_MAX_L = 6144;      // longest vector: w (LDS) plus the static arrays stay below 64 KB
// One CU reads the bases from L2 at ~0.1 TB/s and runs the products one
// thread per row.  Measured on MI355X against the step-by-step launches
// (whose short products carry the first CGS pass and whose short passes sum
// their partials themselves): 19% faster with 2 x 1000 x 21 FP64 bases
// (328 KB; 1000 x 1000, 5 nonzeros per row, p = 20), even at 492 KB (1500 x
// 1500, 7500 nonzeros), 6% slower at 656 KB (2000 x 2000, 10,000 nonzeros)
// and 13-16% slower on 2000 x 1000 with 20,000 nonzeros at p = 20-28
// (492-680 KB).
constexpr int64_t LZS_MAX_NNZ = 8192;
constexpr int64_t LZS_MAX_BASIS_BYTES = 512 << 10;

// w (LDS, L entries) <- (I - Q Q^T)(I - Q Q^T) w, Q = columns 0..j-1 (ld ldq)
__device__ inline void lzs_cgs2(const double *__restrict__ Q, int64_t ldq, int L, int j, double *w,
                                double *sh_h) {
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const int nw = blockDim.x / WAVE;
  for (int pass = 0; pass < 2; ++pass) {
    for (int c = wv; c < j; c += nw) {
      const double *q = Q + c * ldq;
      double s = 0;
      for (int r = lane; r < L; r += WAVE) s += q[r] * w[r];
      s = wave_sum(s);
      if (lane == 0) sh_h[c] = s;
    }
    __syncthreads();
    for (int r = tid; r < L; r += blockDim.x) {
      double s = 0;
      for (int c = 0; c < j; ++c) s += Q[c * ldq + r] * sh_h[c];
      w[r] -= s;
    }
    __syncthreads();
  }
}

// Row r of a CSR product: sum_z a[z] x[col[z]] over z in [z0, z1), eight
// nonzeros at a time (their index and value loads, then their gathers, in
// flight together), added in nonzero order.
template <typename TV>
__device__ __forceinline__ double lzs_row(const int32_t *__restrict__ col, const TV *__restrict__ a,
                                          const double *__restrict__ x, int z0, int z1) {
  double s = 0;
  int z = z0;
  for (; z + 8 <= z1; z += 8) {
    int c[8];
    double v[8], g[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      c[u] = col[z + u];
      v[u] = widen<double>(a[z + u]);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) g[u] = x[c[u]];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u] * g[u];
  }
  for (; z < z1; ++z) s += widen<double>(a[z]) * x[col[z]];
  return s;
}

// |w| of the LDS vector; every thread gets the same value.
__device__ inline double lzs_norm(const double *w, int L, double *sh_d) {
  double s = 0;
  for (int r = threadIdx.x; r < L; r += blockDim.x) s += w[r] * w[r];
  return sqrt(block_sum(s, sh_d));
}

// Breakdown replacement (as breakdown_repair): out = the Philox normal
// vector of stream `stream`, taken twice against Q[:, 0..j-1], normalized;
// built in the LDS vector w.
__device__ inline void lzs_repair(const double *__restrict__ Q, int64_t ldq, int L, int j, double *w,
                                  double *__restrict__ out, uint32_t stream, uint64_t seed, double *sh_d,
                                  double *sh_h) {
  for (int b = threadIdx.x; 2 * b < L; b += blockDim.x) {
    double z0, z1;
    philox_normal_pair(seed, stream, static_cast<uint64_t>(b), z0, z1);
    w[2 * b] = z0;
    if (2 * b + 1 < L) w[2 * b + 1] = z1;
  }
  __syncthreads();
  lzs_cgs2(Q, ldq, L, j, w, sh_h);
  const double inv = 1.0 / lzs_norm(w, L, sh_d);
  for (int r = threadIdx.x; r < L; r += blockDim.x) out[r] = w[r] * inv;
  __syncthreads();
}

// The finish of a step: |w| into T (and into t, in every thread), the scale
// of the stored vector, the running sigma estimate; or on a breakdown the
// replacement vector (taken against Q[:, 0..j-1]) with 0 in T and scale 1.
// out (global) receives w or the replacement; returns the scale.
__device__ inline double lzs_finish(double *w, int L, const double *__restrict__ Q, int64_t ldq, int j,
                                    double *__restrict__ out, double *__restrict__ t_entry, double &t,
                                    double &sig, int *__restrict__ breakdowns, uint64_t seed, double *sh_d,
                                    double *sh_h, int *s_bd) {
  const double nrm = lzs_norm(w, L, sh_d);
  if (nrm > BREAKDOWN_REL * sig) {
    for (int r = threadIdx.x; r < L; r += blockDim.x) out[r] = w[r];
    if (threadIdx.x == 0) *t_entry = nrm;
    t = nrm;
    sig = fmax(sig, nrm);
    __syncthreads();
    return 1.0 / nrm;
  }
  if (threadIdx.x == 0) {
    *s_bd = *breakdowns + 1;
    *breakdowns = *s_bd;
    *t_entry = 0.0;
  }
  t = 0.0;
  __syncthreads();
  lzs_repair(Q, ldq, L, j, w, out, static_cast<uint32_t>(*s_bd), seed, sh_d, sh_h);
  return 1.0;
}

template <typename TV>
__global__ __launch_bounds__(LZS_THREADS) void lanczos_small_kernel(
    int m, int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci, const TV *__restrict__ val,
    const int32_t *__restrict__ trp, const int32_t *__restrict__ tci, const TV *__restrict__ tval,
    double *__restrict__ U, int64_t ldu, double *__restrict__ V, int64_t ldv, double *__restrict__ T, int ld,
    int i0, int p, double *__restrict__ bu, double *__restrict__ bv, double *__restrict__ xs_u,
    double *__restrict__ xs_v, double *__restrict__ sigma_est, int *__restrict__ breakdowns, uint64_t seed) {
  extern __shared__ double w[];  // max(m, n) entries
  __shared__ double sh_h[CGS_MAXJ];
  __shared__ double sh_d[LZS_THREADS / WAVE];
  __shared__ int s_bd;
  const int tid = threadIdx.x, nt = blockDim.x;
  // the scalars of the process stay in registers (the same value in every
  // thread); T receives them as they are formed
  double sig = *sigma_est;
  double xu = *xs_u, xv = *xs_v;
  double alpha = T[i0 * ld + i0], beta = 0.0;
  for (int i = i0; i < p; ++i) {
    // v-step: u_i into U[:, i], w = A^T u_i - alpha_i v_i
    double *Ui = U + i * ldu;
    for (int r = tid; r < m; r += nt) Ui[r] = bu[r] * xu;
    __syncthreads();
    const double *Vi = V + i * ldv;
    for (int c = tid; c < n; c += nt) w[c] = lzs_row(tci, tval, Ui, trp[c], trp[c + 1]) - alpha * Vi[c];
    __syncthreads();
    lzs_cgs2(V, ldv, n, i + 1, w, sh_h);
    xv = lzs_finish(w, n, V, ldv, i + 1, bv, T + i * ld + i + 1, beta, sig, breakdowns, seed, sh_d, sh_h, &s_bd);
    // v_{i+1} into V[:, i+1] (for i = p - 1 that is v_{p+1} of the restart)
    double *Vn = V + (i + 1) * ldv;
    for (int c = tid; c < n; c += nt) Vn[c] = bv[c] * xv;
    __syncthreads();
    if (i == p - 1) break;
    // u-step: w = A v_{i+1} - beta_i u_i
    for (int r = tid; r < m; r += nt) w[r] = lzs_row(ci, val, Vn, rp[r], rp[r + 1]) - beta * Ui[r];
    __syncthreads();
    lzs_cgs2(U, ldu, m, i + 1, w, sh_h);
    xu = lzs_finish(w, m, U, ldu, i + 1, bu, T + (i + 1) * ld + i + 1, alpha, sig, breakdowns, seed, sh_d, sh_h,
                    &s_bd);
  }
  if (tid == 0) {
    *xs_u = xu;
    *xs_v = xv;
    *sigma_est = sig;
  }
}

}  // namespace svds
