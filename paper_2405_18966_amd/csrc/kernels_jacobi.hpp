// Small SVD of T(1:p,1:p), convergence test and restart set-up
// (Alg. 2 steps 4-9, eq. (4), eq. (6)) in ONE workgroup, FP64.
//
// SVD method: one-sided Jacobi (Hestenes 1958).  W <- T, Vh <- I; column
// pairs (i, j) are rotated from the right until every pair is orthogonal to
// working precision: with a = |w_i|^2, b = |w_j|^2, c = w_i . w_j the pair is
// rotated when |c| > tolJ * sqrt(a b), by t = sign(z)/(|z| + sqrt(1+z^2)),
// z = (b - a)/(2c), cs = 1/sqrt(1+t^2), sn = cs t (Rutishauser).  Pairs are
// scheduled in round-robin (tournament) order: each step rotates p/2
// disjoint pairs, one wave per pair; a sweep is p-1 steps.  Then
// sigma_i = |w_i|, Uh_i = w_i / sigma_i, sorted descending.
//
// T is upper triangular (bidiagonal after the first LBP; diagonal block,
// arrow column k+1, then bidiagonal after a restart, Alg. 2 step 9), so the
// general dense SVD is needed.
//
// Outputs (all device, FP64):
//   Uk   p x k   (ld p)     leading left singular vectors of T
//   Vext (p+1) x (k+1) (ld p+1): leading right singular vectors of T with a
//        zero row p, plus column k = e_{p+1}; the restart rotation
//        [V(:,1:p) v_{p+1}] Vext gives [V Vh_k, v_{p+1}] in one product
//        (Alg. 2 steps 8 and 10).
//   sig  k       singular values, res k estimates of eq. (4)
//   rho  k       beta_p Uh(p, j) (eq. (6)); T is rewritten as the restarted
//                matrix [diag(sig), rho] (Alg. 2 step 9).
//   flags[0] = all estimates < tol, flags[1] = leading count below tol,
//   flags[2] = Jacobi sweeps used.
#pragma once
#include "common.hpp"

namespace svds {

constexpr int JAC_THREADS = 1024;

// bytes of the Jacobi work area for a p x p problem
__host__ __device__ inline int64_t jacobi_work_bytes(int p) {
  const int64_t pe = p + (p & 1);
  return (2 * pe * pe + pe) * 8 + pe * 4;
}
constexpr int JAC_MAX_SWEEPS = 30;

__device__ __forceinline__ void rr_pair(int pe, int step, int i, int &a, int &b) {
  // players 1..pe-1 on a ring rotated by `step`; player 0 is fixed
  const int n1 = pe - 1;
  if (i == 0) {
    a = 0;
    b = 1 + (step % n1);
  } else {
    a = 1 + ((step + i) % n1);
    b = 1 + ((step + n1 - i) % n1);
  }
}

template <int RPL>
__global__ __launch_bounds__(JAC_THREADS) void small_svd_kernel(
    double *__restrict__ T, int p, int k, double tol, double *__restrict__ scratch,
    double *__restrict__ Uk, double *__restrict__ Vext,
    double *__restrict__ sig, double *__restrict__ res, double *__restrict__ rho,
    int *__restrict__ flags, double *__restrict__ sigma_est, int use_lds) {
  extern __shared__ double smem[];
  __shared__ int rot_count;
  __shared__ double s_beta;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const int nwaves = blockDim.x / WAVE;
  const int pe = p + (p & 1);
  const int ld = p + 1;
  // layout of the work area (LDS when it fits, else global scratch):
  // W pe x pe | Vh pe x pe | sigma pe | rank pe (int)
  double *base = use_lds ? smem : scratch;
  double *W = base;
  double *Vh = base + static_cast<int64_t>(pe) * pe;

  if (tid == 0) s_beta = T[(p - 1) * ld + p];
  for (int idx = tid; idx < pe * pe; idx += blockDim.x) {
    const int r = idx % pe, c = idx / pe;
    W[idx] = (r < p && c < p) ? T[r * ld + c] : 0.0;
    Vh[idx] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();

  // tolJ: orthogonality to working precision, scaled by sqrt(rows)
  const double tolJ = 0x1.0p-52 * sqrt(static_cast<double>(pe));
  const int npairs = pe / 2;
  // pairs per batch: a wave issues the loads of B pairs (W and Vh columns)
  // before any of them is reduced, so one memory round trip serves B pairs
  constexpr int B = RPL <= 2 ? 4 : (RPL <= 4 ? 3 : 1);
  int sweeps = 0;
  for (int sweep = 0; sweep < JAC_MAX_SWEEPS; ++sweep) {
    if (tid == 0) rot_count = 0;
    __syncthreads();
    for (int step = 0; step < pe - 1; ++step) {
      for (int base = wv; base < npairs; base += nwaves * B) {
        double xi[B][RPL], xj[B][RPL], yi[B][RPL], yj[B][RPL];
        int ci[B], cj[B];
#pragma unroll
        for (int q = 0; q < B; ++q) {
          const int pi = base + q * nwaves;
          ci[q] = cj[q] = -1;
          if (pi < npairs) rr_pair(pe, step, pi, ci[q], cj[q]);
#pragma unroll
          for (int t = 0; t < RPL; ++t) {
            const int r = lane + t * WAVE;
            const bool ok = ci[q] >= 0 && r < pe;
            xi[q][t] = ok ? W[static_cast<int64_t>(ci[q]) * pe + r] : 0.0;
            xj[q][t] = ok ? W[static_cast<int64_t>(cj[q]) * pe + r] : 0.0;
            yi[q][t] = ok ? Vh[static_cast<int64_t>(ci[q]) * pe + r] : 0.0;
            yj[q][t] = ok ? Vh[static_cast<int64_t>(cj[q]) * pe + r] : 0.0;
          }
        }
#pragma unroll
        for (int q = 0; q < B; ++q) {
          if (ci[q] < 0) continue;  // wave-uniform
          double a = 0, bb = 0, c = 0;
#pragma unroll
          for (int t = 0; t < RPL; ++t) {
            a += xi[q][t] * xi[q][t];
            bb += xj[q][t] * xj[q][t];
            c += xi[q][t] * xj[q][t];
          }
          a = wave_sum(a);
          bb = wave_sum(bb);
          c = wave_sum(c);
          if (fabs(c) > tolJ * sqrt(a * bb)) {
            const double z = (bb - a) / (2.0 * c);
            const double tt = (z >= 0 ? 1.0 : -1.0) / (fabs(z) + sqrt(1.0 + z * z));
            const double cs = 1.0 / sqrt(1.0 + tt * tt);
            const double sn = cs * tt;
            double *wi = W + static_cast<int64_t>(ci[q]) * pe, *wj = W + static_cast<int64_t>(cj[q]) * pe;
            double *vi = Vh + static_cast<int64_t>(ci[q]) * pe, *vj = Vh + static_cast<int64_t>(cj[q]) * pe;
#pragma unroll
            for (int t = 0; t < RPL; ++t) {
              const int r = lane + t * WAVE;
              if (r < pe) {
                wi[r] = cs * xi[q][t] - sn * xj[q][t];
                wj[r] = sn * xi[q][t] + cs * xj[q][t];
                vi[r] = cs * yi[q][t] - sn * yj[q][t];
                vj[r] = sn * yi[q][t] + cs * yj[q][t];
              }
            }
            if (lane == 0) atomicAdd(&rot_count, 1);
          }
        }
      }
      __syncthreads();
    }
    sweeps = sweep + 1;
    if (rot_count == 0) break;
    __syncthreads();
  }

  // singular values and descending order (ties: lower column first)
  double *sv = base + 2 * static_cast<int64_t>(pe) * pe;
  int *rank = reinterpret_cast<int *>(sv + pe);
  for (int c = wv; c < p; c += nwaves) {
    double s = 0;
    for (int r = lane; r < pe; r += WAVE) s += W[c * pe + r] * W[c * pe + r];
    s = wave_sum(s);
    if (lane == 0) sv[c] = sqrt(s);
  }
  __syncthreads();
  for (int c = tid; c < p; c += blockDim.x) {
    const double s = sv[c];
    int rk = 0;
    for (int d = 0; d < p; ++d) rk += (sv[d] > s) || (sv[d] == s && d < c);
    rank[c] = rk;
  }
  __syncthreads();
  const double beta = s_beta;
  for (int c = wv; c < p; c += nwaves) {
    const int rk = rank[c];
    if (rk >= k) continue;
    const double s = sv[c];
    const double inv = s > 0 ? 1.0 / s : 0.0;
    for (int r = lane; r < p; r += WAVE) {
      Uk[rk * p + r] = W[c * pe + r] * inv;
      Vext[rk * ld + r] = Vh[c * pe + r];
    }
    if (lane == 0) {
      Vext[rk * ld + p] = 0.0;
      sig[rk] = s;
    }
  }
  for (int r = tid; r <= p; r += blockDim.x) Vext[k * ld + r] = (r == p) ? 1.0 : 0.0;
  __syncthreads();
  __threadfence_block();
  if (tid == 0) {
    const double s1 = sig[0];
    const double floor_ = fmax(0x1.0p-52 * s1, 2.2250738585072014e-308);
    int all = 1, lead = 0, leading = 1;
    for (int r = 0; r < k; ++r) {
      const double u = Uk[r * p + (p - 1)];
      const double e = fabs(beta * u) / fmax(sig[r], floor_);
      res[r] = e;
      rho[r] = beta * u;
      const int ok = e < tol;
      all &= ok;
      if (leading && ok) ++lead;
      else leading = 0;
    }
    flags[0] = all;
    flags[1] = lead;
    flags[2] = sweeps;
    *sigma_est = fmax(*sigma_est, s1);
  }
  __syncthreads();
  // restarted T (Alg. 2 step 9): zeros, diag(sig), arrow column rho
  for (int idx = tid; idx < ld * ld; idx += blockDim.x) {
    const int r = idx / ld, c = idx % ld;
    double v = 0.0;
    if (r < k && c == r) v = sig[r];
    else if (r < k && c == k) v = rho[r];
    T[idx] = v;
  }
}

}  // namespace svds
