// Small SVD of T(1:p,1:p), convergence test and restart set-up
// (Alg. 2 steps 4-9, eq. (4), eq. (6)), FP64.
//
// SVD method: one-sided Jacobi (Hestenes 1958).  W <- T, Vh <- I; column
// pairs (i, j) are rotated from the right until every pair is orthogonal to
// working precision: with a = |w_i|^2, b = |w_j|^2, c = w_i . w_j the pair is
// rotated when |c| > tolJ * sqrt(a b), by t = sign(z)/(|z| + sqrt(1+z^2)),
// z = (b - a)/(2c), cs = 1/sqrt(1+t^2), sn = cs t (Rutishauser).  A sweep
// visits every pair once; the iteration stops after a sweep without a
// rotation (then every pair passed the test on the final W).  Then
// sigma_i = |w_i|, Uh_i = w_i / sigma_i, sorted descending.
//
// T is upper triangular (bidiagonal after the first LBP; diagonal block,
// arrow column k+1, then bidiagonal after a restart, Alg. 2 step 9), so the
// general dense SVD is needed.
//
// Two schedules of the same iteration:
//  * p <= JAC_SMALL_P: one workgroup, W and Vh in LDS, pairs in round-robin
//    (tournament) order, p/2 disjoint pairs per step.
//  * larger p: block Jacobi over several workgroups.  The columns are cut
//    into nb (even) blocks of c columns; a sweep is nb-1 rounds of a
//    round-robin over blocks, each round one kernel in which workgroup g
//    stages its two blocks (W and Vh columns) in LDS and rotates, one pair
//    per group of 16 lanes per step: in round 0 every pair of its 2c columns (this covers
//    the pairs inside each block, as every block appears once per round), in
//    later rounds the c*c pairs across its two blocks.  W and Vh live in
//    global memory between rounds; each round adds its rotation count to a
//    per-sweep counter, and kernels of a sweep that follows a sweep without
//    rotations return at once.
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
constexpr int JAC_MAX_SWEEPS = 30;
constexpr int JAC_SMALL_P = 62;          // single-workgroup schedule up to here
constexpr int BJ_LDS = 160 * 1024 - 1024; // dynamic LDS of a block-Jacobi round
constexpr int BJ_LU = 8;                  // loads in flight per thread when staging

// block shape of the multi-workgroup schedule: c columns per block (16, 8 or
// 4, the largest whose two blocks of W and Vh fit in LDS), nb blocks (even)
__host__ __device__ inline void bjac_shape(int p, int &c, int &nb) {
  c = (2 * 16 * p * 16 <= BJ_LDS) ? 16 : ((2 * 8 * p * 16 <= BJ_LDS) ? 8 : 4);
  nb = static_cast<int>(ceil_div(p, c));
  nb += nb & 1;
}

// bytes of the Jacobi work area in global memory (block schedule): W and Vh
// (p rows x nb*c columns each) and the per-sweep rotation counters
__host__ __device__ inline int64_t jacobi_work_bytes(int p) {
  int c, nb;
  bjac_shape(p, c, nb);
  return 2 * static_cast<int64_t>(p) * nb * c * 8 + JAC_MAX_SWEEPS * 8;
}

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

// One Jacobi pair (columns of `rows` entries, rows spread over the lanes,
// RPL per lane).  Every lane of the wave takes part; returns 1 if rotated
// (wave-uniform).
template <int RPL>
__device__ __forceinline__ int jacobi_pair(double *__restrict__ wi, double *__restrict__ wj,
                                           double *__restrict__ vi, double *__restrict__ vj, int rows,
                                           int lane, double tolJ) {
  double xi[RPL], xj[RPL], yi[RPL], yj[RPL];
  double a = 0, b = 0, c = 0;
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int r = lane + t * WAVE;
    const bool ok = r < rows;
    xi[t] = ok ? wi[r] : 0.0;
    xj[t] = ok ? wj[r] : 0.0;
    yi[t] = ok ? vi[r] : 0.0;
    yj[t] = ok ? vj[r] : 0.0;
    a += xi[t] * xi[t];
    b += xj[t] * xj[t];
    c += xi[t] * xj[t];
  }
  a = wave_sum_u(a);
  b = wave_sum_u(b);
  c = wave_sum_u(c);
  if (!(fabs(c) > tolJ * sqrt(a * b))) return 0;
  const double z = (b - a) / (2.0 * c);
  const double tt = (z >= 0 ? 1.0 : -1.0) / (fabs(z) + sqrt(1.0 + z * z));
  const double cs = 1.0 / sqrt(1.0 + tt * tt);
  const double sn = cs * tt;
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int r = lane + t * WAVE;
    if (r < rows) {
      wi[r] = cs * xi[t] - sn * xj[t];
      wj[r] = sn * xi[t] + cs * xj[t];
      vi[r] = cs * yi[t] - sn * yj[t];
      vj[r] = sn * yi[t] + cs * yj[t];
    }
  }
  return 1;
}

// 1/x and 1/sqrt(x) from the hardware approximations plus two Newton steps
// (quadratic convergence from the approximations' ~2^-23 to working precision).
__device__ __forceinline__ double jac_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}
__device__ __forceinline__ double jac_rsqrt(double q) {
  double y = __builtin_amdgcn_rsq(q);
  y = fma(0.5 * y, fma(-q * y, y, 1.0), y);
  y = fma(0.5 * y, fma(-q * y, y, 1.0), y);
  return y;
}

// Sum over the LPP lanes of a pair group: a DPP row of 16 lanes, or the whole
// wave (scalar result); either way every lane of the group gets the same bits.
template <int LPP> __device__ __forceinline__ double group_sum(double v) {
  static_assert(LPP == 16 || LPP == WAVE, "pair groups of 16 lanes or a whole wave");
  if constexpr (LPP == 16) return row16_sum(v);
  else return wave_sum_u(v);
}

// Same rotation for one pair per group of LPP lanes (16: four pairs per wave,
// whose sums and rotation parameters are computed by the same instructions;
// 64: one pair per wave), RPL rows per lane.  Every lane of the wave takes
// part (a group with no pair passes null columns); returns 1 if this lane's
// pair rotated.
template <int RPL, int LPP>
__device__ __forceinline__ int jacobi_pairg(double *__restrict__ wi, double *__restrict__ wj,
                                            double *__restrict__ vi, double *__restrict__ vj, int rows,
                                            int sl, double tolJ) {
  double xi[RPL], xj[RPL], yi[RPL], yj[RPL];
  double a = 0, b = 0, c = 0;
  const bool has = wi != nullptr;
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int r = sl + t * LPP;
    const bool ok = has && r < rows;
    xi[t] = ok ? wi[r] : 0.0;
    xj[t] = ok ? wj[r] : 0.0;
    yi[t] = ok ? vi[r] : 0.0;
    yj[t] = ok ? vj[r] : 0.0;
    a += xi[t] * xi[t];
    b += xj[t] * xj[t];
    c += xi[t] * xj[t];
  }
  a = group_sum<LPP>(a);
  b = group_sum<LPP>(b);
  c = group_sum<LPP>(c);
  // |c| below 2^-1000 counts as orthogonal: the hardware reciprocal flushes
  // a subnormal 2c to infinity (then the rotation would be NaN), and such a
  // pair (a column that has converged to nothing) needs no rotation
  if (!has || !(fabs(c) > tolJ * sqrt(a * b)) || !(fabs(c) >= 0x1.0p-1000)) return 0;
  // Rutishauser's parameters with hardware reciprocal / reciprocal square
  // root, each refined by two Newton steps (full double accuracy; the
  // rotation only needs cs^2 + sn^2 = 1 to working precision)
  const double z = (b - a) * jac_rcp(2.0 * c);
  double tt;
  if (fabs(z) < 1e100) {
    const double q = fma(z, z, 1.0);
    tt = (z >= 0 ? 1.0 : -1.0) * jac_rcp(fabs(z) + q * jac_rsqrt(q));
  } else {
    tt = 0.5 / z;  // sqrt(1 + z^2) = |z| to working precision
  }
  const double cs = jac_rsqrt(fma(tt, tt, 1.0));
  const double sn = cs * tt;
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int r = sl + t * LPP;
    if (r < rows) {
      wi[r] = cs * xi[t] - sn * xj[t];
      wj[r] = sn * xi[t] + cs * xj[t];
      vi[r] = cs * yi[t] - sn * yj[t];
      vj[r] = sn * yi[t] + cs * yj[t];
    }
  }
  return 1;
}

// As jacobi_pairg with column i held in registers (xi, yi: this lane's RPL
// rows of W and Vh): in the cross rounds of the block schedule a group keeps
// its column for the whole round, so only column j travels through LDS.
template <int RPL, int LPP>
__device__ __forceinline__ int jacobi_pairg_reg(double (&xi)[RPL], double (&yi)[RPL], double *__restrict__ wj,
                                                double *__restrict__ vj, int rows, int sl, double tolJ,
                                                bool has) {
  double xj[RPL], yj[RPL];
  double a = 0, b = 0, c = 0;
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int r = sl + t * LPP;
    const bool ok = has && r < rows;
    xj[t] = ok ? wj[r] : 0.0;
    yj[t] = ok ? vj[r] : 0.0;
    a += xi[t] * xi[t];
    b += xj[t] * xj[t];
    c += xi[t] * xj[t];
  }
  a = group_sum<LPP>(a);
  b = group_sum<LPP>(b);
  c = group_sum<LPP>(c);
  if (!has || !(fabs(c) > tolJ * sqrt(a * b)) || !(fabs(c) >= 0x1.0p-1000)) return 0;  // as jacobi_pairg
  const double z = (b - a) * jac_rcp(2.0 * c);
  double tt;
  if (fabs(z) < 1e100) {
    const double q = fma(z, z, 1.0);
    tt = (z >= 0 ? 1.0 : -1.0) * jac_rcp(fabs(z) + q * jac_rsqrt(q));
  } else {
    tt = 0.5 / z;
  }
  const double cs = jac_rsqrt(fma(tt, tt, 1.0));
  const double sn = cs * tt;
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int r = sl + t * LPP;
    const double wi = cs * xi[t] - sn * xj[t];
    const double vi = cs * yi[t] - sn * yj[t];
    if (r < rows) {
      wj[r] = sn * xi[t] + cs * xj[t];
      vj[r] = sn * yi[t] + cs * yj[t];
    }
    xi[t] = wi;
    yi[t] = vi;
  }
  return 1;
}

// Singular values from the converged W (column norms), descending order
// (ties: lower column first), outputs, eq. (4) estimates, restarted T.
// smallest != 0: the k smallest in ascending order are kept instead (Ritz
// augmentation with the smallest Ritz triplets); the sigma floor of eq. (4)
// still uses the largest.
// W, Vh: p rows, leading dimensions ldw, ldv.  sv/rank: block-shared
// scratch of p entries.  beta = T(p, p+1) read before T is rewritten.
// Entry (r, c) of T is T[(r (p+1) + c) ts] (ts = 1, or the number of
// problems of a batch whose projected matrices are interleaved).
__device__ inline void jacobi_finish(const double *W, int64_t ldw, const double *Vh, int64_t ldv, int p,
                                     int k, double tol, double beta, int sweeps, double *__restrict__ T,
                                     int64_t ts,
                                     double *__restrict__ Uk, double *__restrict__ Vext,
                                     double *__restrict__ sig, double *__restrict__ res,
                                     double *__restrict__ rho, int *__restrict__ flags,
                                     double *__restrict__ sigma_est, double *sv, int *rank, int smallest) {
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const int nwaves = blockDim.x / WAVE;
  const int ld = p + 1;
  for (int c = wv; c < p; c += nwaves) {
    double s = 0;
    for (int r = lane; r < p; r += WAVE) s += W[c * ldw + r] * W[c * ldw + r];
    s = wave_sum_u(s);
    if (lane == 0) sv[c] = sqrt(s);
  }
  __syncthreads();
  for (int c = tid; c < p; c += blockDim.x) {
    const double s = sv[c];
    int rk = 0;
    if (smallest)
      for (int d = 0; d < p; ++d) rk += (sv[d] < s) || (sv[d] == s && d < c);
    else
      for (int d = 0; d < p; ++d) rk += (sv[d] > s) || (sv[d] == s && d < c);
    rank[c] = rk;
  }
  __syncthreads();
  for (int c = wv; c < p; c += nwaves) {
    const int rk = rank[c];
    if (rk >= k) continue;
    const double s = sv[c];
    const double inv = s > 0 ? 1.0 / s : 0.0;
    for (int r = lane; r < p; r += WAVE) {
      Uk[rk * p + r] = W[c * ldw + r] * inv;
      Vext[rk * ld + r] = Vh[c * ldv + r];
    }
    if (lane == 0) {
      Vext[rk * ld + p] = 0.0;
      sig[rk] = s;
    }
  }
  for (int r = tid; r <= p; r += blockDim.x) Vext[k * ld + r] = (r == p) ? 1.0 : 0.0;
  __syncthreads();
  if (tid == 0) {
    double s1 = sig[0];
    if (smallest)
      for (int c = 0; c < p; ++c) s1 = fmax(s1, sv[c]);
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
    T[idx * ts] = v;
  }
}

// tolJ: orthogonality to working precision, scaled by sqrt(rows)
__device__ __forceinline__ double jacobi_tol(int rows) {
  return 0x1.0p-52 * sqrt(static_cast<double>(rows));
}

// ---------------------------------------------------------------------------
// Single-workgroup schedule (p <= JAC_SMALL_P, one row per lane).  Dynamic
// LDS: W and Vh (pe x pe each, pe = p rounded up to even), sv, rank.
// ---------------------------------------------------------------------------
// Sweeps over W and Vh (pe x pe each, in LDS) until one passes without a
// rotation or JAC_MAX_SWEEPS are done; returns the sweeps used.
template <int RPL>
__device__ inline int lds_jacobi_sweeps_r(double *__restrict__ W, double *__restrict__ Vh, int pe) {
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const double tolJ = jacobi_tol(pe);
  const int npairs = pe / 2, n1 = pe - 1;
  // four pairs per wave, one per row of 16 lanes; the launch has one lane
  // group per pair (small_svd_threads), so each group keeps its pair q for
  // every step and steps its ring positions (rr_pair's players) by one
  const int lg = lane >> 4, sl = lane & 15;
  const int q = wv * 4 + lg;
  const bool has = q < npairs;
  int sweeps = 0;
  for (int sweep = 0; sweep < JAC_MAX_SWEEPS; ++sweep) {
    int ia = q % n1, ib = (n1 - q) % n1;  // (step + q) mod n1 and (step + n1 - q) mod n1 at step 0
    int any = 0;
    for (int step = 0; step < n1; ++step) {
      double *wi = nullptr, *wj = nullptr, *vi = nullptr, *vj = nullptr;
      if (has) {
        const int i = q == 0 ? 0 : 1 + ia, j = 1 + ib;  // as rr_pair(pe, step, q, i, j)
        wi = W + i * pe;
        wj = W + j * pe;
        vi = Vh + i * pe;
        vj = Vh + j * pe;
      }
      any |= jacobi_pairg<RPL, 16>(wi, wj, vi, vj, pe, sl, tolJ);
      ia = ia + 1 == n1 ? 0 : ia + 1;
      ib = ib + 1 == n1 ? 0 : ib + 1;
      __syncthreads();
    }
    sweeps = sweep + 1;
    if (!__syncthreads_or(any)) break;
  }
  return sweeps;
}

// One-sided Jacobi sweeps of the pe x pe LDS matrices (pe even, <= 64) until
// a sweep rotates no pair; returns the number of sweeps.  Rows per lane of
// a 16-lane pair group: two up to 32 rows, four above.
__device__ inline int lds_jacobi_sweeps(double *__restrict__ W, double *__restrict__ Vh, int pe) {
  return pe <= 32 ? lds_jacobi_sweeps_r<2>(W, Vh, pe) : lds_jacobi_sweeps_r<4>(W, Vh, pe);
}

__device__ inline void small_svd_body(double *__restrict__ T, int64_t ts, int p, int k, double tol,
                                      double *__restrict__ Uk, double *__restrict__ Vext,
                                      double *__restrict__ sig, double *__restrict__ res,
                                      double *__restrict__ rho, int *__restrict__ flags,
                                      double *__restrict__ sigma_est, int smallest) {
  extern __shared__ double smem[];
  __shared__ double s_beta;
  const int tid = threadIdx.x;
  const int pe = p + (p & 1);
  const int ld = p + 1;
  double *W = smem;
  double *Vh = smem + pe * pe;
  double *sv = Vh + pe * pe;
  int *rank = reinterpret_cast<int *>(sv + pe);

  if (tid == 0) s_beta = T[((p - 1) * ld + p) * ts];
  for (int idx = tid; idx < pe * pe; idx += blockDim.x) {
    const int r = idx % pe, c = idx / pe;
    W[idx] = (r < p && c < p) ? T[(r * ld + c) * ts] : 0.0;
    Vh[idx] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int sweeps = lds_jacobi_sweeps(W, Vh, pe);
  jacobi_finish(W, pe, Vh, pe, p, k, tol, s_beta, sweeps, T, ts, Uk, Vext, sig, res, rho, flags, sigma_est, sv,
                rank, smallest);
}

static __global__ __launch_bounds__(JAC_THREADS) void small_svd_kernel(
    double *__restrict__ T, int p, int k, double tol, double *__restrict__ Uk, double *__restrict__ Vext,
    double *__restrict__ sig, double *__restrict__ res, double *__restrict__ rho, int *__restrict__ flags,
    double *__restrict__ sigma_est, int smallest) {
  small_svd_body(T, 1, p, k, tol, Uk, Vext, sig, res, rho, flags, sigma_est, smallest);
}

// One workgroup per problem of a batch (interleaved T, per-problem outputs
// at fixed strides: Uk p*k, Vext (p+1)(k+1), sig/res/rho k, flags 4);
// problems with active[b] = 0 are skipped.
static __global__ __launch_bounds__(JAC_THREADS) void bsmall_svd_kernel(
    double *__restrict__ T, int nb, int p, int k, double tol, double *__restrict__ Uk, double *__restrict__ Vext,
    double *__restrict__ sig, double *__restrict__ res, double *__restrict__ rho, int *__restrict__ flags,
    double *__restrict__ sigma_est, const int32_t *__restrict__ active) {
  const int64_t b = blockIdx.x;
  if (!active[b]) return;  // converged and frozen: outputs of its last small SVD stay
  small_svd_body(T + b, nb, p, k, tol, Uk + b * p * k, Vext + b * (p + 1) * (k + 1), sig + b * k, res + b * k,
                 rho + b * k, flags + 4 * b, sigma_est + b, 0);
}

// threads of the single-workgroup schedule: four pairs per wave
__host__ __device__ inline int small_svd_threads(int p) {
  const int pe = p + (p & 1);
  return static_cast<int>(ceil_div(pe / 2, 4)) * WAVE;
}

__host__ __device__ inline size_t small_svd_lds_bytes(int p) {
  const int pe = p + (p & 1);
  return static_cast<size_t>(2 * pe * pe + pe) * 8 + pe * 4;
}

// ---------------------------------------------------------------------------
// Block schedule: one round.  Grid nb/2 workgroups of c LPP / 64 waves (one
// pair per group of LPP lanes, RPL rows per lane); dynamic LDS
// 2c columns of W then 2c columns of Vh, p rows each.  Block b holds global
// columns [b c, b c + c); W and Vh in global memory are column-major with
// ld = p and nb*c columns.  In the first round of the first sweep the blocks
// are loaded from T (row-major, row stride ldt; rows from tr on read as
// zero) and the identity instead: ldt = p + 1, tr = p for the small SVD of
// T(1:p, 1:p), ldt = p, tr = p - 1 for the harmonic SVD of the whole stored
// matrix ([T, beta e] and a zero row).
// ---------------------------------------------------------------------------
template <int RPL, int LPP>
__global__ __launch_bounds__(LPP == WAVE ? (RPL <= 6 ? 1024 : 512) : 256) void bjac_round_kernel(const double *__restrict__ T, int ldt, int tr,
                                                                 int from_T, double *__restrict__ W,
                                                                 double *__restrict__ Vh, int p, int c,
                                                                 int nb, int round, int sweep,
                                                                 int *__restrict__ counters) {
  extern __shared__ double smem[];
  __shared__ int s_rot;
  if (sweep > 0 && counters[sweep - 1] == 0) return;  // converged earlier
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const int c2 = 2 * c;
  double *X = smem;
  double *Y = smem + static_cast<int64_t>(c2) * p;
  int ba, bb;
  rr_pair(nb, round, blockIdx.x, ba, bb);
  if (tid == 0) s_rot = 0;
  // staging: a thread issues BJ_LU loads of each matrix before it writes
  // any of them to LDS, so the global-memory latency is paid once per batch
  const int ntot = c2 * p;
  for (int base = tid; base < ntot; base += BJ_LU * blockDim.x) {
    double vx[BJ_LU], vy[BJ_LU];
#pragma unroll
    for (int u = 0; u < BJ_LU; ++u) {
      const int idx = base + u * blockDim.x;
      vx[u] = vy[u] = 0.0;
      if (idx < ntot) {
        const int lc = idx / p, r = idx - lc * p;
        const int gc = lc < c ? ba * c + lc : bb * c + (lc - c);
        if (from_T) {
          vx[u] = (gc < p && r < tr) ? T[static_cast<int64_t>(r) * ldt + gc] : 0.0;
          vy[u] = (r == gc) ? 1.0 : 0.0;
        } else {
          vx[u] = W[static_cast<int64_t>(gc) * p + r];
          vy[u] = Vh[static_cast<int64_t>(gc) * p + r];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < BJ_LU; ++u) {
      const int idx = base + u * blockDim.x;
      if (idx < ntot) {
        X[idx] = vx[u];
        Y[idx] = vy[u];
      }
    }
  }
  __syncthreads();
  const double tolJ = jacobi_tol(p + (p & 1));
  // pair q of a step is handled by lane group q (WAVE / LPP groups per wave)
  const int q = wv * (WAVE / LPP) + lane / LPP, sl = lane % LPP;
  const bool own = q < c;
  int nrot = 0;
  if (round == 0) {
    for (int step = 0; step < c2 - 1; ++step) {
      int i = 0, j = 0;
      if (own) rr_pair(c2, step, q, i, j);
      nrot += jacobi_pairg<RPL, LPP>(own ? X + i * p : nullptr, X + j * p, Y + i * p, Y + j * p, p, sl, tolJ);
      __syncthreads();
    }
  } else {
    // column i = q stays with this group for the round: keep it in registers
    double xi[RPL], yi[RPL];
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int r = sl + t * LPP;
      const bool ok = own && r < p;
      xi[t] = ok ? X[q * p + r] : 0.0;
      yi[t] = ok ? Y[q * p + r] : 0.0;
    }
    for (int step = 0; step < c; ++step) {
      const int j = c + (q + step) % c;
      nrot += jacobi_pairg_reg<RPL, LPP>(xi, yi, X + (own ? j : 0) * p, Y + (own ? j : 0) * p, p, sl, tolJ, own);
      __syncthreads();
    }
    if (own) {
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int r = sl + t * LPP;
        if (r < p) {
          X[q * p + r] = xi[t];
          Y[q * p + r] = yi[t];
        }
      }
    }
    __syncthreads();
  }
  for (int idx = tid; idx < c2 * p; idx += blockDim.x) {
    const int lc = idx / p, r = idx - lc * p;
    const int gc = lc < c ? ba * c + lc : bb * c + (lc - c);
    W[static_cast<int64_t>(gc) * p + r] = X[idx];
    Vh[static_cast<int64_t>(gc) * p + r] = Y[idx];
  }
  if (sl == 0 && nrot) atomicAdd(&s_rot, nrot);
  __syncthreads();
  if (tid == 0 && s_rot) atomicAdd(&counters[sweep], s_rot);
}

// Block schedule: outputs after the last round (one workgroup).  `nsw` =
// sweeps enqueued; the sweeps used are up to the first without rotations.
static __global__ __launch_bounds__(JAC_THREADS) void bjac_finish_kernel(
    const double *__restrict__ W, const double *__restrict__ Vh, const int *__restrict__ counters, int nsw,
    double *__restrict__ T, int p, int k, double tol, double *__restrict__ Uk, double *__restrict__ Vext,
    double *__restrict__ sig, double *__restrict__ res, double *__restrict__ rho, int *__restrict__ flags,
    double *__restrict__ sigma_est, int smallest) {
  extern __shared__ double smem[];
  __shared__ double s_beta;
  __shared__ int s_sweeps;
  double *sv = smem;
  int *rank = reinterpret_cast<int *>(sv + p);
  if (threadIdx.x == 0) {
    s_beta = T[(p - 1) * (p + 1) + p];
    int s = nsw;
    for (int i = 0; i < nsw; ++i)
      if (counters[i] == 0) {
        s = i + 1;
        break;
      }
    s_sweeps = s;
  }
  __syncthreads();
  jacobi_finish(W, p, Vh, p, p, k, tol, s_beta, s_sweeps, T, 1, Uk, Vext, sig, res, rho, flags, sigma_est, sv,
                rank, smallest);
}


// ---------------------------------------------------------------------------
// Harmonic-Ritz restart (SVDS_FLAG_HARMONIC, smallest triplets).  With
// A V_p = U_p T and A^T U_p = V_p T^T + beta_p v_{p+1} e_p^T, the harmonic
// Ritz values of A^T A on span(V_p) are the squared singular values of
// B = [T, beta_p e_p] (p x (p+1)); the harmonic Ritz vectors and the common
// direction of their residuals span V_{p+1} span{y_1..y_k, y_0}, y_j the right
// singular vectors of the k smallest values and y_0 the null vector of B.
// One-sided Jacobi of the stored (p+1) x (p+1) matrix (B and a zero row)
// gives them all: B Vh = W, column norms s_c (one of them ~0: y_0).
// From W and Vh (q = p + 1 columns, rows 0..p; row p of W is zero):
//   M = [y_1..y_k, y_0] (Vh columns); H = I - tau v v^T the Householder
//   reflection with r H = -sign(r_{k+1}) |r| e_{k+1}^T for the last row r of
//   M; Q_C = M H with Q_C(p, 0:k) = 0 and a positive Q_C(p, k)
//   ((p+1) x (k+1), ld p+1: [V_p v_{p+1}] Q_C is the new V_{k+1});
//   Q_M = [x_1..x_k], x_j = W(:, y_j) / s_j the left singular vectors
//   (p x k, ld p: U_p Q_M is the new U_k);
//   R = Q_M^T B Q_C(:, 0:k) = Q_M^T (W_M H)(:, 0:k), W_M = B M the W columns
//   of M (k x k row-major: the new T(1:k, 1:k)).
// Both Lanczos relations then hold with the backward error of the SVD
// alone.  Scratch: sd 4 q doubles, si 2 q ints (block-shared).
// ---------------------------------------------------------------------------
__device__ inline void harm_finish(const double *W, int64_t ldw, const double *Vh, int64_t ldv, int p, int k,
                                   double *__restrict__ QC, double *__restrict__ QM, double *__restrict__ R,
                                   double *sd, int *si) {
  __shared__ double s_tau, s_sgn;
  __shared__ int s_null;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const int nwaves = blockDim.x / WAVE;
  const int q = p + 1;
  double *sv = sd, *y = sd + q, *z = sd + 2 * q, *v = sd + 3 * q;
  int *sel = si;
  for (int c = wv; c < q; c += nwaves) {
    double a = 0;
    for (int r = lane; r < q; r += WAVE) a += W[c * ldw + r] * W[c * ldw + r];
    a = wave_sum_u(a);
    if (lane == 0) sv[c] = sqrt(a);
  }
  __syncthreads();
  if (tid == 0) {  // y_0: the column of least norm (ties: the lower one)
    int nl = 0;
    for (int c = 1; c < q; ++c)
      if (sv[c] < sv[nl]) nl = c;
    s_null = nl;
    sel[k] = nl;
  }
  __syncthreads();
  const int nl = s_null;
  for (int c = tid; c < q; c += blockDim.x) {  // the k smallest of the others, ascending
    if (c == nl) continue;
    const double s = sv[c];
    int rk = 0;
    for (int d = 0; d < q; ++d) rk += (d != nl) && ((sv[d] < s) || (sv[d] == s && d < c));
    if (rk < k) sel[rk] = c;
  }
  __syncthreads();
  if (tid == 0) {  // Householder vector from the last row of M
    double n2 = 0;
    for (int j = 0; j <= k; ++j) {
      const double r = Vh[sel[j] * ldv + p];
      v[j] = r;
      n2 += r * r;
    }
    v[k] += copysign(sqrt(n2), v[k]);
    double vv = 0;
    for (int j = 0; j <= k; ++j) vv += v[j] * v[j];
    s_tau = vv > 0 ? 2.0 / vv : 0.0;
  }
  __syncthreads();
  const double tau = s_tau;
  for (int i = tid; i < q; i += blockDim.x) {  // y = M v
    double a = 0;
    for (int j = 0; j <= k; ++j) a += Vh[sel[j] * ldv + i] * v[j];
    y[i] = a;
  }
  for (int r = tid; r < p; r += blockDim.x) {  // z = W_M v
    double a = 0;
    for (int j = 0; j <= k; ++j) a += W[sel[j] * ldw + r] * v[j];
    z[r] = a;
  }
  __syncthreads();
  if (tid == 0) s_sgn = (Vh[nl * ldv + p] - tau * y[p] * v[k]) < 0 ? -1.0 : 1.0;
  __syncthreads();
  const double sg = s_sgn;
  for (int idx = tid; idx < q * (k + 1); idx += blockDim.x) {
    const int j = idx / q, i = idx - j * q;
    double x = (i == p && j < k) ? 0.0 : Vh[sel[j] * ldv + i] - tau * y[i] * v[j];
    if (j == k) x *= sg;
    QC[static_cast<int64_t>(j) * q + i] = x;
  }
  for (int idx = tid; idx < p * k; idx += blockDim.x) {
    const int j = idx / p, r = idx - j * p;
    const double s = sv[sel[j]];
    QM[static_cast<int64_t>(j) * p + r] = s > 0 ? W[sel[j] * ldw + r] / s : 0.0;
  }
  for (int idx = wv; idx < k * k; idx += nwaves) {  // R(i, j), one wave each
    const int i = idx / k, j = idx - i * k;
    const double *wi = W + sel[i] * ldw, *wj = W + sel[j] * ldw;
    const double tv = tau * v[j];
    double a = 0;
    for (int r = lane; r < p; r += WAVE) a += wi[r] * (wj[r] - tv * z[r]);
    a = wave_sum_u(a);
    if (lane == 0) {
      const double s = sv[sel[i]];
      R[idx] = s > 0 ? a / s : 0.0;
    }
  }
}

// LDS of the harmonic finish: 4 q doubles and 2 q ints
__host__ __device__ inline size_t harm_scratch_bytes(int q) { return static_cast<size_t>(q) * (4 * 8 + 2 * 4); }

// Single-workgroup schedule of the harmonic SVD (p + 1 <= JAC_SMALL_P):
// W <- the stored T (rows 0..p-1; row p zero), Vh <- I, pe = p + 1 rounded
// up to even (a padding column stays zero and is never rotated).
static __global__ __launch_bounds__(JAC_THREADS) void harm_small_kernel(const double *__restrict__ T, int p, int k,
                                                                        double *__restrict__ QC,
                                                                        double *__restrict__ QM,
                                                                        double *__restrict__ R) {
  extern __shared__ double smem[];
  const int q = p + 1, pe = q + (q & 1);
  double *W = smem;
  double *Vh = smem + pe * pe;
  double *sd = Vh + pe * pe;
  int *si = reinterpret_cast<int *>(sd + 4 * q);
  for (int idx = threadIdx.x; idx < pe * pe; idx += blockDim.x) {
    const int r = idx % pe, c = idx / pe;
    W[idx] = (r < p && c < q) ? T[r * q + c] : 0.0;
    Vh[idx] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  (void)lds_jacobi_sweeps(W, Vh, pe);
  harm_finish(W, pe, Vh, pe, p, k, QC, QM, R, sd, si);
}

__host__ __device__ inline size_t harm_small_lds_bytes(int p) {
  const int q = p + 1, pe = q + (q & 1);
  return static_cast<size_t>(2 * pe * pe) * 8 + harm_scratch_bytes(q);
}

// Block schedule of the harmonic SVD: outputs after the last round (one
// workgroup); W and Vh column-major with ld q = p + 1.
static __global__ __launch_bounds__(JAC_THREADS) void harm_bjac_finish_kernel(const double *__restrict__ W,
                                                                              const double *__restrict__ Vh, int p,
                                                                              int k, double *__restrict__ QC,
                                                                              double *__restrict__ QM,
                                                                              double *__restrict__ R) {
  extern __shared__ double smem[];
  const int q = p + 1;
  harm_finish(W, q, Vh, q, p, k, QC, QM, R, smem, reinterpret_cast<int *>(smem + 4 * q));
}

// The restarted T of a harmonic restart: zeros, R in the leading k x k block
// (the arrow column T(0:k, k) is filled after the restart vector's CGS2).
static __global__ void harm_tset_kernel(double *__restrict__ T, int p, int k, const double *__restrict__ R) {
  const int ld = p + 1;
  for (int idx = threadIdx.x; idx < ld * ld; idx += blockDim.x) {
    const int r = idx / ld, c = idx - r * ld;
    T[idx] = (r < k && c < k) ? R[r * k + c] : 0.0;
  }
}

// T(0:k, k) = the two CGS projections of A v_{k+1} on U_k (u_{k+1} =
// (A v_{k+1} - U_k T(0:k, k)) / T(k, k)).
template <typename TB>
__global__ void harm_couple_kernel(double *__restrict__ T, int p, int k, const TB *__restrict__ h1,
                                   const TB *__restrict__ h2) {
  for (int r = threadIdx.x; r < k; r += blockDim.x)
    T[r * (p + 1) + k] = static_cast<double>(h1[r]) + static_cast<double>(h2[r]);
}

}  // namespace svds
