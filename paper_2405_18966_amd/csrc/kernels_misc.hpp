// Restart rotation (Alg. 2 steps 8 and 16: U(:,1:p) Uh(:,1:k),
// V(:,1:p) Vh(:,1:k)), start vector, sign normalization, norms and small
// helpers.
#pragma once
#include "common.hpp"

namespace svds {

// ---------------------------------------------------------------------------
// out(:, 0:kc) = B(:, 0:pc) * Y(0:pc, 0:kc), B L x pc (ld ldb), Y column-major
// FP64 (ld ldy), out L x kc (ld ldo).  Tall-skinny: each wave owns 64 rows,
// columns of the output in groups of ROT_CG accumulated in registers; the
// Y panel of a group is staged in LDS and read as broadcasts.
// ---------------------------------------------------------------------------
constexpr int ROT_THREADS = 256;
constexpr int ROT_CG = 16;
constexpr int ROT_QMAX = 512;  // rows of Y staged per pass

template <typename TB, typename TO>
static __global__ __launch_bounds__(ROT_THREADS) void rotate_kernel(int64_t L, int pc, int kc,
                                                            const TB *__restrict__ B, int64_t ldb,
                                                            const double *__restrict__ Y,
                                                            int64_t ldy, TO *__restrict__ out,
                                                            int64_t ldo) {
  __shared__ TB ys[ROT_QMAX * ROT_CG];
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const int64_t r = (static_cast<int64_t>(blockIdx.x) * (ROT_THREADS / WAVE) + wv) * WAVE + lane;
  const bool valid = r < L;
  for (int g0 = 0; g0 < kc; g0 += ROT_CG) {
    const int ng = min(ROT_CG, kc - g0);
    TB acc[ROT_CG];
#pragma unroll
    for (int c = 0; c < ROT_CG; ++c) acc[c] = 0;
    for (int q0 = 0; q0 < pc; q0 += ROT_QMAX) {
      const int nq = min(ROT_QMAX, pc - q0);
      __syncthreads();
      for (int idx = tid; idx < nq * ROT_CG; idx += ROT_THREADS) {
        const int q = idx / ROT_CG, c = idx % ROT_CG;
        ys[idx] = c < ng ? static_cast<TB>(Y[(g0 + c) * ldy + q0 + q]) : TB(0);
      }
      __syncthreads();
      if (valid) {
        for (int q = 0; q < nq; ++q) {
          const TB b = B[(q0 + q) * ldb + r];
#pragma unroll
          for (int c = 0; c < ROT_CG; ++c) acc[c] += b * ys[q * ROT_CG + c];
        }
      }
    }
    if (valid) {
#pragma unroll
      for (int c = 0; c < ROT_CG; ++c)
        if (c < ng) out[(g0 + c) * ldo + r] = static_cast<TO>(acc[c]);
    }
  }
}

// Philox normal vector (stream `stream` of `seed`), the library's v1 when the
// caller gives none (Alg. 1 step 1: randn(n, 1)).
template <typename T>
static __global__ void philox_fill_kernel(int64_t L, uint64_t seed, uint32_t stream, T *__restrict__ out) {
  const int64_t b = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (2 * b >= L) return;
  double z0, z1;
  philox_normal_pair(seed, stream, static_cast<uint64_t>(b), z0, z1);
  out[2 * b] = static_cast<T>(z0);
  if (2 * b + 1 < L) out[2 * b + 1] = static_cast<T>(z1);
}

// dst = src * (*xs)
template <typename T>
static __global__ void scale_copy_kernel(int64_t L, const T *__restrict__ src, const double *__restrict__ xs,
                                  T *__restrict__ dst) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < L) dst[i] = src[i] * static_cast<T>(*xs);
}

template <typename TI, typename TO>
static __global__ void cast_copy_kernel(int64_t L, const TI *__restrict__ src, TO *__restrict__ dst) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < L) dst[i] = static_cast<TO>(src[i]);
}

// Plain copy (bandwidth reference for traffic counters).
static __global__ void copy_f64_kernel(int64_t L, const double *__restrict__ src, double *__restrict__ dst) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < L) dst[i] = src[i];
}

// Sign convention: flip (u_j, v_j) so the entry of v_j of largest magnitude
// (lowest index on ties) is positive.  One block per column j.
static __global__ __launch_bounds__(256) void signfix_kernel(int64_t m, int64_t n, double *__restrict__ U,
                                                     int64_t ldu, double *__restrict__ V,
                                                     int64_t ldv) {
  __shared__ double smax[256 / WAVE];
  __shared__ int64_t sidx[256 / WAVE];
  __shared__ double sgn;
  const int j = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  double *v = V + j * ldv;
  double best = -1.0;
  int64_t bi = INT64_MAX;
  for (int64_t i = tid; i < n; i += 256) {
    const double a = fabs(v[i]);
    if (a > best) {  // strictly greater keeps the lowest index of this thread
      best = a;
      bi = i;
    }
  }
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    const double ob = __shfl_xor(best, o, WAVE);
    const int64_t oi = __shfl_xor(bi, o, WAVE);
    if (ob > best || (ob == best && oi < bi)) {
      best = ob;
      bi = oi;
    }
  }
  if (lane == 0) {
    smax[wv] = best;
    sidx[wv] = bi;
  }
  __syncthreads();
  if (tid == 0) {
    double b = smax[0];
    int64_t id = sidx[0];
    for (int w = 1; w < 256 / WAVE; ++w)
      if (smax[w] > b || (smax[w] == b && sidx[w] < id)) {
        b = smax[w];
        id = sidx[w];
      }
    sgn = (id < n && v[id] < 0) ? -1.0 : 1.0;
  }
  __syncthreads();
  if (sgn < 0) {
    for (int64_t i = tid; i < n; i += 256) v[i] = -v[i];
    double *u = U + j * ldu;
    for (int64_t i = tid; i < m; i += 256) u[i] = -u[i];
  }
}

// |x|_2 of a length-L vector (FP64 accumulation) for the explicit residuals:
// block partials, then one block adds them in block order.
template <typename T>
static __global__ __launch_bounds__(256) void norm_partials_kernel(int64_t L, const T *__restrict__ x,
                                                                  double *__restrict__ partials) {
  __shared__ double sh[256 / WAVE];
  double s = 0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < L;
       i += static_cast<int64_t>(gridDim.x) * 256)
    s += static_cast<double>(x[i]) * static_cast<double>(x[i]);
  s = block_sum(s, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

static __global__ __launch_bounds__(256) void norm_finish_kernel(const double *__restrict__ partials,
                                                                int n, double *__restrict__ out) {
  __shared__ double sh[256 / WAVE];
  double s = 0;
  for (int g = threadIdx.x; g < n; g += 256) s += partials[g];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) *out = sqrt(s);
}

}  // namespace svds
