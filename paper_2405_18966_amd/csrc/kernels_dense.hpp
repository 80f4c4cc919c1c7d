// Dense mat-vecs for the dense form of the solver (the paper's
// svds_C_dense, Sec. 2.3): y = xs * A x - coef * yprev and
// y = xs * A^T x - coef * yprev, A column-major (ld >= m) stored as FP64, FP32
// or BF16 and widened exactly in registers; accumulation in the basis type.
//
// Both products stream A once; every lane owns 8 consecutive rows of a
// column, read as 16-byte accesses (one for BF16, two for FP32, four for
// FP64) when the operands are aligned (VEC), element by element otherwise.
//
// A x  : 2-D grid of (row tile of 512 rows) x (column slab of DN_SLAB
//        columns); each wave covers the tile's 512 rows for a quarter of the
//        slab's columns (x[c] is a uniform scalar load), waves combine in
//        LDS, the slab partial goes to global memory, and gemv_n_fixup_kernel
//        (next launch) adds the slab partials in slab order.  Deterministic.
// A^T x: one block per group of DN_TCOLS columns; its waves take alternate
//        512-row chunks, a lane loads its 8 entries of x once per chunk and
//        uses them for all the group's columns; fixed-order wave and block
//        reductions.
#pragma once
#include "common.hpp"

namespace svds {

constexpr int DN_ROWS = 512;     // rows per tile (8 per lane)
constexpr int DN_SLAB = 256;     // columns per slab (A x)
constexpr int DN_THREADS = 256;
constexpr int DN_TCOLS = 8;      // columns per block (A^T x)

// 8 consecutive entries of a column starting at row r (r + 8 <= m when VEC)
template <typename TV, typename TB, bool VEC>
__device__ __forceinline__ void load8(const TV *__restrict__ p, int64_t rem, TB (&v)[8]) {
  if (VEC && rem >= 8) {
    TV t[8];
    constexpr int CH = static_cast<int>(8 * sizeof(TV) / 16);  // 16-byte chunks
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const uint4 u = reinterpret_cast<const uint4 *>(p)[q];
      __builtin_memcpy(&t[q * (16 / sizeof(TV))], &u, 16);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = widen<TB>(t[i]);
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = i < rem ? widen<TB>(p[i]) : TB(0);
  }
}

template <typename TV, typename TB, bool VEC>
__global__ __launch_bounds__(DN_THREADS) void gemv_n_kernel(
    int64_t m, int64_t n, const TV *__restrict__ A, int64_t lda, const TB *__restrict__ x,
    const double *__restrict__ xs_ptr,
    TB *__restrict__ partials, TB *__restrict__ side_dst, int64_t side_len) {
  __shared__ TB red[DN_THREADS / WAVE][DN_ROWS];
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const TB xs = xs_ptr ? static_cast<TB>(*xs_ptr) : TB(1);
  const int64_t bid = static_cast<int64_t>(blockIdx.y) * gridDim.x + blockIdx.x;
  if (side_dst) {
    const int64_t nb = static_cast<int64_t>(gridDim.x) * gridDim.y;
    for (int64_t i = bid * DN_THREADS + tid; i < side_len; i += nb * DN_THREADS) side_dst[i] = x[i] * xs;
  }
  const int64_t r = static_cast<int64_t>(blockIdx.x) * DN_ROWS + lane * 8;
  const int64_t c0 = static_cast<int64_t>(blockIdx.y) * DN_SLAB;
  const int64_t c1 = min(n, c0 + DN_SLAB);
  TB acc[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) acc[t] = 0;
  if (r < m) {
    for (int64_t c = c0 + wv; c < c1; c += DN_THREADS / WAVE) {
      const TB xc = x[c];
      TB a[8];
      load8<TV, TB, VEC>(A + c * lda + r, m - r, a);
#pragma unroll
      for (int t = 0; t < 8; ++t) acc[t] += a[t] * xc;
    }
  }
#pragma unroll
  for (int t = 0; t < 8; ++t) red[wv][lane * 8 + t] = acc[t];
  __syncthreads();
  for (int i = tid; i < DN_ROWS; i += DN_THREADS) {
    TB s = 0;
#pragma unroll
    for (int w = 0; w < DN_THREADS / WAVE; ++w) s += red[w][i];
    const int64_t row = static_cast<int64_t>(blockIdx.x) * DN_ROWS + i;
    if (row < m) partials[static_cast<int64_t>(blockIdx.y) * m + row] = s;
  }
}

// y[r] = xs * sum_slab partials[slab][r] - coef * yprev[r]; the slab loop
// keeps 8 loads in flight and adds in slab order.
template <typename TB>
__global__ void gemv_n_fixup_kernel(int64_t m, int nslab, const TB *__restrict__ partials,
                                    const double *__restrict__ xs_ptr, const double *__restrict__ coef_ptr,
                                    const TB *__restrict__ yprev, TB *__restrict__ y) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= m) return;
  const TB xs = xs_ptr ? static_cast<TB>(*xs_ptr) : TB(1);
  const TB coef = coef_ptr ? static_cast<TB>(*coef_ptr) : TB(0);
  TB s = 0;
  int sl = 0;
  for (; sl + 8 <= nslab; sl += 8) {
    TB v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = partials[static_cast<int64_t>(sl + i) * m + r];
#pragma unroll
    for (int i = 0; i < 8; ++i) s += v[i];
  }
  for (; sl < nslab; ++sl) s += partials[static_cast<int64_t>(sl) * m + r];
  y[r] = xs * s - (yprev ? coef * yprev[r] : TB(0));
}

template <typename TV, typename TB, bool VEC>
__global__ __launch_bounds__(DN_THREADS) void gemv_t_kernel(
    int64_t m, int64_t n, const TV *__restrict__ A, int64_t lda, const TB *__restrict__ x,
    const double *__restrict__ xs_ptr, const double *__restrict__ coef_ptr,
    const TB *__restrict__ yprev, TB *__restrict__ y, TB *__restrict__ side_dst, int64_t side_len) {
  constexpr int NW = DN_THREADS / WAVE;
  __shared__ TB red[NW][DN_TCOLS];
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const TB xs = xs_ptr ? static_cast<TB>(*xs_ptr) : TB(1);
  const TB coef = coef_ptr ? static_cast<TB>(*coef_ptr) : TB(0);
  if (side_dst) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * DN_THREADS + tid; i < side_len;
         i += static_cast<int64_t>(gridDim.x) * DN_THREADS)
      side_dst[i] = x[i] * xs;
  }
  // block: DN_TCOLS columns; wave w takes the 512-row chunks w, w + NW, ...
  const int64_t c0 = static_cast<int64_t>(blockIdx.x) * DN_TCOLS;
  const int nc = static_cast<int>(min<int64_t>(DN_TCOLS, n - c0));
  TB acc[DN_TCOLS];
#pragma unroll
  for (int c = 0; c < DN_TCOLS; ++c) acc[c] = 0;
  for (int64_t r = static_cast<int64_t>(wv) * DN_ROWS + lane * 8; r < m; r += NW * DN_ROWS) {
    TB xv[8];
    if (VEC && m - r >= 8) {
#pragma unroll
      for (int q = 0; q < static_cast<int>(8 * sizeof(TB) / 16); ++q) {
        const uint4 u = reinterpret_cast<const uint4 *>(x + r)[q];
        __builtin_memcpy(&xv[q * (16 / sizeof(TB))], &u, 16);
      }
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) xv[i] = r + i < m ? x[r + i] : TB(0);
    }
#pragma unroll
    for (int c = 0; c < DN_TCOLS; ++c) {
      if (c < nc) {
        TB a[8];
        load8<TV, TB, VEC>(A + (c0 + c) * lda + r, m - r, a);
        TB s = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) s += a[i] * xv[i];
        acc[c] += s;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < DN_TCOLS; ++c) {
    const TB s = wave_sum(acc[c]);
    if (lane == 0) red[wv][c] = s;
  }
  __syncthreads();
  if (tid < nc) {
    TB s = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += red[w][tid];
    const int64_t c = c0 + tid;
    y[c] = xs * s - (yprev ? coef * yprev[c] : TB(0));
  }
}

// Exact FP64 copy of a stored dense matrix (column-major, ld m).
template <typename TV>
__global__ void widen_dense_kernel(int64_t m, int64_t n, const TV *__restrict__ A, int64_t lda,
                                   double *__restrict__ out) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < m * n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t c = i / m, r = i - c * m;
    out[i] = widen<double>(A[c * lda + r]);
  }
}

// R(:, j) = S[j] X(:, j), j < k (X, R column-major, ld L).
static __global__ void scale_cols_kernel(int64_t L, int k, const double *__restrict__ X, const double *__restrict__ S,
                                         double *__restrict__ R) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < L * k;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    R[i] = S[i / L] * X[i];
}

// out[j] = |R(:, j)|_2, one block per column, fixed-order block sum.
static __global__ __launch_bounds__(256) void col_norms_kernel(int64_t L, const double *__restrict__ R,
                                                               double *__restrict__ out) {
  __shared__ double sh[256 / WAVE];
  const double *c = R + static_cast<int64_t>(blockIdx.x) * L;
  double s = 0;
  for (int64_t i = threadIdx.x; i < L; i += 256) s += c[i] * c[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = sqrt(s);
}

// out[j] = |C(j, :) - S[j] V(:, j)^T|_2 for C = U^T A (k x n, ld k) and V
// (n x k, ld n): the norms of A^T u_j - s_j v_j.  One block per j, fixed-order
// block sum.
static __global__ __launch_bounds__(256) void row_resid_norms_kernel(int64_t n, int k, const double *__restrict__ C,
                                                                     const double *__restrict__ V,
                                                                     const double *__restrict__ S,
                                                                     double *__restrict__ out) {
  __shared__ double sh[256 / WAVE];
  const int j = blockIdx.x;
  const double sj = S[j];
  const double *v = V + static_cast<int64_t>(j) * n;
  double s = 0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double d = C[i * k + j] - sj * v[i];
    s += d * d;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[j] = sqrt(s);
}

// scratch of the A x kernel: partials (slabs x m of TB <= 8 bytes)
inline int64_t dense_partial_doubles(int64_t m, int64_t n) { return ceil_div(n, DN_SLAB) * m; }

// 16-byte accesses are legal: A, x, and every column start 16-byte aligned
template <typename TV, typename TB>
inline bool dense_vec_ok(const void *A, int64_t lda, const void *x) {
  auto al = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  return al(A) && al(x) && (lda * static_cast<int64_t>(sizeof(TV))) % 16 == 0;
}

}  // namespace svds
