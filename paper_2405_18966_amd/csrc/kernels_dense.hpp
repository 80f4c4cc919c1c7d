// Dense mat-vecs for the dense form of the solver (the paper's
// svds_C_dense, Sec. 2.3): y = xs * A x - coef * yprev and
// y = xs * A^T x - coef * yprev, A column-major (ld >= m) stored as FP64, FP32
// or BF16 and widened exactly in registers; accumulation in the basis type.
//
// A x  : 2-D grid of (row tile of 512 rows) x (column slab of 256 columns);
//        each lane owns 8 rows and walks a quarter of the slab's columns,
//        waves combine in LDS, the slab partial goes to global memory, and
//        gemv_n_fixup_kernel (next launch) adds the slab partials in slab
//        order.  Deterministic.
// A^T x: one wave per column (the column is contiguous), lanes stride the
//        rows with vector loads, fixed-order wave reduction.
#pragma once
#include "common.hpp"

namespace svds {

constexpr int DN_ROWS = 512;     // rows per tile (2 per thread)
constexpr int DN_SLAB = 256;     // columns per slab
constexpr int DN_THREADS = 256;

template <typename TV, typename TB>
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
  // a lane owns rows rbase + t*128 + 2*lane + {0,1}, t = 0..3
  const int64_t rbase = static_cast<int64_t>(blockIdx.x) * DN_ROWS;
  const int64_t c0 = static_cast<int64_t>(blockIdx.y) * DN_SLAB;
  const int64_t c1 = min(n, c0 + DN_SLAB);
  // each wave covers all 512 rows (8 rows per lane: 4 strips of 128) for a
  // quarter of the slab's columns
  TB acc[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) acc[t] = 0;
  for (int64_t c = c0 + wv; c < c1; c += DN_THREADS / WAVE) {
    const TB xc = x[c];
    const TV *col = A + c * lda;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t r = rbase + t * 128 + 2 * lane;
      if (r + 1 < m) {
        acc[2 * t] += widen<TB>(col[r]) * xc;
        acc[2 * t + 1] += widen<TB>(col[r + 1]) * xc;
      } else if (r < m) {
        acc[2 * t] += widen<TB>(col[r]) * xc;
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    red[wv][t * 128 + 2 * lane] = acc[2 * t];
    red[wv][t * 128 + 2 * lane + 1] = acc[2 * t + 1];
  }
  __syncthreads();
  for (int i = tid; i < DN_ROWS; i += DN_THREADS) {
    TB s = 0;
    for (int w = 0; w < DN_THREADS / WAVE; ++w) s += red[w][i];
    const int64_t r = rbase + i;
    if (r < m) partials[static_cast<int64_t>(blockIdx.y) * m + r] = s;
  }
}

// y[r] = xs * sum_slab partials[slab][r] - coef * yprev[r]
template <typename TB>
__global__ void gemv_n_fixup_kernel(int64_t m, int nslab, const TB *__restrict__ partials,
                                    const double *__restrict__ xs_ptr, const double *__restrict__ coef_ptr,
                                    const TB *__restrict__ yprev, TB *__restrict__ y) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= m) return;
  const TB xs = xs_ptr ? static_cast<TB>(*xs_ptr) : TB(1);
  const TB coef = coef_ptr ? static_cast<TB>(*coef_ptr) : TB(0);
  TB s = 0;
  for (int sl = 0; sl < nslab; ++sl) s += partials[static_cast<int64_t>(sl) * m + r];
  y[r] = xs * s - (yprev ? coef * yprev[r] : TB(0));
}

template <typename TV, typename TB>
__global__ __launch_bounds__(DN_THREADS) void gemv_t_kernel(
    int64_t m, int64_t n, const TV *__restrict__ A, int64_t lda, const TB *__restrict__ x,
    const double *__restrict__ xs_ptr, const double *__restrict__ coef_ptr,
    const TB *__restrict__ yprev, TB *__restrict__ y, TB *__restrict__ side_dst, int64_t side_len) {
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const TB xs = xs_ptr ? static_cast<TB>(*xs_ptr) : TB(1);
  const TB coef = coef_ptr ? static_cast<TB>(*coef_ptr) : TB(0);
  if (side_dst) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * DN_THREADS + tid; i < side_len;
         i += static_cast<int64_t>(gridDim.x) * DN_THREADS)
      side_dst[i] = x[i] * xs;
  }
  const int64_t c = static_cast<int64_t>(blockIdx.x) * (DN_THREADS / WAVE) + wv;
  if (c >= n) return;
  const TV *col = A + c * lda;
  TB s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  int64_t r = 4 * lane;
  for (; r + 3 < m; r += 4 * WAVE) {
    s0 += widen<TB>(col[r]) * x[r];
    s1 += widen<TB>(col[r + 1]) * x[r + 1];
    s2 += widen<TB>(col[r + 2]) * x[r + 2];
    s3 += widen<TB>(col[r + 3]) * x[r + 3];
  }
  for (; r < m; ++r) s0 += widen<TB>(col[r]) * x[r];
  TB s = wave_sum((s0 + s1) + (s2 + s3));
  if (lane == 0) y[c] = xs * s - (yprev ? coef * yprev[c] : TB(0));
}

// scratch of the A x kernel: partials (slabs x m of TB <= 8 bytes)
inline int64_t dense_partial_doubles(int64_t m, int64_t n) { return ceil_div(n, DN_SLAB) * m; }

}  // namespace svds
