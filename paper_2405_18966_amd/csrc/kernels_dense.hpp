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
#include <algorithm>

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

// ---------------------------------------------------------------------------
// Block residuals of the dense form (Proposition 1 eq. (2), evaluated
// explicitly for the output triplets, Alg. 2 steps 15-16):
//   R1 = A V - U diag(S)  (m x k),   R2 = A^T U - V diag(S)  (n x k),
// res[j] = |R(:, j)|_2.  One pass over the stored A per side, widened exactly
// to FP64 in registers, with FP64 matrix-core products
// (v_mfma_f64_16x16x4f64: D(16x16) += A(16x4) B(4x16)).
//
// resid_gemm_kernel computes C = op(A) X for one group of at most RD_BN
// columns of X, op(A) = A (M = m, K = n) or A^T (M = n, K = m):
//   - grid (row blocks of RD_BM rows) x (K split in slices) ; 8 waves, each
//     owning 16 rows and NT 16-column tiles of the block's C tile;
//   - per RD_BK-deep chunk of K the block stages op(A)'s RD_BM x RD_BK tile
//     (FP64, widened on the way) and X's RD_BK x 16 NT chunk in LDS; the
//     next chunk's global loads (8 consecutive entries per thread along the
//     contiguous direction of A, 16-byte accesses when aligned) are issued
//     before the current chunk's matrix operations;
//   - operand layout (gfx950): lane l holds A(l % 16, l / 16) and
//     B(l / 16, l % 16); accumulator entry i of lane l is D(4 i + l / 16,
//     l % 16);
//   - each block writes its C tile of its K slice to `part` in fragment order
//     ([wave][tile][entry][lane], 64 consecutive doubles per store).
// resid_finish_kernel adds the slices in slice order, subtracts
// S[c] Sub(r, c) and forms per-row-block column sums of squares;
// resid_colnorm_kernel adds those in row-block order.  Deterministic: fixed
// split, fixed summation order, no atomics.
// ---------------------------------------------------------------------------
constexpr int RD_WAVES = 8;
constexpr int RD_THREADS = RD_WAVES * WAVE;  // 512
constexpr int RD_BM = 16 * RD_WAVES;         // 128 rows of C per block
constexpr int RD_BK = 32;                    // depth of a staged chunk of K
constexpr int RD_BN = 128;                   // columns per group (NT <= 8)
constexpr int RD_TILE = RD_BM * RD_BN;       // doubles of one block's partial tile
constexpr int RD_MAX_SPLIT = 16;
typedef double rd_v4d __attribute__((ext_vector_type(4)));

template <typename TV, bool TRANS, bool VEC, int NT>
__global__ __launch_bounds__(RD_THREADS) void resid_gemm_kernel(
    int64_t M, int64_t K, const TV *__restrict__ A, int64_t lda, const double *__restrict__ X, int64_t ldx,
    int kc, int64_t kslice, double *__restrict__ part) {
  __shared__ double As[RD_BK][RD_BM + 2];
  __shared__ double Xs[RD_BK][16 * NT + 2];
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * RD_BM;
  const int64_t q0 = static_cast<int64_t>(blockIdx.y) * kslice;
  const int64_t q1 = min(K, q0 + kslice);
  // op(A) chunk: 8 consecutive entries per thread along A's columns
  //   A   : entry (r, kk) = A[r0 + r + (q + kk) lda]; thread -> kk = tid / 16, r = 8 (tid % 16) + e
  //   A^T : entry (r, kk) = A[q + kk + (r0 + r) lda]; thread -> r = tid / 4, kk = 8 (tid % 4) + e
  const int a_kk = TRANS ? 8 * (tid & 3) : tid >> 4;
  const int a_r = TRANS ? tid >> 2 : 8 * (tid & 15);
  // X chunk: entry (kk, c) = X[q + kk + c ldx]; thread -> c = tid / 4, kk = 8 (tid % 4) + e
  const int x_c = tid >> 2, x_kk = 8 * (tid & 3);
  const bool x_live = x_c < 16 * NT;
  double ra[8], rx[8];
  auto load = [&](int64_t q) {
    if (TRANS) {
      const int64_t col = r0 + a_r, row = q + a_kk;
      if (col < M) load8<TV, double, VEC>(A + col * lda + row, q1 - row, ra);
      else
#pragma unroll
        for (int e = 0; e < 8; ++e) ra[e] = 0.0;
    } else {
      const int64_t row = r0 + a_r, col = q + a_kk;
      if (col < q1) load8<TV, double, VEC>(A + col * lda + row, M - row, ra);
      else
#pragma unroll
        for (int e = 0; e < 8; ++e) ra[e] = 0.0;
    }
    if (x_live) {
      const int64_t row = q + x_kk;
      if (x_c < kc) load8<double, double, VEC>(X + static_cast<int64_t>(x_c) * ldx + row, q1 - row, rx);
      else
#pragma unroll
        for (int e = 0; e < 8; ++e) rx[e] = 0.0;
    }
  };
  rd_v4d acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = rd_v4d{0.0, 0.0, 0.0, 0.0};
  if (q0 < q1) load(q0);
  const int li = lane & 15, lk = lane >> 4;
  for (int64_t q = q0; q < q1; q += RD_BK) {
    __syncthreads();  // the previous chunk's operand reads are done
    if (TRANS) {
#pragma unroll
      for (int e = 0; e < 8; ++e) As[a_kk + e][a_r] = ra[e];
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) As[a_kk][a_r + e] = ra[e];
    }
    if (x_live)
#pragma unroll
      for (int e = 0; e < 8; ++e) Xs[x_kk + e][x_c] = rx[e];
    __syncthreads();
    if (q + RD_BK < q1) load(q + RD_BK);  // in flight during the products below
#pragma unroll
    for (int k4 = 0; k4 < RD_BK; k4 += 4) {
      const double a = As[k4 + lk][16 * wv + li];
#pragma unroll
      for (int t = 0; t < NT; ++t)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Xs[k4 + lk][16 * t + li], acc[t], 0, 0, 0);
    }
  }
  double *out = part + ((static_cast<int64_t>(blockIdx.y) * gridDim.x + blockIdx.x) * RD_TILE) +
                static_cast<int64_t>(wv) * (RD_BN / 16) * 4 * WAVE;
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) out[(t * 4 + i) * WAVE + lane] = acc[t][i];
}

// colpart[rb * ldc + c0 + c] = sum over the block's rows r of
// (sum_s part_s(r, c) - S[c0 + c] Sub(r, c0 + c))^2, c < kc; one block per
// row block, slices added in slice order, waves in wave order.
template <int NT>
__global__ __launch_bounds__(RD_THREADS) void resid_finish_kernel(
    int64_t M, int nsplit, int nrb, const double *__restrict__ part, const double *__restrict__ Sub, int64_t ldsub,
    const double *__restrict__ S, int c0, int kc, double *__restrict__ colpart, int ldc) {
  __shared__ double red[RD_WAVES][16 * NT];
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t rb = blockIdx.x;
  double sq[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    sq[t] = 0.0;
    const int c = 16 * t + li;
    const double sc = c < kc ? S[c0 + c] : 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t row = rb * RD_BM + 16 * wv + 4 * i + lk;
      const int64_t off = static_cast<int64_t>(wv) * (RD_BN / 16) * 4 * WAVE + (t * 4 + i) * WAVE + lane;
      double v = 0.0;
      for (int s = 0; s < nsplit; ++s) v += part[(static_cast<int64_t>(s) * nrb + rb) * RD_TILE + off];
      if (row < M && c < kc) {
        v -= sc * Sub[static_cast<int64_t>(c0 + c) * ldsub + row];
        sq[t] += v * v;
      }
    }
  }
  // the four lanes of a column (lk = 0..3), then the waves in order
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    double v = sq[t];
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    if (lk == 0) red[wv][16 * t + li] = v;
  }
  __syncthreads();
  for (int c = tid; c < 16 * NT; c += RD_THREADS) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < RD_WAVES; ++w) v += red[w][c];
    if (c < kc) colpart[rb * ldc + c0 + c] = v;
  }
}

// out[c] = sqrt(sum_rb colpart[rb * ldc + c]), one block per column.
static __global__ __launch_bounds__(256) void resid_colnorm_kernel(int nrb, const double *__restrict__ colpart,
                                                                   int ldc, double *__restrict__ out) {
  __shared__ double sh[256 / WAVE];
  const int c = blockIdx.x;
  double s = 0;
  for (int rb = threadIdx.x; rb < nrb; rb += 256) s += colpart[static_cast<int64_t>(rb) * ldc + c];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[c] = sqrt(s);
}

// K split of resid_gemm_kernel: about 1024 blocks per column group, slices a
// multiple of RD_BK deep and at least 4 chunks, at most RD_MAX_SPLIT.
inline void resid_split(int64_t M, int64_t K, int &nsplit, int64_t &kslice) {
  const int64_t nrb = ceil_div(M, RD_BM);
  int64_t ns = std::max<int64_t>(1, std::min<int64_t>(ceil_div(1024, nrb), ceil_div(K, 4 * RD_BK)));
  ns = std::min<int64_t>(ns, RD_MAX_SPLIT);
  kslice = ceil_div(ceil_div(K, ns), RD_BK) * RD_BK;
  nsplit = static_cast<int>(ceil_div(K, kslice));
}

// device scratch (doubles) of the dense residuals of an m x n matrix with k
// triplets: the partial tiles of the larger side and the column partials
inline int64_t resid_dense_doubles(int64_t m, int64_t n, int k) {
  int64_t most = 0;
  for (int side = 0; side < 2; ++side) {
    const int64_t M = side ? n : m, K = side ? m : n;
    int ns;
    int64_t ks;
    resid_split(M, K, ns, ks);
    most = std::max<int64_t>(most, ceil_div(M, RD_BM) * ns * RD_TILE);
  }
  return most + ceil_div(std::max(m, n), RD_BM) * static_cast<int64_t>(k);
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
