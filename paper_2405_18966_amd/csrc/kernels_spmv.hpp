// Sparse matrix-vector product y = xs * (A x) - coef * yprev over 0-based CSR.
//
// The product is the mat-vec of Alg. 1 steps 2, 5 and 7 (A v and A^T u with
// the -beta u / -alpha v terms fused); A^T u runs the same kernel over the
// CSR of A^T built on the device.
//
// Work decomposition (fixed at plan time, so results are deterministic):
//  * MULTI item: a run of consecutive rows whose total nnz <= SPMV_NNZ_BLK and
//    whose count <= SPMV_ROWS_BLK.  The block stages the products val*x[col]
//    in LDS with coalesced loads, then reduces each row from LDS, one thread
//    per row (short rows) or one wave per row (long rows).
//  * PIECE item: a slice of SPMV_PIECE nonzeros of a row longer than
//    SPMV_NNZ_BLK; the block writes its partial sum, and
//    spmv_longrow_fixup_kernel (next launch) adds the partials of each long
//    row in piece order and writes y.  Power-law rows (the heaviest columns of
//    a Zipf matrix seen through A^T) are spread over many blocks this way.
//  * Optional side task: dst[i] = src[i] * xs for i < side_len, spread over
//    the grid.  The solver uses it to write the normalized previous Lanczos
//    vector into its basis column while the product consumes the
//    unnormalized copy.
//
// Several independent problems can share one launch as the blocks of a
// block-diagonal matrix (the batched solver): every item then carries its
// problem's index (item.z of a MULTI item, LongRow::inst of a long row) and
// the scale factors xs, coef are per-problem arrays; the side task finds the
// problem of entry i from x_tile_inst[i / 256] (problems are padded to
// multiples of 256 rows).  A single problem has index 0 everywhere.
#pragma once
#include "common.hpp"

namespace svds {

constexpr int SPMV_THREADS = 256;
constexpr int SPMV_NNZ_BLK = 2048;
constexpr int SPMV_ROWS_BLK = 256;
constexpr int SPMV_PIECE = 4096;

// item.x >= 0: MULTI rows [x, y) of problem z.   item.x < 0: PIECE of long
// row id -x-1, nonzeros [z, w), written to partials[item.y].
struct LongRow {
  int32_t row, first_piece, npieces, inst;
};
constexpr int SPMV_TILE_SHIFT = 8;  // 256-row tiles of the problem map

template <typename TV, typename TB>
__global__ __launch_bounds__(SPMV_THREADS) void spmv_csr_kernel(
    const int4 *__restrict__ items, const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const TV *__restrict__ val, const TB *__restrict__ x, const double *__restrict__ xs_ptr,
    const double *__restrict__ coef_ptr, const TB *__restrict__ yprev, TB *__restrict__ y,
    TB *__restrict__ partials, TB *__restrict__ side_dst, int64_t side_len,
    const int32_t *__restrict__ x_tile_inst, const int32_t *__restrict__ active) {
  __shared__ TB prod[SPMV_NNZ_BLK];
  __shared__ TB red[SPMV_THREADS / WAVE];
  __shared__ int rps[SPMV_ROWS_BLK + 1];
  __shared__ TB rsum[SPMV_ROWS_BLK];
  const int tid = threadIdx.x;
  const int lane = tid & (WAVE - 1);
  const int wv = tid / WAVE;

  if (side_dst) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * SPMV_THREADS + tid; i < side_len;
         i += static_cast<int64_t>(gridDim.x) * SPMV_THREADS) {
      const int inst = x_tile_inst ? x_tile_inst[i >> SPMV_TILE_SHIFT] : 0;
      if (active && !active[inst]) continue;
      side_dst[i] = x[i] * (xs_ptr ? static_cast<TB>(xs_ptr[inst]) : TB(1));
    }
  }

  const int4 it = items[blockIdx.x];
  if (active && it.x >= 0 && !active[it.z]) return;  // problem already converged (batched)
  if (it.x >= 0) {
    const TB xs = xs_ptr ? static_cast<TB>(xs_ptr[it.z]) : TB(1);
    const TB coef = coef_ptr ? static_cast<TB>(coef_ptr[it.z]) : TB(0);
    const int r0 = it.x, r1 = it.y;
    const int nrows = r1 - r0;
    // the item's row pointers go to LDS first: the row loops below then read
    // no global memory (a global load per row serializes a wave per row)
    for (int i = tid; i <= nrows; i += SPMV_THREADS) rps[i] = row_ptr[r0 + i];
    __syncthreads();
    const int base = rps[0];
    const int cnt = rps[nrows] - base;
    // staging: all index and value loads of the thread first, then all the
    // gathers of x, so each thread has SPMV_NNZ_BLK / SPMV_THREADS loads in
    // flight per round trip instead of one dependent pair per iteration
    constexpr int UPT = SPMV_NNZ_BLK / SPMV_THREADS;
    int ci[UPT];
    TV cv[UPT];
#pragma unroll
    for (int u = 0; u < UPT; ++u) {
      const int z = tid + u * SPMV_THREADS;
      // indices and values are streamed once: non-temporal loads keep them
      // from displacing the gathered x in L2
      ci[u] = z < cnt ? __builtin_nontemporal_load(col + base + z) : 0;
      cv[u] = z < cnt ? __builtin_nontemporal_load(val + base + z) : TV(0);
    }
#pragma unroll
    for (int u = 0; u < UPT; ++u) {
      const int z = tid + u * SPMV_THREADS;
      if (z < cnt) prod[z] = widen<TB>(cv[u]) * x[ci[u]];
    }
    __syncthreads();
    if (cnt >= 32 * nrows) {
      // few long rows: one wave per row
      for (int r = wv; r < nrows; r += SPMV_THREADS / WAVE) {
        const int a = rps[r] - base, b = rps[r + 1] - base;
        TB s = 0;
        for (int z = a + lane; z < b; z += WAVE) s += prod[z];
        s = wave_sum(s);
        if (lane == 0) rsum[r] = s;
      }
    } else {
      for (int r = tid; r < nrows; r += SPMV_THREADS) {
        const int a = rps[r] - base, b = rps[r + 1] - base;
        TB s = 0;
        for (int z = a; z < b; ++z) s += prod[z];
        rsum[r] = s;
      }
    }
    __syncthreads();
    for (int r = tid; r < nrows; r += SPMV_THREADS) {
      const int64_t row = r0 + r;
      y[row] = xs * rsum[r] - (yprev ? coef * yprev[row] : TB(0));
    }
  } else {
    const int z0 = it.z, z1 = it.w;
    TB s = 0;
    for (int zb = z0 + tid; zb < z1; zb += 4 * SPMV_THREADS) {
      int ci[4];
      TV cv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int z = zb + u * SPMV_THREADS;
        ci[u] = z < z1 ? __builtin_nontemporal_load(col + z) : 0;
        cv[u] = z < z1 ? __builtin_nontemporal_load(val + z) : TV(0);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int z = zb + u * SPMV_THREADS;
        if (z < z1) s += widen<TB>(cv[u]) * x[ci[u]];
      }
    }
    s = wave_sum(s);
    if (lane == 0) red[wv] = s;
    __syncthreads();
    if (tid == 0) {
      TB t = 0;
      for (int i = 0; i < SPMV_THREADS / WAVE; ++i) t += red[i];
      partials[it.y] = t;
    }
  }
}

// y[row] = xs * (sum of the row's piece partials) - coef * yprev[row]; one
// wave per long row (lanes take interleaved pieces, fixed-order reduction).
template <typename TB>
__global__ __launch_bounds__(WAVE) void spmv_longrow_fixup_kernel(const LongRow *__restrict__ longrows,
                                                                  int nlong, const TB *__restrict__ partials,
                                                                  const double *__restrict__ xs_ptr,
                                                                  const double *__restrict__ coef_ptr,
                                                                  const TB *__restrict__ yprev,
                                                                  TB *__restrict__ y,
                                                                  const int32_t *__restrict__ active) {
  const int i = blockIdx.x;
  if (i >= nlong) return;
  const LongRow L = longrows[i];
  if (active && !active[L.inst]) return;
  const TB xs = xs_ptr ? static_cast<TB>(xs_ptr[L.inst]) : TB(1);
  const TB coef = coef_ptr ? static_cast<TB>(coef_ptr[L.inst]) : TB(0);
  TB t = 0;
  for (int q = threadIdx.x; q < L.npieces; q += WAVE) t += partials[L.first_piece + q];
  t = wave_sum(t);
  if (threadIdx.x == 0) y[L.row] = xs * t - (yprev ? coef * yprev[L.row] : TB(0));
}

}  // namespace svds
