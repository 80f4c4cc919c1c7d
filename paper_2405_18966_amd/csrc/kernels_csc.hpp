// Device construction of the CSR of A^T (a column-major copy of A) from the
// CSR of A, for the product A^T u of Alg. 1 step 5; the same sort with
// panel-offset keys builds the stacked transpose of the panelled product.
//
// The CSR of A lists entries in (row, col) order, so a *stable* sort by
// column yields (col, row) order: every column's entries come out in
// increasing row order -- a canonical, run-to-run identical layout.
// The sort is an LSD radix sort (8-bit digits) of the column keys carrying the
// entry's position; each pass is histogram -> exclusive scan -> stable
// scatter, where the within-tile rank of an element among equal digits is
// found with wave ballots.  Integer work only: bit-exact.
#pragma once
#include "common.hpp"

namespace svds {

constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 8;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;  // keys per tile
constexpr int RS_BITS = 8;
constexpr int RS_BINS = 1 << RS_BITS;

// rowof[z] = row of entry z; keys[z] = col[z] + (row / rows_per_panel) * n;
// perm[z] = z.  With rows_per_panel >= m every key is the column (the plain
// transpose); with panels of rows the sort yields the stacked transpose
// [A_0^T; A_1^T; ...], A_g = rows [g rpp, (g + 1) rpp) of A.
// CSC_EXPAND_LANES lanes per row, each taking every CSC_EXPAND_LANES-th
// entry, so that neighbouring lanes write neighbouring entries (one thread
// per row wrote rows of ~100 entries with strided stores: 5.7 ms for the
// 128M nonzeros of a 256-problem batch).
constexpr int CSC_EXPAND_LANES = 16;
static __global__ void csc_expand_kernel(int64_t m, const int32_t *__restrict__ row_ptr,
                                  const int32_t *__restrict__ col, int64_t rows_per_panel, int64_t n,
                                  int32_t *__restrict__ rowof, int32_t *__restrict__ keys,
                                  int32_t *__restrict__ perm) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t r = t / CSC_EXPAND_LANES;
  if (r >= m) return;
  const int32_t off = static_cast<int32_t>((r / rows_per_panel) * n);
  const int32_t z1 = row_ptr[r + 1];
  for (int32_t z = row_ptr[r] + static_cast<int32_t>(t % CSC_EXPAND_LANES); z < z1; z += CSC_EXPAND_LANES) {
    rowof[z] = static_cast<int32_t>(r);
    keys[z] = col[z] + off;
    perm[z] = z;
  }
}

// hist[d * ntiles + tile] = number of keys of the tile with digit d.
static __global__ __launch_bounds__(RS_THREADS) void radix_hist_kernel(const int32_t *__restrict__ keys,
                                                                int64_t nnz, int shift,
                                                                int32_t *__restrict__ hist,
                                                                int64_t ntiles) {
  __shared__ int32_t cnt[RS_BINS];
  for (int i = threadIdx.x; i < RS_BINS; i += RS_THREADS) cnt[i] = 0;
  __syncthreads();
  const int64_t base = static_cast<int64_t>(blockIdx.x) * RS_TILE;
  for (int i = 0; i < RS_ITEMS; ++i) {
    const int64_t z = base + i * RS_THREADS + threadIdx.x;
    if (z < nnz) atomicAdd(&cnt[(keys[z] >> shift) & (RS_BINS - 1)], 1);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < RS_BINS; d += RS_THREADS)
    hist[static_cast<int64_t>(d) * ntiles + blockIdx.x] = cnt[d];
}

// Stable scatter: element e of the tile goes to offs[d*ntiles+tile] + (number
// of earlier elements of the tile with the same digit d).
static __global__ __launch_bounds__(RS_THREADS) void radix_scatter_kernel(
    const int32_t *__restrict__ keys_in, const int32_t *__restrict__ vals_in, int64_t nnz,
    int shift, const int32_t *__restrict__ offs, int64_t ntiles, int32_t *__restrict__ keys_out,
    int32_t *__restrict__ vals_out) {
  constexpr int NW = RS_THREADS / WAVE;
  __shared__ int32_t running[RS_BINS];
  __shared__ int32_t wcnt[NW][RS_BINS];
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  for (int d = tid; d < RS_BINS; d += RS_THREADS)
    running[d] = offs[static_cast<int64_t>(d) * ntiles + blockIdx.x];
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
  const int64_t base = static_cast<int64_t>(blockIdx.x) * RS_TILE;
  for (int i = 0; i < RS_ITEMS; ++i) {
    for (int d = lane; d < RS_BINS; d += WAVE) wcnt[wv][d] = 0;
    __syncthreads();
    const int64_t z = base + i * RS_THREADS + tid;
    const bool valid = z < nnz;
    int32_t key = 0, v = 0, dg = -1;
    if (valid) {
      key = keys_in[z];
      v = vals_in[z];
      dg = (key >> shift) & (RS_BINS - 1);
    }
    // lanes of this wave holding the same digit
    uint64_t same = __ballot(valid);
#pragma unroll
    for (int b = 0; b < RS_BITS; ++b) {
      const bool bit = valid && ((dg >> b) & 1);
      const uint64_t bb = __ballot(bit);
      same &= bit ? bb : ~bb;
    }
    const int rank_w = __popcll(same & lt_mask);
    const int leader = valid ? (__ffsll(static_cast<long long>(same)) - 1) : -1;
    if (valid && lane == leader) wcnt[wv][dg] = __popcll(same);
    __syncthreads();
    if (valid) {
      int pos = running[dg] + rank_w;
      for (int w = 0; w < wv; ++w) pos += wcnt[w][dg];
      keys_out[pos] = key;
      vals_out[pos] = v;
    }
    __syncthreads();
    for (int d = tid; d < RS_BINS; d += RS_THREADS) {
      int s = 0;
      for (int w = 0; w < NW; ++w) s += wcnt[w][d];
      running[d] += s;
    }
    __syncthreads();
  }
}

// Exclusive scan of int32 (three kernels: tile sums, scan of tile sums,
// tile scan with offset).
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__device__ __forceinline__ int32_t block_exclusive_scan_i32(int32_t v, int32_t *sh, int32_t &total) {
  // sh: SCAN_THREADS/WAVE + 1 ints
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  int32_t incl = v;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const int32_t t = __shfl_up(incl, o, WAVE);
    if (lane >= o) incl += t;
  }
  if (lane == WAVE - 1) sh[wv] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t s = 0;
    for (int w = 0; w < static_cast<int>(blockDim.x / WAVE); ++w) {
      const int32_t t = sh[w];
      sh[w] = s;
      s += t;
    }
    sh[blockDim.x / WAVE] = s;
  }
  __syncthreads();
  const int32_t excl = incl - v + sh[wv];
  total = sh[blockDim.x / WAVE];
  __syncthreads();
  return excl;
}

static __global__ __launch_bounds__(SCAN_THREADS) void scan_tile_sums_kernel(const int32_t *__restrict__ in,
                                                                      int64_t n,
                                                                      int32_t *__restrict__ sums) {
  __shared__ int32_t sh[SCAN_THREADS / WAVE + 1];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  int32_t s = 0;
  for (int i = 0; i < SCAN_ITEMS; ++i)
    if (base + i < n) s += in[base + i];
  int32_t total;
  block_exclusive_scan_i32(s, sh, total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// single block: exclusive scan of `sums` in place (any length)
static __global__ __launch_bounds__(SCAN_THREADS) void scan_sums_kernel(int32_t *__restrict__ sums,
                                                                 int64_t nt) {
  __shared__ int32_t sh[SCAN_THREADS / WAVE + 1];
  int32_t carry = 0;
  for (int64_t b = 0; b < nt; b += SCAN_TILE) {
    const int64_t base = b + threadIdx.x * SCAN_ITEMS;
    int32_t loc[SCAN_ITEMS];
    int32_t s = 0;
    for (int i = 0; i < SCAN_ITEMS; ++i) {
      loc[i] = (base + i < nt) ? sums[base + i] : 0;
      s += loc[i];
    }
    int32_t total;
    int32_t e = block_exclusive_scan_i32(s, sh, total) + carry;
    for (int i = 0; i < SCAN_ITEMS; ++i) {
      if (base + i < nt) sums[base + i] = e;
      e += loc[i];
    }
    carry += total;
  }
}

static __global__ __launch_bounds__(SCAN_THREADS) void scan_apply_kernel(const int32_t *__restrict__ in,
                                                                  int64_t n,
                                                                  const int32_t *__restrict__ sums,
                                                                  int32_t *__restrict__ out) {
  __shared__ int32_t sh[SCAN_THREADS / WAVE + 1];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  int32_t loc[SCAN_ITEMS];
  int32_t s = 0;
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    loc[i] = (base + i < n) ? in[base + i] : 0;
    s += loc[i];
  }
  int32_t total;
  int32_t e = block_exclusive_scan_i32(s, sh, total) + sums[blockIdx.x];
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    if (base + i < n) out[base + i] = e;
    e += loc[i];
  }
}

// Final gather: transposed row index / value of every sorted entry.
template <typename TV>
static __global__ void csc_gather_kernel(int64_t nnz, const int32_t *__restrict__ perm,
                                  const int32_t *__restrict__ rowof, const TV *__restrict__ val,
                                  int32_t *__restrict__ t_col, TV *__restrict__ t_val) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= nnz) return;
  const int32_t z = perm[q];
  t_col[q] = rowof[z];
  t_val[q] = val[z];
}

// Column pointers from the sorted keys: t_rowptr[c] = first q with key >= c,
// for c = 0..n, one thread per column by binary search (a thread per
// nonzero filling the gap before it wrote long runs of empty columns
// serially: 13 ms for a 500,000-column matrix of 30 nonzeros).
static __global__ void csc_colptr_kernel(int64_t nnz, int64_t n, const int32_t *__restrict__ skeys,
                                  int32_t *__restrict__ t_rowptr) {
  const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c > n) return;
  int64_t lo = 0, hi = nnz;  // first q in [lo, hi) with skeys[q] >= c
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (skeys[mid] < c) lo = mid + 1;
    else hi = mid;
  }
  t_rowptr[c] = static_cast<int32_t>(lo);
}

static __global__ void fill_i32_kernel(int64_t n, int32_t v, int32_t *__restrict__ out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = v;
}

}  // namespace svds
