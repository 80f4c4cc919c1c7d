// Sparse matrix-vector product y = xs * (A x) - coef * yprev over 0-based CSR.
//
// The product is the mat-vec of Alg. 1 steps 2, 5 and 7 (A v and A^T u with
// the -beta u / -alpha v terms fused); A^T u runs the same kernel over the
// CSR of A^T built on the device.
//
// Work decomposition (fixed at plan time, so results are deterministic):
//  * MULTI item: a run of consecutive rows whose total nnz <= SPMV_NNZ_BLK and
//    whose count <= SPMV_ROWS_BLK.  The block stages the products val*x[col]
//    in LDS with coalesced loads, then reduces each row from LDS: one thread
//    per row (short rows), 16 lanes per row (mean length >= SPMV_GROUP_ROW;
//    2% faster on a batch of uniform 0.5%-dense problems) or one wave per row
//    (mean length >= SPMV_WAVE_ROW).
//  * PIECE item: a slice of SPMV_PIECE nonzeros of a row longer than
//    SPMV_NNZ_BLK; the block writes its partial sum, and
//    spmv_longrow_fixup_kernel (next launch) adds the partials of each long
//    row in piece order and writes y.  Power-law rows (the heaviest columns of
//    a Zipf matrix seen through A^T) are spread over many blocks this way.
//  * Column-sorted items (optional): a plan stores each MULTI item's nonzeros
//    sorted by column with their row-order positions (spos), built once by
//    sort_items_kernel.  Gathers of neighbouring lanes then often share a
//    cache line (1.5x on a block-diagonal batch, 7% on a Zipf matrix, 3%
//    slower on uniformly random columns, measured on MI355X); the products
//    are placed in LDS at their row-order positions, so the result is
//    bit-identical to the row-ordered layout.  PIECE ranges stay in row order.
//  * Optional side task: dst[i] = src[i] * xs for i < side_len, spread over
//    the grid.  The solver uses it to write the normalized previous Lanczos
//    vector into its basis column while the product consumes the
//    unnormalized copy.
//
// Several independent problems can share one launch as the blocks of a
// block-diagonal matrix (the batched solver): every item then carries its
// problem's index (in item.w of a MULTI item, LongRow::inst of a long row) and
// the scale factors xs, coef are per-problem arrays; the side task finds the
// problem of entry i from x_tile_inst[i / 256] (problems are padded to
// multiples of 256 rows), restricted to the tiles in side_tiles when given.
// A single problem has index 0 everywhere.
#pragma once
#include "common.hpp"

namespace svds {

constexpr int SPMV_THREADS = 256;
constexpr int SPMV_NNZ_BLK = 2048;
constexpr int SPMV_ROWS_BLK = 256;
constexpr int SPMV_PIECE = 4096;
constexpr int SPMV_CNT_BITS = 12;   // MULTI item: w = nnz count | problem << 12
static_assert(SPMV_NNZ_BLK < (1 << SPMV_CNT_BITS), "item count field");
constexpr int SPMV_WAVE_ROW = 128;  // mean row length from which a MULTI item reduces a wave per row
constexpr int SPMV_GROUP_ROW = 32;  // ... and 16 lanes per row (below: one thread per row)

// Sum over each DPP row of 16 lanes (quad swaps, half-row and row mirrors);
// all 16 lanes end with the same bits.  Every lane of the wave must be active.
template <typename T> __device__ __forceinline__ T spmv_row16_sum(T v) {
  if constexpr (sizeof(T) == 8) {
    v += dpp_f64<0xB1>(v);
    v += dpp_f64<0x4E>(v);
    v += dpp_f64<0x141>(v);
    v += dpp_f64<0x140>(v);
  } else {
    v += dpp_f32<0xB1>(v);
    v += dpp_f32<0x4E>(v);
    v += dpp_f32<0x141>(v);
    v += dpp_f32<0x140>(v);
  }
  return v;
}
static_assert(SPMV_ROWS_BLK <= SPMV_THREADS, "one thread per row of an item");

// item.x >= 0: MULTI rows [x, y), nonzeros from z, w = count | problem << 12.
// item.x < 0: PIECE of long row id -x-1, nonzeros [z, w), written to
// partials[item.y].
struct LongRow {
  int32_t row, first_piece, npieces, inst;
};
constexpr int SPMV_TILE_SHIFT = 8;  // 256-row tiles of the problem map

// Optional epilogue of a MULTI item, for short products of a single problem
// without long rows: the item's rows of y projected on the first jq columns
// of Q (column-major, leading dimension ldq),
//   qpart[c * gridDim.x + item] = sum over the item's rows r of Q[r, c] y[r],
// the partials of the first CGS pass over the vector y becomes (the pass
// then needs no launch of its own).  Only in the PROJ instantiation.
template <typename TB>
struct SpmvProj {
  const TB *Q;
  int64_t ldq;
  int jq;
  TB *qpart;
};

constexpr int SPMV_PT_LD = SPMV_THREADS + 8;  // padded: the four groups of a wave on other banks
static_assert(SPMV_THREADS == 16 * 16, "one 16-lane group per column of a 16-column chunk");

template <typename TV, typename TB, bool PROJ = false>
__global__ __launch_bounds__(SPMV_THREADS) void spmv_csr_kernel(
    const int4 *__restrict__ items, const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const TV *__restrict__ val, const uint16_t *__restrict__ spos, const TB *__restrict__ x,
    const double *__restrict__ xs_ptr,
    const double *__restrict__ coef_ptr, const TB *__restrict__ yprev, TB *__restrict__ y,
    TB *__restrict__ partials, TB *__restrict__ side_dst, int64_t side_len,
    const int32_t *__restrict__ x_tile_inst, const int32_t *__restrict__ active,
    const int32_t *__restrict__ side_tiles, int side_ntiles, SpmvProj<TB> pj) {
  __shared__ TB prod[SPMV_NNZ_BLK];
  __shared__ TB red[SPMV_THREADS / WAVE];
  __shared__ int rps[SPMV_ROWS_BLK + 1];
  __shared__ TB rsum[SPMV_ROWS_BLK];
  __shared__ TB ptr_[PROJ ? 16 * SPMV_PT_LD : 1];  // SpmvProj epilogue: products by column
  const int tid = threadIdx.x;
  const int lane = tid & (WAVE - 1);
  const int wv = tid / WAVE;

  if (side_dst && side_tiles) {
    // only the listed 256-row tiles (the active problems' rows)
    const int64_t len = static_cast<int64_t>(side_ntiles) << SPMV_TILE_SHIFT;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * SPMV_THREADS + tid; i < len;
         i += static_cast<int64_t>(gridDim.x) * SPMV_THREADS) {
      const int32_t t = side_tiles[i >> SPMV_TILE_SHIFT];
      const int64_t r = (static_cast<int64_t>(t) << SPMV_TILE_SHIFT) + (i & ((1 << SPMV_TILE_SHIFT) - 1));
      const int inst = x_tile_inst[t];
      if (active && !active[inst]) continue;
      side_dst[r] = x[r] * (xs_ptr ? static_cast<TB>(xs_ptr[inst]) : TB(1));
    }
  } else if (side_dst && active) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * SPMV_THREADS + tid; i < side_len;
         i += static_cast<int64_t>(gridDim.x) * SPMV_THREADS) {
      const int inst = x_tile_inst ? x_tile_inst[i >> SPMV_TILE_SHIFT] : 0;
      if (!active[inst]) continue;
      side_dst[i] = x[i] * (xs_ptr ? static_cast<TB>(xs_ptr[inst]) : TB(1));
    }
  }
  // Without a problem mask (no block returns early) the side task's first
  // entry per thread is loaded here, with the item's loads in flight, and
  // stored at the end (the loads of short products are one dependent round
  // trip fewer); further entries follow it there.
  const bool side_late = side_dst && !side_tiles && !active;
  const int64_t side_i0 = static_cast<int64_t>(blockIdx.x) * SPMV_THREADS + tid;
  TB side_v0 = 0;
  if (side_late && side_i0 < side_len) {
    const int inst = x_tile_inst ? x_tile_inst[side_i0 >> SPMV_TILE_SHIFT] : 0;
    side_v0 = x[side_i0] * (xs_ptr ? static_cast<TB>(xs_ptr[inst]) : TB(1));
  }

  const int4 it = items[blockIdx.x];
  if (active && it.x >= 0 && !active[it.w >> SPMV_CNT_BITS]) return;  // problem already converged (batched)
  if (it.x >= 0) {
    const int inst = it.w >> SPMV_CNT_BITS;
    const TB xs = xs_ptr ? static_cast<TB>(xs_ptr[inst]) : TB(1);
    const TB coef = coef_ptr ? static_cast<TB>(coef_ptr[inst]) : TB(0);
    const int r0 = it.x, r1 = it.y;
    const int nrows = r1 - r0;
    const int base = it.z;                                   // first nonzero of the item
    const int cnt = it.w & ((1 << SPMV_CNT_BITS) - 1);       // its nonzero count
    // The descriptor carries the nonzero range, so the index/value loads, the
    // row pointers (to LDS: the row loops below then read no global memory)
    // and yprev are all issued at once.
    for (int i = tid; i <= nrows; i += SPMV_THREADS) rps[i] = row_ptr[r0 + i];
    const TB yp = (yprev && tid < nrows) ? yprev[r0 + tid] : TB(0);
    // staging: all index and value loads of the thread first, then all the
    // gathers of x, so each thread has SPMV_NNZ_BLK / SPMV_THREADS loads in
    // flight per round trip instead of one dependent pair per iteration
    constexpr int UPT = SPMV_NNZ_BLK / SPMV_THREADS;
    int ci[UPT], ps[UPT];
    TV cv[UPT];
#pragma unroll
    for (int u = 0; u < UPT; ++u) {
      const int z = tid + u * SPMV_THREADS;
      // indices and values are streamed once: non-temporal loads keep them
      // from displacing the gathered x in L2
      ci[u] = z < cnt ? __builtin_nontemporal_load(col + base + z) : 0;
      cv[u] = z < cnt ? __builtin_nontemporal_load(val + base + z) : TV(0);
      ps[u] = spos ? (z < cnt ? static_cast<int>(__builtin_nontemporal_load(spos + base + z)) : 0) : z;
    }
    // with spos the item's nonzeros are stored sorted by column (neighbouring
    // lanes gather from shared cache lines) and each product goes back to its
    // row-order slot, so the row sums below are unchanged bit for bit
#pragma unroll
    for (int u = 0; u < UPT; ++u) {
      const int z = tid + u * SPMV_THREADS;
      if (z < cnt) prod[ps[u]] = widen<TB>(cv[u]) * x[ci[u]];
    }
    __syncthreads();  // products and row pointers in LDS
    if (cnt >= SPMV_WAVE_ROW * nrows) {
      // few long rows: one wave per row (a wave reduces its rows one after the
      // other, so rows of moderate length go to one thread each instead)
      for (int r = wv; r < nrows; r += SPMV_THREADS / WAVE) {
        const int a = rps[r] - base, b = rps[r + 1] - base;
        TB s = 0;
        for (int z = a + lane; z < b; z += WAVE) s += prod[z];
        s = wave_sum(s);
        if (lane == 0) rsum[r] = s;
      }
    } else if (cnt >= SPMV_GROUP_ROW * nrows) {
      // medium rows: 16 lanes per row, 16 rows at a time (the loop bound is
      // uniform across each wave, as the DPP sums need every lane)
      const int g = tid >> 4, sl = tid & 15;
      for (int r0 = 0; r0 < nrows; r0 += SPMV_THREADS / 16) {
        const int r = r0 + g;
        TB s = 0;
        if (r < nrows) {
          const int a = rps[r] - base, b = rps[r + 1] - base;
          for (int z = a + sl; z < b; z += 16) s += prod[z];
        }
        s = spmv_row16_sum(s);
        if (sl == 0 && r < nrows) rsum[r] = s;
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
    const TB yv = tid < nrows ? xs * rsum[tid] - coef * yp : TB(0);  // nrows <= SPMV_THREADS
    if (tid < nrows) y[r0 + tid] = yv;
    if constexpr (PROJ) {
      // one row per thread, sixteen columns' loads in flight; the products
      // go to LDS column by column and each 16-lane group adds one column's
      // 256 rows (16 each, then a DPP row sum), so a chunk costs one row sum
      // per group instead of a wave sum per column (loading the columns with
      // the item's loads was slower: they then delay the gathers)
      const int g = tid >> 4, l = tid & 15;
      for (int c0 = 0; c0 < pj.jq; c0 += 16) {
        const int nc = min(16, pj.jq - c0);
        TB q[16];
#pragma unroll
        for (int u = 0; u < 16; ++u)
          q[u] = (tid < nrows && u < nc) ? pj.Q[static_cast<int64_t>(c0 + u) * pj.ldq + r0 + tid] : TB(0);
#pragma unroll
        for (int u = 0; u < 16; ++u) ptr_[u * SPMV_PT_LD + tid] = q[u] * yv;
        __syncthreads();
        TB t = 0;
#pragma unroll
        for (int e = 0; e < SPMV_THREADS / 16; ++e) t += ptr_[g * SPMV_PT_LD + l + 16 * e];
        t = spmv_row16_sum(t);
        if (l == 0 && g < nc) pj.qpart[static_cast<int64_t>(c0 + g) * gridDim.x + blockIdx.x] = t;
        __syncthreads();
      }
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
  if (side_late) {
    const int64_t gs = static_cast<int64_t>(gridDim.x) * SPMV_THREADS;
    if (side_i0 < side_len) side_dst[side_i0] = side_v0;
    for (int64_t i = side_i0 + gs; i < side_len; i += gs) {
      const int inst = x_tile_inst ? x_tile_inst[i >> SPMV_TILE_SHIFT] : 0;
      side_dst[i] = x[i] * (xs_ptr ? static_cast<TB>(xs_ptr[inst]) : TB(1));
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
  TB t = strided_sum(partials + L.first_piece, static_cast<int>(threadIdx.x), L.npieces, WAVE, TB(0));
  t = wave_sum(t);
  if (threadIdx.x == 0) y[L.row] = xs * t - (yprev ? coef * yprev[L.row] : TB(0));
}

// Column-sorted copy of a plan's nonzeros: for a MULTI item, (scol, sval)
// = the item's (col, val) ordered by (column, position) and spos = the
// position within the item; a PIECE range is copied as it is.  One block per
// item: keys (column << 11 | position) and values staged in LDS, bitonic sort,
// written back, so scol/sval may alias col/val (in-place sort).
template <typename TV>
__global__ __launch_bounds__(SPMV_THREADS) void sort_items_kernel(const int4 *__restrict__ items,
                                                                  const int32_t *col, const TV *val,
                                                                  int32_t *scol, TV *sval,
                                                                  uint16_t *__restrict__ spos) {
  static_assert(SPMV_NNZ_BLK <= 2048, "11-bit positions");
  __shared__ uint64_t key[SPMV_NNZ_BLK];
  __shared__ TV sv[SPMV_NNZ_BLK];
  const int tid = threadIdx.x;
  const int4 it = items[blockIdx.x];
  if (it.x < 0) {
    if (scol != col)
      for (int z = it.z + tid; z < it.w; z += SPMV_THREADS) scol[z] = col[z], sval[z] = val[z];
    return;
  }
  const int base = it.z, cnt = it.w & ((1 << SPMV_CNT_BITS) - 1);
  int p2 = 1;
  while (p2 < cnt) p2 <<= 1;
  for (int i = tid; i < p2; i += SPMV_THREADS) {
    key[i] = i < cnt ? (static_cast<uint64_t>(static_cast<uint32_t>(col[base + i])) << 11) | static_cast<uint64_t>(i)
                     : ~0ull;
    if (i < cnt) sv[i] = val[base + i];
  }
  __syncthreads();
  for (int k = 2; k <= p2; k <<= 1)
    for (int jj = k >> 1; jj > 0; jj >>= 1) {
      for (int i = tid; i < p2; i += SPMV_THREADS) {
        const int l = i ^ jj;
        if (l > i) {
          const uint64_t a = key[i], b = key[l];
          if ((a > b) == ((i & k) == 0)) key[i] = b, key[l] = a;
        }
      }
      __syncthreads();
    }
  for (int i = tid; i < cnt; i += SPMV_THREADS) {
    const int pos = static_cast<int>(key[i] & 2047u);
    scol[base + i] = static_cast<int32_t>(key[i] >> 11);
    sval[base + i] = sv[pos];
    spos[base + i] = static_cast<uint16_t>(pos);
  }
}

// Column panels of the transpose product.  When u is much larger than one
// XCD's L2, A^T u is computed as sum_g A_g^T u_g over row panels A_g of A
// (column panels of A^T): the stacked CSR [A_0^T; ...; A_{P-1}^T] runs
// through spmv_csr_kernel with its work items interleaved so that block b
// works on panel (b mod 8) mod P (workgroups are dispatched to the 8 XCDs
// round-robin), so each XCD gathers from one slice of u that stays in its L2.
// This kernel adds the panel partials in panel order and applies the
// -coef * yprev term: y[r] = sum_g ypart[g n + r] - coef * yprev[r].
template <typename TB>
__global__ void spmv_panel_sum_kernel(int64_t n, int np, const TB *__restrict__ ypart,
                                      const double *__restrict__ coef_ptr, const TB *__restrict__ yprev,
                                      TB *__restrict__ y) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= n) return;
  TB s = 0;
  for (int g = 0; g < np; ++g) s += ypart[g * n + r];
  const TB coef = coef_ptr ? static_cast<TB>(*coef_ptr) : TB(0);
  y[r] = s - (yprev ? coef * yprev[r] : TB(0));
}
constexpr int SPMV_MAX_PANELS = 8;
constexpr int64_t SPMV_PANEL_BYTES = int64_t(2) << 20;  // FP64 slice of u per panel
constexpr int SPMV_PANEL_MIN_NNZ = 4;                   // mean entries per stacked row

}  // namespace svds

namespace svds {

// ---------------------------------------------------------------------------
// Explicit residual norms of RG output triplets at once (Proposition 1,
// eq. (2)): for g < RG, |A x_g - s_g y_g|^2 over the rows of this launch.
// X (ncols x RG) and Y (nrows x RG) are row-major panels of the triplets'
// vectors (RG consecutive doubles per row: one 64-byte line per gathered
// row for RG = 8).  Same work items as the product: a MULTI item gives one
// thread per row (one wave per row for long rows) and writes the item's
// partial squared norms to part[item][g]; a PIECE item writes its partial
// row sums to pieces[piece][g] and resid_longrow_kernel finishes long rows.
// ---------------------------------------------------------------------------
constexpr int RG = 8;

template <typename TV>
__global__ __launch_bounds__(SPMV_THREADS) void resid_spmm_kernel(
    const int4 *__restrict__ items, const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const TV *__restrict__ val, const double *__restrict__ X, const double *__restrict__ Y,
    const double *__restrict__ s, double *__restrict__ part, double *__restrict__ pieces) {
  __shared__ double red[SPMV_THREADS / WAVE][RG];
  __shared__ double wsum[SPMV_THREADS / WAVE][RG];
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const int4 it = items[blockIdx.x];
  double sg[RG];
#pragma unroll
  for (int g = 0; g < RG; ++g) sg[g] = s[g];
  double sq[RG];
#pragma unroll
  for (int g = 0; g < RG; ++g) sq[g] = 0.0;
  auto gather = [&](int c, double (&acc)[RG], double a) {
    const double4 *xr = reinterpret_cast<const double4 *>(X + static_cast<int64_t>(c) * RG);
    const double4 x0 = xr[0], x1 = xr[1];
    acc[0] += a * x0.x; acc[1] += a * x0.y; acc[2] += a * x0.z; acc[3] += a * x0.w;
    acc[4] += a * x1.x; acc[5] += a * x1.y; acc[6] += a * x1.z; acc[7] += a * x1.w;
  };
  if (it.x >= 0) {
    const int r0 = it.x, r1 = it.y, nrows = r1 - r0;
    const int cnt = it.w & ((1 << SPMV_CNT_BITS) - 1);
    if (cnt >= SPMV_WAVE_ROW * nrows) {
      for (int r = wv; r < nrows; r += SPMV_THREADS / WAVE) {
        const int a = row_ptr[r0 + r], b = row_ptr[r0 + r + 1];
        double acc[RG];
#pragma unroll
        for (int g = 0; g < RG; ++g) acc[g] = 0.0;
        for (int z = a + lane; z < b; z += WAVE) gather(col[z], acc, static_cast<double>(val[z]));
#pragma unroll
        for (int g = 0; g < RG; ++g) acc[g] = wave_sum(acc[g]);
        if (lane == 0) {
          const int64_t row = r0 + r;
#pragma unroll
          for (int g = 0; g < RG; ++g) {
            const double d = acc[g] - sg[g] * Y[row * RG + g];
            sq[g] += d * d;
          }
        }
      }
    } else {
      for (int r = tid; r < nrows; r += SPMV_THREADS) {
        const int a = row_ptr[r0 + r], b = row_ptr[r0 + r + 1];
        double acc[RG];
#pragma unroll
        for (int g = 0; g < RG; ++g) acc[g] = 0.0;
        for (int z = a; z < b; ++z) gather(col[z], acc, static_cast<double>(val[z]));
        const int64_t row = r0 + r;
#pragma unroll
        for (int g = 0; g < RG; ++g) {
          const double d = acc[g] - sg[g] * Y[row * RG + g];
          sq[g] += d * d;
        }
      }
    }
  } else {
    double acc[RG];
#pragma unroll
    for (int g = 0; g < RG; ++g) acc[g] = 0.0;
    for (int z = it.z + tid; z < it.w; z += SPMV_THREADS) gather(col[z], acc, static_cast<double>(val[z]));
#pragma unroll
    for (int g = 0; g < RG; ++g) {
      const double v = wave_sum(acc[g]);
      if (lane == 0) wsum[wv][g] = v;
    }
    __syncthreads();
    if (tid < RG) {
      double t = 0;
      for (int w = 0; w < SPMV_THREADS / WAVE; ++w) t += wsum[w][tid];
      pieces[static_cast<int64_t>(it.y) * RG + tid] = t;
    }
    if (tid < RG) part[static_cast<int64_t>(blockIdx.x) * RG + tid] = 0.0;
    return;
  }
#pragma unroll
  for (int g = 0; g < RG; ++g) {
    const double v = wave_sum(sq[g]);
    if (lane == 0) red[wv][g] = v;
  }
  __syncthreads();
  if (tid < RG) {
    double t = 0;
    for (int w = 0; w < SPMV_THREADS / WAVE; ++w) t += red[w][tid];
    part[static_cast<int64_t>(blockIdx.x) * RG + tid] = t;
  }
}

// Long rows: the row's piece sums in piece order, minus s_g Y, squared, into
// lpart[longrow][g].  One thread per (long row, g).
static __global__ void resid_longrow_kernel(const LongRow *__restrict__ longrows, int nlong,
                                            const double *__restrict__ pieces, const double *__restrict__ Y,
                                            const double *__restrict__ s, double *__restrict__ lpart) {
  const int i = blockIdx.x * (256 / RG) + threadIdx.x / RG, g = threadIdx.x % RG;
  if (i >= nlong) return;
  const LongRow L = longrows[i];
  double t = 0;
  for (int q = 0; q < L.npieces; ++q) t += pieces[static_cast<int64_t>(L.first_piece + q) * RG + g];
  const double d = t - s[g] * Y[static_cast<int64_t>(L.row) * RG + g];
  lpart[static_cast<int64_t>(i) * RG + g] = d * d;
}

// res[g] = sqrt(sum over items of part[item][g] + sum over long rows of
// lpart[row][g]), in index order; one wave per g.
static __global__ void resid_finish_kernel(const double *__restrict__ part, int nitems,
                                           const double *__restrict__ lpart, int nlong, int ng,
                                           double *__restrict__ res) {
  const int g = blockIdx.x, lane = threadIdx.x;
  if (g >= ng) return;
  double t = 0;
  for (int i = lane; i < nitems; i += WAVE) t += part[static_cast<int64_t>(i) * RG + g];
  for (int i = lane; i < nlong; i += WAVE) t += lpart[static_cast<int64_t>(i) * RG + g];
  t = wave_sum(t);
  if (lane == 0) res[g] = sqrt(t);
}

// s8[g] = S[c0 + g] for c0 + g < nc, 0 beyond.
static __global__ void resid_svals_kernel(const double *__restrict__ S, int c0, int nc, double *__restrict__ s8) {
  const int g = threadIdx.x;
  if (g < RG) s8[g] = c0 + g < nc ? S[c0 + g] : 0.0;
}

// Panel of RG columns, row-major: P[r * RG + g] = M[(c0 + g) * ld + r] for
// c0 + g < nc, 0 beyond.
static __global__ void resid_panel_kernel(int64_t L, const double *__restrict__ M, int64_t ld, int c0, int nc,
                                          double *__restrict__ P) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < L * RG;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t r = i / RG;
    const int g = static_cast<int>(i % RG);
    P[i] = c0 + g < nc ? M[(c0 + g) * ld + r] : 0.0;
  }
}

}  // namespace svds
