// Full re-orthogonalization of a new Lanczos vector (Sec. 2.1, after Alg. 1:
// u <- (I - U U^T) u, v <- (I - V V^T) v), done as classical Gram-Schmidt
// applied twice (CGS2), plus the norm that becomes alpha or beta
// (Alg. 1 steps 6 and 8).
//
// Q is the basis, column-major with leading dimension ldq, columns [0, j);
// w has L entries.  Three passes over Q, the minimum with Q in HBM:
//   cgs_proj      : partials of h1 = Q^T w
//   cgs_upd_proj  : w1 = w - Q h1 and partials of h2 = Q^T w1 from the same
//                   read of Q
//   cgs_upd_norm  : w2 = w1 - Q h2 and partials of |w2|^2
// Cross-block sums are finished by small kernels at the kernel boundary
// (reduce_cols_kernel, finish_norm_kernel): on MI355X a device-scope fence or
// a shared arrival counter in every block costs ~0.1 us per block, serialized,
// far more than one extra launch.  For short vectors, whose passes leave at
// most CGS_FUSE_NP partials per column, the next pass sums them itself
// (CgsCoef) and the reduction launch is skipped.  Sums are in fixed order
// (deterministic).
#pragma once
#include <algorithm>
#include <hip/hip_cooperative_groups.h>
#include "common.hpp"

namespace svds {

constexpr int CGS_THREADS = 256;
constexpr int CGS_PCG = 8;      // columns per block column-group in cgs_proj
constexpr int CGS_FUSED_MAXJ = 320;  // widest basis of the fused pass (16 waves x 20 columns)
constexpr int CGS_MAXJ = 1024;  // largest basis width supported
constexpr int CGS_MAX_SLABS = 1024;  // partials per column (cgs_proj / cgs_upd_proj)
constexpr int NORM_MAX_BLOCKS = 2048;
constexpr double BREAKDOWN_REL = 1e-14;

// Row vectors of N consecutive entries per lane.  N = 16 / sizeof(T) turns a
// lane's access into one 16-byte load or store (measured on MI355X: 6.3 TB/s
// for the projection pattern against 5.7 TB/s with 8-byte accesses); it
// needs 16-byte aligned vectors and a leading dimension divisible by N.
// `rem` = entries left in the vector from p on; entries past the end read 0
// and are not written.
template <typename T, int N>
__device__ __forceinline__ void load_rows(const T *__restrict__ p, int64_t rem, T (&v)[N]) {
  if (N * sizeof(T) == 16 && rem >= N) {
    const uint4 u = *reinterpret_cast<const uint4 *>(p);
    __builtin_memcpy(&v[0], &u, 16);
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = i < rem ? p[i] : T(0);
  }
}
template <typename T, int N>
__device__ __forceinline__ void store_rows(T *__restrict__ p, int64_t rem, const T (&v)[N]) {
  if (N * sizeof(T) == 16 && rem >= N) {
    uint4 u;
    __builtin_memcpy(&u, &v[0], 16);
    *reinterpret_cast<uint4 *>(p) = u;
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (i < rem) p[i] = v[i];
  }
}

// out[c] = sum_{i < nv} src[c * ld + i] for c < nc.  One wave per column,
// lanes take interleaved indices, fixed-order wave reduction.
template <typename T>
__global__ __launch_bounds__(256) void reduce_cols_kernel(const T *__restrict__ src, int64_t ld, int nv,
                                                          int nc, T *__restrict__ out) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int c = blockIdx.x * (256 / WAVE) + threadIdx.x / WAVE;
  if (c >= nc) return;
  const T *p = src + static_cast<int64_t>(c) * ld;
  T s = strided_sum(p, lane, nv, WAVE, T(0));
  s = wave_sum(s);
  if (lane == 0) out[c] = s;
}

// Where a pass finds the coefficients of the previous projection: h (global,
// from reduce_cols_kernel) or, with hp non-null, that projection's np
// partials per column (column-major, [j][np]), which the pass sums itself:
// for short vectors the partials are few and the summing costs less than a
// reduction launch.  Workgroup 0 then also stores the sums to hout.
template <typename T>
struct CgsCoef {
  const T *hp;
  int np;
  T *hout;
};

// sh[c] = h[c] for c < j and 0 for j <= c < npad; one thread per column,
// partials added in order (every workgroup gets the same sums).  Ends with
// a barrier.
constexpr int CGS_FUSE_NP = 32;  // at most two batches of 16 loads per thread
template <typename T>
__device__ inline void cgs_load_coeffs(T *sh, int j, int npad, const T *__restrict__ h, const CgsCoef<T> &cf) {
  for (int c = threadIdx.x; c < npad; c += blockDim.x) {
    T v = 0;
    if (c < j) {
      if (cf.hp) {
        v = strided_sum(cf.hp + static_cast<int64_t>(c) * cf.np, 0, cf.np, 1, T(0));
        if (blockIdx.x == 0) cf.hout[c] = v;
      } else {
        v = h[c];
      }
    }
    sh[c] = v;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Pass 1: partials of h = Q^T w.  Grid (row slabs, column groups of 8).
// Each wave walks tiles of 64 N rows of its block's slab (N rows per lane)
// keeping 8 column accumulators per lane (narrow groups and many blocks
// stream fastest on MI355X; 32-column groups reach half the rate).
// part: [j][nslab]; with normw the blocks of column group 0 also write the
// partials of |w|^2 as column j (read by the selective second pass).
// MASK: only the columns c with cmask[c] != 0 are read (partial
// re-orthogonalization); the others get zero partials, and a block none of
// whose columns is selected writes its zeros without reading anything.
// ---------------------------------------------------------------------------
template <typename T, int N, bool MASK = false>
__global__ __launch_bounds__(CGS_THREADS) void cgs_proj_kernel(const T *__restrict__ Q, int64_t ldq,
                                                              int64_t L, int j, const T *__restrict__ w,
                                                              T *__restrict__ part, int normw,
                                                              const int *__restrict__ cmask) {
  constexpr int NW = CGS_THREADS / WAVE;
  __shared__ T red[NW][CGS_PCG + 1];
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const int nslab = gridDim.x, slab = blockIdx.x;
  const int c0 = blockIdx.y * CGS_PCG;
  int nc = min(CGS_PCG, j - c0);
  bool en[CGS_PCG];
#pragma unroll
  for (int c = 0; c < CGS_PCG; ++c) en[c] = c < nc && (!MASK || cmask[c0 + c] != 0);
  if (MASK) {
    bool any = false;
#pragma unroll
    for (int c = 0; c < CGS_PCG; ++c) any = any || en[c];
    if (!any && !(normw && blockIdx.y == 0)) {
      if (tid < nc) part[static_cast<int64_t>(c0 + tid) * nslab + slab] = T(0);
      return;
    }
  }
  const int64_t R = static_cast<int64_t>(WAVE) * N;
  const int64_t tiles = ceil_div(L, R);
  const int64_t per = ceil_div(tiles, nslab);
  const int64_t t0 = slab * per, t1 = min(tiles, t0 + per);
  const T *Qc = Q + c0 * ldq;
  const bool dn = normw && blockIdx.y == 0;
  T acc[CGS_PCG], nw = 0;
#pragma unroll
  for (int c = 0; c < CGS_PCG; ++c) acc[c] = 0;
  for (int64_t t = t0 + wv; t < t1; t += NW) {
    const int64_t r = t * R + lane * N;
    if (r < L) {
      T wr[N];
      load_rows<T, N>(w + r, L - r, wr);
      if (dn)
#pragma unroll
        for (int i = 0; i < N; ++i) nw += wr[i] * wr[i];
#pragma unroll
      for (int c = 0; c < CGS_PCG; ++c) {
        if (MASK ? en[c] : c < nc) {
          T q[N];
          load_rows<T, N>(Qc + c * ldq + r, L - r, q);
#pragma unroll
          for (int i = 0; i < N; ++i) acc[c] += q[i] * wr[i];
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < CGS_PCG; ++c) {
    const T s = wave_sum(acc[c]);
    if (lane == 0) red[wv][c] = s;
  }
  if (dn) {
    const T s = wave_sum(nw);
    if (lane == 0) red[wv][CGS_PCG] = s;
  }
  __syncthreads();
  if (tid < nc) {
    T s = 0;
    for (int v = 0; v < NW; ++v) s += red[v][tid];
    part[static_cast<int64_t>(c0 + tid) * nslab + slab] = s;
  }
  if (dn && tid == CGS_PCG) {
    T s = 0;
    for (int v = 0; v < NW; ++v) s += red[v][CGS_PCG];
    part[static_cast<int64_t>(j) * nslab + slab] = s;
  }
}

// ---------------------------------------------------------------------------
// Pass 2 fused with the update of pass 1: w1 = w - Q h1 (written out) and
// partials of h2 = Q^T w1.  Block = ceil(j/CPW) waves (<= 16); a block walks
// tiles of 64 N rows; wave v holds columns [CPW v, CPW v + CPW) of the tile in
// registers, so Q is read once for both the update and the projection.  The
// cross-wave row sums go through a double-buffered LDS array (one barrier per
// tile).  Narrow register tiles (CPW <= 12 with one row per lane) keep
// occupancy high: measured on MI355X, two rows per lane with 12-16 columns
// per wave stream at a third of the rate or less.  Bases of 161-320 columns
// take CPW = 20 without prefetch (one 16-wave block per CU, as with
// CPW = 10); wider ones use a separate update pass plus cgs_proj instead.
// part: [j][nblk]; with normw1 also the partials of |w1|^2 as column j.
// MASK: only the columns with cmask[c] != 0 are read (the others have h1 = 0
// and get zero partials).
// ---------------------------------------------------------------------------
template <typename T, int CPW, bool PF, int N, bool MASK = false>
__global__ __launch_bounds__(1024) void cgs_upd_proj_kernel(const T *__restrict__ Q, int64_t ldq,
                                                           int64_t L, int j, const T *__restrict__ w,
                                                           const T *__restrict__ h1,
                                                           T *__restrict__ w1out, T *__restrict__ part,
                                                           int normw1, const int *__restrict__ cmask,
                                                           CgsCoef<T> cf) {
  __shared__ T sh_h[CGS_MAXJ];
  __shared__ T xch[2][16][WAVE * N];
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const int NW = blockDim.x / WAVE;
  const int nblk = gridDim.x, blk = blockIdx.x;
  cgs_load_coeffs(sh_h, j, NW * CPW, h1, cf);  // padding columns 0
  const int c0 = wv * CPW;
  const int nc = max(0, min(CPW, j - c0));
  bool en[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) en[c] = c < nc && (!MASK || cmask[c0 + c] != 0);
  __syncthreads();
  const int64_t R = static_cast<int64_t>(WAVE) * N;
  const int64_t tiles = ceil_div(L, R);
  const int64_t per = ceil_div(tiles, nblk);
  const int64_t t0 = static_cast<int64_t>(blk) * per;
  const int64_t t1 = min(tiles, t0 + per);
  const T *Qc = Q + c0 * ldq;
  T acc[CPW], q[CPW][N], qn[CPW][N];
  T wn[N], nw1 = 0;
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    acc[c] = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) qn[c][i] = 0;
  }
#pragma unroll
  for (int i = 0; i < N; ++i) wn[i] = 0;
  auto load = [&](int64_t t) {
    const int64_t r = t * R + lane * N;
    if (r < L) {
#pragma unroll
      for (int c = 0; c < CPW; ++c)
        if (MASK ? en[c] : c < nc) load_rows<T, N>(Qc + c * ldq + r, L - r, qn[c]);
      load_rows<T, N>(w + r, L - r, wn);
    }
  };
  if (PF && t0 < t1) load(t0);
  int buf = 0;
  for (int64_t t = t0; t < t1; ++t) {
    const int64_t r = t * R + lane * N;
    if (!PF) load(t);
    T wr[N];
#pragma unroll
    for (int i = 0; i < N; ++i) wr[i] = wn[i];
#pragma unroll
    for (int c = 0; c < CPW; ++c)
#pragma unroll
      for (int i = 0; i < N; ++i) q[c][i] = qn[c][i];
    if (PF && t + 1 < t1) load(t + 1);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T s = 0;
#pragma unroll
      for (int c = 0; c < CPW; ++c) s += q[c][i] * sh_h[c0 + c];
      xch[buf][wv][lane * N + i] = s;
    }
    __syncthreads();
    T w1[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T u = 0;
      for (int v = 0; v < NW; ++v) u += xch[buf][v][lane * N + i];
      w1[i] = (r + i < L) ? wr[i] - u : T(0);
    }
    if (wv == 0 && r < L) store_rows<T, N>(w1out + r, L - r, w1);
    if (normw1 && wv == 0)
#pragma unroll
      for (int i = 0; i < N; ++i) nw1 += w1[i] * w1[i];
#pragma unroll
    for (int c = 0; c < CPW; ++c)
#pragma unroll
      for (int i = 0; i < N; ++i) acc[c] += q[c][i] * w1[i];
    buf ^= 1;
  }
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const T s = wave_sum(acc[c]);
    if (lane == 0 && c < nc) part[static_cast<int64_t>(c0 + c) * nblk + blk] = s;
  }
  if (normw1 && wv == 0) {
    const T s = wave_sum(nw1);
    if (lane == 0) part[static_cast<int64_t>(j) * nblk + blk] = s;
  }
}

// The fused pass for bases of 161-320 columns: 20 columns per wave, one row
// per lane, each tile's 20 loads issued together (no prefetch of the next
// tile, so the 20 columns and 20 accumulators fit the 128 VGPRs a 16-wave
// block may use).  Same outputs as cgs_upd_proj_kernel.
template <typename T, bool MASK = false>
__global__ __launch_bounds__(1024) void cgs_upd_proj_wide_kernel(const T *__restrict__ Q, int64_t ldq, int64_t L,
                                                                int j, const T *__restrict__ w,
                                                                const T *__restrict__ h1, T *__restrict__ w1out,
                                                                T *__restrict__ part, int normw1,
                                                                const int *__restrict__ cmask, CgsCoef<T> cf) {
  constexpr int CPW = 20;
  __shared__ T sh_h[CGS_MAXJ];
  __shared__ T xch[2][16][WAVE];
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const int NW = blockDim.x / WAVE;
  const int nblk = gridDim.x, blk = blockIdx.x;
  cgs_load_coeffs(sh_h, j, NW * CPW, h1, cf);  // padding columns 0
  const int c0 = wv * CPW;
  const int nc = max(0, min(CPW, j - c0));
  unsigned en = 0;  // bit c: column c0 + c is read
  for (int c = 0; c < nc; ++c)
    if (!MASK || cmask[c0 + c] != 0) en |= 1u << c;
  en = __builtin_amdgcn_readfirstlane(en);
  __syncthreads();
  const int64_t tiles = ceil_div(L, static_cast<int64_t>(WAVE));
  const int64_t per = ceil_div(tiles, nblk);
  const int64_t t0 = static_cast<int64_t>(blk) * per;
  const int64_t t1 = min(tiles, t0 + per);
  const T *Qc = Q + c0 * ldq;
  T acc[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) acc[c] = 0;
  T nw1 = 0;
  int buf = 0;
  for (int64_t t = t0; t < t1; ++t) {
    const int64_t r = t * WAVE + lane;
    const bool ok = r < L;
    T q[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) q[c] = (ok && ((en >> c) & 1u)) ? Qc[c * ldq + r] : T(0);
    const T wr = ok ? w[r] : T(0);
    T s = 0;
#pragma unroll
    for (int c = 0; c < CPW; ++c) s += q[c] * sh_h[c0 + c];
    xch[buf][wv][lane] = s;
    __syncthreads();
    T u = 0;
    for (int v = 0; v < NW; ++v) u += xch[buf][v][lane];
    const T w1 = ok ? wr - u : T(0);
    if (wv == 0 && ok) w1out[r] = w1;
    if (normw1 && wv == 0) nw1 += w1 * w1;
#pragma unroll
    for (int c = 0; c < CPW; ++c) acc[c] += q[c] * w1;
    buf ^= 1;
  }
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const T sc = wave_sum(acc[c]);
    if (lane == 0 && c < nc) part[static_cast<int64_t>(c0 + c) * nblk + blk] = sc;
  }
  if (normw1 && wv == 0) {
    const T sc = wave_sum(nw1);
    if (lane == 0) part[static_cast<int64_t>(j) * nblk + blk] = sc;
  }
}

// Selective second pass: with sel non-null the pass is skipped (out = w1, no
// read of Q) when |w1|^2 >= |w|^2 / 2, i.e. the first projection removed at
// most 1/sqrt(2) of w's norm (the test of Daniel, Gragg, Kaufman and Stewart,
// 1976); sel[0] = |w|^2 and h[j] = |w1|^2 come from the first two passes.
// Every block takes the same decision from the same two values; block 0
// counts the passes that ran in *ran.
template <typename T>
__device__ __forceinline__ int cgs_second_pass_width(int j, const T *h, const T *sel, int *ran) {
  if (!sel) return j;
  const bool run = h[j] < T(0.5) * sel[0];
  if (run && ran && blockIdx.x == 0 && threadIdx.x == 0) *ran += 1;
  return run ? j : 0;
}

// ---------------------------------------------------------------------------
// Pass 3: out = w1 - Q h; with `npart` non-null, partials of |out|^2 (FP64).
// Grid-stride rows, the column loop unrolled 8-wide for loads in flight.
// ---------------------------------------------------------------------------
// MASK: only the columns with cmask[c] != 0 are read.
template <typename T, int N, bool MASK = false>
__global__ __launch_bounds__(CGS_THREADS) void cgs_upd_norm_kernel(
    const T *__restrict__ Q, int64_t ldq, int64_t L, int j, const T *__restrict__ w1,
    const T *__restrict__ h, T *__restrict__ out, double *__restrict__ npart, const T *__restrict__ sel,
    int *__restrict__ ran, const int *__restrict__ cmask, CgsCoef<T> cf) {
  __shared__ T sh_h[CGS_MAXJ];
  __shared__ int sh_c[MASK ? CGS_MAXJ : 1];
  __shared__ double sh_d[CGS_THREADS / WAVE];
  const int tid = threadIdx.x;
  j = cgs_second_pass_width(j, h, sel, ran);
  cgs_load_coeffs(sh_h, j, j, h, cf);
  if (MASK) {
    // the selected columns, in increasing order (one wave compacts them)
    __shared__ int sh_n;
    if (tid < WAVE) {
      int base = 0;
      for (int c0 = 0; c0 < j; c0 += WAVE) {
        const int c = c0 + tid;
        const bool on = c < j && cmask[c] != 0;
        const uint64_t bal = __ballot(on);
        if (on) sh_c[base + __popcll(bal & ((uint64_t(1) << tid) - 1))] = c;
        base += __popcll(bal);
      }
      if (tid == 0) sh_n = base;
    }
    __syncthreads();
    j = sh_n;
  }
  __syncthreads();
  double nrm2 = 0;
  for (int64_t r = (static_cast<int64_t>(blockIdx.x) * CGS_THREADS + tid) * N; r < L;
       r += static_cast<int64_t>(gridDim.x) * CGS_THREADS * N) {
    T u[8][N];
#pragma unroll
    for (int g = 0; g < 8; ++g)
#pragma unroll
      for (int i = 0; i < N; ++i) u[g][i] = 0;
    int c = 0;
    for (; c + 8 <= j; c += 8) {
#pragma unroll
      for (int g = 0; g < 8; ++g) {
        const int col = MASK ? sh_c[c + g] : c + g;
        T q[N];
        load_rows<T, N>(Q + col * ldq + r, L - r, q);
#pragma unroll
        for (int i = 0; i < N; ++i) u[g][i] += q[i] * sh_h[col];
      }
    }
    for (; c < j; ++c) {
      const int col = MASK ? sh_c[c] : c;
      T q[N];
      load_rows<T, N>(Q + col * ldq + r, L - r, q);
#pragma unroll
      for (int i = 0; i < N; ++i) u[0][i] += q[i] * sh_h[col];
    }
    T wv[N], x[N];
    load_rows<T, N>(w1 + r, L - r, wv);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      x[i] = wv[i] - (((u[0][i] + u[1][i]) + (u[2][i] + u[3][i])) + ((u[4][i] + u[5][i]) + (u[6][i] + u[7][i])));
      if (r + i < L) nrm2 += static_cast<double>(x[i]) * static_cast<double>(x[i]);
    }
    store_rows<T, N>(out + r, L - r, x);
  }
  if (!npart) return;
  nrm2 = block_sum(nrm2, sh_d);
  if (tid == 0) npart[blockIdx.x] = nrm2;
}

// ---------------------------------------------------------------------------
// Pass 3 for short vectors (few row tiles, e.g. a dense matrix's bases):
// out = w1 - Q h with one tile of 64 N rows per block, so that the grid has a
// block per tile instead of a few hundred threads per CU.  Wave v multiplies
// the tile by columns [CPW v, CPW v + CPW) of Q; the waves' partial updates
// are added in LDS in wave order; wave 0 writes the tile of out and, with
// `npart` non-null, the tile's squared norm (FP64) to npart[tile].
// Measured on MI355X (L = 20000, j = 250, FP64): 9 us against 23 us for the
// row-per-thread pass.
// ---------------------------------------------------------------------------
constexpr int CGS_TILE_CPW = 16;
constexpr int CGS_TILE_MAXJ = 16 * CGS_TILE_CPW;  // 16 waves

template <typename T, int N, bool MASK = false>
__global__ __launch_bounds__(1024) void cgs_tile_upd_kernel(const T *__restrict__ Q, int64_t ldq, int64_t L,
                                                            int j, const T *__restrict__ w1,
                                                            const T *__restrict__ h, T *__restrict__ out,
                                                            double *__restrict__ npart, const T *__restrict__ sel,
                                                            int *__restrict__ ran, const int *__restrict__ cmask,
                                                            CgsCoef<T> cf) {
  constexpr int CPW = CGS_TILE_CPW;
  j = cgs_second_pass_width(j, h, sel, ran);
  __shared__ T sh_h[CGS_TILE_MAXJ];
  __shared__ T xch[16][WAVE * N];
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const int NW = blockDim.x / WAVE;
  cgs_load_coeffs(sh_h, j, NW * CPW, h, cf);
  const int64_t tile = blockIdx.x;
  const int64_t r = tile * (WAVE * N) + lane * N;
  const int c0 = wv * CPW;
  const int nc = max(0, min(CPW, j - c0));
  T s[N];
#pragma unroll
  for (int i = 0; i < N; ++i) s[i] = 0;
  if (r < L) {
    T q[CPW][N];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      if (c < nc && (!MASK || cmask[c0 + c] != 0)) load_rows<T, N>(Q + (c0 + c) * ldq + r, L - r, q[c]);
      else
#pragma unroll
        for (int i = 0; i < N; ++i) q[c][i] = 0;
    }
#pragma unroll
    for (int c = 0; c < CPW; ++c)
#pragma unroll
      for (int i = 0; i < N; ++i) s[i] += q[c][i] * sh_h[c0 + c];
  }
#pragma unroll
  for (int i = 0; i < N; ++i) xch[wv][lane * N + i] = s[i];
  __syncthreads();
  if (wv != 0) return;
  double nrm2 = 0;
  if (r < L) {
    T wr[N], x[N];
    load_rows<T, N>(w1 + r, L - r, wr);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T u = 0;
      for (int v = 0; v < NW; ++v) u += xch[v][lane * N + i];
      x[i] = wr[i] - u;
      if (r + i < L) nrm2 += static_cast<double>(x[i]) * static_cast<double>(x[i]);
    }
    store_rows<T, N>(out + r, L - r, x);
  }
  if (!npart) return;
  nrm2 = wave_sum(nrm2);
  if (lane == 0) npart[tile] = nrm2;
}

// Rows per lane of the CGS kernels for these operands: 16-byte accesses when
// every vector is 16-byte aligned and ldq is a multiple of the row count.
template <typename T>
inline int cgs_rows_per_lane(const void *Q, int64_t ldq, const void *a, const void *b, const void *c) {
  constexpr int N = 16 / sizeof(T);
  auto al = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  return (ldq % N == 0 && al(Q) && al(a) && al(b) && al(c)) ? N : 1;
}

// ---------------------------------------------------------------------------
// Norm finish (one block): adds the norm partials in block order, then by mode
//   MODE_NORM   : xs = 1 / |w|                               (start vector)
//   MODE_LANCZOS: T entry = |w|, xs = 1/|w|, sigma_est update; on breakdown
//                 (|w| <= 1e-14 sigma_est) the vector is replaced in place by
//                 a Philox normal vector re-orthogonalized against Q (CGS2)
//                 and normalized, T entry = 0, xs = 1.
// ---------------------------------------------------------------------------
enum { MODE_NORM = 1, MODE_LANCZOS = 2 };

struct FinishArgs {
  double *t_entry;      // T(i,i) or T(i,i+1)
  double *xs;           // reciprocal norm of the stored vector
  double *sigma_est;    // running max of alpha, beta, sigma_1
  int *breakdowns;      // breakdown counter of the solve
  uint64_t seed;
  // partial re-orthogonalization (om_row non-null): the new vector's
  // orthogonality estimates against the j earlier ones of its side become
  // om_row[0..j) and om_row[j] = 1: the pending estimates (om_pend, made
  // with the norm *om_nrm0 before re-orthogonalization) rescaled to the final
  // norm, EPS for the columns it was re-orthogonalized against (om_mask), and
  // EPS everywhere when om_full or on a breakdown (taken against the whole
  // basis; a breakdown also clears the side's forced set om_force).
  double *om_row;
  const double *om_pend;
  const int *om_mask;
  const double *om_nrm0;
  int *om_force;
  int om_full;
};

constexpr double OMEGA_EPS = 0x1.0p-52;

__device__ __forceinline__ void omega_fix(const FinishArgs &fa, int j, double nrm, bool all_eps) {
  if (!fa.om_row) return;
  const double scale = (!all_eps && nrm > 0) ? *fa.om_nrm0 / nrm : 0.0;
  for (int l = threadIdx.x; l < j; l += blockDim.x) {
    fa.om_row[l] = (all_eps || fa.om_full || fa.om_mask[l]) ? OMEGA_EPS : fa.om_pend[l] * scale;
    if (all_eps) fa.om_force[l] = 0;
  }
  if (threadIdx.x == 0) fa.om_row[j] = 1.0;
}

// Breakdown replacement (one block): out = a Philox normal vector (stream
// `stream` of `seed`), taken twice against Q[:, 0:j] by classical
// Gram-Schmidt, then normalized.  The projections run eight columns at a
// time (one read of the eight columns and of out per chunk, eight block sums
// in column order), the updates add the columns eight at a time per row: each
// pass reads Q once, whatever j is.
template <typename T>
__device__ void breakdown_repair(const T *__restrict__ Q, int64_t ldq, int64_t L, int j,
                                 T *__restrict__ out, uint32_t stream, uint64_t seed,
                                 double *sh_d, T *sh_h) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int64_t b = tid; 2 * b < L; b += nt) {
    double z0, z1;
    philox_normal_pair(seed, stream, static_cast<uint64_t>(b), z0, z1);
    out[2 * b] = static_cast<T>(z0);
    if (2 * b + 1 < L) out[2 * b + 1] = static_cast<T>(z1);
  }
  __threadfence_block();
  __syncthreads();
  constexpr int CH = 8;
  for (int pass = 0; pass < 2; ++pass) {
    for (int c0 = 0; c0 < j; c0 += CH) {
      const int nc = min(CH, j - c0);
      T acc[CH];
#pragma unroll
      for (int g = 0; g < CH; ++g) acc[g] = 0;
      for (int64_t r = tid; r < L; r += nt) {
        const T x = out[r];
#pragma unroll
        for (int g = 0; g < CH; ++g)
          if (g < nc) acc[g] += Q[static_cast<int64_t>(c0 + g) * ldq + r] * x;
      }
#pragma unroll
      for (int g = 0; g < CH; ++g) {
        const T sg = block_sum(acc[g], reinterpret_cast<T *>(sh_d));
        if (tid == 0 && g < nc) sh_h[c0 + g] = sg;
      }
    }
    __syncthreads();
    for (int64_t r = tid; r < L; r += nt) {
      T u[CH];
#pragma unroll
      for (int g = 0; g < CH; ++g) u[g] = 0;
      int c = 0;
      for (; c + CH <= j; c += CH)
#pragma unroll
        for (int g = 0; g < CH; ++g) u[g] += Q[static_cast<int64_t>(c + g) * ldq + r] * sh_h[c + g];
      for (; c < j; ++c) u[0] += Q[static_cast<int64_t>(c) * ldq + r] * sh_h[c];
      out[r] -= ((u[0] + u[1]) + (u[2] + u[3])) + ((u[4] + u[5]) + (u[6] + u[7]));
    }
    __threadfence_block();
    __syncthreads();
  }
  double s = 0;
  for (int64_t r = tid; r < L; r += nt) s += static_cast<double>(out[r]) * out[r];
  s = block_sum(s, sh_d);
  const double inv = 1.0 / sqrt(s);
  for (int64_t r = tid; r < L; r += nt) out[r] = static_cast<T>(out[r] * inv);
}

constexpr int FINISH_THREADS = 1024;  // a breakdown's repair streams the basis with one block

template <typename T>
__global__ __launch_bounds__(FINISH_THREADS) void finish_norm_kernel(const double *__restrict__ npart,
                                                                    int nparts, int mode, FinishArgs fa,
                                                                    const T *__restrict__ Q, int64_t ldq,
                                                                    int64_t L, int j, T *__restrict__ out) {
  __shared__ double sh_d[FINISH_THREADS / WAVE];
  __shared__ T sh_h[CGS_MAXJ];
  __shared__ int bd;
  const int tid = threadIdx.x;
  double tot = strided_sum(npart, tid, nparts, static_cast<int>(blockDim.x), 0.0);
  tot = block_sum(tot, sh_d);
  const double nrm = sqrt(tot);
  if (mode == MODE_NORM) {
    if (tid == 0) *fa.xs = 1.0 / nrm;
    return;
  }
  const double sig = *fa.sigma_est;
  if (nrm > BREAKDOWN_REL * sig) {
    if (tid == 0) {
      *fa.t_entry = nrm;
      *fa.xs = 1.0 / nrm;
      *fa.sigma_est = fmax(sig, nrm);
    }
    omega_fix(fa, j, nrm, false);
    return;
  }
  omega_fix(fa, j, 0.0, true);
  // Breakdown: the new vector lies in the span of Q (an invariant subspace was
  // found).  Replace it by a re-orthogonalized random vector, store 0 in T.
  if (tid == 0) {
    bd = *fa.breakdowns + 1;
    *fa.breakdowns = bd;
    *fa.t_entry = 0.0;
    *fa.xs = 1.0;
  }
  __syncthreads();
  breakdown_repair<T>(Q, ldq, L, j, out, static_cast<uint32_t>(bd), fa.seed, sh_d, sh_h);
}

// The finish step over G workgroups of a cooperative launch, for long bases
// (the one-workgroup finish_norm_kernel streams a 10^6 x 40 basis for a
// breakdown at one CU's bandwidth, ~26 ms).  Every workgroup forms |w| from
// the same partials in the same order, so all take the same branch; on the
// usual path workgroup 0 does what finish_norm_kernel does and the others
// return.  On a breakdown workgroup b owns rows [L b / G, L (b+1) / G): it
// draws those rows of the same Philox vector, and for each of the two
// classical Gram-Schmidt passes and for the norm writes its partial sums to
// `part` (double; two halves of G x (j + 1) used alternately, so a workgroup
// never overwrites sums another is still adding), passes a grid barrier, and
// adds the G partials in workgroup order: every workgroup holds the same
// coefficients.  Three grid barriers per breakdown.  The breakdown counter is
// read by all before the first barrier and advanced after it.
template <typename T>
__global__ __launch_bounds__(FINISH_THREADS) void finish_norm_coop_kernel(
    const double *__restrict__ npart, int nparts, int mode, FinishArgs fa, const T *__restrict__ Q, int64_t ldq,
    int64_t L, int j, T *__restrict__ out, double *__restrict__ part) {
  __shared__ double sh_d[FINISH_THREADS / WAVE];
  __shared__ T sh_h[CGS_MAXJ];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int G = gridDim.x, b = blockIdx.x;
  double tot = strided_sum(npart, tid, nparts, nt, 0.0);
  tot = block_sum(tot, sh_d);
  const double nrm = sqrt(tot);
  if (mode == MODE_NORM) {
    if (b == 0 && tid == 0) *fa.xs = 1.0 / nrm;
    return;
  }
  // workgroup 0 raises sigma_est only on the usual path, where the others
  // return whichever value they read (nrm > REL sig implies nrm > REL max(sig, nrm))
  const double sig = *fa.sigma_est;
  if (nrm > BREAKDOWN_REL * sig) {
    if (b != 0) return;
    if (tid == 0) {
      *fa.t_entry = nrm;
      *fa.xs = 1.0 / nrm;
      *fa.sigma_est = fmax(sig, nrm);
    }
    omega_fix(fa, j, nrm, false);
    return;
  }
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  const int bd = *fa.breakdowns + 1;
  if (b == 0) omega_fix(fa, j, 0.0, true);
  const int64_t r0 = L * b / G, r1 = L * (b + 1) / G;
  for (int64_t r = r0 + tid; r < r1; r += nt) {
    double z0, z1;
    philox_normal_pair(fa.seed, static_cast<uint32_t>(bd), static_cast<uint64_t>(r >> 1), z0, z1);
    out[r] = static_cast<T>((r & 1) ? z1 : z0);
  }
  __syncthreads();
  const int ps = j + 1;
  constexpr int CH = 8;
  for (int pass = 0; pass < 2; ++pass) {
    double *P = part + (pass & 1) * G * ps;
    for (int c0 = 0; c0 < j; c0 += CH) {
      const int nc = min(CH, j - c0);
      T acc[CH];
#pragma unroll
      for (int g = 0; g < CH; ++g) acc[g] = 0;
      for (int64_t r = r0 + tid; r < r1; r += nt) {
        const T x = out[r];
#pragma unroll
        for (int g = 0; g < CH; ++g)
          if (g < nc) acc[g] += Q[static_cast<int64_t>(c0 + g) * ldq + r] * x;
      }
#pragma unroll
      for (int g = 0; g < CH; ++g) {
        const T sg = block_sum(acc[g], reinterpret_cast<T *>(sh_d));
        if (tid == 0 && g < nc) P[b * ps + c0 + g] = static_cast<double>(sg);
      }
    }
    grid.sync();
    if (pass == 0 && b == 0 && tid == 0) {
      *fa.breakdowns = bd;
      *fa.t_entry = 0.0;
      *fa.xs = 1.0;
    }
    for (int c = tid; c < j; c += nt) {
      double h = 0;
      for (int q = 0; q < G; ++q) h += P[q * ps + c];
      sh_h[c] = static_cast<T>(h);
    }
    __syncthreads();
    for (int64_t r = r0 + tid; r < r1; r += nt) {
      T u[CH];
#pragma unroll
      for (int g = 0; g < CH; ++g) u[g] = 0;
      int c = 0;
      for (; c + CH <= j; c += CH)
#pragma unroll
        for (int g = 0; g < CH; ++g) u[g] += Q[static_cast<int64_t>(c + g) * ldq + r] * sh_h[c + g];
      for (; c < j; ++c) u[0] += Q[static_cast<int64_t>(c) * ldq + r] * sh_h[c];
      out[r] -= ((u[0] + u[1]) + (u[2] + u[3])) + ((u[4] + u[5]) + (u[6] + u[7]));
    }
    __syncthreads();
  }
  double s = 0;
  for (int64_t r = r0 + tid; r < r1; r += nt) s += static_cast<double>(out[r]) * out[r];
  s = block_sum(s, sh_d);
  if (tid == 0) part[b * ps] = s;  // first half again: its last readers passed the second barrier
  grid.sync();
  double n2 = 0;
  for (int q = 0; q < G; ++q) n2 += part[q * ps];
  const double inv = 1.0 / sqrt(n2);
  for (int64_t r = r0 + tid; r < r1; r += nt) out[r] = static_cast<T>(out[r] * inv);
}

// ---------------------------------------------------------------------------
// Partial re-orthogonalization (one block of CGS_THREADS threads per step).
// The loss of orthogonality of the new, unnormalized vector w against every
// earlier vector of its side follows from the two Lanczos relations
// A V = U T and A^T U = V T^T (T row-major, leading dimension ld):
//   V side, w = A^T u_i - T(i,i) v_i, estimates for l <= i:
//     v_l^T w = sum_{r<=l} T(r,l) mu[r] - T(i,i) nu[l]
//   U side, w = A v_i - T(i-1,i) u_{i-1}, estimates for l < i:
//     u_l^T w = sum_{c<=i} T(l,c) nu[c] - T(i-1,i) mu[l]
// with mu / nu the estimate rows of the newest u and v (their own entry 1),
// plus a local rounding term EPS sigma_est with the sign of the sum, divided
// by |w| (from the norm partials of w).  An estimate above `tau` triggers a
// re-orthogonalization against the columns whose estimate is above `eta`,
// together with the columns `force` holds (the set of the previous vector of
// this side, when that one triggered); a trigger also sets `force` for the
// next vector of the side.  Outputs: cmask (the columns to take w against),
// the pending estimates and |w| for the finish step (omega_fix), and
// counters stats[0] += 1 and stats[1] += selected columns when any column is
// selected, stats[2] += j.
// ---------------------------------------------------------------------------
struct OmegaArgs {
  const double *T;
  int ld;
  int side;  // 0: the new vector is v_{i+1}; 1: it is u_i
  int i;
  const double *npart;
  int nparts;
  const double *sigma_est;
  const double *mu, *nu;
  int *force, *cmask;
  double *pend, *nrm0;
  long long *stats;
  double tau, eta;
};

static __global__ __launch_bounds__(CGS_THREADS) void omega_kernel(OmegaArgs a) {
  __shared__ double sh_d[CGS_THREADS / WAVE];
  const int tid = threadIdx.x;
  double tot = strided_sum(a.npart, tid, a.nparts, CGS_THREADS, 0.0);
  tot = block_sum(tot, sh_d);
  const double nrm = sqrt(tot);
  const double rnd = OMEGA_EPS * *a.sigma_est;
  const int i = a.i, ld = a.ld;
  const int j = a.side == 0 ? i + 1 : i;  // earlier vectors of the side
  int trig = 0, forced = 0;
  for (int l = tid; l < j; l += CGS_THREADS) {
    double x;
    if (a.side == 0) {
      x = -a.T[i * ld + i] * a.nu[l];
      for (int r = 0; r <= l; ++r) x += a.T[r * ld + l] * a.mu[r];
    } else {
      x = -a.T[(i - 1) * ld + i] * a.mu[l];
      for (int c = 0; c <= i; ++c) x += a.T[l * ld + c] * a.nu[c];
    }
    const double om = nrm > 0 ? (x + (x >= 0 ? rnd : -rnd)) / nrm : INFINITY;
    a.pend[l] = om;
    trig |= fabs(om) > a.tau;
    forced |= a.force[l] != 0;
  }
  trig = __syncthreads_or(trig);
  forced = __syncthreads_or(forced);
  int cnt = 0;
  for (int l = tid; l < j; l += CGS_THREADS) {
    const bool on = (trig || forced) && (fabs(a.pend[l]) > a.eta || a.force[l] != 0);
    a.cmask[l] = on ? 1 : 0;
    a.force[l] = (trig && on) ? 1 : 0;
    cnt += on ? 1 : 0;
  }
  cnt = static_cast<int>(block_sum(static_cast<double>(cnt), sh_d));
  if (tid == 0) {
    *a.nrm0 = nrm;
    if (cnt > 0) {
      a.stats[0] += 1;
      a.stats[1] += cnt;
    }
    a.stats[2] += j;
  }
}

// Restart (Alg. 2 step 10): v_{k+1} = v_{p+1}, so its estimates against the
// kept Ritz vectors V Vh(:, l) are nu_new[l] = sum_c Vh(c, l) nu[c], c < p
// (Vext column-major, leading dimension p + 1); nu[k] = 1, the rest 0; the
// forced sets of both sides are cleared.  One block; pend is scratch.
static __global__ __launch_bounds__(CGS_THREADS) void omega_restart_kernel(const double *__restrict__ Vext, int p, int k,
                                                                   double *nu, double *pend, int *force_u,
                                                                   int *force_v) {
  const int tid = threadIdx.x;
  for (int l = tid; l < k; l += CGS_THREADS) {
    double x = 0;
    for (int c = 0; c < p; ++c) x += Vext[static_cast<int64_t>(l) * (p + 1) + c] * nu[c];
    pend[l] = x;
  }
  __syncthreads();
  for (int l = tid; l <= p + 1; l += CGS_THREADS) {
    nu[l] = l < k ? pend[l] : (l == k ? 1.0 : 0.0);
    force_u[l] = 0;
    force_v[l] = 0;
  }
}

// Start of a solve: estimate rows of u_1 and v_1 (their own entry 1), no
// forced sets, the 8 counters (both sides) zero.
static __global__ void omega_init_kernel(int p, double *mu, double *nu, int *force_u, int *force_v, long long *stats) {
  for (int l = threadIdx.x; l <= p + 1; l += blockDim.x) {
    mu[l] = l == 0 ? 1.0 : 0.0;
    nu[l] = l == 0 ? 1.0 : 0.0;
    force_u[l] = 0;
    force_v[l] = 0;
  }
  if (threadIdx.x < 8) stats[threadIdx.x] = 0;
}

// Launch shapes (host side), tuned on MI355X.
inline void cgs_proj_shape(int64_t L, int j, int &nslab, int &ngrp_c) {
  // 8-column groups x row slabs of >= 32 tiles of 64 rows, at most 512 slabs;
  // short vectors or narrow bases get more slabs (up to ~2048 blocks, at
  // least 256 rows per slab): a 20000-row basis of 250 columns projects in
  // 9 us with 64 slabs against 16 us with 9
  ngrp_c = static_cast<int>(ceil_div(j, CGS_PCG));
  const int64_t tiles = ceil_div(L, WAVE);
  const int64_t base = std::max<int64_t>(1, std::min<int64_t>(512, tiles / 32));
  const int64_t wide = std::min<int64_t>({ceil_div(2048, ngrp_c), ceil_div(L, 256), CGS_MAX_SLABS});
  int64_t ns = std::max(base, wide);
  // a grid of more than one round of the ~2048 blocks the chip holds at once
  // is cut to a whole number (>= 2) of rounds, so that no partial last round
  // leaves CUs idle (measured: 1,000,000 x 150 basis 214 -> 202 us,
  // 500,000 x 150 117 -> 105 us)
  constexpr int64_t RESIDENT = 2048;
  const double rounds = static_cast<double>(ns * ngrp_c) / RESIDENT;
  if (rounds > 1.0) {
    const int64_t k = std::max<int64_t>(2, static_cast<int64_t>(rounds + 0.3));
    const int64_t ns2 = ceil_div(RESIDENT * k, ngrp_c);
    if (ns2 <= CGS_MAX_SLABS && ns2 <= ceil_div(L, 256)) ns = ns2;
  }
  nslab = static_cast<int>(ns);
}
inline int cgs_updproj_blocks(int64_t L, int j) {
  // a quarter of the 64-row tiles, at most 512 blocks; at least ~160 blocks
  // for short vectors, and up to 1024 for one- or two-wave blocks (j <= 16)
  const int64_t tiles = ceil_div(L, WAVE);
  int64_t nb = std::min<int64_t>(512, ceil_div(tiles, 4));
  nb = std::max(nb, std::min<int64_t>(tiles, 160));
  if (j <= 16) nb = std::max(nb, std::min<int64_t>(CGS_MAX_SLABS, ceil_div(tiles, 2)));
  return static_cast<int>(std::max<int64_t>(1, nb));
}
// the tile-per-block update applies (its norm partials fit NORM_MAX_BLOCKS)
inline bool cgs_tile_upd_ok(int64_t L, int j, int rows_per_lane) {
  return j <= CGS_TILE_MAXJ && ceil_div(L, static_cast<int64_t>(WAVE) * rows_per_lane) <= NORM_MAX_BLOCKS;
}
// columns per wave of the fused pass for a basis of width j (0: use the split
// path).  FP64: 8 up to j = 80, then 10 (both one row per lane with register
// prefetch; measured on MI355X, 10 columns are 2-7% faster from j ~ 90 on).
// FP32: 8 up to 128, then 10 with 16-byte rows.
// Columns per wave of the fused pass: 8, 10, or 20 (no register prefetch:
// with it 20 columns would not fit the 128 VGPRs of a 16-wave block) for
// 160 < j <= 320.
inline int cgs_fused_cpw(int j, int elem_bytes) {
  if (j > CGS_FUSED_MAXJ) return 0;
  if (j > 160) return 20;
  return j <= (elem_bytes == 8 ? 80 : 128) ? 8 : 10;
}
inline int cgs_updnorm_blocks(int64_t L) {
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(NORM_MAX_BLOCKS, ceil_div(L, CGS_THREADS))));
}

}  // namespace svds
