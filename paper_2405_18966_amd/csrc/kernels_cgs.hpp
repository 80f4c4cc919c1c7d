// Full re-orthogonalization of a new Lanczos vector (Sec. 2.1, after Alg. 1:
// u <- (I - U U^T) u, v <- (I - V V^T) v), done as classical Gram-Schmidt
// applied twice (CGS2), plus the norm that becomes alpha or beta
// (Alg. 1 steps 6 and 8).
//
// Q is the basis, column-major with leading dimension ldq, columns [0, j);
// w has L entries.  Three passes over Q, the minimum with Q in HBM:
//   cgs_proj      : h1 = Q^T w
//   cgs_upd_proj  : w1 = w - Q h1 and h2 = Q^T w1 from the same read of Q
//   cgs_upd_norm  : w2 = w1 - Q h2, |w2|; the last block turns the norm into
//                   T(i,i) / T(i,i+1), the reciprocal scale of the vector,
//                   and handles breakdown.
// Reductions across blocks: each block writes per-column partial sums, the
// last block to finish (arrival counter) adds them in block order.  No float
// atomics anywhere, so every run gives bitwise the same result.
#pragma once
#include "common.hpp"

namespace svds {

constexpr int CGS_THREADS = 256;
constexpr int CGS_CC = 8;       // columns per chunk in cgs_proj
constexpr int CGS_CPW = 16;     // columns per wave in cgs_upd_proj
constexpr int CGS_MAXJ = 1024;  // largest basis width supported
constexpr double BREAKDOWN_REL = 1e-14;

// Row slab [r0, r1) of block g out of G for vectors of length L, 64-aligned.
__device__ __forceinline__ void block_slab(int64_t L, int64_t &r0, int64_t &r1) {
  const int64_t tiles = ceil_div(L, WAVE);
  const int64_t per = ceil_div(tiles, gridDim.x);
  r0 = static_cast<int64_t>(blockIdx.x) * per * WAVE;
  r1 = r0 + per * WAVE;
  if (r1 > L) r1 = L;
  if (r0 > L) r0 = L;
}

// Last block: out[c] = sum_g partials[c*G + g], c < j.  One wave per column,
// lanes stride over g, fixed-order wave reduction.
template <typename T>
__device__ __forceinline__ void reduce_partials(const T *__restrict__ partials, int j,
                                                T *__restrict__ out) {
  const int G = gridDim.x;
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  const int nw = blockDim.x / WAVE;
  for (int c = wv; c < j; c += nw) {
    T s = 0;
    for (int g = lane; g < G; g += WAVE) s += partials[static_cast<int64_t>(c) * G + g];
    s = wave_sum(s);
    if (lane == 0) out[c] = s;
  }
}

// ---------------------------------------------------------------------------
// Pass 1: h = Q^T w.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(CGS_THREADS) void cgs_proj_kernel(
    const T *__restrict__ Q, int64_t ldq, int64_t L, int j, const T *__restrict__ w,
    T *__restrict__ partials, T *__restrict__ h, unsigned int *__restrict__ counter) {
  constexpr int NW = CGS_THREADS / WAVE;
  __shared__ T red[NW][CGS_CC];
  __shared__ int flag;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  int64_t r0, r1;
  block_slab(L, r0, r1);
  const int G = gridDim.x;
  for (int c0 = 0; c0 < j; c0 += CGS_CC) {
    const int nc = min(CGS_CC, j - c0);
    T acc[CGS_CC];
#pragma unroll
    for (int c = 0; c < CGS_CC; ++c) acc[c] = 0;
    for (int64_t r = r0 + tid; r < r1; r += CGS_THREADS) {
      const T wr = w[r];
#pragma unroll
      for (int c = 0; c < CGS_CC; ++c)
        if (c < nc) acc[c] += Q[(c0 + c) * ldq + r] * wr;
    }
#pragma unroll
    for (int c = 0; c < CGS_CC; ++c) {
      const T s = wave_sum(acc[c]);
      if (lane == 0) red[wv][c] = s;
    }
    __syncthreads();
    if (tid < nc) {
      T s = 0;
      for (int v = 0; v < NW; ++v) s += red[v][tid];
      partials[static_cast<int64_t>(c0 + tid) * G + blockIdx.x] = s;
    }
    __syncthreads();
  }
  if (elect_last_block(counter, &flag)) reduce_partials(partials, j, h);
}

// ---------------------------------------------------------------------------
// Pass 2 fused with the update of pass 1: w1 = w - Q h1 (written out) and
// h2 = Q^T w1.  Block = NW waves; a block walks 64-row tiles, wave v holds
// columns [16v, 16v+16) of the tile in registers, so Q is read once for both
// the update and the projection.  NW = ceil(j/16) <= 16 (j <= 256) -- wider
// bases loop over column groups of 256.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(1024) void cgs_upd_proj_kernel(
    const T *__restrict__ Q, int64_t ldq, int64_t L, int j, const T *__restrict__ w,
    const T *__restrict__ h1, T *__restrict__ w1out, T *__restrict__ partials,
    T *__restrict__ h2, unsigned int *__restrict__ counter) {
  __shared__ T sh_h[CGS_MAXJ];
  __shared__ T part[16][WAVE];
  __shared__ int flag;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const int NW = blockDim.x / WAVE;
  const int G = gridDim.x;
  for (int c = tid; c < j; c += blockDim.x) sh_h[c] = h1[c];
  __syncthreads();
  const int64_t tiles = ceil_div(L, WAVE);
  const int64_t per = ceil_div(tiles, G);
  const int64_t t0 = static_cast<int64_t>(blockIdx.x) * per;
  const int64_t t1 = min(tiles, t0 + per);
  // Basis wider than the block's register tile: fall back to the generic
  // path below (two sweeps of the block's rows, still one launch).
  const bool tiled = j <= NW * CGS_CPW;
  if (tiled) {
    const int c0 = wv * CGS_CPW;
    const int nc = max(0, min(CGS_CPW, j - c0));
    T acc[CGS_CPW];
#pragma unroll
    for (int c = 0; c < CGS_CPW; ++c) acc[c] = 0;
    for (int64_t t = t0; t < t1; ++t) {
      const int64_t r = t * WAVE + lane;
      const bool valid = r < L;
      T q[CGS_CPW];
      T s = 0;
#pragma unroll
      for (int c = 0; c < CGS_CPW; ++c) {
        q[c] = (valid && c < nc) ? Q[(c0 + c) * ldq + r] : T(0);
        s += q[c] * sh_h[c0 + c < j ? c0 + c : 0];
      }
      part[wv][lane] = s;
      __syncthreads();
      T w1 = 0;
      if (valid) {
        T u = 0;
        for (int v = 0; v < NW; ++v) u += part[v][lane];
        w1 = w[r] - u;
        if (wv == 0) w1out[r] = w1;
      }
#pragma unroll
      for (int c = 0; c < CGS_CPW; ++c) acc[c] += q[c] * w1;
      __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < CGS_CPW; ++c) {
      const T s = wave_sum(acc[c]);
      if (lane == 0 && c < nc) partials[static_cast<int64_t>(c0 + c) * G + blockIdx.x] = s;
    }
  }
  if (!tiled) {
    // generic path: thread-per-row update, then column-chunked projection
    const int64_t r0 = t0 * WAVE, r1 = min(L, t1 * WAVE);
    for (int64_t r = r0 + tid; r < r1; r += blockDim.x) {
      T u = 0;
      for (int c = 0; c < j; ++c) u += Q[c * ldq + r] * sh_h[c];
      w1out[r] = w[r] - u;
    }
    __syncthreads();
    __threadfence_block();
    T *red = &part[0][0];
    for (int c0 = 0; c0 < j; c0 += CGS_CC) {
      const int nc = min(CGS_CC, j - c0);
      T acc[CGS_CC];
#pragma unroll
      for (int c = 0; c < CGS_CC; ++c) acc[c] = 0;
      for (int64_t r = r0 + tid; r < r1; r += blockDim.x) {
        const T x = w1out[r];
#pragma unroll
        for (int c = 0; c < CGS_CC; ++c)
          if (c < nc) acc[c] += Q[(c0 + c) * ldq + r] * x;
      }
#pragma unroll
      for (int c = 0; c < CGS_CC; ++c) {
        const T s = wave_sum(acc[c]);
        if (lane == 0) red[wv * CGS_CC + c] = s;
      }
      __syncthreads();
      if (tid < nc) {
        T s = 0;
        for (int v = 0; v < NW; ++v) s += red[v * CGS_CC + tid];
        partials[static_cast<int64_t>(c0 + tid) * G + blockIdx.x] = s;
      }
      __syncthreads();
    }
  }
  if (elect_last_block(counter, &flag)) reduce_partials(partials, j, h2);
}

// ---------------------------------------------------------------------------
// Pass 3: w2 = w1 - Q h (written to out), then, by mode:
//   MODE_UPDATE : nothing else (restart: u_{k+1} = A v_{k+1} - Uk rho, eq. (7))
//   MODE_NORM   : xs = 1 / |w2|                              (start vector)
//   MODE_LANCZOS: T entry = |w2|, xs = 1/|w2|, breakdown handling
// ---------------------------------------------------------------------------
enum { MODE_UPDATE = 0, MODE_NORM = 1, MODE_LANCZOS = 2 };

struct FinishArgs {
  double *t_entry;      // T(i,i) or T(i,i+1)
  double *xs;           // reciprocal norm of the stored vector
  double *sigma_est;    // running max of alpha, beta, sigma_1
  int *breakdowns;      // breakdown counter of the solve
  uint64_t seed;
};

// Single-block CGS2 of the Philox vector that replaces a vector lost to a
// breakdown: out <- normalize(CGS2(z, Q)).  Only the elected last block of
// cgs_upd_norm runs this, and only on breakdown.
template <typename T>
__device__ void breakdown_repair(const T *__restrict__ Q, int64_t ldq, int64_t L, int j,
                                 T *__restrict__ out, uint32_t stream, uint64_t seed,
                                 double *sh_d, T *sh_h) {
  const int tid = threadIdx.x;
  for (int64_t b = tid; 2 * b < L; b += blockDim.x) {
    double z0, z1;
    philox_normal_pair(seed, stream, static_cast<uint64_t>(b), z0, z1);
    out[2 * b] = static_cast<T>(z0);
    if (2 * b + 1 < L) out[2 * b + 1] = static_cast<T>(z1);
  }
  __threadfence_block();
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
    for (int c = 0; c < j; ++c) {
      T s = 0;
      for (int64_t r = tid; r < L; r += blockDim.x) s += Q[c * ldq + r] * out[r];
      s = block_sum(s, reinterpret_cast<T *>(sh_d));
      if (tid == 0) sh_h[c] = s;
    }
    __syncthreads();
    for (int64_t r = tid; r < L; r += blockDim.x) {
      T u = 0;
      for (int c = 0; c < j; ++c) u += Q[c * ldq + r] * sh_h[c];
      out[r] -= u;
    }
    __threadfence_block();
    __syncthreads();
  }
  double s = 0;
  for (int64_t r = tid; r < L; r += blockDim.x) s += static_cast<double>(out[r]) * out[r];
  s = block_sum(s, sh_d);
  const double inv = 1.0 / sqrt(s);
  for (int64_t r = tid; r < L; r += blockDim.x) out[r] = static_cast<T>(out[r] * inv);
  __threadfence_block();
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(CGS_THREADS) void cgs_upd_norm_kernel(
    const T *__restrict__ Q, int64_t ldq, int64_t L, int j, const T *__restrict__ w1,
    const T *__restrict__ h, T *__restrict__ out, double *__restrict__ partials,
    unsigned int *__restrict__ counter, int mode, FinishArgs fa) {
  __shared__ T sh_h[CGS_MAXJ];
  __shared__ double sh_d[CGS_THREADS / WAVE];
  __shared__ int flag;
  const int tid = threadIdx.x;
  for (int c = tid; c < j; c += CGS_THREADS) sh_h[c] = h[c];
  __syncthreads();
  int64_t r0, r1;
  block_slab(L, r0, r1);
  double nrm2 = 0;
  for (int64_t r = r0 + tid; r < r1; r += CGS_THREADS) {
    T u0 = 0, u1 = 0, u2 = 0, u3 = 0;
    int c = 0;
    for (; c + 4 <= j; c += 4) {
      u0 += Q[(c + 0) * ldq + r] * sh_h[c + 0];
      u1 += Q[(c + 1) * ldq + r] * sh_h[c + 1];
      u2 += Q[(c + 2) * ldq + r] * sh_h[c + 2];
      u3 += Q[(c + 3) * ldq + r] * sh_h[c + 3];
    }
    for (; c < j; ++c) u0 += Q[c * ldq + r] * sh_h[c];
    const T x = w1[r] - ((u0 + u1) + (u2 + u3));
    out[r] = x;
    nrm2 += static_cast<double>(x) * static_cast<double>(x);
  }
  if (mode == MODE_UPDATE) return;
  nrm2 = block_sum(nrm2, sh_d);
  if (tid == 0) partials[blockIdx.x] = nrm2;
  if (!elect_last_block(counter, &flag)) return;
  double tot = 0;
  if (tid == 0)
    for (int g = 0; g < static_cast<int>(gridDim.x); ++g) tot += partials[g];
  if (tid == 0) sh_d[0] = tot;
  __syncthreads();
  const double nrm = sqrt(sh_d[0]);
  __syncthreads();
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
    return;
  }
  // Breakdown: the new vector lies in the span of Q (an invariant subspace was
  // found).  Replace it by a re-orthogonalized random vector, store 0 in T.
  __shared__ int bd;
  if (tid == 0) {
    bd = *fa.breakdowns + 1;
    *fa.breakdowns = bd;
    *fa.t_entry = 0.0;
    *fa.xs = 1.0;
  }
  __syncthreads();
  breakdown_repair<T>(Q, ldq, L, j, out, static_cast<uint32_t>(bd), fa.seed, sh_d, sh_h);
}

}  // namespace svds
