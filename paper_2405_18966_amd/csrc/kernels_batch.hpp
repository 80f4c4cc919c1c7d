// Kernels of the batched solver: many independent problems advance through
// Alg. 2 in lockstep, every launch serving all of them.
//
// Layout.  The problems are stacked as one block-diagonal matrix; problem b
// owns rows [mo_b, mo_b + mp_b) of every U-side vector and rows
// [no_b, no_b + np_b) of every V-side vector, mp_b and np_b being m_b and
// n_b rounded up to BT = 256.  Padding rows are zero in A, in every basis
// vector and in every work vector, so they change no dot product or norm.
// A 256-row tile therefore belongs to exactly one problem (tile maps
// tile_inst); per-tile partial sums are added per problem in tile order
// (deterministic).  Problems that have converged are masked out (active[b]
// = 0): kernels skip their tiles, and the per-step kernels take a list of
// the active problems' tiles (tl, block i works on tile tl[i]) so that their
// grids shrink as problems freeze.  Per-problem FP64 scalars are arrays indexed by problem;
// the projected matrices are interleaved: entry (r, c) of problem b's T is
// T[(r (p+1) + c) B + b], so one pointer per entry serves every problem.
#pragma once
#include "common.hpp"
#include "kernels_cgs.hpp"

namespace svds {

constexpr int BT = 256;        // rows per tile; problem segments are multiples of BT
constexpr int BHJ = 64;        // widest basis of the batched CGS kernels (p + 1 <= 64)

struct BProb {
  int64_t mo, no;              // first row of the problem's U-side / V-side segment
  int32_t m, n;                // true sizes
  int32_t tu0, ntu, tv0, ntv;  // tile ranges of the segments
};

// per-problem tile range of one side
__device__ __forceinline__ void bside(const BProb &q, int side_v, int64_t &off, int32_t &len, int32_t &t0,
                                      int32_t &nt) {
  if (side_v) {
    off = q.no, len = q.n, t0 = q.tv0, nt = q.ntv;
  } else {
    off = q.mo, len = q.m, t0 = q.tu0, nt = q.ntu;
  }
}

// part[c][tile] = sum over the tile's rows of Q[r, c] w[r], c < j.
template <typename T>
__global__ __launch_bounds__(BT) void bproj_kernel(const T *__restrict__ Q, int64_t ldq, int j,
                                                  const T *__restrict__ w, const int32_t *__restrict__ tile_inst,
                                                  const int32_t *__restrict__ active, const int32_t *__restrict__ tl,
                                                  int64_t ntiles, T *__restrict__ part) {
  __shared__ T red[BT / WAVE][BHJ];
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const int64_t tile = tl ? tl[blockIdx.x] : blockIdx.x;
  if (!active[tile_inst[tile]]) return;
  const int64_t r = tile * BT + tid;
  const T wr = w[r];
  for (int c0 = 0; c0 < j; c0 += 8) {
    T v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = (c0 + i < j) ? Q[(c0 + i) * ldq + r] * wr : T(0);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const T s = wave_sum(v[i]);
      if (lane == 0 && c0 + i < j) red[wv][c0 + i] = s;
    }
  }
  __syncthreads();
  if (tid < j) {
    T s = 0;
#pragma unroll
    for (int v = 0; v < BT / WAVE; ++v) s += red[v][tid];
    part[tid * ntiles + tile] = s;
  }
}

// h[b * hs + c] = sum over the problem's tiles of part[c][tile] (tile order).
template <typename T>
__global__ void bseg_sum_kernel(const T *__restrict__ part, int64_t ntiles, int j, const BProb *__restrict__ pr,
                                int side_v, const int32_t *__restrict__ active, T *__restrict__ h, int hs) {
  const int b = blockIdx.x, c = threadIdx.x;
  if (c >= j || !active[b]) return;
  int64_t off;
  int32_t len, t0, nt;
  bside(pr[b], side_v, off, len, t0, nt);
  // tile order; 8 loads in flight
  T s = 0;
  int t = 0;
  for (; t + 8 <= nt; t += 8) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[c * ntiles + t0 + t + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; t < nt; ++t) s += part[c * ntiles + t0 + t];
  h[static_cast<int64_t>(b) * hs + c] = s;
}

// w1 = w - Q h[problem] (written), part[c][tile] = sum of Q[r, c] w1[r].
// The row's j basis entries stay in registers between the two uses (JM >= j).
template <typename T, int JM>
__global__ __launch_bounds__(BT) void bupd_proj_kernel(const T *__restrict__ Q, int64_t ldq, int j,
                                                      const T *__restrict__ w, const T *__restrict__ h, int hs,
                                                      const int32_t *__restrict__ tile_inst,
                                                      const int32_t *__restrict__ active,
                                                      const int32_t *__restrict__ tl, int64_t ntiles,
                                                      T *__restrict__ w1out, T *__restrict__ part) {
  __shared__ T sh[BHJ];
  __shared__ T red[BT / WAVE][BHJ];
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const int64_t tile = tl ? tl[blockIdx.x] : blockIdx.x;
  const int inst = tile_inst[tile];
  if (!active[inst]) return;
  if (tid < j) sh[tid] = h[static_cast<int64_t>(inst) * hs + tid];
  __syncthreads();
  const int64_t r = tile * BT + tid;
  T q[JM];
  T u = 0;
#pragma unroll
  for (int c = 0; c < JM; ++c) {
    q[c] = c < j ? Q[c * ldq + r] : T(0);
    u += q[c] * (c < j ? sh[c] : T(0));
  }
  const T w1 = w[r] - u;
  w1out[r] = w1;
#pragma unroll
  for (int c = 0; c < JM; ++c) {
    if (c < j) {  // uniform
      const T s = wave_sum(q[c] * w1);
      if (lane == 0) red[wv][c] = s;
    }
  }
  __syncthreads();
  if (tid < j) {
    T s = 0;
#pragma unroll
    for (int v = 0; v < BT / WAVE; ++v) s += red[v][tid];
    part[tid * ntiles + tile] = s;
  }
}

// out = w1 - Q h[problem]; with npart, npart[tile] = sum of out^2 (FP64).
template <typename T>
__global__ __launch_bounds__(BT) void bupd_norm_kernel(const T *__restrict__ Q, int64_t ldq, int j,
                                                      const T *__restrict__ w1, const T *__restrict__ h, int hs,
                                                      const int32_t *__restrict__ tile_inst,
                                                      const int32_t *__restrict__ active,
                                                      const int32_t *__restrict__ tl,
                                                      T *__restrict__ out, double *__restrict__ npart) {
  __shared__ T sh[BHJ];
  __shared__ double shd[BT / WAVE];
  const int tid = threadIdx.x;
  const int64_t tile = tl ? tl[blockIdx.x] : blockIdx.x;
  const int inst = tile_inst[tile];
  if (!active[inst]) return;
  if (tid < j) sh[tid] = h[static_cast<int64_t>(inst) * hs + tid];
  __syncthreads();
  const int64_t r = tile * BT + tid;
  T u[4] = {0, 0, 0, 0};
  int c = 0;
  for (; c + 4 <= j; c += 4) {
#pragma unroll
    for (int i = 0; i < 4; ++i) u[i] += Q[(c + i) * ldq + r] * sh[c + i];
  }
  for (; c < j; ++c) u[0] += Q[c * ldq + r] * sh[c];
  const T x = w1[r] - ((u[0] + u[1]) + (u[2] + u[3]));
  out[r] = x;
  if (!npart) return;
  const double s = block_sum(static_cast<double>(x) * static_cast<double>(x), shd);
  if (tid == 0) npart[tile] = s;
}

// Per problem: |out| from the tile partials, then as finish_norm_kernel:
//   MODE_NORM   : xs[b] = 1 / |w|
//   MODE_LANCZOS: T entry (interleaved, t_entry[b]) = |w|, xs[b] = 1/|w|,
//                 sigma_est[b] update; on breakdown the problem's true rows
//                 of out are replaced by a re-orthogonalized Philox vector
//                 (seed + b, stream 1 + breakdowns) and T entry = 0, xs = 1.
template <typename T>
__global__ __launch_bounds__(CGS_THREADS) void bfinish_norm_kernel(
    const double *__restrict__ npart, const BProb *__restrict__ pr, int side_v, const int32_t *__restrict__ active,
    int mode, double *__restrict__ t_entry, double *__restrict__ xs, double *__restrict__ sigma_est,
    int *__restrict__ breakdowns, uint64_t seed, const T *__restrict__ Q, int64_t ldq, int j,
    T *__restrict__ out) {
  __shared__ double sh_d[CGS_THREADS / WAVE];
  __shared__ T sh_h[CGS_MAXJ];
  __shared__ int bd;
  const int b = blockIdx.x, tid = threadIdx.x;
  if (!active[b]) return;
  int64_t off;
  int32_t len, t0, nt;
  bside(pr[b], side_v, off, len, t0, nt);
  double tot = strided_sum(npart + t0, tid, nt, CGS_THREADS, 0.0);
  tot = block_sum(tot, sh_d);
  const double nrm = sqrt(tot);
  if (mode == MODE_NORM) {
    if (tid == 0) xs[b] = 1.0 / nrm;
    return;
  }
  const double sig = sigma_est[b];
  if (nrm > BREAKDOWN_REL * sig) {
    if (tid == 0) {
      t_entry[b] = nrm;
      xs[b] = 1.0 / nrm;
      sigma_est[b] = fmax(sig, nrm);
    }
    return;
  }
  if (tid == 0) {
    bd = breakdowns[b] + 1;
    breakdowns[b] = bd;
    t_entry[b] = 0.0;
    xs[b] = 1.0;
  }
  __syncthreads();
  breakdown_repair<T>(Q + off, ldq, len, j, out + off, static_cast<uint32_t>(bd), seed + b, sh_d, sh_h);
}

// Start vectors: problem b's true rows from Philox stream 0 of seed + b (or
// from the caller's unpadded concatenation v0, problem b at v0o[b]); padding 0.
template <typename T>
__global__ void bstart_kernel(int64_t Ntot, const int32_t *__restrict__ tile_inst_v, const BProb *__restrict__ pr,
                              uint64_t seed, const double *__restrict__ v0, const int64_t *__restrict__ v0o,
                              T *__restrict__ out) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < Ntot;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int b = tile_inst_v[i / BT];
    const int64_t loc = i - pr[b].no;
    T v = 0;
    if (loc < pr[b].n) {
      if (v0) {
        v = static_cast<T>(v0[v0o[b] + loc]);
      } else {
        double z0, z1;
        philox_normal_pair(seed + b, 0u, static_cast<uint64_t>(loc >> 1), z0, z1);
        v = static_cast<T>((loc & 1) ? z1 : z0);
      }
    }
    out[i] = v;
  }
}

// Per-problem scaled copy: dst[i] = src[i] * xs[problem of i].
template <typename T>
__global__ void bscale_copy_kernel(int64_t L, const int32_t *__restrict__ tile_inst,
                                   const int32_t *__restrict__ active, const T *__restrict__ src,
                                   const double *__restrict__ xs, T *__restrict__ dst) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < L;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int b = tile_inst[i / BT];
    if (active[b]) dst[i] = src[i] * static_cast<T>(xs[b]);
  }
}

// Problems flagged in `freeze` stop: their restart panels become the identity
// (Uk_b = [I_k; 0], Vext_b = [I_k 0; 0 1] in its leading columns), so every
// later rotation copies their first k basis columns, which the restart that
// preceded hold their Ritz vectors; active[b] = 0.
static __global__ void bfreeze_kernel(int nb, const int32_t *__restrict__ freeze, int32_t *__restrict__ active,
                                      double *__restrict__ Uk, double *__restrict__ Vext, int p, int k) {
  const int b = blockIdx.x;
  if (b >= nb || !freeze[b]) return;
  double *u = Uk + static_cast<int64_t>(b) * p * k;
  double *v = Vext + static_cast<int64_t>(b) * (p + 1) * (k + 1);
  for (int i = threadIdx.x; i < p * k; i += blockDim.x) u[i] = (i % p == i / p) ? 1.0 : 0.0;
  for (int i = threadIdx.x; i < (p + 1) * (k + 1); i += blockDim.x) {
    const int r = i % (p + 1), c = i / (p + 1);
    v[i] = (c < k) ? (r == c ? 1.0 : 0.0) : (r == p ? 1.0 : 0.0);
  }
  if (threadIdx.x == 0) active[b] = 0;
}

// Yt_b = Y_b^T zero-padded (row stride ldyt), for every problem b:
// Y_b = Y + b * ys (column-major, ld ldy), Yt_b = Yt + b * yts.
static __global__ void brot_transpose_kernel(int nb, int pc, int kc, const double *__restrict__ Y, int64_t ys,
                                             int64_t ldy, double *__restrict__ Yt, int64_t yts, int ldyt) {
  const int64_t per = static_cast<int64_t>(pc) * ldyt;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < per * nb;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int b = static_cast<int>(i / per);
    const int64_t e = i - b * per;
    const int q = static_cast<int>(e / ldyt), c = static_cast<int>(e % ldyt);
    Yt[b * yts + e] = c < kc ? Y[b * ys + c * ldy + q] : 0.0;
  }
}

// out(:, 0:kcv) = B(:, 0:pc) Y_problem for every row of the stacked basis (one
// tile per block: the problem's panel Yt_b is uniform across the block and is
// read with scalar loads).  Rows of one thread accumulate in q order.
template <typename TB, typename TO, int KC>
__global__ __launch_bounds__(BT) void brotate_kernel(int pc, int kcv, const TB *__restrict__ B, int64_t ldb,
                                                    const double *__restrict__ Yt, int64_t yts, int ldyt,
                                                    const int32_t *__restrict__ tile_inst, TO *__restrict__ out,
                                                    int64_t ldo) {
  const int64_t tile = blockIdx.x;
  const int inst = tile_inst[tile];
  const double *Y = Yt + inst * yts;
  const int64_t r = tile * BT + threadIdx.x;
  TB acc[KC];
#pragma unroll
  for (int c = 0; c < KC; ++c) acc[c] = TB(0);
  for (int q = 0; q < pc; ++q) {
    const TB bq = B[q * ldb + r];
    const double *y = Y + static_cast<int64_t>(q) * ldyt;
#pragma unroll
    for (int c = 0; c < KC; ++c) acc[c] += bq * static_cast<TB>(y[c]);
  }
#pragma unroll
  for (int c = 0; c < KC; ++c)
    if (c < kcv) out[c * ldo + r] = static_cast<TO>(acc[c]);
}

// Signs per problem and output column (one block each): the entry of largest
// magnitude of V_b(:, c) (lowest index on ties) made positive; the column of
// V (stacked, ld ldv) is flipped in place and column c of Uk_b scaled alike.
static __global__ __launch_bounds__(256) void bsign_kernel(const BProb *__restrict__ pr, double *__restrict__ V,
                                                           int64_t ldv, double *__restrict__ Uk, int p, int k) {
  __shared__ double smax[256 / WAVE];
  __shared__ int64_t sidx[256 / WAVE];
  __shared__ double s_sg;
  const int c = blockIdx.x, b = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  double *v = V + c * ldv + pr[b].no;
  const int64_t n = pr[b].n;
  double best = -1.0;
  int64_t bi = INT64_MAX;
  for (int64_t i = tid; i < n; i += 256) {
    const double a = fabs(v[i]);
    if (a > best) {
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
    double bb = smax[0];
    int64_t id = sidx[0];
    for (int w = 1; w < 256 / WAVE; ++w)
      if (smax[w] > bb || (smax[w] == bb && sidx[w] < id)) {
        bb = smax[w];
        id = sidx[w];
      }
    s_sg = (id < n && v[id] < 0) ? -1.0 : 1.0;
  }
  __syncthreads();
  if (s_sg < 0) {
    for (int64_t i = tid; i < n; i += 256) v[i] = -v[i];
    double *u = Uk + (static_cast<int64_t>(b) * k + c) * p;
    for (int i = tid; i < p; i += 256) u[i] = -u[i];
  }
}

// Per-problem copy of the stacked outputs into the caller's buffers:
// dst_b(r, c) = src(off_b + r, c) for r < len_b, c < k.
static __global__ void bcopy_out_kernel(const BProb *__restrict__ pr, int side_v, int k, const double *__restrict__ src,
                                        int64_t lds, double *const *__restrict__ dst) {
  const int b = blockIdx.y;
  int64_t off;
  int32_t len, t0, nt;
  bside(pr[b], side_v, off, len, t0, nt);
  double *d = dst[b];
  const int64_t tot = static_cast<int64_t>(len) * k;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < tot;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t c = i / len, r = i - c * len;
    d[c * len + r] = src[c * lds + off + r];
  }
}

// npart[tile] = sum of x^2 over the tile (FP64).
template <typename T>
__global__ __launch_bounds__(BT) void btile_sq_kernel(const T *__restrict__ x, double *__restrict__ npart) {
  __shared__ double shd[BT / WAVE];
  const int64_t r = static_cast<int64_t>(blockIdx.x) * BT + threadIdx.x;
  const double v = static_cast<double>(x[r]);
  const double s = block_sum(v * v, shd);
  if (threadIdx.x == 0) npart[blockIdx.x] = s;
}

// out[b * os] = sqrt(sum of the problem's tile partials) (tile order).
static __global__ void bseg_norm_kernel(const double *__restrict__ npart, const BProb *__restrict__ pr, int side_v,
                                        double *__restrict__ out, int os) {
  __shared__ double sh_d[CGS_THREADS / WAVE];
  const int b = blockIdx.x;
  int64_t off;
  int32_t len, t0, nt;
  bside(pr[b], side_v, off, len, t0, nt);
  double tot = strided_sum(npart + t0, static_cast<int>(threadIdx.x), nt, CGS_THREADS, 0.0);
  tot = block_sum(tot, sh_d);
  if (threadIdx.x == 0) out[static_cast<int64_t>(b) * os] = sqrt(tot);
}

// Per-problem scalar gather: dst[b] = src[b * ss] (e.g. sigma_j of every problem).
static __global__ void bgather_kernel(int nb, const double *__restrict__ src, int64_t ss, double *__restrict__ dst) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nb) dst[b] = src[b * ss];
}

}  // namespace svds
