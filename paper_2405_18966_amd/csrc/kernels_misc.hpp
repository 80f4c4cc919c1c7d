// Restart rotation (Alg. 2 steps 8 and 16: U(:,1:p) Uh(:,1:k),
// V(:,1:p) Vh(:,1:k)), start vector, sign normalization, norms and small
// helpers.
#pragma once
#include <algorithm>
#include <type_traits>

#include "common.hpp"

namespace svds {

// ---------------------------------------------------------------------------
// out(:, 0:kc) = B(:, 0:pc) * Y(0:pc, 0:kc), B L x pc (ld ldb), Y column-major
// FP64 (ld ldy), out L x kc (ld ldo).  Tall-skinny and bound by reading B:
// each thread owns one row of B and accumulates up to ROT_KC output columns
// in registers, so B is read once per group of ROT_KC columns (once for
// kc <= 64).  Y is first transposed into a row-major, zero-padded copy Yt;
// the kernel's loads of Yt are uniform across the wave (same q, same c) and
// compile to scalar loads, so no LDS is involved.  Accumulation in q order.
// The solver uses the matrix-core kernel below; this vector kernel is kept
// as the reference form (svds_op_rotate with its `vector` switch).
// ---------------------------------------------------------------------------
constexpr int ROT_THREADS = 256;
constexpr int ROT_KC = 64;  // output columns per launch

// row stride of Yt for kc columns: kc rounded up to 8, plus ROT_KC of zero
// padding so a launch for the last column group may read ROT_KC columns
__host__ __device__ inline int rot_ldyt(int kc) { return ((kc + 7) / 8) * 8 + ROT_KC; }
__host__ __device__ inline int64_t rot_yt_doubles(int pc, int kc) {
  return static_cast<int64_t>(pc) * rot_ldyt(kc);
}

static __global__ void rot_transpose_kernel(int pc, int kc, const double *__restrict__ Y, int64_t ldy,
                                            double *__restrict__ Yt, int ldyt) {
  const int64_t n = static_cast<int64_t>(pc) * ldyt;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int q = static_cast<int>(i / ldyt), c = static_cast<int>(i % ldyt);
    Yt[i] = c < kc ? Y[c * ldy + q] : 0.0;
  }
}

template <typename TB, typename TO, int KC>
static __global__ __launch_bounds__(ROT_THREADS) void rotate_kernel(int64_t L, int pc, int kcv,
                                                                    const TB *__restrict__ B, int64_t ldb,
                                                                    const double *__restrict__ Yt, int ldyt,
                                                                    TO *__restrict__ out, int64_t ldo) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * ROT_THREADS + threadIdx.x;
  if (r >= L) return;
  TB acc[KC];
#pragma unroll
  for (int c = 0; c < KC; ++c) acc[c] = TB(0);
  int q = 0;
  for (; q + 4 <= pc; q += 4) {
    TB b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) b[u] = B[static_cast<int64_t>(q + u) * ldb + r];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double *y = Yt + static_cast<int64_t>(q + u) * ldyt;
#pragma unroll
      for (int c = 0; c < KC; ++c) acc[c] += b[u] * static_cast<TB>(y[c]);
    }
  }
  for (; q < pc; ++q) {
    const TB bq = B[static_cast<int64_t>(q) * ldb + r];
    const double *y = Yt + static_cast<int64_t>(q) * ldyt;
#pragma unroll
    for (int c = 0; c < KC; ++c) acc[c] += bq * static_cast<TB>(y[c]);
  }
#pragma unroll
  for (int c = 0; c < KC; ++c)
    if (c < kcv) out[c * ldo + r] = static_cast<TO>(acc[c]);
}

// ---------------------------------------------------------------------------
// Rotation on the matrix cores: v_mfma_f64_16x16x4f64 for FP64 bases,
// v_mfma_f32_16x16x4f32 for FP32 bases (FP32 accumulation, as the vector
// kernel); D(16x16) += A(16x4) B(4x16).  A block of ROTM_WAVES waves covers
// 16 ROTM_WAVES rows of B; each wave owns one 16-row tile and NT 16-column
// tiles of out, and steps through pc four columns of B at a time (four steps
// per loop iteration, all their loads issued first): lane l loads
// A(l % 16, l / 16) = B(r0 + l % 16, q + l / 16) and the B-operand entries
// Yt(q + l / 16, 16 t + l % 16).  Accumulator entry i of lane l holds
// D(4 i + l / 16, l % 16) for FP64 and D(4 (l / 16) + i, l % 16) for FP32
// (both measured on gfx950 with one-hot A operands).  The tile is written
// back through LDS so that each store covers 16 consecutive rows of a
// column.  Out-of-range rows and k-steps read as 0.
// Measured on MI355X for a 1,000,000 x 150 FP64 basis and 50 columns: ~610
// us, the same rate as the one-row-per-thread vector kernel (the strided
// reads of B's row tiles, not the arithmetic, bound both); double-buffered
// loads and four row tiles per wave were slower.
// ---------------------------------------------------------------------------
constexpr int ROTM_WAVES = 4;
typedef double rot_v4d __attribute__((ext_vector_type(4)));
typedef float rot_v4f __attribute__((ext_vector_type(4)));

template <typename TB, typename TO, int NT>
static __global__ __launch_bounds__(ROTM_WAVES * WAVE) void rotate_mfma_kernel(
    int64_t L, int pc, int kcv, const TB *__restrict__ B, int64_t ldb, const double *__restrict__ Yt,
    int ldyt, TO *__restrict__ out, int64_t ldo) {
  constexpr bool F64 = sizeof(TB) == 8;
  using acc_t = typename std::conditional<F64, rot_v4d, rot_v4f>::type;
  __shared__ TB tile[ROTM_WAVES][16 * NT][17];  // [wave][column][row], padded
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  const int64_t r0 = (static_cast<int64_t>(blockIdx.x) * ROTM_WAVES + wv) * 16;
  const bool live = r0 < L;  // wave-uniform; every wave reaches the barrier
  const int li = lane & 15, lk = lane >> 4;
  const int64_t ra = r0 + li;
  const bool rin = ra < L;
  acc_t acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = acc_t{TB(0), TB(0), TB(0), TB(0)};
  for (int q = 0; live && q < pc; q += 16) {
    TB a[4], b[4][NT];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int qk = q + 4 * u + lk;
      const bool kin = qk < pc;
      a[u] = (rin && kin) ? B[static_cast<int64_t>(qk) * ldb + ra] : TB(0);
      const double *y = Yt + static_cast<int64_t>(kin ? qk : 0) * ldyt + li;
#pragma unroll
      for (int t = 0; t < NT; ++t) b[u][t] = kin ? static_cast<TB>(y[16 * t]) : TB(0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if constexpr (F64)
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u][t], acc[t], 0, 0, 0);
        else
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u], b[u][t], acc[t], 0, 0, 0);
      }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) tile[wv][16 * t + li][F64 ? 4 * i + lk : 4 * lk + i] = acc[t][i];
  __syncthreads();
  // lanes: row li of the tile, columns lk, lk + 4, ...
  const int64_t row = r0 + li;
  if (live && row < L)
    for (int c = lk; c < 16 * NT; c += 4)
      if (c < kcv) out[static_cast<int64_t>(c) * ldo + row] = static_cast<TO>(tile[wv][c][li]);
}

// Enqueues Yt = Y^T (padded) and the launches of all column groups.  Yt holds
// rot_yt_doubles(pc, kc) doubles of device scratch.  use_mfma: the matrix
// core kernel (default), else the vector kernel.
template <typename TB, typename TO>
inline hipError_t rotate_launch(hipStream_t st, int64_t L, int pc, int kc, const TB *B, int64_t ldb,
                                const double *Y, int64_t ldy, double *Yt, TO *out, int64_t ldo,
                                bool use_mfma = true) {
  const int ldyt = rot_ldyt(kc);
  hipLaunchKernelGGL(rot_transpose_kernel, dim3(static_cast<unsigned>(
                                               std::min<int64_t>(1024, ceil_div(rot_yt_doubles(pc, kc), 256)))),
                     dim3(256), 0, st, pc, kc, Y, ldy, Yt, ldyt);
  const unsigned g = static_cast<unsigned>(ceil_div(L, ROT_THREADS));
  for (int g0 = 0; g0 < kc; g0 += ROT_KC) {
    const int kcv = std::min(ROT_KC, kc - g0);
    const double *yt = Yt + g0;
    TO *o = out + g0 * ldo;
    if (use_mfma) {
      const dim3 gm(static_cast<unsigned>(ceil_div(L, 16 * ROTM_WAVES)));
#define ROTM_GO(NT)                                                                                          \
  hipLaunchKernelGGL((rotate_mfma_kernel<TB, TO, NT>), gm, dim3(ROTM_WAVES * WAVE), 0, st, L, pc, kcv, B, ldb, \
                     yt, ldyt, o, ldo)
      if (kcv <= 16) ROTM_GO(1);
      else if (kcv <= 32) ROTM_GO(2);
      else if (kcv <= 48) ROTM_GO(3);
      else ROTM_GO(4);
#undef ROTM_GO
      continue;
    }
#define ROT_GO(K)                                                                                         \
  hipLaunchKernelGGL((rotate_kernel<TB, TO, K>), dim3(g), dim3(ROT_THREADS), 0, st, L, pc, kcv, B, ldb, yt, \
                     ldyt, o, ldo)
    if (kcv <= 8) ROT_GO(8);
    else if (kcv <= 16) ROT_GO(16);
    else if (kcv <= 24) ROT_GO(24);
    else if (kcv <= 32) ROT_GO(32);
    else if (kcv <= 40) ROT_GO(40);
    else if (kcv <= 48) ROT_GO(48);
    else if (kcv <= 56) ROT_GO(56);
    else ROT_GO(64);
#undef ROT_GO
  }
  return hipGetLastError();
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

// Gather copy out[i] = x[idx[i]] (gather-rate reference for the sparse
// products: per entry it streams the same 12 bytes as the CSR product, a
// 4-byte index and an 8-byte value, plus the gather).  Entries are cut into
// segments (seg[0..nseg]) and each segment into chunks of GATHER_CHUNK; block
// b takes chunk b / nseg of segment b % nseg, so with nseg = 8 the blocks of
// one XCD gather one segment only, as the column-panel product's do.  Each
// thread keeps its 8 index loads, then its 8 gathers, in flight.
constexpr int GATHER_CHUNK = 2048;
static __global__ __launch_bounds__(256) void gather_copy_kernel(const int32_t *__restrict__ idx,
                                                                 const double *__restrict__ x,
                                                                 double *__restrict__ out, int nseg,
                                                                 const int64_t *__restrict__ seg) {
  const int g = static_cast<int>(blockIdx.x % nseg);
  const int64_t c = blockIdx.x / nseg;
  const int64_t start = seg[g] + c * GATHER_CHUNK;
  const int64_t end = min(start + GATHER_CHUNK, seg[g + 1]);
  if (start >= end) return;
  int32_t id[8];
  double v[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int64_t i = start + threadIdx.x + u * 256;
    id[u] = i < end ? idx[i] : -1;
  }
#pragma unroll
  for (int u = 0; u < 8; ++u) v[u] = id[u] >= 0 ? x[id[u]] : 0.0;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int64_t i = start + threadIdx.x + u * 256;
    if (i < end) out[i] = v[u];
  }
}

// Sign convention: flip (u_j, v_j) so the entry of v_j of largest magnitude
// (lowest index on ties) is positive.  Three steps over V (n x k):
//  absmax_partials_kernel  grid (nslab, k): max |v| and its first index per
//                          slab of SIGN_SLAB rows of a column;
//  sign_pick_kernel        one wave per column: the column's winner in slab
//                          order, sgn[j] = -1 if that entry is negative, and
//                          column j of Uk scaled by sgn[j] (so U = U_basis Uk
//                          formed afterwards carries the sign);
//  flip_cols_kernel        V(:, j) *= -1 where sgn[j] < 0 (other columns are
//                          not touched).
constexpr int SIGN_SLAB = 8192;
constexpr int SIGN_MAX_SLABS = 256;
__host__ __device__ inline int64_t sign_slab_rows(int64_t n) {
  return std::max<int64_t>(SIGN_SLAB, ceil_div(n, SIGN_MAX_SLABS));
}

static __global__ __launch_bounds__(256) void absmax_partials_kernel(int64_t n, int64_t slab,
                                                                     const double *__restrict__ V, int64_t ldv,
                                                                     double *__restrict__ pval,
                                                                     int64_t *__restrict__ pidx) {
  __shared__ double smax[256 / WAVE];
  __shared__ int64_t sidx[256 / WAVE];
  const int j = blockIdx.y, sl = blockIdx.x, nslab = gridDim.x;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const double *v = V + j * ldv;
  const int64_t i0 = sl * slab, i1 = std::min<int64_t>(n, i0 + slab);
  double best = -1.0;
  int64_t bi = INT64_MAX;
  for (int64_t i = i0 + tid; i < i1; i += 256) {
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
    pval[j * nslab + sl] = b;
    pidx[j * nslab + sl] = id;
  }
}

static __global__ __launch_bounds__(WAVE) void sign_pick_kernel(int nslab, const double *__restrict__ pval,
                                                                const int64_t *__restrict__ pidx,
                                                                const double *__restrict__ V, int64_t ldv,
                                                                int64_t n, double *__restrict__ sgn,
                                                                double *__restrict__ Uk, int p) {
  __shared__ double s_sign;
  const int j = blockIdx.x, lane = threadIdx.x;
  double best = -1.0;
  int64_t bi = INT64_MAX;
  for (int s = lane; s < nslab; s += WAVE) {
    const double b = pval[j * nslab + s];
    const int64_t id = pidx[j * nslab + s];
    if (b > best || (b == best && id < bi)) {
      best = b;
      bi = id;
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
    const double sg = (bi < n && V[j * ldv + bi] < 0) ? -1.0 : 1.0;
    sgn[j] = sg;
    s_sign = sg;
  }
  __syncthreads();
  const double sg = s_sign;
  if (sg < 0)
    for (int r = lane; r < p; r += WAVE) Uk[j * p + r] = -Uk[j * p + r];
}

static __global__ __launch_bounds__(256) void flip_cols_kernel(int64_t n, double *__restrict__ V, int64_t ldv,
                                                               const double *__restrict__ sgn) {
  const int j = blockIdx.y;
  if (!(sgn[j] < 0)) return;
  double *v = V + j * ldv;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * 256)
    v[i] = -v[i];
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
  double s = strided_sum(partials, static_cast<int>(threadIdx.x), n, 256, 0.0);
  s = block_sum(s, sh);
  if (threadIdx.x == 0) *out = sqrt(s);
}

}  // namespace svds
