// Shared device/host helpers of the HIP implementation (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <cstdint>
#include <cstddef>

namespace svds {

constexpr int WAVE = 64;

// ---------------------------------------------------------------------------
// Error handling: every HIP call in host code goes through HIP_TRY, which
// returns SVDS_EDEVICE from the enclosing int-returning function.
// ---------------------------------------------------------------------------
#define HIP_TRY(expr)                                                         \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess) {                                                   \
      ::svds::set_last_error(e_, #expr, __FILE__, __LINE__);                  \
      return SVDS_EDEVICE;                                                    \
    }                                                                         \
  } while (0)

void set_last_error(hipError_t e, const char *what, const char *file, int line);
const char *last_error_text();

// ---------------------------------------------------------------------------
// Value loads: every stored type widens exactly to the accumulation type.
// ---------------------------------------------------------------------------
template <typename Acc, typename V> __device__ __forceinline__ Acc widen(V v) {
  return static_cast<Acc>(v);
}
template <> __device__ __forceinline__ float widen<float, uint16_t>(uint16_t b) {
  return __uint_as_float(static_cast<uint32_t>(b) << 16);
}
template <> __device__ __forceinline__ double widen<double, uint16_t>(uint16_t b) {
  return static_cast<double>(__uint_as_float(static_cast<uint32_t>(b) << 16));
}

// ---------------------------------------------------------------------------
// Reductions.  Block sums combine waves in index order; all reductions in
// this library are deterministic (no float atomics).
//
// Full-wave sums run in a fixed order with the result held in a scalar
// register, so every lane sees the same bits by construction (a plain xor
// butterfly does not guarantee that: the compiler may fuse the caller's
// product into the first butterfly add, so partners round differently, and
// the Jacobi rotation test branches on such sums).  DPP steps: swap lanes
// within quads (xor 1, xor 2), mirror half-rows and rows (row sums in all 16
// lanes), then row_bcast:15 / row_bcast:31 accumulate the four row sums into
// row 3; lane 63 holds the total and is read out.  Every lane of the wave
// must be active at the call.  No LDS traffic is involved.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return static_cast<uint32_t>(
      __builtin_amdgcn_update_dpp(0, static_cast<int>(v), CTRL, ROW_MASK, 0xF, false));
}
template <int CTRL, int ROW_MASK = 0xF> __device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t u = static_cast<uint64_t>(__double_as_longlong(v));
  const uint32_t lo = dpp_u32<CTRL, ROW_MASK>(static_cast<uint32_t>(u));
  const uint32_t hi = dpp_u32<CTRL, ROW_MASK>(static_cast<uint32_t>(u >> 32));
  return __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(hi) << 32) | lo));
}
template <int CTRL, int ROW_MASK = 0xF> __device__ __forceinline__ float dpp_f32(float v) {
  return __uint_as_float(dpp_u32<CTRL, ROW_MASK>(__float_as_uint(v)));
}
__device__ __forceinline__ double wave_sum_u(double v) {
  v += dpp_f64<0xB1>(v);        // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);        // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);       // row_half_mirror
  v += dpp_f64<0x140>(v);       // row_mirror
  v += dpp_f64<0x142, 0xA>(v);  // row_bcast:15 -> rows 1, 3
  v += dpp_f64<0x143, 0xC>(v);  // row_bcast:31 -> rows 2, 3
  const uint64_t u = static_cast<uint64_t>(__double_as_longlong(v));
  const uint32_t lo = __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(u)), WAVE - 1);
  const uint32_t hi = __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(u >> 32)), WAVE - 1);
  return __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(hi) << 32) | lo));
}
__device__ __forceinline__ float wave_sum_u(float v) {
  v += dpp_f32<0xB1>(v);
  v += dpp_f32<0x4E>(v);
  v += dpp_f32<0x141>(v);
  v += dpp_f32<0x140>(v);
  v += dpp_f32<0x142, 0xA>(v);
  v += dpp_f32<0x143, 0xC>(v);
  return __uint_as_float(static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(__float_as_uint(v)), WAVE - 1)));
}
template <typename T> __device__ __forceinline__ T wave_sum(T v) { return wave_sum_u(v); }

// s + p[i0] + p[i0 + stride] + ... over i < n, added in increasing i.  The
// loads are issued 16 at a time before their adds: partial sums are read
// straight after the kernel that wrote them, from L2 or beyond, and one load
// per dependent add would pay that latency once per entry.
template <typename T>
__device__ __forceinline__ T strided_sum(const T *__restrict__ p, int i0, int n, int stride, T s) {
  constexpr int U = 16;
  for (; i0 < n; i0 += U * stride) {
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = i0 + u * stride < n ? p[i0 + u * stride] : T(0);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i0 + u * stride < n) s += v[u];
  }
  return s;
}

// Sum over each row of 16 lanes (DPP rows): quad swaps, half-row and row
// mirrors.  Every add combines two values in both orders on the two lanes
// involved, so all 16 lanes of a row end with the same bits.  Every lane of
// the wave must be active.
__device__ __forceinline__ double row16_sum(double v) {
  v = __dadd_rn(v, dpp_f64<0xB1>(v));   // quad_perm [1,0,3,2]
  v = __dadd_rn(v, dpp_f64<0x4E>(v));   // quad_perm [2,3,0,1]
  v = __dadd_rn(v, dpp_f64<0x141>(v));  // row_half_mirror
  v = __dadd_rn(v, dpp_f64<0x140>(v));  // row_mirror
  return v;
}


// Sum over the block; result valid in every thread.  `sh` holds >= 16 T.
template <typename T> __device__ __forceinline__ T block_sum(T v, T *sh) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  const int nw = (blockDim.x + WAVE - 1) / WAVE;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  T s = 0;
  for (int i = 0; i < nw; ++i) s += sh[i];
  __syncthreads();
  return s;
}

__host__ __device__ __forceinline__ int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and the library's normal
// vector encoding: block b of stream q under seed s gives two normals by
// Box-Muller from counter (b_lo, b_hi, q, 0), key (s_lo, s_hi).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c[0];
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c[2];
    const uint32_t hi0 = static_cast<uint32_t>(p0 >> 32), lo0 = static_cast<uint32_t>(p0);
    const uint32_t hi1 = static_cast<uint32_t>(p1 >> 32), lo1 = static_cast<uint32_t>(p1);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__device__ __forceinline__ void philox_normal_pair(uint64_t seed, uint32_t stream, uint64_t block,
                                                   double &z0, double &z1) {
  uint32_t c[4] = {static_cast<uint32_t>(block), static_cast<uint32_t>(block >> 32), stream, 0u};
  philox4x32_10(c, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
  const uint64_t a = ((static_cast<uint64_t>(c[1]) << 32) | c[0]) >> 11;
  const uint64_t b = ((static_cast<uint64_t>(c[3]) << 32) | c[2]) >> 11;
  const double u1 = (static_cast<double>(a) + 1.0) * 0x1.0p-53;
  const double u2 = static_cast<double>(b) * 0x1.0p-53;
  const double rad = sqrt(-2.0 * log(u1));
  double s, co;
  sincos(2.0 * 3.141592653589793238462643383279502884 * u2, &s, &co);
  z0 = rad * co;
  z1 = rad * s;
}

}  // namespace svds
