// common.hpp -- device helpers shared by the step kernels and the adjoint
// kernels: launch-shape helpers, grid-stride indices, deterministic wave and
// block reductions, Bessel functions of the first kind.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "kernels.hpp"

// Compile-time dispatch over the internal key word count and over the
// lattice shape (axes, modes per site).
#define PACES_DISPATCH_W(Wi, ...)                           \
  switch (Wi) {                                             \
    case 1: { constexpr int WW = 1; __VA_ARGS__; } break;   \
    case 2: { constexpr int WW = 2; __VA_ARGS__; } break;   \
    case 3: { constexpr int WW = 3; __VA_ARGS__; } break;   \
    case 4: { constexpr int WW = 4; __VA_ARGS__; } break;   \
    case 6: { constexpr int WW = 6; __VA_ARGS__; } break;   \
    case 8: { constexpr int WW = 8; __VA_ARGS__; } break;   \
    case 10: { constexpr int WW = 10; __VA_ARGS__; } break; \
    case 16: { constexpr int WW = 16; __VA_ARGS__; } break; \
    default: break;                                         \
  }

#define PACES_DISPATCH_SHAPE(ND, NV, ...)                        \
  switch ((ND) * 8 + (NV)) {                                     \
    case 9: { constexpr int A = 1, B = 1; __VA_ARGS__; } break;  \
    case 10: { constexpr int A = 1, B = 2; __VA_ARGS__; } break; \
    case 11: { constexpr int A = 1, B = 3; __VA_ARGS__; } break; \
    case 12: { constexpr int A = 1, B = 4; __VA_ARGS__; } break; \
    case 17: { constexpr int A = 2, B = 1; __VA_ARGS__; } break; \
    case 18: { constexpr int A = 2, B = 2; __VA_ARGS__; } break; \
    case 19: { constexpr int A = 2, B = 3; __VA_ARGS__; } break; \
    case 20: { constexpr int A = 2, B = 4; __VA_ARGS__; } break; \
    case 25: { constexpr int A = 3, B = 1; __VA_ARGS__; } break; \
    case 26: { constexpr int A = 3, B = 2; __VA_ARGS__; } break; \
    case 27: { constexpr int A = 3, B = 3; __VA_ARGS__; } break; \
    case 28: { constexpr int A = 3, B = 4; __VA_ARGS__; } break; \
    default: break;                                              \
  }

namespace paces {
namespace {

constexpr int kItems = 8;
constexpr int kTile = kBlock * kItems;
// Grid-stride kernels launch at most this many blocks (4M threads, several
// times what the 256 CUs hold): blocks beyond the work are dispatched only
// to exit, and with grids sized from a row estimate they cost the
// expansion rounds about a sixth of their time.
constexpr int kMaxGrid = 16384;
constexpr int kFold = 256;  // blocks of the second reduction level

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) {
  return (a + b - 1) / b;
}

// Grid for a grid-stride kernel over at most `bound` items.
inline int grid_for(int64_t bound, int64_t cap = kMaxGrid) {
  int64_t g = cdiv(bound, kBlock);
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return int(g);
}
// Launch of a kBlock-thread kernel on s.  With events the dispatch itself
// records its start and stop (no marker packets between launches), so
// timing a kernel costs no idle time on the stream.
template <typename... K, typename... A>
inline void launch_ev(void (*kern)(K...), int grid, hipStream_t s,
                      hipEvent_t ev_a, hipEvent_t ev_b, A... args) {
  if (ev_a)
    hipExtLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, s, ev_a, ev_b,
                          0u, K(args)...);
  else
    kern<<<grid, kBlock, 0, s>>>(K(args)...);
}

// Grid for a kernel striding over tiles of kTile items.
inline int tiles_for(int64_t bound) {
  int64_t g = cdiv(bound, kTile);
  if (g < 1) g = 1;
  if (g > 2048) g = 2048;
  return int(g);
}

// |c|^2 as fl(fl(re*re) + fl(im*im)) in FP64 (FP32 amplitudes widened
// first), compared with theta^2 and ranked by the truncation: the same
// predicate on every path.  HIP device code contracts a*b + c into an FMA
// by default (and __dmul_rn / __dadd_rn are plain operators there), which
// rounds once instead of twice and can reorder weights one ulp apart, so
// contraction is switched off here.
__device__ __forceinline__ double weight(double2 c) {
#pragma clang fp contract(off)
  return c.x * c.x + c.y * c.y;
}
__device__ __forceinline__ double weight(float2 c) {
#pragma clang fp contract(off)
  const double x = c.x, y = c.y;
  return x * x + y * y;
}
__device__ __forceinline__ double2 widen(double2 c) { return c; }
__device__ __forceinline__ double2 widen(float2 c) {
  return make_double2(c.x, c.y);
}

// Loads of streams read once per launch, with the non-temporal hint, so
// that they do not push the gathered vector out of the caches.
template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
  return __builtin_nontemporal_load(p);
}
__device__ __forceinline__ double2 ld_stream(const double2* p) {
  const double* q = reinterpret_cast<const double*>(p);
  return make_double2(__builtin_nontemporal_load(q),
                      __builtin_nontemporal_load(q + 1));
}
__device__ __forceinline__ float2 ld_stream(const float2* p) {
  const float* q = reinterpret_cast<const float*>(p);
  return make_float2(__builtin_nontemporal_load(q),
                     __builtin_nontemporal_load(q + 1));
}

// The D ELL columns of one row (row-major, D int32 per row), read as a
// stream with the widest aligned vector loads: rows start at multiples of
// 16 bytes for D % 4 == 0 and of 8 bytes for even D.
typedef int32_t v4i32 __attribute__((ext_vector_type(4)));
typedef int32_t v2i32 __attribute__((ext_vector_type(2)));
template <int D>
__device__ __forceinline__ void load_cols(const int32_t* row, int32_t (&c)[D]) {
  if constexpr (D % 4 == 0) {
#pragma unroll
    for (int q = 0; q < D / 4; ++q) {
      const v4i32 v = __builtin_nontemporal_load(
          reinterpret_cast<const v4i32*>(row) + q);
      c[4 * q] = v.x;
      c[4 * q + 1] = v.y;
      c[4 * q + 2] = v.z;
      c[4 * q + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int q = 0; q < D / 2; ++q) {
      const v2i32 v = __builtin_nontemporal_load(
          reinterpret_cast<const v2i32*>(row) + q);
      c[2 * q] = v.x;
      c[2 * q + 1] = v.y;
    }
  }
}

__device__ __forceinline__ int64_t gtid() {
  return int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
}
__device__ __forceinline__ int64_t gstride() {
  return int64_t(gridDim.x) * blockDim.x;
}

// ---- deterministic block reductions ---------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
// Sum over the block; every lane gets the result.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double s[kBlock / 64];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) s[wid] = v;
  __syncthreads();
  double r = 0;
  for (int w = 0; w < kBlock / 64; ++w) r += s[w];
  return r;
}
__device__ __forceinline__ double block_min(double v) {
  __shared__ double s[kBlock / 64];
  v = wave_min(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) s[wid] = v;
  __syncthreads();
  double r = s[0];
  for (int w = 1; w < kBlock / 64; ++w) r = fmin(r, s[w]);
  return r;
}
__device__ __forceinline__ double block_max(double v) {
  __shared__ double s[kBlock / 64];
  v = wave_max(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) s[wid] = v;
  __syncthreads();
  double r = s[0];
  for (int w = 1; w < kBlock / 64; ++w) r = fmax(r, s[w]);
  return r;
}

// Exclusive scan over the block of one u32 per lane; total to *tot.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v,
                                                    uint32_t* tot) {
  __shared__ uint32_t s[kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  __syncthreads();
  if (lane == 63) s[wid] = x;
  __syncthreads();
  uint32_t base = 0, all = 0;
  for (int w = 0; w < kBlock / 64; ++w) {
    if (w < wid) base += s[w];
    all += s[w];
  }
  *tot = all;
  return base + x - v;
}

// Per-realization integer counters (deterministic: integer sums commute):
// LDS bins per block, one global add per nonzero bin.
__device__ __forceinline__ void count_flush(int R, uint32_t* lds,
                                            uint32_t* global) {
  __syncthreads();
  for (int r = threadIdx.x; r < R; r += blockDim.x)
    if (lds[r]) atomicAdd(&global[r], lds[r]);
}

// J_k(x) by its power series sum_j (-1)^j (x/2)^(2j+k) / (j! (j+k)!); for
// x <= 2 every term shrinks and no cancellation occurs.
__device__ double bessel_series(double x, int k) {
  const double h = 0.5 * x, h2 = h * h;
  double lead = 1.0;
  for (int q = 1; q <= k; ++q) lead *= h / q;
  if (lead == 0.0) return 0.0;
  double term = lead, sum = lead;
  for (int j = 1; j < 60; ++j) {
    term *= -h2 / (double(j) * double(j + k));
    sum += term;
    if (fabs(term) <= 1e-18 * fabs(sum)) break;
  }
  return sum;
}

// J_0..J_kmax for x > 2: Miller's backward recurrence normalised by
// J_0 + 2 sum_k J_2k = 1 (Miller 1952; Abramowitz & Stegun 9.12).
__device__ void bessel_miller(double x, int kmax, double* out) {
  int start = kmax > int(x) ? kmax : int(x);
  start += 20 + int(sqrt(40.0 * start));
  start += start & 1;
  double fp1 = 0.0, f = 1e-280, norm = 0.0;
  for (int k = 0; k <= kmax; ++k) out[k] = 0.0;
  for (int k = start; k >= 0; --k) {
    if (k <= kmax) out[k] = f;
    if ((k & 1) == 0) norm += (k == 0 ? 1.0 : 2.0) * f;
    const double fm1 = (k > 0) ? (2.0 * k / x) * f - fp1 : 0.0;
    fp1 = f;
    f = fm1;
    if (fabs(f) > 1e250) {
      f *= 1e-250;
      fp1 *= 1e-250;
      norm *= 1e-250;
      for (int q = k; q <= kmax; ++q) out[q] *= 1e-250;
    }
  }
  for (int k = 0; k <= kmax; ++k) out[k] /= norm;
}

}  // namespace
}  // namespace paces
