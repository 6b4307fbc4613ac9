// cap.hip -- kernels of the state cap (top-q cut of the selection).
//
// The composite order is (weight descending, tie-break hash ascending,
// canonical key ascending).  Weight keys are the bit patterns of the
// non-negative FP64 weights complemented, so ascending integers are
// descending weights; the hash is the splitmix64 output function (Steele,
// Lea & Flood 2014) chained over the canonical key words, most significant
// first, from 0.  A radix select walks 8-bit digits of (weight key, hash,
// key words) from the top; rows of a realization are decided in bulk once
// their digit differs from the realization's split digit.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "cap.hpp"
#include "common.hpp"

namespace paces {

namespace {

__device__ __forceinline__ uint64_t splitmix_mix(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Canonical word w (0 = most significant) of an internal key: the last W
// internal words, with the bits at and above B (realization id) cleared.
template <int Wi>
__device__ __forceinline__ uint64_t canon_word(const uint64_t (&k)[Wi], int W,
                                               int B, int w) {
  uint64_t v = k[Wi - W + w];
  if (w == 0) {
    const int top = B - 64 * (W - 1);  // bits held by word 0
    if (top < 64) v &= (uint64_t(1) << top) - 1;
  }
  return v;
}

template <int Wi>
__device__ __forceinline__ int cap_digit(int pass, uint64_t wk, uint64_t hk,
                                         const uint64_t (&k)[Wi], int W,
                                         int B) {
  if (pass < 8) return int((wk >> (56 - 8 * pass)) & 255u);
  if (pass < 16) return int((hk >> (56 - 8 * (pass - 8))) & 255u);
  const int p = pass - 16, w = p >> 3, b = p & 7;
  return int((canon_word<Wi>(k, W, B, w) >> (56 - 8 * b)) & 255u);
}

__global__ void k_cap_zero(uint32_t* ball, int R, const int* err) {
  if (*err) return;
  for (int r = threadIdx.x; r < R; r += blockDim.x) ball[r] = 0;
}

__global__ void __launch_bounds__(kBlock)
    k_cap_count(DevModel m, const StepCtl* ctl, const uint64_t* pay,
                uint32_t* ball, const int* err) {
  __shared__ uint32_t bins[kMaxReal];
  if (*err) return;
  const int64_t n = ctl->n_new;
  if (m.R == 1) {
    if (gtid() == 0) ball[0] = uint32_t(n);
    return;
  }
  for (int r = threadIdx.x; r < m.R; r += blockDim.x) bins[r] = 0;
  __syncthreads();
  for (int64_t i = gtid(); i < n; i += gstride())
    atomicAdd(&bins[pay_real(pay[i])], 1u);
  __syncthreads();
  for (int r = threadIdx.x; r < m.R; r += blockDim.x)
    if (bins[r]) atomicAdd(&ball[r], bins[r]);
}

__global__ void __launch_bounds__(kBlock)
    k_count_real(DevModel m, const uint64_t* pay, const uint32_t* idx,
                 int64_t n, uint32_t* out) {
  __shared__ uint32_t bins[kMaxReal];
  for (int r = threadIdx.x; r < m.R; r += blockDim.x) bins[r] = 0;
  __syncthreads();
  for (int64_t i = gtid(); i < n; i += gstride())
    atomicAdd(&bins[pay_real(pay[idx ? int64_t(idx[i]) : i])], 1u);
  __syncthreads();
  for (int r = threadIdx.x; r < m.R; r += blockDim.x)
    if (bins[r]) atomicAdd(&out[r], bins[r]);
}

__global__ void __launch_bounds__(kBlock)
    k_iota_u32(uint32_t* p, int64_t n) {
  for (int64_t i = gtid(); i < n; i += gstride()) p[i] = uint32_t(i);
}

__global__ void k_cap_over(const uint32_t* ball, int R, int64_t cap,
                            int* err) {
  if (*err) return;
  bool over = false;
  for (int r = threadIdx.x; r < R; r += blockDim.x)
    if (int64_t(ball[r]) > cap) over = true;
  if (over) atomicOr(err, kErrCap);
}

template <int Wi, typename Amp>
__global__ void __launch_bounds__(kBlock)
    k_cap_prepare(DevModel m, int W, const uint32_t* midx, int64_t nM,
                  const uint64_t* keys, const uint64_t* pay, const Amp* psi,
                  const int8_t* capped, uint64_t* wkey, uint64_t* hkey,
                  uint8_t* status) {
  for (int64_t j = gtid(); j < nM; j += gstride()) {
    const int64_t i = midx[j];
    const int r = pay_real(pay[i]);
    if (!capped[r]) {
      status[j] = 1;
      continue;
    }
    status[j] = 0;
    wkey[j] = ~uint64_t(__double_as_longlong(weight(psi[i])));
    uint64_t k[Wi];
    load_key<Wi>(keys, i, k);
    uint64_t h = 0;
    for (int w = 0; w < W; ++w) h = splitmix_mix(h ^ canon_word<Wi>(k, W, m.B, w));
    hkey[j] = h;
  }
}

// Digit histogram of the open rows per realization.  Up to kLdsReal
// realizations the block counts in LDS and adds each nonzero bin once: the
// leading weight digits are shared by almost every row, and global atomics
// on those few bins serialise the whole pass.
constexpr int kLdsReal = 32;  // 32 * 256 counters = 32 KiB of LDS

template <int Wi>
__global__ void __launch_bounds__(kBlock)
    k_cap_hist(DevModel m, int W, int pass, const uint32_t* midx, int64_t nM,
               const uint64_t* keys, const uint64_t* pay,
               const uint64_t* wkey, const uint64_t* hkey,
               const uint8_t* status, uint32_t* hist) {
  __shared__ uint32_t bins[kLdsReal * 256];
  const bool lds = m.R <= kLdsReal;
  if (lds) {
    for (int q = threadIdx.x; q < m.R * 256; q += blockDim.x) bins[q] = 0;
    __syncthreads();
  }
  for (int64_t j = gtid(); j < nM; j += gstride()) {
    if (status[j] != 0) continue;
    const int64_t i = midx[j];
    uint64_t k[Wi] = {};
    if (pass >= 16) load_key<Wi>(keys, i, k);
    const int d = cap_digit<Wi>(pass, wkey[j], hkey[j], k, W, m.B);
    const int b = pay_real(pay[i]) * 256 + d;
    if (lds)
      atomicAdd(&bins[b], 1u);
    else
      atomicAdd(&hist[b], 1u);
  }
  if (lds) {
    __syncthreads();
    for (int q = threadIdx.x; q < m.R * 256; q += blockDim.x)
      if (bins[q]) atomicAdd(&hist[q], bins[q]);
  }
}

template <int Wi>
__global__ void __launch_bounds__(kBlock)
    k_cap_apply(DevModel m, int W, int pass, const uint32_t* midx,
                int64_t nM, const uint64_t* keys, const uint64_t* pay,
                const uint64_t* wkey, const uint64_t* hkey,
                const int32_t* mode, const int32_t* dstar, uint8_t* status) {
  for (int64_t j = gtid(); j < nM; j += gstride()) {
    if (status[j] != 0) continue;
    const int64_t i = midx[j];
    const int r = pay_real(pay[i]);
    const int md = mode[r];
    if (md == kCapSkip) continue;
    if (md == kCapDrop) {
      status[j] = 2;
      continue;
    }
    if (md == kCapKeep) {
      status[j] = 1;
      continue;
    }
    uint64_t k[Wi] = {};
    if (pass >= 16) load_key<Wi>(keys, i, k);
    const int d = cap_digit<Wi>(pass, wkey[j], hkey[j], k, W, m.B);
    const int ds = dstar[r];
    if (d < ds)
      status[j] = 1;
    else if (d > ds)
      status[j] = 2;
    else if (md == kCapCut)
      status[j] = 1;
  }
}

__global__ void __launch_bounds__(kBlock)
    k_cap_clear(uint8_t* keep, int64_t n) {
  for (int64_t i = gtid(); i < n; i += gstride()) keep[i] = 0;
}

__global__ void __launch_bounds__(kBlock)
    k_cap_flags(const uint32_t* midx, int64_t nM, const uint8_t* status,
                uint8_t* keep) {
  for (int64_t j = gtid(); j < nM; j += gstride())
    if (status[j] == 1) keep[midx[j]] = 1;
}

}  // namespace

void cap_check(const DevModel& m, const StepCtl* ctl, const uint64_t* pay,
               int64_t est, int64_t cap, uint32_t* ball, int* err,
               hipStream_t s) {
  k_cap_zero<<<1, kBlock, 0, s>>>(ball, m.R, err);
  const int g = m.R == 1 ? 1 : std::min(grid_for(est), 2048);
  k_cap_count<<<g, kBlock, 0, s>>>(m, ctl, pay, ball, err);
  k_cap_over<<<1, kBlock, 0, s>>>(ball, m.R, cap, err);
}

void count_per_real(const DevModel& m, const uint64_t* pay, int64_t n,
                    uint32_t* out, hipStream_t s, const uint32_t* idx) {
  (void)hipMemsetAsync(out, 0, size_t(m.R) * 4, s);
  if (n <= 0) return;
  k_count_real<<<std::min(grid_for(n), 2048), kBlock, 0, s>>>(m, pay, idx, n,
                                                              out);
}

void iota_u32(uint32_t* p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_iota_u32<<<grid_for(n), kBlock, 0, s>>>(p, n);
}

void cap_prepare(const DevModel& m, int Wi, int W, int prec,
                 const uint32_t* midx, int64_t nM, const uint64_t* keys,
                 const uint64_t* pay, const void* psi, const int8_t* capped,
                 uint64_t* wkey, uint64_t* hkey, uint8_t* status,
                 hipStream_t s) {
  if (nM <= 0) return;
  const int g = grid_for(nM);
  if (prec == 64) {
    PACES_DISPATCH_W(Wi, k_cap_prepare<WW, double2><<<g, kBlock, 0, s>>>(
                             m, W, midx, nM, keys, pay, (const double2*)psi,
                             capped, wkey, hkey, status));
  } else {
    PACES_DISPATCH_W(Wi, k_cap_prepare<WW, float2><<<g, kBlock, 0, s>>>(
                             m, W, midx, nM, keys, pay, (const float2*)psi,
                             capped, wkey, hkey, status));
  }
}

void cap_hist(const DevModel& m, int Wi, int W, int pass, const uint32_t* midx,
              int64_t nM, const uint64_t* keys, const uint64_t* pay,
              const uint64_t* wkey, const uint64_t* hkey,
              const uint8_t* status, uint32_t* hist, hipStream_t s) {
  if (nM <= 0) return;
  PACES_DISPATCH_W(Wi, k_cap_hist<WW><<<grid_for(nM), kBlock, 0, s>>>(
                           m, W, pass, midx, nM, keys, pay, wkey, hkey,
                           status, hist));
}

void cap_apply(const DevModel& m, int Wi, int W, int pass,
               const uint32_t* midx, int64_t nM, const uint64_t* keys,
               const uint64_t* pay, const uint64_t* wkey,
               const uint64_t* hkey, const int32_t* mode,
               const int32_t* dstar, uint8_t* status, hipStream_t s) {
  if (nM <= 0) return;
  PACES_DISPATCH_W(Wi, k_cap_apply<WW><<<grid_for(nM), kBlock, 0, s>>>(
                           m, W, pass, midx, nM, keys, pay, wkey, hkey, mode,
                           dstar, status));
}

void cap_flags(const uint32_t* midx, int64_t nM, const uint8_t* status,
               uint8_t* keep, int64_t n_old, hipStream_t s) {
  if (n_old > 0) k_cap_clear<<<grid_for(n_old), kBlock, 0, s>>>(keep, n_old);
  if (nM > 0)
    k_cap_flags<<<grid_for(nM), kBlock, 0, s>>>(midx, nM, status, keep);
}

}  // namespace paces
