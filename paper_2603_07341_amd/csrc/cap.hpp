// cap.hpp -- state cap: when the new set of a realization would exceed the
// cap, its selection M is cut to the q heaviest rows in the order (weight
// descending, splitmix64 hash of the canonical key ascending, canonical key
// ascending) by an MSD radix select over 8-bit digits of that composite key
// (weight bits, then hash, then key words), one digit per pass, the host
// choosing the split digit of every realization between passes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace paces {

// Passes of the radix select for W canonical key words.
inline int cap_passes(int W) { return 16 + 8 * W; }

// Rows of the new set per realization into ball[R]; latches kErrCap when
// one exceeds cap.
void cap_check(const DevModel& m, const StepCtl* ctl, const uint64_t* pay,
               int64_t est, int64_t cap, uint32_t* ball, int* err,
               hipStream_t s);
// Rows of a set per realization (out[R], cleared first; eager use only:
// the clear is a memset).
void count_per_real(const DevModel& m, const uint64_t* pay, int64_t n,
                    uint32_t* out, hipStream_t s,
                    const uint32_t* idx = nullptr);
// p[i] = i for i < n.
void iota_u32(uint32_t* p, int64_t n, hipStream_t s);
// Per selected row j (row midx[j] of the old side): status 1 (kept) for
// realizations not capped, 0 (undecided) otherwise; the weight key and the
// tie-break hash.
void cap_prepare(const DevModel& m, int Wi, int W, int prec,
                 const uint32_t* midx, int64_t nM, const uint64_t* keys,
                 const uint64_t* pay, const void* psi, const int8_t* capped,
                 uint64_t* wkey, uint64_t* hkey, uint8_t* status,
                 hipStream_t s);
// Histogram hist[R][256] of digit `pass` over undecided rows.
void cap_hist(const DevModel& m, int Wi, int W, int pass, const uint32_t* midx,
              int64_t nM, const uint64_t* keys, const uint64_t* pay,
              const uint64_t* wkey, const uint64_t* hkey,
              const uint8_t* status, uint32_t* hist, hipStream_t s);
// Decide undecided rows of realization r by mode[r]:
//   0 skip; 1 digit < dstar kept, > dstar dropped, = dstar undecided;
//   2 digit <= dstar kept, > dstar dropped; 3 all dropped; 4 all kept.
enum : int32_t { kCapSkip = 0, kCapSplit = 1, kCapCut = 2, kCapDrop = 3,
                 kCapKeep = 4 };
void cap_apply(const DevModel& m, int Wi, int W, int pass,
               const uint32_t* midx, int64_t nM, const uint64_t* keys,
               const uint64_t* pay, const uint64_t* wkey,
               const uint64_t* hkey, const int32_t* mode,
               const int32_t* dstar, uint8_t* status, hipStream_t s);
// keep[midx[j]] = status[j] == 1 (keep cleared first over n_old rows).
void cap_flags(const uint32_t* midx, int64_t nM, const uint8_t* status,
               uint8_t* keep, int64_t n_old, hipStream_t s);

}  // namespace paces
