// device.hpp -- device-side model description, key edits, hashing and the
// HBM hash table used by every stage of the step.
//
// Key layout (App. "Lossless bit-level compression of state information"):
// a basis state is a B-bit integer, occupations n_{i,nu} most significant
// first, exciton site j in the lowest bits.  It is stored in W 64-bit words
// per row, word 0 most significant, rows contiguous (the paper's table C).
// Kernels are instantiated for a compile-time word count so that keys live
// in registers; a runtime word index is resolved with unrolled selects,
// never by indexing a private array.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace paces {

constexpr int kMaxW = 16;   // up to 1024 key bits
constexpr int kMaxV = 4;    // modes per site
constexpr int kMaxD = 14;   // 2*3 hops + 2*4 exciton-phonon slots
constexpr int kBlock = 256;
constexpr uint64_t kEmpty = ~0ull;       // free hash slot
// Longest probe sequence an insert may take.  An insert that would go
// further latches kErrTableFull (the step is repeated with a larger
// table), so every key of a completed table lies within kMaxProbe slots of
// its home and a lookup can stop there.  At the load factors the host
// keeps (at most 1/2) sequences this long do not occur; when a set outgrows
// its estimate the table fills up and the latch fires early instead of
// after a walk through the whole table.
constexpr uint64_t kMaxProbe = 4096;
constexpr uint32_t kCand = 0x80000000u;  // ref names a candidate, not a row
constexpr uint32_t kNone = 0xFFFFFFFFu;  // no slot / no column
// Distance byte of a row that is a hole: a row of an in-place step's set
// whose state was dropped (no key in the table, amplitude 0, no columns,
// and no column of another row points at it).
constexpr uint8_t kHole = 0xFE;
constexpr int kGsqStride = 256;          // g*sqrt(n) table row length

// Device error latch bits.
enum : int {
  kErrTableFull = 1,
  kErrCapacity = 2,
  kErrNonFinite = 4,
  kErrTerms = 8,       // series longer than the allowed maximum
  kErrNeedTerms = 16,  // more series launches needed than enqueued
  kErrCap = 32,        // a realization's new set exceeds the state cap
  kErrChunks = 64,     // a round's frontier needs more candidate chunks
  kErrInput = 128,     // a given key is out of range or repeated
};

// Model constants passed by value to every kernel.
struct DevModel {
  int N, V, ndim, D, W, B, bj, P;
  int R, br;            // disorder realizations, bits of the realization id
  int bnu[kMaxV];       // bits per mode field
  int cut[kMaxV];       // occupation cutoffs
  int sub[kMaxV];       // offset of mode nu inside one site's bit group
  double omega[kMaxV];
  double J[3];
  uint64_t mul[kMaxW];  // odd multipliers of the key hash
  const int32_t* nbr;   // [N][2*ndim] hop targets, -1 if absent
  const double* gsq;    // [V][kGsqStride]: g_nu * sqrt(n)
  const double* eps;    // [R][N] site energies
  uint32_t hop_mask;    // bit a set iff J[a] != 0
  uint32_t eph_mask;    // bit nu set iff g[nu] != 0
};

// Per-row payload, one 64-bit word: exciton site j in bits 0..11, the
// occupation of each mode at the exciton site in 8-bit fields from bit 12,
// for at most two modes the total occupation T_nu of each mode in 14-bit
// fields from bit 28, and the realization id in bits 56..63.  With more
// modes the totals live in a second word per row (16 bits per mode).  The
// diagonal eps_j + sum_nu omega_nu T_nu is recomputed from these integers
// wherever it is needed.
__device__ __forceinline__ int pay_site(uint64_t p) { return int(p & 0xFFFu); }
__device__ __forceinline__ int pay_occ(uint64_t p, int nu) {
  return int((p >> (12 + 8 * nu)) & 0xFFu);
}
__device__ __forceinline__ int pay_real(uint64_t p) { return int(p >> 56); }
__device__ __forceinline__ int tot_of(uint64_t t, int nu) {
  return int((t >> (16 * nu)) & 0xFFFFu);
}
// Total occupation of mode nu: from the payload (V <= 2) or the totals word.
__device__ __forceinline__ int row_total(int V, uint64_t pay, uint64_t tot,
                                         int nu) {
  return V <= 2 ? int((pay >> (28 + 14 * nu)) & 0x3FFFu) : tot_of(tot, nu);
}
__device__ __forceinline__ uint64_t make_pay(int V, int j, const int* nj,
                                             const int* T, int r) {
  uint64_t p = uint64_t(j) | (uint64_t(r) << 56);
  for (int nu = 0; nu < V; ++nu) p |= uint64_t(nj[nu]) << (12 + 8 * nu);
  if (V <= 2)
    for (int nu = 0; nu < V; ++nu) p |= uint64_t(T[nu]) << (28 + 14 * nu);
  return p;
}
__device__ __forceinline__ uint64_t make_tot(int V, const int* T) {
  uint64_t t = 0;
  for (int nu = 0; nu < V; ++nu) t |= uint64_t(T[nu]) << (16 * nu);
  return t;
}

// Bit offset (from the least significant end) of field (site i, mode nu).
__device__ __forceinline__ int field_off(const DevModel& m, int i, int nu) {
  return m.bj + (m.N - 1 - i) * m.P + m.sub[nu];
}

template <int W>
__device__ __forceinline__ uint64_t word_at(const uint64_t (&k)[W], int w) {
  uint64_t v = 0;
#pragma unroll
  for (int q = 0; q < W; ++q)
    if (q == w) v = k[q];
  return v;
}

// Field of width <= 32 at bit offset off; may straddle two words.
template <int W>
__device__ __forceinline__ uint32_t get_field(const uint64_t (&k)[W], int off,
                                              int width) {
  const int w = W - 1 - (off >> 6), sh = off & 63;
  uint64_t v = word_at<W>(k, w) >> sh;
  if (sh + width > 64) v |= word_at<W>(k, w - 1) << (64 - sh);
  return uint32_t(v & ((uint64_t(1) << width) - 1));
}

// key +/- 2^off on the W-word integer.  The edited field never leaves its
// range, so a carry or borrow reaches at most the next word up.
template <int W>
__device__ __forceinline__ void add_pow2(uint64_t (&k)[W], int off,
                                         bool subtract) {
  const int w = W - 1 - (off >> 6);
  const uint64_t d = uint64_t(1) << (off & 63);
  bool carry = false;
#pragma unroll
  for (int q = 0; q < W; ++q)
    if (q == w) {
      const uint64_t old = k[q];
      k[q] = subtract ? old - d : old + d;
      carry = subtract ? (old < d) : (k[q] < old);
    }
#pragma unroll
  for (int q = 0; q < W; ++q)
    if (q == w - 1 && carry) k[q] = subtract ? k[q] - 1 : k[q] + 1;
}

template <int W>
__device__ __forceinline__ void load_key(const uint64_t* keys, int64_t row,
                                         uint64_t (&k)[W]) {
  const uint64_t* p = keys + row * W;
#pragma unroll
  for (int q = 0; q < W; ++q) k[q] = p[q];
}
template <int W>
__device__ __forceinline__ void store_key(uint64_t* keys, int64_t row,
                                          const uint64_t (&k)[W]) {
  uint64_t* p = keys + row * W;
#pragma unroll
  for (int q = 0; q < W; ++q) p[q] = k[q];
}
template <int W>
__device__ __forceinline__ bool key_eq(const uint64_t (&a)[W],
                                       const uint64_t* b) {
  bool eq = true;
#pragma unroll
  for (int q = 0; q < W; ++q) eq &= (a[q] == b[q]);
  return eq;
}

// Realization id of a key: the br bits above the B bits of the state.
template <int W>
__device__ __forceinline__ int key_real(const DevModel& m,
                                        const uint64_t (&k)[W]) {
  return m.br ? int(get_field<W>(k, m.B, m.br)) : 0;
}

// 64-bit hash: a multiply-add over the words followed by the murmur3
// 64-bit finalizer (Appleby, public domain).
__device__ __forceinline__ uint64_t fmix64(uint64_t h) {
  h ^= h >> 33;
  h *= 0xff51afd7ed558ccdull;
  h ^= h >> 33;
  h *= 0xc4ceb9fe1a85ec53ull;
  h ^= h >> 33;
  return h;
}
template <int W>
__device__ __forceinline__ uint64_t key_hash(const DevModel& m,
                                             const uint64_t (&k)[W]) {
  uint64_t L = 0;
#pragma unroll
  for (int q = 0; q < W; ++q) L += k[q] * m.mul[q];
  return fmix64(L);
}
__device__ __forceinline__ uint32_t hash_tag(uint64_t h) {
  const uint32_t t = uint32_t(h >> 32);
  return t == 0xFFFFFFFFu ? 0xFFFFFFFEu : t;  // never the empty pattern
}

// Slot s of a row: the neighbour key and the matrix element value.  Slot
// order: for each axis the +1 then the -1 hop; then for each mode the
// lowering then the raising term at the exciton site.  Returns false when
// the slot is structurally zero (J or g zero, a missing open-boundary
// neighbour, or an occupation at 0 / at the cutoff).
template <int W>
__device__ __forceinline__ bool slot_target(const DevModel& m,
                                            const uint64_t (&parent)[W],
                                            uint64_t pay, int s,
                                            uint64_t (&out)[W]) {
  const int j = pay_site(pay);
#pragma unroll
  for (int q = 0; q < W; ++q) out[q] = parent[q];
  if (s < 2 * m.ndim) {
    const int a = s >> 1;
    if (!((m.hop_mask >> a) & 1u)) return false;
    const int jn = m.nbr[j * 2 * m.ndim + s];
    if (jn < 0) return false;
    const uint64_t lowmask = (uint64_t(1) << m.bj) - 1;
    out[W - 1] = (out[W - 1] & ~lowmask) | uint64_t(jn);
    return true;
  }
  const int e = s - 2 * m.ndim, nu = e >> 1;
  const bool lower = (e & 1) == 0;
  if (!((m.eph_mask >> nu) & 1u)) return false;
  const int n = pay_occ(pay, nu);
  if (lower ? n == 0 : n >= m.cut[nu]) return false;
  add_pow2<W>(out, field_off(m, j, nu), lower);
  return true;
}

// Value of slot s for a row with payload pay (the slot must exist).
__device__ __forceinline__ double slot_value(const DevModel& m, uint64_t pay,
                                             int s) {
  if (s < 2 * m.ndim) return m.J[s >> 1];
  const int e = s - 2 * m.ndim, nu = e >> 1;
  const int n = pay_occ(pay, nu);
  return m.gsq[nu * kGsqStride + ((e & 1) ? n + 1 : n)];
}

// Payload and totals of the slot-s neighbour of a row.
template <int W>
__device__ __forceinline__ void slot_row_info(const DevModel& m,
                                              const uint64_t (&target)[W],
                                              uint64_t pay, uint64_t tot, int s,
                                              uint64_t& pay_out,
                                              uint64_t& tot_out) {
  int nj[kMaxV], T[kMaxV];
  for (int nu = 0; nu < m.V; ++nu) T[nu] = row_total(m.V, pay, tot, nu);
  int j = pay_site(pay);
  if (s < 2 * m.ndim) {
    j = int(target[W - 1] & ((uint64_t(1) << m.bj) - 1));
    for (int nu = 0; nu < m.V; ++nu)
      nj[nu] = int(get_field<W>(target, field_off(m, j, nu), m.bnu[nu]));
  } else {
    const int e = s - 2 * m.ndim, nu = e >> 1;
    const int delta = (e & 1) ? 1 : -1;
    for (int q = 0; q < m.V; ++q) nj[q] = pay_occ(pay, q);
    nj[nu] += delta;
    T[nu] += delta;
  }
  pay_out = make_pay(m.V, j, nj, T, pay_real(pay));
  tot_out = make_tot(m.V, T);
}

// Diagonal eps_j + sum_nu omega_nu * T_nu, evaluated in this order with
// separately rounded products (no contraction), as Eq. (holstein) reads
// term by term.
__device__ __forceinline__ double row_diag(const DevModel& m, uint64_t pay,
                                           uint64_t tot) {
#pragma clang fp contract(off)
  double d = m.eps[pay_real(pay) * m.N + pay_site(pay)];
  for (int nu = 0; nu < m.V; ++nu)
    d = d + m.omega[nu] * double(row_total(m.V, pay, tot, nu));
  return d;
}

// Look a key up in the table; returns its row or -1.
template <int W>
__device__ __forceinline__ int64_t table_find(const uint64_t* table,
                                              uint64_t mask,
                                              const uint64_t* keys,
                                              const uint64_t (&k)[W],
                                              uint64_t h) {
  const uint32_t tag = hash_tag(h);
  uint64_t i = h & mask;
  for (uint64_t probes = 0; probes <= mask && probes < kMaxProbe; ++probes) {
    const uint64_t e = table[i];
    if (e == kEmpty) return -1;
    if (uint32_t(e >> 32) == tag) {
      const uint32_t r = uint32_t(e);
      if (!(r & kCand) && key_eq<W>(k, keys + int64_t(r) * W)) return int64_t(r);
    }
    i = (i + 1) & mask;
  }
  return -1;
}

}  // namespace paces
