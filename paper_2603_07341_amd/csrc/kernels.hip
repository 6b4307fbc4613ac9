// kernels.hip -- HIP kernels of one co-evolving-subspace step on gfx950.
//
// The step is sparse, memory-bound gather/scatter: every kernel streams
// rows with one row (or one row slot) per lane, wave64, 256-lane blocks,
// and no matrix cores.  Reductions are deterministic: fixed lane-to-row
// mapping, wave shuffles in a fixed order, and per-block partials summed in
// block order by a single block.
//
// Stages (paper: Sec. "Formal operator representation and notes on
// parallelization"):
//   select     rows of psi with |c|^2 >= theta^2, compacted in row order
//              (Sec. "Truncation & post-adaptation detruncation")
//   expand     k rounds of neighbour generation on packed keys with
//              insert-if-absent into an HBM hash table (Eqs. (def_neighbor_k),
//              (H_eff)); candidates resolve duplicates by the smallest
//              candidate id, so the row order is deterministic
//   transfer   old amplitudes moved to their rows in the new set, weight of
//              the dropped rows summed (post-adaptation detruncation)
//   build      ELL columns come out of the expansion; values are implied by
//              the slot and the row payload (Sec. "Generating the effective
//              Hamiltonian from the effective Hilbert space")
//   propagate  exp(-i H dt) phi by a Chebyshev series evaluated with
//              Clenshaw's recurrence, one fused SpMV kernel per term
//              (App. "The action of the exponential of a sparse matrix"
//              names series of SpMVs; Chebyshev replaces Taylor here)
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.hpp"

namespace paces {

namespace {

constexpr int kItems = 8;
constexpr int kTile = kBlock * kItems;

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline int grid_for(int64_t n, int64_t cap = 1 << 20) {
  int64_t g = cdiv(n, kBlock);
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return int(g);
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

// ---- fills ------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
    k_fill_u64(uint64_t* p, int64_t n, uint64_t v) {
  for (int64_t i = gtid(); i < n; i += gstride()) p[i] = v;
}
__global__ void __launch_bounds__(kBlock)
    k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t i = gtid(); i < n; i += gstride()) p[i] = v;
}
__global__ void __launch_bounds__(kBlock) k_iota_u32(uint32_t* p, int64_t n) {
  for (int64_t i = gtid(); i < n; i += gstride()) p[i] = uint32_t(i);
}

// ---- scan -------------------------------------------------------------------
// Tile t covers elements [t*kTile, (t+1)*kTile); lane l of the block owns the
// kItems consecutive elements starting at t*kTile + l*kItems.
__global__ void __launch_bounds__(kBlock)
    k_scan_reduce(const uint32_t* in, int64_t n, uint32_t* bsum) {
  const int64_t base = int64_t(blockIdx.x) * kTile + threadIdx.x * kItems;
  uint32_t v = 0;
#pragma unroll
  for (int q = 0; q < kItems; ++q)
    if (base + q < n) v += in[base + q];
  uint32_t tot;
  block_excl_scan(v, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Single block: exclusive scan of nb block sums in place, grand total out.
__global__ void __launch_bounds__(kBlock)
    k_scan_bsum(uint32_t* bsum, int64_t nb, uint32_t* total) {
  uint32_t carry = 0;
  for (int64_t c = 0; c < nb; c += kTile) {
    const int64_t base = c + threadIdx.x * kItems;
    uint32_t loc[kItems];
    uint32_t v = 0;
#pragma unroll
    for (int q = 0; q < kItems; ++q) {
      loc[q] = (base + q < nb) ? bsum[base + q] : 0u;
      v += loc[q];
    }
    uint32_t tot;
    uint32_t off = block_excl_scan(v, &tot) + carry;
#pragma unroll
    for (int q = 0; q < kItems; ++q) {
      if (base + q < nb) bsum[base + q] = off;
      off += loc[q];
    }
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ void __launch_bounds__(kBlock)
    k_scan_apply(const uint32_t* in, int64_t n, const uint32_t* bsum,
                 uint32_t* out) {
  const int64_t base = int64_t(blockIdx.x) * kTile + threadIdx.x * kItems;
  uint32_t loc[kItems];
  uint32_t v = 0;
#pragma unroll
  for (int q = 0; q < kItems; ++q) {
    loc[q] = (base + q < n) ? in[base + q] : 0u;
    v += loc[q];
  }
  uint32_t tot;
  uint32_t off = block_excl_scan(v, &tot) + bsum[blockIdx.x];
#pragma unroll
  for (int q = 0; q < kItems; ++q) {
    if (base + q < n) out[base + q] = off;
    off += loc[q];
  }
}

// ---- select -----------------------------------------------------------------
// |c|^2 as fl(fl(re*re) + fl(im*im)) in FP64 (FP32 amplitudes widened
// first), compared with theta^2: the same predicate on every path.
__device__ __forceinline__ double weight(double2 c) {
  return __dadd_rn(__dmul_rn(c.x, c.x), __dmul_rn(c.y, c.y));
}
__device__ __forceinline__ double weight(float2 c) {
  const double x = c.x, y = c.y;
  return __dadd_rn(__dmul_rn(x, x), __dmul_rn(y, y));
}

template <typename Amp>
__global__ void __launch_bounds__(kBlock)
    k_select_count(const Amp* psi, int64_t n, double th2, uint32_t* bsum) {
  const int64_t base = int64_t(blockIdx.x) * kTile + threadIdx.x * kItems;
  uint32_t v = 0;
#pragma unroll
  for (int q = 0; q < kItems; ++q)
    if (base + q < n && weight(psi[base + q]) >= th2) ++v;
  uint32_t tot;
  block_excl_scan(v, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

template <typename Amp>
__global__ void __launch_bounds__(kBlock)
    k_select_write(const Amp* psi, int64_t n, double th2, const uint32_t* bsum,
                   uint32_t* midx) {
  const int64_t base = int64_t(blockIdx.x) * kTile + threadIdx.x * kItems;
  bool keep[kItems];
  uint32_t v = 0;
#pragma unroll
  for (int q = 0; q < kItems; ++q) {
    keep[q] = base + q < n && weight(psi[base + q]) >= th2;
    v += keep[q] ? 1u : 0u;
  }
  uint32_t tot;
  uint32_t off = block_excl_scan(v, &tot) + bsum[blockIdx.x];
#pragma unroll
  for (int q = 0; q < kItems; ++q)
    if (keep[q]) midx[off++] = uint32_t(base + q);
}

// ---- row metadata from keys -------------------------------------------------
template <int W>
__global__ void __launch_bounds__(kBlock)
    k_row_info(DevModel m, const uint64_t* keys, int64_t n, uint64_t* pay,
               uint64_t* tot, double* diag) {
  for (int64_t r = gtid(); r < n; r += gstride()) {
    uint64_t k[W];
    load_key<W>(keys, r, k);
    const int j = int(k[W - 1] & ((uint64_t(1) << m.bj) - 1));
    int nj[kMaxV];
    uint64_t t = 0;
    for (int nu = 0; nu < m.V; ++nu) {
      nj[nu] = int(get_field<W>(k, field_off(m, j, nu), m.bnu[nu]));
      uint32_t T = 0;
      for (int i = 0; i < m.N; ++i)
        T += get_field<W>(k, field_off(m, i, nu), m.bnu[nu]);
      t |= uint64_t(T) << (16 * nu);
    }
    const uint64_t p = make_pay(j, nj, m.V);
    pay[r] = p;
    tot[r] = t;
    diag[r] = row_diag(m, p, t);
  }
}

// ---- insert the selected rows as rows 0..nM-1 of the new set ----------------
template <int W>
__global__ void __launch_bounds__(kBlock)
    k_insert_rows(DevModel m, const uint64_t* keys_o, const uint64_t* pay_o,
                  const uint64_t* tot_o, const double* diag_o,
                  const uint32_t* midx, int64_t nM, uint64_t* keys_n,
                  uint64_t* pay_n, uint64_t* tot_n, double* diag_n,
                  uint64_t* table, uint64_t mask, int* err) {
  for (int64_t i = gtid(); i < nM; i += gstride()) {
    const int64_t r = midx[i];
    uint64_t k[W];
    load_key<W>(keys_o, r, k);
    store_key<W>(keys_n, i, k);
    pay_n[i] = pay_o[r];
    tot_n[i] = tot_o[r];
    diag_n[i] = diag_o[r];
    const uint64_t h = key_hash<W>(m, k);
    const uint64_t mine = (uint64_t(hash_tag(h)) << 32) | uint64_t(i);
    uint64_t s = h & mask;
    bool done = false;
    for (uint64_t p = 0; p <= mask; ++p) {
      if (table[s] == kEmpty && atomicCAS((unsigned long long*)(table + s),
                                          (unsigned long long)kEmpty,
                                          (unsigned long long)mine) == kEmpty) {
        done = true;
        break;
      }
      s = (s + 1) & mask;
    }
    if (!done) atomicOr(err, kErrTableFull);
  }
}

// ---- expansion round --------------------------------------------------------
// Candidate c = (parent f0 + c / D, slot c % D) of the current chunk.
//
// Probe: insert-if-absent.  A slot holds (tag << 32 | ref); ref is a row of
// the new set or, during the round, kCand | candidate id.  Candidates with
// equal keys meet in one slot and keep the smallest candidate id (atomicMin:
// equal keys share the tag, so the minimum is over the id).  Entries only
// move EMPTY -> CAND(x) -> CAND(y < x) inside this kernel, so a stale read is
// repaired by the compare-and-swap or is harmless.
template <int W>
__global__ void __launch_bounds__(kBlock)
    k_expand_probe(DevModel m, const uint64_t* keys, const uint64_t* pay,
                   int64_t f0, int64_t rows, uint64_t* table, uint64_t mask,
                   uint32_t* c_slot, uint32_t* c_ref, int* err) {
  const int D = m.D;
  const int64_t nc = rows * D;
  for (int64_t c = gtid(); c < nc; c += gstride()) {
    const int64_t p = f0 + c / D;
    const int s = int(c % D);
    uint64_t par[W], k[W];
    load_key<W>(keys, p, par);
    const uint64_t py = pay[p];
    if (!slot_target<W>(m, par, py, s, k)) {
      c_slot[c] = kNone;
      c_ref[c] = kNone;
      continue;
    }
    const uint64_t h = key_hash<W>(m, k);
    const uint32_t tag = hash_tag(h);
    const uint64_t mine = (uint64_t(tag) << 32) | uint64_t(kCand | uint32_t(c));
    uint64_t i = h & mask;
    uint32_t rslot = kNone, rref = kNone;
    for (uint64_t probes = 0; probes <= mask; ++probes) {
      uint64_t e = table[i];
      if (e == kEmpty) {
        const uint64_t old = atomicCAS((unsigned long long*)(table + i),
                                       (unsigned long long)kEmpty,
                                       (unsigned long long)mine);
        if (old == kEmpty) {
          rslot = uint32_t(i);
          rref = kCand;
          break;
        }
        e = old;
      }
      if (uint32_t(e >> 32) == tag) {
        const uint32_t r = uint32_t(e);
        bool same;
        if (r & kCand) {
          const int64_t c2 = int64_t(r & ~kCand);
          uint64_t par2[W], k2[W];
          load_key<W>(keys, f0 + c2 / D, par2);
          slot_target<W>(m, par2, pay[f0 + c2 / D], int(c2 % D), k2);
          same = true;
#pragma unroll
          for (int q = 0; q < W; ++q) same &= (k2[q] == k[q]);
        } else {
          same = key_eq<W>(k, keys + int64_t(r) * W);
        }
        if (same) {
          if (r & kCand) {
            atomicMin((unsigned long long*)(table + i),
                      (unsigned long long)mine);
            rslot = uint32_t(i);
            rref = kCand;
          } else {
            rref = r;
          }
          break;
        }
      }
      i = (i + 1) & mask;
    }
    if (rref == kNone) atomicOr(err, kErrTableFull);
    c_slot[c] = rslot;
    c_ref[c] = rref;
  }
}

// Resolve each pending candidate to its owner; count owners per parent.
__global__ void __launch_bounds__(kBlock)
    k_expand_resolve(int D, int64_t rows, const uint64_t* table,
                     const uint32_t* c_slot, uint32_t* c_ref,
                     uint32_t* rowcnt) {
  for (int64_t p = gtid(); p < rows; p += gstride()) {
    uint32_t cnt = 0;
    for (int s = 0; s < D; ++s) {
      const int64_t c = p * D + s;
      if (c_ref[c] != kCand) continue;
      const uint32_t owner = uint32_t(table[c_slot[c]]) & ~kCand;
      c_ref[c] = kCand | owner;
      if (int64_t(owner) == c) ++cnt;
    }
    rowcnt[p] = cnt;
  }
}

// Owners append their key as a new row (numbered in candidate order), fix
// the table slot to point at the row, and fill the parents' columns.
template <int W, typename Amp>
__global__ void __launch_bounds__(kBlock)
    k_expand_commit(DevModel m, uint64_t* keys, uint64_t* pay, uint64_t* tot,
                    double* diag, int64_t f0, int64_t rows, int64_t n_cur,
                    uint64_t* table, const uint32_t* c_slot,
                    const uint32_t* c_ref, const uint32_t* rowbase,
                    uint32_t* crow, int32_t* col, int64_t stride, Amp* phi) {
  const int D = m.D;
  for (int64_t pl = gtid(); pl < rows; pl += gstride()) {
    const int64_t p = f0 + pl;
    uint64_t par[W];
    load_key<W>(keys, p, par);
    const uint64_t py = pay[p], pt = tot[p];
    uint32_t run = 0;
    for (int s = 0; s < D; ++s) {
      const int64_t c = pl * D + s;
      const uint32_t r = c_ref[c];
      if (r == kNone) {
        col[int64_t(s) * stride + p] = -1;
      } else if (r & kCand) {
        if (int64_t(r & ~kCand) != c) continue;  // linked afterwards
        const int64_t row = n_cur + rowbase[pl] + run++;
        uint64_t k[W];
        slot_target<W>(m, par, py, s, k);
        store_key<W>(keys, row, k);
        uint64_t np, nt;
        slot_row_info<W>(m, k, py, pt, s, np, nt);
        pay[row] = np;
        tot[row] = nt;
        diag[row] = row_diag(m, np, nt);
        const uint64_t e = table[c_slot[c]];
        table[c_slot[c]] = (e & 0xFFFFFFFF00000000ull) | uint64_t(row);
        crow[c] = uint32_t(row);
        col[int64_t(s) * stride + p] = int32_t(row);
        Amp z;
        z.x = 0;
        z.y = 0;
        phi[row] = z;
      } else {
        col[int64_t(s) * stride + p] = int32_t(r);
      }
    }
  }
}

__global__ void __launch_bounds__(kBlock)
    k_expand_link(int D, int64_t f0, int64_t rows, const uint32_t* c_ref,
                  const uint32_t* crow, int32_t* col, int64_t stride) {
  const int64_t nc = rows * D;
  for (int64_t c = gtid(); c < nc; c += gstride()) {
    const uint32_t r = c_ref[c];
    if (r == kNone || !(r & kCand)) continue;
    const uint32_t owner = r & ~kCand;
    if (int64_t(owner) == c) continue;
    col[int64_t(c % D) * stride + f0 + c / D] = int32_t(crow[owner]);
  }
}

template <int W>
__global__ void __launch_bounds__(kBlock)
    k_lookup_cols(DevModel m, const uint64_t* keys, const uint64_t* pay,
                  int64_t f0, int64_t rows, const uint64_t* table,
                  uint64_t mask, int32_t* col, int64_t stride) {
  const int D = m.D;
  const int64_t nc = rows * D;
  for (int64_t c = gtid(); c < nc; c += gstride()) {
    const int64_t p = f0 + c / D;
    const int s = int(c % D);
    uint64_t par[W], k[W];
    load_key<W>(keys, p, par);
    int32_t out = -1;
    if (slot_target<W>(m, par, pay[p], s, k))
      out = int32_t(table_find<W>(table, mask, keys, k, key_hash<W>(m, k)));
    col[int64_t(s) * stride + p] = out;
  }
}

// ---- transfer ---------------------------------------------------------------
__device__ __forceinline__ double2 widen(double2 c) { return c; }
__device__ __forceinline__ double2 widen(float2 c) {
  return make_double2(c.x, c.y);
}

template <int W, typename Amp>
__global__ void __launch_bounds__(kBlock)
    k_transfer(DevModel m, const uint64_t* keys_o, const Amp* psi_o,
               int64_t n_old, const uint64_t* table, uint64_t mask,
               const uint64_t* keys_n, Amp* phi, double* mass_part) {
  double lost = 0;
  for (int64_t i = gtid(); i < n_old; i += gstride()) {
    uint64_t k[W];
    load_key<W>(keys_o, i, k);
    const int64_t r = table_find<W>(table, mask, keys_n, k, key_hash<W>(m, k));
    const Amp v = psi_o[i];
    if (r >= 0)
      phi[r] = v;
    else
      lost += weight(v);
  }
  lost = block_sum(lost);
  if (threadIdx.x == 0) mass_part[blockIdx.x] = lost;
}

// ---- Gershgorin bounds and Chebyshev coefficients ---------------------------
__global__ void __launch_bounds__(kBlock)
    k_bounds(DevModel m, const uint64_t* pay, const double* diag,
             const int32_t* col, int64_t stride, int64_t n, double* part) {
  double lo = INFINITY, hi = -INFINITY;
  for (int64_t r = gtid(); r < n; r += gstride()) {
    const uint64_t p = pay[r];
    double rad = 0;
    for (int s = 0; s < m.D; ++s)
      if (col[int64_t(s) * stride + r] >= 0) rad += fabs(slot_value(m, p, s));
    const double d = diag[r];
    lo = fmin(lo, d - rad);
    hi = fmax(hi, d + rad);
  }
  lo = block_min(lo);
  hi = block_max(hi);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = lo;
    part[2 * blockIdx.x + 1] = hi;
  }
}

// J_k(x), k = 0..kmax: power series for x <= 2 (all terms shrink, no
// cancellation), Miller's backward recurrence normalised by
// J_0 + 2 sum_k J_2k = 1 above (Miller 1952; see Abramowitz & Stegun 9.12).
__device__ void bessel_j(double x, int kmax, double* out) {
  for (int k = 0; k <= kmax; ++k) out[k] = 0.0;
  if (x == 0.0) {
    out[0] = 1.0;
    return;
  }
  if (x <= 2.0) {
    const double h = 0.5 * x, h2 = h * h;
    double lead = 1.0;  // (x/2)^k / k!
    for (int k = 0; k <= kmax; ++k) {
      if (k > 0) lead *= h / k;
      if (lead == 0.0) break;
      double term = lead, sum = lead;
      for (int j = 1; j < 60; ++j) {
        term *= -h2 / (double(j) * double(j + k));
        sum += term;
        if (fabs(term) <= 1e-18 * fabs(sum)) break;
      }
      out[k] = sum;
    }
    return;
  }
  int start = kmax > int(x) ? kmax : int(x);
  start += 20 + int(sqrt(40.0 * start));
  start += start & 1;  // even
  double fp1 = 0.0, f = 1e-280, norm = 0.0;
  for (int k = start; k >= 0; --k) {
    if (k <= kmax) out[k] = f;
    if ((k & 1) == 0) norm += (k == 0 ? 1.0 : 2.0) * f;
    const double fm1 = (k > 0) ? (2.0 * k / x) * f - fp1 : 0.0;
    fp1 = f;
    f = fm1;
    if (fabs(f) > 1e250) {  // rescale everything kept so far
      f *= 1e-250;
      fp1 *= 1e-250;
      norm *= 1e-250;
      for (int q = k; q <= kmax; ++q) out[q] *= 1e-250;
    }
  }
  for (int k = 0; k <= kmax; ++k) out[k] /= norm;
}

__global__ void __launch_bounds__(kBlock)
    k_coef(const double* part, int nparts, double dt, double tol, int k_max,
           ChebCoef* cc, int* err) {
  double lo = INFINITY, hi = -INFINITY;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
    lo = fmin(lo, part[2 * i]);
    hi = fmax(hi, part[2 * i + 1]);
  }
  lo = block_min(lo);
  hi = block_max(hi);
  if (threadIdx.x != 0) return;
  if (lo > hi) lo = hi = 0.0;  // empty set
  // widen by 1e-12 of the magnitude so the interval strictly contains the
  // spectrum
  const double pad = 1e-12 * (fabs(hi) + fabs(lo));
  const double emin = lo - pad, emax = hi + pad;
  double a = 0.5 * (emax - emin);
  const double b = 0.5 * (emax + emin);
  if (!(a > 1e-300)) a = 1e-300;
  cc->emin = emin;
  cc->emax = emax;
  cc->a = a;
  cc->b = b;
  cc->alpha = 1.0 / a;
  cc->beta = -b / a;
  double sn, cs;
  sincos(b * dt, &sn, &cs);
  cc->phase[0] = cs;
  cc->phase[1] = -sn;
  double J[kMaxTerms + 1];
  int kcap = k_max < kMaxTerms ? k_max : kMaxTerms;
  bessel_j(a * dt, kcap, J);
  const double thresh = ldexp(tol, -8);
  int K = 1;
  for (int k = 0; k <= kcap; ++k)
    if (fabs(J[k]) > thresh) K = k + 1;
  if (K > kcap) {
    atomicOr(err, kErrTerms);
    K = kcap;
  }
  cc->K = K;
  for (int k = 0; k < K; ++k) {
    const double v = (k == 0 ? 1.0 : 2.0) * J[k];
    // (-i)^k
    const int q = k & 3;
    cc->c[k][0] = (q == 0) ? v : (q == 2 ? -v : 0.0);
    cc->c[k][1] = (q == 1) ? -v : (q == 3 ? v : 0.0);
  }
}

// ---- Clenshaw term ----------------------------------------------------------
// For the series y = sum_{k<K} c_k T_k(H~) phi, Clenshaw's recurrence runs
// b_k = c_k phi + 2 H~ b_{k+1} - b_{k+2} from k = K-1 down to 1 and ends with
// y = c_0 phi + H~ b_1 - b_2.  One launch computes
//   out = c[ck] phi + fac * s_in * H~(in) - s_prev * prev
// with H~ = alpha H + beta, H applied as an ELL SpMV whose values follow
// from the slot and the row payload.  Compared with the forward
// three-term recurrence plus an accumulator this streams one vector less
// per term.
template <typename R>
struct VecT;
template <>
struct VecT<double> {
  using T = double2;
};
template <>
struct VecT<float> {
  using T = float2;
};

template <typename R, int ND, int NV>
__global__ void __launch_bounds__(kBlock)
    k_cheb_term(DevModel m, int64_t n, const int32_t* __restrict__ col,
                int64_t stride, const uint64_t* __restrict__ pay,
                const double* __restrict__ diag,
                const ChebCoef* __restrict__ cc, TermArgs ta,
                const typename VecT<R>::T* __restrict__ phi,
                const typename VecT<R>::T* __restrict__ in,
                const typename VecT<R>::T* prev, typename VecT<R>::T* out,
                double* e_part, double* n2_part, double* pop_part) {
  using Amp = typename VecT<R>::T;
  constexpr int D = 2 * ND + 2 * NV;
  extern __shared__ double pop_lds[];
  const R alpha = R(cc->alpha), beta = R(cc->beta);
  const R ckr = R(cc->c[ta.ck][0]), cki = R(cc->c[ta.ck][1]);
  R sir = R(ta.fac), sii = 0;
  if (ta.in_coef >= 0) {
    sir = R(ta.fac * cc->c[ta.in_coef][0]);
    sii = R(ta.fac * cc->c[ta.in_coef][1]);
  }
  R spr = 1, spi = 0;
  if (ta.prev_coef >= 0) {
    spr = R(cc->c[ta.prev_coef][0]);
    spi = R(cc->c[ta.prev_coef][1]);
  }
  const R phr = R(cc->phase[0]), phi_i = R(cc->phase[1]);
  R jv[3], gv[NV][2];
#pragma unroll
  for (int a = 0; a < ND; ++a) jv[a] = R(m.J[a]);
  if (ta.final_)
    for (int j = threadIdx.x; j < m.N; j += blockDim.x) pop_lds[j] = 0.0;
  if (ta.final_) __syncthreads();
  double esum = 0, n2 = 0;
  for (int64_t i = gtid(); i < n; i += gstride()) {
    const Amp xi = in[i];
    const uint64_t p = pay[i];
    const R d = R(diag[i]);
    R hr = d * xi.x, hi = d * xi.y;
#pragma unroll
    for (int nu = 0; nu < NV; ++nu) {
      const int occ = pay_occ(p, nu);
      gv[nu][0] = R(m.gsq[nu * kGsqStride + occ]);
      gv[nu][1] = R(m.gsq[nu * kGsqStride + occ + 1]);
    }
#pragma unroll
    for (int s = 0; s < D; ++s) {
      const int32_t c = col[int64_t(s) * stride + i];
      if (c >= 0) {
        const R v = s < 2 * ND ? jv[s >> 1] : gv[(s - 2 * ND) >> 1][(s - 2 * ND) & 1];
        const Amp xj = in[c];
        hr += v * xj.x;
        hi += v * xj.y;
      }
    }
    if (ta.energy) esum += double(xi.x) * double(hr) + double(xi.y) * double(hi);
    const R tr = alpha * hr + beta * xi.x, ti = alpha * hi + beta * xi.y;
    R yr = sir * tr - sii * ti, yi = sir * ti + sii * tr;
    const Amp f = phi[i];
    yr += ckr * f.x - cki * f.y;
    yi += ckr * f.y + cki * f.x;
    if (prev) {
      const Amp q = prev[i];
      yr -= spr * q.x - spi * q.y;
      yi -= spr * q.y + spi * q.x;
    }
    if (ta.final_) {
      const R zr = phr * yr - phi_i * yi, zi = phr * yi + phi_i * yr;
      yr = zr;
      yi = zi;
      Amp o;
      o.x = yr;
      o.y = yi;
      const double w = weight(o);
      n2 += w;
      atomicAdd(&pop_lds[pay_site(p)], w);
    }
    Amp o;
    o.x = yr;
    o.y = yi;
    out[i] = o;
  }
  if (ta.energy) {
    esum = block_sum(esum);
    if (threadIdx.x == 0) e_part[blockIdx.x] = esum;
  }
  if (ta.final_) {
    n2 = block_sum(n2);
    if (threadIdx.x == 0) n2_part[blockIdx.x] = n2;
    __syncthreads();
    for (int j = threadIdx.x; j < m.N; j += blockDim.x)
      pop_part[int64_t(blockIdx.x) * m.N + j] = pop_lds[j];
  }
}

template <typename R>
__global__ void __launch_bounds__(kBlock)
    k_cheb_scale(int64_t n, const ChebCoef* cc,
                 const typename VecT<R>::T* phi, typename VecT<R>::T* out,
                 double* n2_part, double* pop_part, const uint64_t* pay,
                 int N) {
  using Amp = typename VecT<R>::T;
  extern __shared__ double pop_lds[];
  for (int j = threadIdx.x; j < N; j += blockDim.x) pop_lds[j] = 0.0;
  __syncthreads();
  // c_0 * exp(-i b dt); c_0 is real
  const R zr = R(cc->c[0][0] * cc->phase[0]), zi = R(cc->c[0][0] * cc->phase[1]);
  double n2 = 0;
  for (int64_t i = gtid(); i < n; i += gstride()) {
    const Amp f = phi[i];
    Amp o;
    o.x = zr * f.x - zi * f.y;
    o.y = zr * f.y + zi * f.x;
    out[i] = o;
    const double w = weight(o);
    n2 += w;
    atomicAdd(&pop_lds[pay_site(pay[i])], w);
  }
  n2 = block_sum(n2);
  if (threadIdx.x == 0) n2_part[blockIdx.x] = n2;
  __syncthreads();
  for (int j = threadIdx.x; j < N; j += blockDim.x)
    pop_part[int64_t(blockIdx.x) * N + j] = pop_lds[j];
}

template <typename R>
__global__ void __launch_bounds__(kBlock)
    k_energy(DevModel m, int64_t n, const int32_t* col, int64_t stride,
             const uint64_t* pay, const double* diag,
             const typename VecT<R>::T* x, double* e_part) {
  using Amp = typename VecT<R>::T;
  double esum = 0;
  for (int64_t i = gtid(); i < n; i += gstride()) {
    const Amp xi = x[i];
    const uint64_t p = pay[i];
    double hr = diag[i] * double(xi.x), hi = diag[i] * double(xi.y);
    for (int s = 0; s < m.D; ++s) {
      const int32_t c = col[int64_t(s) * stride + i];
      if (c >= 0) {
        const double v = slot_value(m, p, s);
        hr += v * double(x[c].x);
        hi += v * double(x[c].y);
      }
    }
    esum += double(xi.x) * hr + double(xi.y) * hi;
  }
  esum = block_sum(esum);
  if (threadIdx.x == 0) e_part[blockIdx.x] = esum;
}

// ---- autocorrelation <psi0|psi(t)> ------------------------------------------
template <int W, typename Amp>
__global__ void __launch_bounds__(kBlock)
    k_autocorr(DevModel m, const uint64_t* keys0, const double* amps0,
               int64_t n0, const uint64_t* table, uint64_t mask,
               const uint64_t* keys, const Amp* psi, double* out2) {
  double re = 0, im = 0;
  for (int64_t i = threadIdx.x; i < n0; i += blockDim.x) {
    uint64_t k[W];
    load_key<W>(keys0, i, k);
    const int64_t r = table_find<W>(table, mask, keys, k, key_hash<W>(m, k));
    if (r < 0) continue;
    const double2 v = widen(psi[r]);
    const double ar = amps0[2 * i], ai = amps0[2 * i + 1];
    // conj(a0) * v
    re += ar * v.x + ai * v.y;
    im += ar * v.y - ai * v.x;
  }
  re = block_sum(re);
  im = block_sum(im);
  if (threadIdx.x == 0) {
    out2[0] = re;
    out2[1] = im;
  }
}

// ---- observation record -----------------------------------------------------
__global__ void __launch_bounds__(kBlock)
    k_obs_final(ObsArgs oa, int nparts, const double* mass_part,
                const double* n2_part, const double* e_part,
                const double* pop_part, const double* a2, const ChebCoef* cc,
                double* mass_total, double* rec, int* err) {
  double ms = 0, n2 = 0, en = 0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
    ms += mass_part[i];
    n2 += n2_part[i];
    if (oa.want_energy) en += e_part[i];
  }
  ms = block_sum(ms);
  n2 = block_sum(n2);
  en = block_sum(en);
  for (int j = threadIdx.x; j < oa.N; j += blockDim.x) {
    double s = 0;
    for (int b = 0; b < nparts; ++b) s += pop_part[int64_t(b) * oa.N + j];
    rec[kObsFields + j] = s;
  }
  if (threadIdx.x == 0) {
    const double tot = *mass_total + ms;
    *mass_total = tot;
    rec[0] = oa.t;
    rec[1] = n2;
    rec[2] = oa.want_energy ? en : NAN;
    rec[3] = a2[0];
    rec[4] = a2[1];
    rec[5] = ms;
    rec[6] = tot;
    rec[7] = oa.nS;
    rec[8] = oa.nM;
    rec[9] = double(cc->K);
    rec[10] = cc->emin;
    rec[11] = cc->emax;
    if (!isfinite(n2)) atomicOr(err, kErrNonFinite);
  }
}

// ---- precision conversion ---------------------------------------------------
__global__ void __launch_bounds__(kBlock)
    k_f32_to_f64(const float2* src, double* dst, int64_t n) {
  for (int64_t i = gtid(); i < n; i += gstride()) {
    dst[2 * i] = src[i].x;
    dst[2 * i + 1] = src[i].y;
  }
}
__global__ void __launch_bounds__(kBlock)
    k_f64_to_f32(const double* src, float2* dst, int64_t n) {
  for (int64_t i = gtid(); i < n; i += gstride())
    dst[i] = make_float2(float(src[2 * i]), float(src[2 * i + 1]));
}

}  // namespace

// ============================================================================
// host wrappers
// ============================================================================
int supported_words(int W) {
  static const int ws[] = {1, 2, 3, 4, 6, 8, 10, 16};
  for (int w : ws)
    if (w >= W) return w;
  return 0;
}

#define PACES_DISPATCH_W(Wi, ...)          \
  switch (Wi) {                            \
    case 1: { constexpr int WW = 1; __VA_ARGS__; } break;   \
    case 2: { constexpr int WW = 2; __VA_ARGS__; } break;   \
    case 3: { constexpr int WW = 3; __VA_ARGS__; } break;   \
    case 4: { constexpr int WW = 4; __VA_ARGS__; } break;   \
    case 6: { constexpr int WW = 6; __VA_ARGS__; } break;   \
    case 8: { constexpr int WW = 8; __VA_ARGS__; } break;   \
    case 10: { constexpr int WW = 10; __VA_ARGS__; } break; \
    case 16: { constexpr int WW = 16; __VA_ARGS__; } break; \
    default: break;                        \
  }

void fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s) {
  if (n <= 0) return;
  k_fill_u64<<<grid_for(n, 8192), kBlock, 0, s>>>(p, n, v);
}
void fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return;
  k_fill_u32<<<grid_for(n, 8192), kBlock, 0, s>>>(p, n, v);
}
void iota_u32(uint32_t* p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_iota_u32<<<grid_for(n, 8192), kBlock, 0, s>>>(p, n);
}

int64_t scan_tmp_words(int64_t n) { return cdiv(n, kTile) + 16; }

void exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n,
                    uint32_t* tmp, uint32_t* total, hipStream_t s) {
  const int64_t nb = cdiv(n, kTile);
  if (n <= 0) {
    k_fill_u32<<<1, kBlock, 0, s>>>(total, 1, 0u);
    return;
  }
  k_scan_reduce<<<int(nb), kBlock, 0, s>>>(in, n, tmp);
  k_scan_bsum<<<1, kBlock, 0, s>>>(tmp, nb, total);
  k_scan_apply<<<int(nb), kBlock, 0, s>>>(in, n, tmp, out);
}

void select_rows(int prec, const void* psi, int64_t n, double th2,
                 uint32_t* midx, uint32_t* tmp, uint32_t* count,
                 hipStream_t s) {
  const int64_t nb = cdiv(n, kTile);
  if (n <= 0) {
    k_fill_u32<<<1, kBlock, 0, s>>>(count, 1, 0u);
    return;
  }
  if (prec == 64) {
    k_select_count<double2><<<int(nb), kBlock, 0, s>>>((const double2*)psi, n, th2, tmp);
    k_scan_bsum<<<1, kBlock, 0, s>>>(tmp, nb, count);
    k_select_write<double2><<<int(nb), kBlock, 0, s>>>((const double2*)psi, n, th2, tmp, midx);
  } else {
    k_select_count<float2><<<int(nb), kBlock, 0, s>>>((const float2*)psi, n, th2, tmp);
    k_scan_bsum<<<1, kBlock, 0, s>>>(tmp, nb, count);
    k_select_write<float2><<<int(nb), kBlock, 0, s>>>((const float2*)psi, n, th2, tmp, midx);
  }
}

void row_info(const DevModel& m, int Wi, const uint64_t* keys, int64_t n,
              uint64_t* pay, uint64_t* tot, double* diag, hipStream_t s) {
  if (n <= 0) return;
  PACES_DISPATCH_W(Wi, k_row_info<WW><<<grid_for(n, 8192), kBlock, 0, s>>>(
                           m, keys, n, pay, tot, diag));
}

void insert_rows(const DevModel& m, int Wi, const uint64_t* keys_o,
                 const uint64_t* pay_o, const uint64_t* tot_o,
                 const double* diag_o, const uint32_t* midx, int64_t nM,
                 uint64_t* keys_n, uint64_t* pay_n, uint64_t* tot_n,
                 double* diag_n, uint64_t* table, uint64_t mask, int* err,
                 hipStream_t s) {
  if (nM <= 0) return;
  PACES_DISPATCH_W(Wi, k_insert_rows<WW><<<grid_for(nM), kBlock, 0, s>>>(
                           m, keys_o, pay_o, tot_o, diag_o, midx, nM, keys_n,
                           pay_n, tot_n, diag_n, table, mask, err));
}

void expand_chunk(const DevModel& m, int Wi, int prec, uint64_t* keys,
                  uint64_t* pay, uint64_t* tot, double* diag, int64_t f0,
                  int64_t rows, int64_t n_cur, uint64_t* table, uint64_t mask,
                  const RoundBufs& rb, int32_t* col, int64_t stride, void* phi,
                  int* err, hipStream_t s) {
  if (rows <= 0) return;
  const int64_t nc = rows * m.D;
  PACES_DISPATCH_W(Wi, k_expand_probe<WW><<<grid_for(nc), kBlock, 0, s>>>(
                           m, keys, pay, f0, rows, table, mask, rb.c_slot,
                           rb.c_ref, err));
  k_expand_resolve<<<grid_for(rows), kBlock, 0, s>>>(m.D, rows, table,
                                                    rb.c_slot, rb.c_ref,
                                                    rb.rowcnt);
  exclusive_scan(rb.rowcnt, rb.rowbase, rows, rb.scan_tmp, rb.total, s);
  if (prec == 64) {
    PACES_DISPATCH_W(Wi, k_expand_commit<WW, double2><<<grid_for(rows), kBlock, 0, s>>>(
                             m, keys, pay, tot, diag, f0, rows, n_cur, table,
                             rb.c_slot, rb.c_ref, rb.rowbase, rb.crow, col,
                             stride, (double2*)phi));
  } else {
    PACES_DISPATCH_W(Wi, k_expand_commit<WW, float2><<<grid_for(rows), kBlock, 0, s>>>(
                             m, keys, pay, tot, diag, f0, rows, n_cur, table,
                             rb.c_slot, rb.c_ref, rb.rowbase, rb.crow, col,
                             stride, (float2*)phi));
  }
  k_expand_link<<<grid_for(nc), kBlock, 0, s>>>(m.D, f0, rows, rb.c_ref,
                                               rb.crow, col, stride);
}

void lookup_cols(const DevModel& m, int Wi, const uint64_t* keys,
                 const uint64_t* pay, int64_t f0, int64_t rows,
                 const uint64_t* table, uint64_t mask, int32_t* col,
                 int64_t stride, hipStream_t s) {
  if (rows <= 0) return;
  const int64_t nc = rows * m.D;
  PACES_DISPATCH_W(Wi, k_lookup_cols<WW><<<grid_for(nc), kBlock, 0, s>>>(
                           m, keys, pay, f0, rows, table, mask, col, stride));
}

void transfer(const DevModel& m, int Wi, int prec, const uint64_t* keys_o,
              const void* psi_o, int64_t n_old, const uint64_t* table,
              uint64_t mask, const uint64_t* keys_n, void* phi,
              double* mass_part, hipStream_t s) {
  if (prec == 64) {
    PACES_DISPATCH_W(Wi, k_transfer<WW, double2><<<kPartBlocks, kBlock, 0, s>>>(
                             m, keys_o, (const double2*)psi_o, n_old, table,
                             mask, keys_n, (double2*)phi, mass_part));
  } else {
    PACES_DISPATCH_W(Wi, k_transfer<WW, float2><<<kPartBlocks, kBlock, 0, s>>>(
                             m, keys_o, (const float2*)psi_o, n_old, table,
                             mask, keys_n, (float2*)phi, mass_part));
  }
}

void bounds_and_coef(const DevModel& m, const uint64_t* pay,
                     const double* diag, const int32_t* col, int64_t stride,
                     int64_t n, double dt, double tol, int k_max,
                     double* part, ChebCoef* cc, int* err, hipStream_t s) {
  k_bounds<<<kPartBlocks, kBlock, 0, s>>>(m, pay, diag, col, stride, n, part);
  k_coef<<<1, kBlock, 0, s>>>(part, kPartBlocks, dt, tol, k_max, cc, err);
}

#define PACES_DISPATCH_SHAPE(ND, NV, ...)                                 \
  switch ((ND) * 8 + (NV)) {                                              \
    case 9: { constexpr int A = 1, B = 1; __VA_ARGS__; } break;           \
    case 10: { constexpr int A = 1, B = 2; __VA_ARGS__; } break;          \
    case 11: { constexpr int A = 1, B = 3; __VA_ARGS__; } break;          \
    case 12: { constexpr int A = 1, B = 4; __VA_ARGS__; } break;          \
    case 17: { constexpr int A = 2, B = 1; __VA_ARGS__; } break;          \
    case 18: { constexpr int A = 2, B = 2; __VA_ARGS__; } break;          \
    case 19: { constexpr int A = 2, B = 3; __VA_ARGS__; } break;          \
    case 20: { constexpr int A = 2, B = 4; __VA_ARGS__; } break;          \
    case 25: { constexpr int A = 3, B = 1; __VA_ARGS__; } break;          \
    case 26: { constexpr int A = 3, B = 2; __VA_ARGS__; } break;          \
    case 27: { constexpr int A = 3, B = 3; __VA_ARGS__; } break;          \
    case 28: { constexpr int A = 3, B = 4; __VA_ARGS__; } break;          \
    default: break;                                                       \
  }

void cheb_term(const DevModel& m, int prec, int64_t n, const int32_t* col,
               int64_t stride, const uint64_t* pay, const double* diag,
               const ChebCoef* cc, const TermArgs& ta, const void* phi,
               const void* in, const void* prev, void* out, double* e_part,
               double* n2_part, double* pop_part, hipStream_t s) {
  const size_t lds = ta.final_ ? sizeof(double) * m.N : 0;
  const bool part = ta.final_ || ta.energy;
  const int grid = part ? kPartBlocks : grid_for(n);
  if (prec == 64) {
    PACES_DISPATCH_SHAPE(m.ndim, m.V,
        k_cheb_term<double, A, B><<<grid, kBlock, lds, s>>>(
            m, n, col, stride, pay, diag, cc, ta, (const double2*)phi,
            (const double2*)in, (const double2*)prev, (double2*)out, e_part,
            n2_part, pop_part));
  } else {
    PACES_DISPATCH_SHAPE(m.ndim, m.V,
        k_cheb_term<float, A, B><<<grid, kBlock, lds, s>>>(
            m, n, col, stride, pay, diag, cc, ta, (const float2*)phi,
            (const float2*)in, (const float2*)prev, (float2*)out, e_part,
            n2_part, pop_part));
  }
}

void cheb_scale(int prec, int64_t n, const ChebCoef* cc, const void* phi,
                void* out, double* n2_part, double* pop_part,
                const uint64_t* pay, int N, hipStream_t s) {
  const size_t lds = sizeof(double) * N;
  if (prec == 64)
    k_cheb_scale<double><<<kPartBlocks, kBlock, lds, s>>>(
        n, cc, (const double2*)phi, (double2*)out, n2_part, pop_part, pay, N);
  else
    k_cheb_scale<float><<<kPartBlocks, kBlock, lds, s>>>(
        n, cc, (const float2*)phi, (float2*)out, n2_part, pop_part, pay, N);
}

void energy_only(const DevModel& m, int prec, int64_t n, const int32_t* col,
                 int64_t stride, const uint64_t* pay, const double* diag,
                 const void* x, double* e_part, hipStream_t s) {
  if (prec == 64)
    k_energy<double><<<kPartBlocks, kBlock, 0, s>>>(m, n, col, stride, pay, diag,
                                                    (const double2*)x, e_part);
  else
    k_energy<float><<<kPartBlocks, kBlock, 0, s>>>(m, n, col, stride, pay, diag,
                                                   (const float2*)x, e_part);
}

void autocorr(const DevModel& m, int Wi, int prec, const uint64_t* keys0,
              const double* amps0, int64_t n0, const uint64_t* table,
              uint64_t mask, const uint64_t* keys, const void* psi,
              double* out2, hipStream_t s) {
  if (prec == 64) {
    PACES_DISPATCH_W(Wi, k_autocorr<WW, double2><<<1, kBlock, 0, s>>>(
                             m, keys0, amps0, n0, table, mask, keys,
                             (const double2*)psi, out2));
  } else {
    PACES_DISPATCH_W(Wi, k_autocorr<WW, float2><<<1, kBlock, 0, s>>>(
                             m, keys0, amps0, n0, table, mask, keys,
                             (const float2*)psi, out2));
  }
}

void obs_final(const ObsArgs& oa, const double* mass_part,
               const double* n2_part, const double* e_part,
               const double* pop_part, const double* a2, const ChebCoef* cc,
               double* mass_total, double* rec, int* err, hipStream_t s) {
  k_obs_final<<<1, kBlock, 0, s>>>(oa, kPartBlocks, mass_part, n2_part,
                                   e_part, pop_part, a2, cc, mass_total, rec,
                                   err);
}

void amps_to_f64(int prec, const void* src, double* dst, int64_t n,
                 hipStream_t s) {
  if (n <= 0) return;
  if (prec == 64)
    (void)hipMemcpyAsync(dst, src, size_t(n) * 16, hipMemcpyDeviceToDevice, s);
  else
    k_f32_to_f64<<<grid_for(n, 8192), kBlock, 0, s>>>((const float2*)src, dst, n);
}
void amps_from_f64(int prec, const double* src, void* dst, int64_t n,
                   hipStream_t s) {
  if (n <= 0) return;
  if (prec == 64)
    (void)hipMemcpyAsync(dst, src, size_t(n) * 16, hipMemcpyDeviceToDevice, s);
  else
    k_f64_to_f32<<<grid_for(n, 8192), kBlock, 0, s>>>(src, (float2*)dst, n);
}

}  // namespace paces
