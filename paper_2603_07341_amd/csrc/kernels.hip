// kernels.hip -- HIP kernels of one co-evolving-subspace step on gfx950.
//
// The step is sparse, memory-bound gather/scatter: kernels stream rows with
// one row (or one row slot) per lane, wave64, 256-lane blocks, and no
// matrix cores.  Row counts live in device memory (StepCtl); kernels run on
// grid-stride grids, clamp counts to the allocated capacity and latch
// overflows, and every kernel after a latching one returns at once when the
// latch is set, so a failed step touches nothing out of bounds and leaves
// the previous state intact for a retry.  Sums over rows use a fixed
// lane-to-row mapping, wave shuffles in a fixed order and per-block
// partials summed in block order; population and per-realization bins use
// LDS atomics, whose order within a block is not fixed.
//
// Stages (paper: Sec. "Formal operator representation and notes on
// parallelization"):
//   select     rows of psi with |c|^2 >= theta^2, compacted in row order
//              (Sec. "Truncation & post-adaptation detruncation")
//   expand     k rounds of neighbour generation on packed keys with
//              insert-if-absent into an HBM hash table (Eqs. (def_neighbor_k),
//              (H_eff)); the candidate whose compare-and-swap claims a key
//              owns it, so new rows are numbered in an order that may vary
//              between runs while every amplitude, taken per basis state,
//              is reproduced bit for bit
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

#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "kernels.hpp"

namespace paces {

namespace {

// ---- fills and step control -------------------------------------------------
__global__ void __launch_bounds__(kBlock)
    k_fill_u64(uint64_t* p, int64_t n, uint64_t v) {
  for (int64_t i = gtid(); i < n; i += gstride()) p[i] = v;
}

// A dispatch that does nothing: a marker that kernel traces and counter
// runs show in stream order.
__global__ void k_mark(int tag) { (void)tag; }

__global__ void k_clear_err(int* err) { *err = 0; }

// ---- a given set of states (stateless propagation) --------------------------
// Canonical keys of W words to the internal width Wi >= W (leading zero
// words; one realization, so no realization bits).
__global__ void __launch_bounds__(kBlock)
    k_pad_keys(int W, int Wi, const uint64_t* in, uint64_t* out, int64_t n) {
  const int64_t total = n * Wi;
  for (int64_t e = gtid(); e < total; e += gstride()) {
    const int64_t i = e / Wi;
    const int w = int(e % Wi) - (Wi - W);
    out[e] = w >= 0 ? in[i * W + w] : 0ull;
  }
}

// Counts of a step whose set is rows [0, n) in place: frontier 0 is the
// whole set.
__global__ void k_set_begin(StepCtl* ctl, int* err, uint32_t n) {
  *err = 0;
  ctl->n_old = n;
  ctl->nM = n;
  ctl->fstart[0] = 0;
  ctl->fstart[1] = n;
  ctl->n_new = n;
  ctl->kmax = 0;
  ctl->r_need = 0;
}

// Every row's key names a basis state (site below N, occupations within
// the cutoffs, no bits above the state's B bits) and finds itself in the
// table (no other row holds the same key); else kErrInput.
template <int W>
__global__ void __launch_bounds__(kBlock)
    k_check_set(DevModel m, const uint64_t* keys, int64_t n,
                const uint64_t* table, uint64_t mask, int* err) {
  for (int64_t i = gtid(); i < n; i += gstride()) {
    uint64_t k[W];
    load_key<W>(keys, i, k);
    bool ok = true;
#pragma unroll
    for (int q = 0; q < W; ++q) {
      const int lo = 64 * (W - 1 - q);  // bit position of the word's bit 0
      if (lo + 64 <= m.B) continue;
      const uint64_t above = lo >= m.B ? ~0ull : ~((uint64_t(1) << (m.B - lo)) - 1);
      ok &= (k[q] & above) == 0;
    }
    const int j = int(k[W - 1] & ((uint64_t(1) << m.bj) - 1));
    ok &= j < m.N;
    for (int s = 0; s < m.N && ok; ++s)
      for (int nu = 0; nu < m.V; ++nu)
        ok &= int(get_field<W>(k, field_off(m, s, nu), m.bnu[nu])) <= m.cut[nu];
    if (ok) ok = table_find<W>(table, mask, keys, k, key_hash<W>(m, k)) == i;
    if (!ok) atomicOr(err, kErrInput);
  }
}

__global__ void k_begin_step(StepCtl* ctl, int* err, uint32_t* cnt, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) cnt[i] = 0u;
  if (threadIdx.x == 0) {
    *err = 0;
    ctl->fstart[0] = 0;
    ctl->nM = 0;
    ctl->n_new = 0;
    ctl->kmax = 0;
    ctl->r_need = 0;
    ctl->w_moved = 0;  // an in-place step has not committed
  }
}

// ---- scan over a device-sized array ----------------------------------------
// Tile t covers elements [t*kTile, (t+1)*kTile); element t*kTile + q*kBlock
// + lane belongs to lane `lane` (q = 0..kItems-1), so every load of the block
// is one contiguous run of kBlock elements.  Blocks stride over tiles.
__global__ void __launch_bounds__(kBlock)
    k_scan_reduce(const uint32_t* in, const uint32_t* nptr, uint32_t* bsum,
                  const int* err) {
  if (*err) return;
  const int64_t n = *nptr, ntiles = cdiv(n, kTile);
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    uint32_t v = 0;
#pragma unroll
    for (int q = 0; q < kItems; ++q) {
      const int64_t e = t * kTile + q * kBlock + threadIdx.x;
      if (e < n) v += in[e];
    }
    uint32_t tot;
    block_excl_scan(v, &tot);
    if (threadIdx.x == 0) bsum[t] = tot;
  }
}

// Single block: exclusive scan of the tile sums in place; the grand total
// goes to *out1 (and *out2 when given).  Each lane takes kScanRun
// consecutive sums per pass, so one pass covers kBlock * kScanRun tiles.
constexpr int kScanRun = 16;
__global__ void __launch_bounds__(kBlock)
    k_scan_bsum(uint32_t* bsum, const uint32_t* nptr, uint32_t* out1,
                uint32_t* out2, const int* err) {
  if (*err) return;
  const int64_t nb = cdiv(int64_t(*nptr), kTile);
  uint32_t carry = 0;
  for (int64_t c = 0; c < nb; c += int64_t(kBlock) * kScanRun) {
    const int64_t e0 = c + int64_t(threadIdx.x) * kScanRun;
    uint32_t v[kScanRun];
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < kScanRun; ++j) {
      v[j] = e0 + j < nb ? bsum[e0 + j] : 0u;
      sum += v[j];
    }
    uint32_t tot;
    uint32_t off = block_excl_scan(sum, &tot) + carry;
#pragma unroll
    for (int j = 0; j < kScanRun; ++j) {
      if (e0 + j < nb) bsum[e0 + j] = off;
      off += v[j];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) {
    *out1 = carry;
    if (out2) *out2 = carry;
  }
}

__global__ void __launch_bounds__(kBlock)
    k_scan_apply(const uint32_t* in, const uint32_t* nptr,
                 const uint32_t* bsum, uint32_t* out, const int* err) {
  if (*err) return;
  const int64_t n = *nptr, ntiles = cdiv(n, kTile);
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    uint32_t run = bsum[t];
#pragma unroll
    for (int q = 0; q < kItems; ++q) {
      const int64_t e = t * kTile + q * kBlock + threadIdx.x;
      const uint32_t v = e < n ? in[e] : 0u;
      uint32_t tot;
      const uint32_t off = block_excl_scan(v, &tot) + run;
      if (e < n) out[e] = off;
      run += tot;
    }
  }
}

// ---- select -----------------------------------------------------------------

// Rows that are holes (dist == kHole, left by dropped rows of in-place
// steps) are never selected; dist may be null (no holes).
__device__ __forceinline__ bool is_hole(const uint8_t* dist, int64_t e) {
  return dist && dist[e] == kHole;
}

template <typename Amp>
__global__ void __launch_bounds__(kBlock)
    k_select_count(const Amp* psi, const uint8_t* dist, const StepCtl* ctl,
                   double th2, uint32_t* bsum) {
  const int64_t n = ctl->n_old, ntiles = cdiv(n, kTile);
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    uint32_t v = 0;
#pragma unroll
    for (int q = 0; q < kItems; ++q) {
      const int64_t e = t * kTile + q * kBlock + threadIdx.x;
      if (e < n && weight(psi[e]) >= th2 && !is_hole(dist, e)) ++v;
    }
    uint32_t tot;
    block_excl_scan(v, &tot);
    if (threadIdx.x == 0) bsum[t] = tot;
  }
}

// Selected rows are written in ascending order: tile offset from the scan,
// then one block scan per run of kBlock rows.
template <typename Amp>
__global__ void __launch_bounds__(kBlock)
    k_select_write(const Amp* psi, const uint8_t* dist, const StepCtl* ctl,
                   double th2, const uint32_t* bsum, uint32_t* midx) {
  const int64_t n = ctl->n_old, ntiles = cdiv(n, kTile);
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    uint32_t run = bsum[t];
#pragma unroll
    for (int q = 0; q < kItems; ++q) {
      const int64_t e = t * kTile + q * kBlock + threadIdx.x;
      const bool keep = e < n && weight(psi[e]) >= th2 && !is_hole(dist, e);
      uint32_t tot;
      const uint32_t off = block_excl_scan(keep ? 1u : 0u, &tot) + run;
      if (keep) midx[off] = uint32_t(e);
      run += tot;
    }
  }
}

// Selection given as one flag per old row (state cap): same tile layout.
__global__ void __launch_bounds__(kBlock)
    k_flag_count(const uint8_t* keep, const StepCtl* ctl, uint32_t* bsum) {
  const int64_t n = ctl->n_old, ntiles = cdiv(n, kTile);
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    uint32_t v = 0;
#pragma unroll
    for (int q = 0; q < kItems; ++q) {
      const int64_t e = t * kTile + q * kBlock + threadIdx.x;
      if (e < n && keep[e]) ++v;
    }
    uint32_t tot;
    block_excl_scan(v, &tot);
    if (threadIdx.x == 0) bsum[t] = tot;
  }
}

__global__ void __launch_bounds__(kBlock)
    k_flag_write(const uint8_t* keep, const StepCtl* ctl,
                 const uint32_t* bsum, uint32_t* midx) {
  const int64_t n = ctl->n_old, ntiles = cdiv(n, kTile);
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    uint32_t run = bsum[t];
#pragma unroll
    for (int q = 0; q < kItems; ++q) {
      const int64_t e = t * kTile + q * kBlock + threadIdx.x;
      const bool k = e < n && keep[e];
      uint32_t tot;
      const uint32_t off = block_excl_scan(k ? 1u : 0u, &tot) + run;
      if (k) midx[off] = uint32_t(e);
      run += tot;
    }
  }
}

__global__ void __launch_bounds__(kBlock)
    k_select_all(StepCtl* ctl, uint32_t* midx) {
  const int64_t n = ctl->n_old;
  for (int64_t i = gtid(); i < n; i += gstride()) midx[i] = uint32_t(i);
  if (gtid() == 0) {
    ctl->nM = uint32_t(n);
    ctl->fstart[1] = uint32_t(n);
  }
}

// ---- row metadata from keys -------------------------------------------------
template <int W>
__global__ void __launch_bounds__(kBlock)
    k_row_info(DevModel m, const uint64_t* keys, int64_t n, uint64_t* pay,
               uint64_t* tot) {
  for (int64_t r = gtid(); r < n; r += gstride()) {
    uint64_t k[W];
    load_key<W>(keys, r, k);
    const int j = int(k[W - 1] & ((uint64_t(1) << m.bj) - 1));
    int nj[kMaxV], T[kMaxV];
    for (int nu = 0; nu < m.V; ++nu) {
      nj[nu] = int(get_field<W>(k, field_off(m, j, nu), m.bnu[nu]));
      int s = 0;
      for (int i = 0; i < m.N; ++i)
        s += int(get_field<W>(k, field_off(m, i, nu), m.bnu[nu]));
      T[nu] = s;
    }
    pay[r] = make_pay(m.V, j, nj, T, key_real<W>(m, k));
    tot[r] = make_tot(m.V, T);
  }
}


// ---- insert rows into the cleared table -------------------------------------
// Row i of the new set is row midx[i] of the old one (keys_o given) or is
// already in place (rehash after growth, keys_o null).  With phi given, the
// row's amplitude moves along (the transfer then skips rows of M).
template <int W, typename Amp>
__global__ void __launch_bounds__(kBlock)
    k_insert_rows(DevModel m, const uint64_t* keys_o, const uint64_t* pay_o,
                  const uint64_t* tot_o, const uint32_t* midx,
                  const uint32_t* nptr, int64_t n_fixed, uint64_t* keys_n,
                  uint64_t* pay_n, uint64_t* tot_n, uint64_t* table,
                  uint64_t mask, uint32_t* cnt_r, const Amp* psi_o, Amp* phi,
                  int* err) {
  __shared__ uint32_t bins[kMaxReal];
  if (*err) return;
  for (int r = threadIdx.x; r < m.R; r += blockDim.x) bins[r] = 0;
  __syncthreads();
  const int64_t nM = nptr ? int64_t(*nptr) : n_fixed;
  for (int64_t i = gtid(); i < nM; i += gstride()) {
    uint64_t k[W];
    if (keys_o) {
      const int64_t r = midx[i];
      load_key<W>(keys_o, r, k);
      store_key<W>(keys_n, i, k);
      pay_n[i] = pay_o[r];
      tot_n[i] = tot_o[r];
      if (phi) phi[i] = psi_o[r];
      if (cnt_r) atomicAdd(&bins[pay_real(pay_o[r])], 1u);
    } else {
      load_key<W>(keys_n, i, k);
    }
    const uint64_t h = key_hash<W>(m, k);
    const uint64_t mine = (uint64_t(hash_tag(h)) << 32) | uint64_t(i);
    uint64_t s = h & mask;
    bool done = false;
    for (uint64_t p = 0; p <= mask && p < kMaxProbe; ++p) {
      if (table[s] == kEmpty &&
          atomicCAS((unsigned long long*)(table + s), (unsigned long long)kEmpty,
                    (unsigned long long)mine) == kEmpty) {
        done = true;
        break;
      }
      s = (s + 1) & mask;
    }
    if (!done) atomicOr(err, kErrTableFull);
  }
  if (cnt_r) count_flush(m.R, bins, cnt_r);
}

// ---- expansion round --------------------------------------------------------
// Parameters of chunk `chunk` of round r: parents [f0 + chunk * per,
// f0 + (chunk + 1) * per) of frontier r-1 = [f0, f1), per = cand_cap / D.
// The first chunk starts the row count of the round at fstart[r]; the last
// one enqueued latches kErrChunks when parents are left over.
__global__ void k_round_prep(StepCtl* ctl, int r, int chunk, int last, int D,
                             int64_t cand_cap, int* err) {
  if (*err) return;
  const int64_t f0 = ctl->fstart[r - 1], f1 = ctl->fstart[r];
  const int64_t per = cand_cap / D;
  const int64_t start = f0 + int64_t(chunk) * per;
  int64_t rows = f1 - start;
  if (rows < 0) rows = 0;
  if (rows > per) {
    if (last) {
      atomicOr(err, kErrChunks);
      const uint32_t need = uint32_t(cdiv(f1 - f0, per));
      if (need > ctl->r_need) ctl->r_need = need;
    }
    rows = per;
  }
  ctl->r_f0 = uint32_t(start < f1 ? start : f1);
  ctl->r_rows = uint32_t(rows);
  ctl->r_ncand = uint32_t(rows * D);
  ctl->r_ntiles = uint32_t(cdiv(rows * D, kBlock));
  if (chunk == 0) ctl->r_ncur = ctl->fstart[r];
  ctl->r_total = 0;
}

// The chunk's new rows join the set; after the last chunk they close
// frontier r.
__global__ void k_round_finish(StepCtl* ctl, int r, int last, int64_t cap,
                               int* err) {
  if (*err) return;
  int64_t n = int64_t(ctl->r_ncur) + ctl->r_total;
  if (n > cap) {
    atomicOr(err, kErrCapacity);
    n = cap;
  }
  ctl->r_ncur = uint32_t(n);
  if (last) ctl->fstart[r + 1] = uint32_t(n);
}

// Probe: insert-if-absent of candidate c = (parent f0 + c / D, slot c % D).
// A table slot holds (tag << 32 | ref); ref is a row of the new set or,
// during the round, kCand | candidate id.  The candidate whose
// compare-and-swap fills an empty slot owns that key.  Entries only move
// EMPTY -> CAND(owner) inside this kernel, so a stale read is repaired by
// the compare-and-swap.  Outcomes per candidate:
//   structural zero      col = -1
//   key already a row    col = that row
//   owner                c_ref = kOwner, c_slot = probe distance of the
//                        claimed slot from the key's home
//   key owned by c2      c_ref = c2 (column linked after the commit)
// Candidates are processed in tiles of one block; the owners of each tile
// are counted into tile_cnt so that new rows are numbered by a scan.
constexpr uint32_t kOwner = 0xFFFFFFFEu;

template <int W>
__global__ void __launch_bounds__(kBlock)
    k_expand_probe(DevModel m, const uint64_t* keys, const uint64_t* pay,
                   const StepCtl* ctl, int64_t cap, uint64_t* table,
                   uint64_t mask, uint32_t* c_slot, uint32_t* c_ref,
                   uint32_t* tile_cnt, int32_t* col, int* err) {
  if (*err) return;
  const int D = m.D;
  const int64_t f0 = ctl->r_f0, nc = ctl->r_ncand;
  const int64_t ntiles = cdiv(nc, kBlock);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t c = tile * kBlock + threadIdx.x;
    uint32_t owner = 0;
    if (c < nc) {
      const int64_t p = f0 + c / D;
      const int s = int(c % D);
      uint64_t par[W], k[W];
      load_key<W>(keys, p, par);
      const uint64_t py = pay[p];
      uint32_t rref = kNone;
      if (!slot_target<W>(m, par, py, s, k)) {
        col[p * D + s] = -1;
      } else {
        const uint64_t h = key_hash<W>(m, k);
        const uint32_t tag = hash_tag(h);
        const uint64_t mine =
            (uint64_t(tag) << 32) | uint64_t(kCand | uint32_t(c));
        uint64_t i = h & mask;
        bool done = false;
        for (uint64_t probes = 0; probes <= mask && probes < kMaxProbe;
             ++probes) {
          uint64_t e = table[i];
          if (e == kEmpty) {
            const uint64_t old = atomicCAS((unsigned long long*)(table + i),
                                           (unsigned long long)kEmpty,
                                           (unsigned long long)mine);
            if (old == kEmpty) {
              rref = kOwner;
              c_slot[c] = uint32_t(probes);
              owner = 1;
              done = true;
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
              if (r & kCand)
                rref = r & ~kCand;
              else
                col[p * D + s] = int32_t(r);
              done = true;
              break;
            }
          }
          i = (i + 1) & mask;
        }
        if (!done) atomicOr(err, kErrTableFull);
      }
      c_ref[c] = rref;
    }
    uint32_t tot;
    block_excl_scan(owner, &tot);
    if (threadIdx.x == 0) tile_cnt[tile] = tot;
  }
}

// Owners append their key as a new row: row = n_cur + tile base + rank of
// the owner inside its tile.  The table slot is pointed at the row.
template <int W, typename Amp>
__global__ void __launch_bounds__(kBlock)
    k_expand_commit(DevModel m, uint64_t* keys, uint64_t* pay, uint64_t* tot,
                    const StepCtl* ctl, int64_t cap, uint64_t* table,
                    uint64_t mask, const uint32_t* c_slot, const uint32_t* c_ref,
                    const uint32_t* tile_base, uint32_t* crow, int32_t* col,
                    Amp* phi, int* err) {
  if (*err) return;
  const int D = m.D;
  const int64_t f0 = ctl->r_f0, nc = ctl->r_ncand, n_cur = ctl->r_ncur;
  const int64_t ntiles = cdiv(nc, kBlock);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t c = tile * kBlock + threadIdx.x;
    const bool own = c < nc && c_ref[c] == kOwner;
    uint32_t tot_in_tile;
    const uint32_t rank = block_excl_scan(own ? 1u : 0u, &tot_in_tile);
    if (!own) continue;
    const int64_t p = f0 + c / D;
    const int s = int(c % D);
    const int64_t row = n_cur + tile_base[tile] + rank;
    if (row >= cap) {
      atomicOr(err, kErrCapacity);
      crow[c] = kNone;
      col[p * D + s] = -1;
      continue;
    }
    uint64_t par[W], k[W];
    load_key<W>(keys, p, par);
    const uint64_t py = pay[p];
    slot_target<W>(m, par, py, s, k);
    store_key<W>(keys, row, k);
    uint64_t np, nt;
    slot_row_info<W>(m, k, py, tot[p], s, np, nt);
    pay[row] = np;
    tot[row] = nt;
    // the slot holds (tag | candidate); the tag and the home follow from
    // the key, so the entry is rewritten without reading it back
    const uint64_t h = key_hash<W>(m, k);
    table[((h & mask) + c_slot[c]) & mask] =
        (uint64_t(hash_tag(h)) << 32) | uint64_t(row);
    crow[c] = uint32_t(row);
    col[p * D + s] = int32_t(row);
    Amp z;
    z.x = 0;
    z.y = 0;
    phi[row] = z;
  }
}

// Candidates whose key another candidate owns take that candidate's row.
__global__ void __launch_bounds__(kBlock)
    k_expand_link(int D, const StepCtl* ctl, int64_t cap, const uint32_t* c_ref,
                  const uint32_t* crow, int32_t* col, const int* err) {
  if (*err) return;
  const int64_t f0 = ctl->r_f0, nc = ctl->r_ncand;
  for (int64_t c = gtid(); c < nc; c += gstride()) {
    const uint32_t r = c_ref[c];
    if (r >= kOwner) continue;  // kOwner or kNone
    const uint32_t row = crow[r];
    col[f0 * D + c] = row == kNone ? -1 : int32_t(row);
  }
}

template <int W>
__global__ void __launch_bounds__(kBlock)
    k_lookup_cols(DevModel m, const uint64_t* keys, const uint64_t* pay,
                  StepCtl* ctl, int k, const uint64_t* table, uint64_t mask,
                  int32_t* col, int64_t cap, const int* err) {
  if (*err) return;
  const int D = m.D;
  const int64_t f0 = ctl->fstart[k];
  const int64_t f1 = ctl->fstart[k + 1];
  const int64_t nc = (f1 - f0) * D;
  if (gtid() == 0) ctl->n_new = uint32_t(f1);
  for (int64_t c = gtid(); c < nc; c += gstride()) {
    const int64_t p = f0 + c / D;
    const int s = int(c % D);
    uint64_t par[W], key[W];
    load_key<W>(keys, p, par);
    int32_t out = -1;
    if (slot_target<W>(m, par, pay[p], s, key))
      out = int32_t(table_find<W>(table, mask, keys, key, key_hash<W>(m, key)));
    col[p * D + s] = out;
  }
}

// ---- transfer ---------------------------------------------------------------

// Old row i goes to its row of the new set, or counts as discarded weight.
// skip 1 (threshold selection) and 2 (preset flags keep[i]): rows of M are
// already in place (insert) and are passed over.
template <int W, typename Amp>
__global__ void __launch_bounds__(kBlock)
    k_transfer(DevModel m, const uint64_t* keys_o, const uint8_t* o_dist,
               const Amp* psi_o,
               const StepCtl* ctl, const uint64_t* table, uint64_t mask,
               const uint64_t* keys_n, Amp* phi, double* mass_part,
               int32_t* tmap, int skip, double th2, const uint8_t* keep,
               const int* err) {
  __shared__ double bins[kMaxReal];
  if (*err) return;
  const int R = m.R;
  if (R > 1) {
    for (int r = threadIdx.x; r < R; r += blockDim.x) bins[r] = 0.0;
    __syncthreads();
  }
  const int64_t n_old = ctl->n_old;
  double lost = 0;
  for (int64_t i = gtid(); i < n_old; i += gstride()) {
    if (is_hole(o_dist, i)) {
      if (tmap) tmap[i] = -1;
      continue;
    }
    const Amp v = psi_o[i];
    if ((skip == 1 && weight(v) >= th2) || (skip == 2 && keep[i])) continue;
    uint64_t k[W];
    load_key<W>(keys_o, i, k);
    const int64_t r = table_find<W>(table, mask, keys_n, k, key_hash<W>(m, k));
    if (tmap) tmap[i] = int32_t(r);
    if (r >= 0)
      phi[r] = v;
    else if (R > 1)
      atomicAdd(&bins[key_real<W>(m, k)], weight(v));
    else
      lost += weight(v);
  }
  if (R > 1) {
    __syncthreads();
    for (int r = threadIdx.x; r < R; r += blockDim.x)
      mass_part[int64_t(blockIdx.x) * R + r] = bins[r];
  } else {
    lost = block_sum(lost);
    if (threadIdx.x == 0) mass_part[blockIdx.x] = lost;
  }
}

// ---- Gershgorin bounds and Chebyshev coefficients ---------------------------
// Order-preserving map of doubles to signed 64-bit integers, so that
// integer min / max (exact, order independent) give the double min / max.
__device__ __forceinline__ long long ord_of(double x) {
  const long long b = __double_as_longlong(x);
  return b >= 0 ? b : (b ^ 0x7FFFFFFFFFFFFFFFll);
}
__device__ __forceinline__ double dbl_of(long long o) {
  return __longlong_as_double(o >= 0 ? o : (o ^ 0x7FFFFFFFFFFFFFFFll));
}

// Gershgorin interval per realization: rows stride over a fixed grid; per
// block the (lo, hi) of each realization go to part[block][r][2].  DT: the
// slot count at compile time (a row's columns in one vector load), or 0
// for m.D at run time; the radius sums the slots in order either way.
template <int DT>
__global__ void __launch_bounds__(kBlock)
    k_bounds(DevModel m, const uint64_t* pay, const uint64_t* tot,
             const uint8_t* dist, const int32_t* col, int64_t cap,
             const StepCtl* ctl, double* part, const int* err) {
  __shared__ long long blo[kMaxReal], bhi[kMaxReal];
  if (*err) return;
  const int R = m.R;
  if (R > 1) {
    for (int r = threadIdx.x; r < R; r += blockDim.x) {
      blo[r] = ord_of(INFINITY);
      bhi[r] = ord_of(-INFINITY);
    }
    __syncthreads();
  }
  const int64_t n = ctl->n_new;
  double lo = INFINITY, hi = -INFINITY;
  for (int64_t r = gtid(); r < n; r += gstride()) {
    if (is_hole(dist, r)) continue;
    const uint64_t p = ld_stream(pay + r);
    double rad = 0;
    if constexpr (DT > 0) {
      int32_t cs[DT];
      load_cols<DT>(col + r * DT, cs);
#pragma unroll
      for (int s = 0; s < DT; ++s)
        if (cs[s] >= 0) rad += fabs(slot_value(m, p, s));
    } else {
      for (int s = 0; s < m.D; ++s)
        if (col[r * m.D + s] >= 0) rad += fabs(slot_value(m, p, s));
    }
    const double d = row_diag(m, p, m.V > 2 ? tot[r] : 0);
    if (R > 1) {
      atomicMin(&blo[pay_real(p)], ord_of(d - rad));
      atomicMax(&bhi[pay_real(p)], ord_of(d + rad));
    } else {
      lo = fmin(lo, d - rad);
      hi = fmax(hi, d + rad);
    }
  }
  if (R > 1) {
    __syncthreads();
    for (int r = threadIdx.x; r < R; r += blockDim.x) {
      part[(int64_t(blockIdx.x) * R + r) * 2] = dbl_of(blo[r]);
      part[(int64_t(blockIdx.x) * R + r) * 2 + 1] = dbl_of(bhi[r]);
    }
  } else {
    lo = block_min(lo);
    hi = block_max(hi);
    if (threadIdx.x == 0) {
      part[2 * blockIdx.x] = lo;
      part[2 * blockIdx.x + 1] = hi;
    }
  }
}

// One block per realization: fold the per-block bounds, pad them, and
// compute the Chebyshev coefficients and the number of terms K_r.
__global__ void __launch_bounds__(kBlock)
    k_coef(const double* part, int nparts, int R, double dt, double tol,
           int k_max, int launched, ChebCoef* cc_all, StepCtl* ctl,
           int* err) {
  __shared__ double J[kMaxTerms + 1];
  if (*err) return;
  const int rr = blockIdx.x;
  ChebCoef* cc = cc_all + rr;
  double lo = INFINITY, hi = -INFINITY;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
    lo = fmin(lo, part[(int64_t(i) * R + rr) * 2]);
    hi = fmax(hi, part[(int64_t(i) * R + rr) * 2 + 1]);
  }
  lo = block_min(lo);
  hi = block_max(hi);
  if (lo > hi) lo = hi = 0.0;  // empty set
  // widen by 1e-12 of the magnitude so the interval strictly contains the
  // spectrum
  const double pad = 1e-12 * (fabs(hi) + fabs(lo));
  const double emin = lo - pad, emax = hi + pad;
  double a = 0.5 * (emax - emin);
  const double b = 0.5 * (emax + emin);
  if (!(a > 1e-300)) a = 1e-300;
  const double x = a * dt;
  const int kcap = k_max < kMaxTerms ? k_max : kMaxTerms;
  // the series needs more than x terms: a spectrum too wide for the step
  // (or not finite) is reported before any Bessel recurrence runs
  if (!(x <= double(kcap))) {
    if (threadIdx.x == 0) atomicOr(err, isfinite(x) ? kErrTerms : kErrNonFinite);
    return;
  }
  if (x <= 2.0) {
    for (int k = threadIdx.x; k <= kcap; k += blockDim.x)
      J[k] = bessel_series(x, k);
  } else if (threadIdx.x == 0) {
    bessel_miller(x, kcap, J);
  }
  __syncthreads();
  // K = 1 + the last k with |J_k| above tol / 4.  Beyond x each J_k is
  // below half the one before (J_{k+1} / J_k < x / (2k + 2) before the
  // first zero of J_k), so the omitted tail sum_{k>=K} |c_k| =
  // 2 sum |J_k| <= 4 |J_K| stays within tol (|T_k| <= 1 on the interval)
  const double thresh = ldexp(tol, -2);
  double last = 0;
  for (int k = threadIdx.x; k <= kcap; k += blockDim.x)
    if (fabs(J[k]) > thresh) last = fmax(last, double(k));
  last = block_max(last);
  int K = int(last) + 1;
  if (K > kcap) K = kcap + 1;
  if (threadIdx.x == 0) {
    if (K > kcap)
      atomicOr(err, kErrTerms);
    else if (K > launched)
      atomicOr(err, kErrNeedTerms);
    atomicMax(&ctl->kmax, uint32_t(K));
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
    cc->K = K;
  }
  for (int k = threadIdx.x; k < K && k < kMaxTerms; k += blockDim.x) {
    const double v = (k == 0 ? 1.0 : 2.0) * J[k];
    const int q = k & 3;  // (-i)^k
    cc->c[k][0] = (q == 0) ? v : (q == 2 ? -v : 0.0);
    cc->c[k][1] = (q == 1) ? -v : (q == 3 ? v : 0.0);
  }
}

// ---- Clenshaw term ----------------------------------------------------------
// y = sum_{k<K} c_k T_k(H~) phi by Clenshaw's recurrence
//   b_k = c_k phi + 2 H~ b_{k+1} - b_{k+2}   (k = K-1 .. 1),
//   y   = c_0 phi + H~ b_1 - b_2,
// with b_K = b_{K+1} = 0 and b_{K-1} = c_{K-1} phi folded into the first
// launch.  Launch kk computes b_kk into buffer kk & 1, in place over
// b_{kk+2}; launches with kk > K-2 return at once, so the host enqueues a
// fixed number of launches before K is known.  H~ = alpha H + beta; H is
// applied as an ELL SpMV whose values follow from the slot and the row
// payload.  Against the forward three-term recurrence plus an accumulator
// this streams one vector less per term.
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

// MID only names the launches the host expects to be middle terms (neither
// first nor last for the previous step's K), so that profiles can tell them
// apart; the code is the same and still decides its role from the device K.
template <typename R, int ND, int NV, bool MID>
__global__ void __launch_bounds__(kBlock)
    k_cheb_term(DevModel m, int kk, int want_energy,
                const StepCtl* __restrict__ ctl, const int* __restrict__ err,
                const int32_t* __restrict__ col, int64_t cap,
                const uint64_t* __restrict__ pay,
                const uint64_t* __restrict__ tot,
                const ChebCoef* __restrict__ cc,
                const typename VecT<R>::T* __restrict__ phi,
                typename VecT<R>::T* b0, typename VecT<R>::T* b1,
                double* e_part) {
  using Amp = typename VecT<R>::T;
  constexpr int D = 2 * ND + 2 * NV;
  if (*err) return;
  const int K = cc->K;
  if (kk > K - 2 && !(K == 1 && kk == 0)) return;
  const int64_t n = ctl->n_new;
  const bool first = (kk == K - 2) || K == 1;
  const bool fin = kk == 0;
  const bool energy = first && want_energy;
  const Amp* in = first ? phi : (((kk + 1) & 1) ? b1 : b0);
  const Amp* prev = first ? nullptr : (kk == K - 3 ? phi : ((kk & 1) ? b1 : b0));
  Amp* out = (kk & 1) ? b1 : b0;
  const R alpha = R(cc->alpha), beta = R(cc->beta);
  const R ckr = R(cc->c[kk][0]), cki = R(cc->c[kk][1]);
  const double fac = fin ? 1.0 : 2.0;
  R sir = R(fac), sii = 0;
  if (first) {
    sir = K == 1 ? R(0) : R(fac * cc->c[K - 1][0]);
    sii = K == 1 ? R(0) : R(fac * cc->c[K - 1][1]);
  }
  R spr = 1, spi = 0;
  if (kk == K - 3) {
    spr = R(cc->c[K - 1][0]);
    spi = R(cc->c[K - 1][1]);
  }
  // the final launch also applies exp(-i b dt)
  const R phr = fin ? R(cc->phase[0]) : R(1), phim = fin ? R(cc->phase[1]) : R(0);
  R jv[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < ND; ++a) jv[a] = R(m.J[a]);
  double esum = 0;
  for (int64_t i = gtid(); i < n; i += gstride()) {
    const Amp xi = in[i];
    const uint64_t p = ld_stream(pay + i);
    const R d = R(row_diag(m, p, NV > 2 ? ld_stream(tot + i) : 0));
    R hr = d * xi.x, hi = d * xi.y;
    R gv[NV][2];
#pragma unroll
    for (int nu = 0; nu < NV; ++nu) {
      const int occ = pay_occ(p, nu);
      gv[nu][0] = R(m.gsq[nu * kGsqStride + occ]);
      gv[nu][1] = R(m.gsq[nu * kGsqStride + occ + 1]);
    }
    int32_t cols[D];
    load_cols<D>(col + i * D, cols);
#pragma unroll
    for (int s = 0; s < D; ++s) {
      const int32_t c = cols[s];
      if (c >= 0) {
        const R v = s < 2 * ND ? jv[s >> 1] : gv[(s - 2 * ND) >> 1][(s - 2 * ND) & 1];
        const Amp xj = in[c];
        hr += v * xj.x;
        hi += v * xj.y;
      }
    }
    if (energy) esum += double(xi.x) * double(hr) + double(xi.y) * double(hi);
    const R tr = alpha * hr + beta * xi.x, ti = alpha * hi + beta * xi.y;
    R yr = sir * tr - sii * ti, yi = sir * ti + sii * tr;
    const Amp f = ld_stream(phi + i);
    yr += ckr * f.x - cki * f.y;
    yi += ckr * f.y + cki * f.x;
    if (prev) {
      const Amp q = ld_stream(prev + i);
      yr -= spr * q.x - spi * q.y;
      yi -= spr * q.y + spi * q.x;
    }
    Amp o;
    o.x = phr * yr - phim * yi;
    o.y = phr * yi + phim * yr;
    out[i] = o;
  }
  if (energy) {
    esum = block_sum(esum);
    if (threadIdx.x == 0) e_part[blockIdx.x] = esum;
  }
}

// Batched form of the Clenshaw launch: rows of different disorder
// realizations carry their own spectral interval, coefficients and term
// count K_r (cc_all[r]); each row takes its role from its own K_r, so a
// realization's rows do exactly the arithmetic of a single-realization run
// (neighbours of a row always belong to the same realization).  Launches
// beyond a realization's K_r leave its rows untouched.  The energy term
// <phi|H|phi> is left per row in e_row for a segmented reduction.
template <typename R, int ND, int NV>
__global__ void __launch_bounds__(kBlock)
    k_cheb_batch(DevModel m, int kk, int want_energy,
                 const StepCtl* __restrict__ ctl, const int* __restrict__ err,
                 const int32_t* __restrict__ col, int64_t cap,
                 const uint64_t* __restrict__ pay,
                 const uint64_t* __restrict__ tot,
                 const ChebCoef* __restrict__ cc_all,
                 const typename VecT<R>::T* __restrict__ phi,
                 typename VecT<R>::T* b0, typename VecT<R>::T* b1,
                 double* e_row) {
  using Amp = typename VecT<R>::T;
  constexpr int D = 2 * ND + 2 * NV;
  if (*err) return;
  const int64_t n = ctl->n_new;
  R jv[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < ND; ++a) jv[a] = R(m.J[a]);
  for (int64_t i = gtid(); i < n; i += gstride()) {
    const uint64_t p = ld_stream(pay + i);
    const ChebCoef* cc = cc_all + pay_real(p);
    const int K = cc->K;
    if (kk > K - 2 && !(K == 1 && kk == 0)) continue;
    const bool first = (kk == K - 2) || K == 1;
    const bool fin = kk == 0;
    const Amp* in = first ? phi : (((kk + 1) & 1) ? b1 : b0);
    const Amp* prev = first ? nullptr : (kk == K - 3 ? phi : ((kk & 1) ? b1 : b0));
    Amp* out = (kk & 1) ? b1 : b0;
    const R alpha = R(cc->alpha), beta = R(cc->beta);
    const R ckr = R(cc->c[kk][0]), cki = R(cc->c[kk][1]);
    const double fac = fin ? 1.0 : 2.0;
    R sir = R(fac), sii = 0;
    if (first) {
      sir = K == 1 ? R(0) : R(fac * cc->c[K - 1][0]);
      sii = K == 1 ? R(0) : R(fac * cc->c[K - 1][1]);
    }
    R spr = 1, spi = 0;
    if (kk == K - 3) {
      spr = R(cc->c[K - 1][0]);
      spi = R(cc->c[K - 1][1]);
    }
    const R phr = fin ? R(cc->phase[0]) : R(1), phim = fin ? R(cc->phase[1]) : R(0);
    const Amp xi = in[i];
    const R d = R(row_diag(m, p, NV > 2 ? ld_stream(tot + i) : 0));
    R hr = d * xi.x, hi = d * xi.y;
    R gv[NV][2];
#pragma unroll
    for (int nu = 0; nu < NV; ++nu) {
      const int occ = pay_occ(p, nu);
      gv[nu][0] = R(m.gsq[nu * kGsqStride + occ]);
      gv[nu][1] = R(m.gsq[nu * kGsqStride + occ + 1]);
    }
    int32_t cols[D];
    load_cols<D>(col + i * D, cols);
#pragma unroll
    for (int s = 0; s < D; ++s) {
      const int32_t c = cols[s];
      if (c >= 0) {
        const R v = s < 2 * ND ? jv[s >> 1] : gv[(s - 2 * ND) >> 1][(s - 2 * ND) & 1];
        const Amp xj = in[c];
        hr += v * xj.x;
        hi += v * xj.y;
      }
    }
    if (first && want_energy)
      e_row[i] = double(xi.x) * double(hr) + double(xi.y) * double(hi);
    const R tr = alpha * hr + beta * xi.x, ti = alpha * hi + beta * xi.y;
    R yr = sir * tr - sii * ti, yi = sir * ti + sii * tr;
    const Amp f = ld_stream(phi + i);
    yr += ckr * f.x - cki * f.y;
    yi += ckr * f.y + cki * f.x;
    if (prev) {
      const Amp q = ld_stream(prev + i);
      yr -= spr * q.x - spi * q.y;
      yi -= spr * q.y + spi * q.x;
    }
    Amp o;
    o.x = phr * yr - phim * yi;
    o.y = phr * yi + phim * yr;
    out[i] = o;
  }
}

// Population bins in LDS: with one realization and up to kPrivBins sites
// every lane of a wave owns a column (bin j, lane l at j*64 + l), so the
// four waves of a block meet on an address at most four at a time; other
// shapes share one bin per (realization, site).
constexpr int kPrivBins = 120;  // N * 64 + 3 doubles fit in 64 KiB
constexpr int kRegBins = 16;

// Norm, exciton populations, row counts and (batched) energy of psi per
// realization as per-block partials.  Rows are visited in the select
// kernels' tile layout, so the same pass also counts, per tile, the rows
// the next step will select.
template <typename R>
__global__ void __launch_bounds__(kBlock)
    k_pop_norm(int N, int Rn, double th2, const StepCtl* ctl,
               const typename VecT<R>::T* psi, const uint64_t* pay,
               const uint8_t* dist,
               const double* e_row, double* n2_part, double* en_part,
               double* pop_part, uint32_t* sel_bsum, uint32_t* cnt_s,
               const int* err) {
  extern __shared__ double lds[];
  if (*err) return;
  const int64_t n = ctl->n_new, ntiles = cdiv(n, kTile);
  const bool priv = Rn == 1 && N <= kPrivBins;
  // up to kRegBins sites: each thread sums its rows' weights per site in
  // registers and adds them to its lane's LDS bins once at the end
  const bool regs = priv && N <= kRegBins;
  double acc[kRegBins];
#pragma unroll
  for (int q = 0; q < kRegBins; ++q) acc[q] = 0.0;
  const int npop = priv ? N * 64 : Rn * N;
  double* pop_lds = lds;
  double* n2_lds = lds + npop;          // Rn (batched only)
  double* en_lds = n2_lds + Rn;         // Rn
  uint32_t* cnt_lds = reinterpret_cast<uint32_t*>(en_lds + Rn);  // Rn
  for (int j = threadIdx.x; j < npop; j += blockDim.x) pop_lds[j] = 0.0;
  for (int j = threadIdx.x; j < Rn; j += blockDim.x) {
    n2_lds[j] = 0.0;
    en_lds[j] = 0.0;
    cnt_lds[j] = 0u;
  }
  __syncthreads();
  double n2 = 0;
  uint32_t rows = 0;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    uint32_t keep = 0;
#pragma unroll
    for (int q = 0; q < kItems; ++q) {
      const int64_t e = t * kTile + q * kBlock + threadIdx.x;
      if (e < n && !is_hole(dist, e)) {
        const double w = weight(psi[e]);
        const uint64_t p = pay[e];
        keep += w >= th2 ? 1u : 0u;
        if (Rn == 1) {
          n2 += w;
          ++rows;
          if (regs) {
            const int j = pay_site(p);
#pragma unroll
            for (int q = 0; q < kRegBins; ++q) acc[q] += q == j ? w : 0.0;
          } else if (priv) {
            atomicAdd(&pop_lds[pay_site(p) * 64 + (threadIdx.x & 63)], w);
          } else {
            atomicAdd(&pop_lds[pay_site(p)], w);
          }
        } else {
          const int r = pay_real(p);
          atomicAdd(&n2_lds[r], w);
          atomicAdd(&cnt_lds[r], 1u);
          atomicAdd(&pop_lds[r * N + pay_site(p)], w);
          if (e_row) atomicAdd(&en_lds[r], e_row[e]);
        }
      }
    }
    uint32_t tot;
    block_excl_scan(keep, &tot);
    if (threadIdx.x == 0) sel_bsum[t] = tot;
  }
  if (regs) {
#pragma unroll
    for (int q = 0; q < kRegBins; ++q)
      if (q < N) atomicAdd(&pop_lds[q * 64 + (threadIdx.x & 63)], acc[q]);
  }
  if (Rn == 1) {
    n2 = block_sum(n2);
    uint32_t all;
    block_excl_scan(rows, &all);
    if (threadIdx.x == 0) {
      n2_part[blockIdx.x] = n2;
      if (all) atomicAdd(&cnt_s[0], all);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < N; j += blockDim.x) {
      double v = 0;
      if (priv)
        for (int l = 0; l < 64; ++l) v += pop_lds[j * 64 + l];
      else
        v = pop_lds[j];
      pop_part[int64_t(blockIdx.x) * N + j] = v;
    }
  } else {
    __syncthreads();
    for (int r = threadIdx.x; r < Rn; r += blockDim.x) {
      n2_part[int64_t(blockIdx.x) * Rn + r] = n2_lds[r];
      en_part[int64_t(blockIdx.x) * Rn + r] = en_lds[r];
      if (cnt_lds[r]) atomicAdd(&cnt_s[r], cnt_lds[r]);
    }
    for (int j = threadIdx.x; j < Rn * N; j += blockDim.x)
      pop_part[int64_t(blockIdx.x) * Rn * N + j] = pop_lds[j];
  }
}

// Second level of a deterministic reduction: block b folds partials
// b, b + gridDim.x, ... into out[b].
__global__ void __launch_bounds__(kBlock)
    k_fold_sum(const double* in, int n, double* out, const int* err) {
  if (*err) return;
  double s = 0;
  for (int i = blockIdx.x + gridDim.x * threadIdx.x; i < n;
       i += gridDim.x * blockDim.x)
    s += in[i];
  s = block_sum(s);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// ---- autocorrelation <psi0|psi(t)> ------------------------------------------
// Block r: the n0 initial states of realization r.
template <int W, typename Amp>
__global__ void __launch_bounds__(kBlock)
    k_autocorr(DevModel m, const uint64_t* keys0, const double* amps0,
               int64_t n0, const uint64_t* table, uint64_t mask,
               const uint64_t* keys, const Amp* psi, double* out2,
               int32_t* p0map, const int* err) {
  if (*err) return;
  const int64_t base = int64_t(blockIdx.x) * n0;
  double re = 0, im = 0;
  for (int64_t i = base + threadIdx.x; i < base + n0; i += blockDim.x) {
    uint64_t k[W];
    load_key<W>(keys0, i, k);
    const int64_t r = table_find<W>(table, mask, keys, k, key_hash<W>(m, k));
    if (p0map) p0map[i] = int32_t(r);
    if (r < 0) continue;
    const double2 v = widen(psi[r]);
    const double ar = amps0[2 * i], ai = amps0[2 * i + 1];
    re += ar * v.x + ai * v.y;  // conj(a0) * v
    im += ar * v.y - ai * v.x;
  }
  re = block_sum(re);
  im = block_sum(im);
  if (threadIdx.x == 0) {
    out2[2 * blockIdx.x] = re;
    out2[2 * blockIdx.x + 1] = im;
  }
}

// ---- observation record -----------------------------------------------------
// Block (x, r): x < N reduces population (r, x), x = N the scalars of
// realization r; each folds the per-block partials with a fixed lane
// mapping.  Records of one step are stored realization after realization.
__global__ void __launch_bounds__(kBlock)
    k_obs_final(int N, int Rn, int want_energy, double dt, int n_mass, int n_e,
                int n_pop, const double* mass_part, const double* n2_part,
                const double* e_part, const double* en_part,
                const double* pop_part, const double* a2, const ChebCoef* cc,
                const StepCtl* ctl, const uint32_t* cnt,
                const double* mass_tot, double* ring, int rec_doubles,
                int64_t ring_cap, int* err) {
  if (*err) return;
  if (int64_t(ctl->nrec) + 1 > ring_cap) return;  // the host keeps room
  const int r = blockIdx.y;
  double* rec = ring + (int64_t(ctl->nrec) * Rn + r) * rec_doubles;
  if (int(blockIdx.x) < N) {
    double s = 0;
    for (int b = threadIdx.x; b < n_pop; b += blockDim.x)
      s += pop_part[(int64_t(b) * Rn + r) * N + blockIdx.x];
    s = block_sum(s);
    if (threadIdx.x == 0) rec[kObsFields + blockIdx.x] = s;
    return;
  }
  double ms = 0, n2 = 0, en = 0;
  for (int i = threadIdx.x; i < n_mass; i += blockDim.x)
    ms += mass_part[int64_t(i) * Rn + r];
  for (int i = threadIdx.x; i < n_pop; i += blockDim.x)
    n2 += n2_part[int64_t(i) * Rn + r];
  if (want_energy) {
    if (Rn == 1)
      for (int i = threadIdx.x; i < n_e; i += blockDim.x) en += e_part[i];
    else
      for (int i = threadIdx.x; i < n_pop; i += blockDim.x)
        en += en_part[int64_t(i) * Rn + r];
  }
  ms = block_sum(ms);
  n2 = block_sum(n2);
  en = block_sum(en);
  if (threadIdx.x == 0) {
    rec[0] = ctl->t + dt;
    rec[1] = n2;
    rec[2] = want_energy ? en : NAN;
    rec[3] = a2[2 * r];
    rec[4] = a2[2 * r + 1];
    rec[5] = ms;
    rec[6] = mass_tot[r] + ms;
    rec[7] = double(cnt[Rn + r]);
    rec[8] = double(cnt[r]);
    rec[9] = double(cc[r].K);
    rec[10] = cc[r].emin;
    rec[11] = cc[r].emax;
    if (!isfinite(n2)) atomicOr(err, kErrNonFinite);
  }
}

// Commit the step on the device: time, cumulative discarded weight per
// realization, record count and the row count of the current set.
// The last kernel of a step also mirrors the counts and the error latch into
// mapped pinned host memory, so the host reads them after one stream
// synchronisation without copy dispatches.
__global__ void k_end_step(StepCtl* ctl, int Rn, const double* ring,
                           int rec_doubles, double* mass_tot, const int* err,
                           uint32_t* h_ctl, int* h_err) {
  const int e = *err;
  if (threadIdx.x == 0 && !e) {
    const double* rec = ring + int64_t(ctl->nrec) * Rn * rec_doubles;
    for (int r = 0; r < Rn; ++r) mass_tot[r] = rec[int64_t(r) * rec_doubles + 6];
    ctl->t = rec[0];
    ctl->n_old = ctl->n_new;
    ctl->nrec += 1;
  }
  __syncthreads();
  const uint32_t* src = reinterpret_cast<const uint32_t*>(ctl);
  for (int i = threadIdx.x; i < int(sizeof(StepCtl) / 4); i += blockDim.x)
    h_ctl[i] = src[i];
  if (threadIdx.x == 0) *h_err = e;
  __threadfence_system();
}

__global__ void k_clear_u32(uint32_t* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
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

int64_t scan_tmp_words(int64_t n) { return cdiv(n, kTile) + 16; }

void fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s) {
  if (n <= 0) return;
  k_fill_u64<<<grid_for(n), kBlock, 0, s>>>(p, n, v);
}

void mark(int tag, hipStream_t s) { k_mark<<<1, 64, 0, s>>>(tag); }

void clear_latch(int* err, hipStream_t s) { k_clear_err<<<1, 1, 0, s>>>(err); }

void pad_keys(int W, int Wi, const uint64_t* in, uint64_t* out, int64_t n,
              hipStream_t s) {
  if (n <= 0) return;
  k_pad_keys<<<grid_for(n * Wi), kBlock, 0, s>>>(W, Wi, in, out, n);
}

void set_begin(StepCtl* ctl, int* err, int64_t n, hipStream_t s) {
  k_set_begin<<<1, 1, 0, s>>>(ctl, err, uint32_t(n));
}

void check_set(const DevModel& m, int Wi, const uint64_t* keys, int64_t n,
               const uint64_t* table, uint64_t mask, int* err,
               hipStream_t s) {
  if (n <= 0) return;
  PACES_DISPATCH_W(Wi, k_check_set<WW><<<grid_for(n), kBlock, 0, s>>>(
                           m, keys, n, table, mask, err));
}

void begin_step(StepCtl* ctl, int* err, uint32_t* cnt, int R,
                hipStream_t s) {
  k_begin_step<<<1, kBlock, 0, s>>>(ctl, err, cnt, 2 * R);
}

void select_rows(int prec, const void* psi, const uint8_t* dist, double th2,
                 bool select_all, bool counted, StepCtl* ctl, uint32_t* midx,
                 uint32_t* tmp, int64_t cap, int* err, hipStream_t s) {
  if (select_all) {
    k_select_all<<<grid_for(cap), kBlock, 0, s>>>(ctl, midx);
    return;
  }
  const int g = tiles_for(cap);
  if (!counted) {
    if (prec == 64)
      k_select_count<double2><<<g, kBlock, 0, s>>>((const double2*)psi, dist, ctl, th2, tmp);
    else
      k_select_count<float2><<<g, kBlock, 0, s>>>((const float2*)psi, dist, ctl, th2, tmp);
  }
  k_scan_bsum<<<1, kBlock, 0, s>>>(tmp, &ctl->n_old, &ctl->nM, &ctl->fstart[1],
                                   err);
  if (prec == 64)
    k_select_write<double2><<<g, kBlock, 0, s>>>((const double2*)psi, dist, ctl, th2, tmp, midx);
  else
    k_select_write<float2><<<g, kBlock, 0, s>>>((const float2*)psi, dist, ctl, th2, tmp, midx);
}

void select_flags(const uint8_t* keep, StepCtl* ctl, uint32_t* midx,
                  uint32_t* tmp, int64_t cap, int* err, hipStream_t s) {
  const int g = tiles_for(cap);
  k_flag_count<<<g, kBlock, 0, s>>>(keep, ctl, tmp);
  k_scan_bsum<<<1, kBlock, 0, s>>>(tmp, &ctl->n_old, &ctl->nM, &ctl->fstart[1],
                                   err);
  k_flag_write<<<g, kBlock, 0, s>>>(keep, ctl, tmp, midx);
}

void insert_rows(const DevModel& m, int Wi, int prec, const Side& o,
                 const Side& n, const uint32_t* midx, const StepCtl* ctl,
                 uint64_t* table, uint64_t mask, uint32_t* cnt_m,
                 const void* psi_o, void* phi, int* err, hipStream_t s) {
  const int g = grid_for(int64_t(mask + 1) / 2);
  if (prec == 64) {
    PACES_DISPATCH_W(Wi, k_insert_rows<WW, double2><<<g, kBlock, 0, s>>>(
                             m, o.keys, o.pay, o.tot, midx, &ctl->nM, 0,
                             n.keys, n.pay, n.tot, table, mask, cnt_m,
                             (const double2*)psi_o, (double2*)phi, err));
  } else {
    PACES_DISPATCH_W(Wi, k_insert_rows<WW, float2><<<g, kBlock, 0, s>>>(
                             m, o.keys, o.pay, o.tot, midx, &ctl->nM, 0,
                             n.keys, n.pay, n.tot, table, mask, cnt_m,
                             (const float2*)psi_o, (float2*)phi, err));
  }
}

void rehash_rows(const DevModel& m, int Wi, const Side& n, uint32_t* midx,
                 int64_t rows, uint64_t* table, uint64_t mask, int* err,
                 hipStream_t s) {
  (void)midx;
  if (rows <= 0) return;
  PACES_DISPATCH_W(Wi, k_insert_rows<WW, double2><<<grid_for(rows), kBlock, 0, s>>>(
                           m, nullptr, nullptr, nullptr, nullptr, nullptr,
                           rows, n.keys, n.pay, n.tot, table, mask, nullptr,
                           nullptr, nullptr, err));
}

void expand_round(const DevModel& m, int Wi, int prec, const Side& n, int r,
                  StepCtl* ctl, int64_t cap, int64_t est, uint64_t* table,
                  uint64_t mask, const RoundBufs& rb, int32_t* col, void* phi,
                  int chunks, int* err, hipStream_t s) {
  const int D = m.D;
  const int64_t nc_bound = std::min<int64_t>(rb.cand_cap, est * D);
  const int g = grid_for(nc_bound);
  for (int q = 0; q < chunks; ++q) {
  const int last = q == chunks - 1 ? 1 : 0;
  k_round_prep<<<1, 1, 0, s>>>(ctl, r, q, last, D, rb.cand_cap, err);
  PACES_DISPATCH_W(Wi, k_expand_probe<WW><<<g, kBlock, 0, s>>>(
                           m, n.keys, n.pay, ctl, cap, table, mask, rb.c_slot,
                           rb.c_ref, rb.tile_cnt, col, err));
  const int gt = tiles_for(cdiv(nc_bound, kBlock));
  k_scan_reduce<<<gt, kBlock, 0, s>>>(rb.tile_cnt, &ctl->r_ntiles, rb.scan_tmp,
                                      err);
  k_scan_bsum<<<1, kBlock, 0, s>>>(rb.scan_tmp, &ctl->r_ntiles, &ctl->r_total,
                                   nullptr, err);
  k_scan_apply<<<gt, kBlock, 0, s>>>(rb.tile_cnt, &ctl->r_ntiles, rb.scan_tmp,
                                     rb.tile_base, err);
  if (prec == 64) {
    PACES_DISPATCH_W(Wi, k_expand_commit<WW, double2><<<g, kBlock, 0, s>>>(
                             m, n.keys, n.pay, n.tot, ctl, cap, table, mask,
                             rb.c_slot, rb.c_ref, rb.tile_base, rb.crow, col,
                             (double2*)phi, err));
  } else {
    PACES_DISPATCH_W(Wi, k_expand_commit<WW, float2><<<g, kBlock, 0, s>>>(
                             m, n.keys, n.pay, n.tot, ctl, cap, table, mask,
                             rb.c_slot, rb.c_ref, rb.tile_base, rb.crow, col,
                             (float2*)phi, err));
  }
  k_expand_link<<<g, kBlock, 0, s>>>(D, ctl, cap, rb.c_ref, rb.crow, col, err);
  k_round_finish<<<1, 1, 0, s>>>(ctl, r, last, cap, err);
  }
}

void tile_scan(const uint32_t* cnt, const uint32_t* ntiles, int64_t bound,
               uint32_t* tmp, uint32_t* base, uint32_t* total, int* err,
               hipStream_t s) {
  const int gt = tiles_for(bound);
  k_scan_reduce<<<gt, kBlock, 0, s>>>(cnt, ntiles, tmp, err);
  k_scan_bsum<<<1, kBlock, 0, s>>>(tmp, ntiles, total, nullptr, err);
  k_scan_apply<<<gt, kBlock, 0, s>>>(cnt, ntiles, tmp, base, err);
}

void tile_sums_scan(uint32_t* bsum, const uint32_t* nrows, uint32_t* total,
                    int* err, hipStream_t s) {
  k_scan_bsum<<<1, kBlock, 0, s>>>(bsum, nrows, total, nullptr, err);
}

void lookup_last(const DevModel& m, int Wi, const Side& n, int k,
                 StepCtl* ctl, int64_t est, const uint64_t* table,
                 uint64_t mask, int32_t* col, int64_t cap, int* err,
                 hipStream_t s) {
  PACES_DISPATCH_W(Wi, k_lookup_cols<WW><<<grid_for(est * m.D), kBlock, 0, s>>>(
                           m, n.keys, n.pay, ctl, k, table, mask, col, cap,
                           err));
}

int part_grid(int64_t rows) { return grid_for(rows); }

int transfer(const DevModel& m, int Wi, int prec, const Side& o,
             const void* psi_o, int64_t n_old, const StepCtl* ctl,
             const uint64_t* table, uint64_t mask, const uint64_t* keys_n,
             void* phi, double* mass_part, int32_t* tmap, int skip, double th2,
             const uint8_t* keep, int* err, hipStream_t s) {
  const int g = m.R > 1 ? std::min(grid_for(n_old), kPartBlocks) : grid_for(n_old);
  if (prec == 64) {
    PACES_DISPATCH_W(Wi, k_transfer<WW, double2><<<g, kBlock, 0, s>>>(
                             m, o.keys, o.dist, (const double2*)psi_o, ctl, table, mask,
                             keys_n, (double2*)phi, mass_part, tmap, skip, th2,
                             keep, err));
  } else {
    PACES_DISPATCH_W(Wi, k_transfer<WW, float2><<<g, kBlock, 0, s>>>(
                             m, o.keys, o.dist, (const float2*)psi_o, ctl, table, mask,
                             keys_n, (float2*)phi, mass_part, tmap, skip, th2,
                             keep, err));
  }
  return g;
}

namespace {
void launch_bounds_kernel(const DevModel& m, const Side& n, const int32_t* col,
                          int64_t cap, int g, const StepCtl* ctl, double* part,
                          const int* err, hipStream_t s) {
#define PACES_BOUNDS(DT) \
  k_bounds<DT><<<g, kBlock, 0, s>>>(m, n.pay, n.tot, n.dist, col, cap, ctl, part, err)
  switch (m.D) {
    case 4: PACES_BOUNDS(4); break;
    case 6: PACES_BOUNDS(6); break;
    case 8: PACES_BOUNDS(8); break;
    case 10: PACES_BOUNDS(10); break;
    case 12: PACES_BOUNDS(12); break;
    default: PACES_BOUNDS(0); break;
  }
#undef PACES_BOUNDS
}
}  // namespace

int bounds_part(const DevModel& m, const Side& n, const int32_t* col,
                int64_t cap, int64_t est, const StepCtl* ctl, double* part,
                const int* err, hipStream_t s) {
  const int g = std::min(grid_for(est), kPartBlocks);
  launch_bounds_kernel(m, n, col, cap, g, ctl, part, err, s);
  return g;
}

void bounds_and_coef(const DevModel& m, const Side& n, const int32_t* col,
                     int64_t cap, int64_t est, StepCtl* ctl, double dt,
                     double tol, int k_max, int launched, double* part,
                     ChebCoef* cc, int* err, hipStream_t s) {
  // a bounded grid: each block reduces many rows, and k_coef folds few
  // partials
  const int g = std::min(grid_for(est), kPartBlocks);
  launch_bounds_kernel(m, n, col, cap, g, ctl, part, err, s);
  k_coef<<<m.R, kBlock, 0, s>>>(part, g, m.R, dt, tol, k_max, launched, cc,
                                ctl, err);
}

int fold_sum(const double* in, int n, double* out, int* err, hipStream_t s) {
  const int f = std::max(1, std::min(n, kFold));
  k_fold_sum<<<f, kBlock, 0, s>>>(in, n, out, err);
  return f;
}

int cheb_term(const DevModel& m, int prec, int kk, bool energy, bool mid,
              int64_t est, const StepCtl* ctl, const int32_t* col, int64_t cap,
              const Side& n, const ChebCoef* cc, const void* phi, void* b0,
              void* b1, double* e_part, double* e_row, int* err,
              hipEvent_t ev_a, hipEvent_t ev_b, hipStream_t s) {
  const int e = energy ? 1 : 0;
  const int g = grid_for(est);
  if (m.R > 1) {
    if (prec == 64) {
      PACES_DISPATCH_SHAPE(m.ndim, m.V,
          launch_ev(k_cheb_batch<double, A, B>, g, s, ev_a, ev_b,
                    m, kk, e, ctl, err, col, cap, n.pay, n.tot, cc,
                    (const double2*)phi, (double2*)b0, (double2*)b1, e_row));
    } else {
      PACES_DISPATCH_SHAPE(m.ndim, m.V,
          launch_ev(k_cheb_batch<float, A, B>, g, s, ev_a, ev_b,
                    m, kk, e, ctl, err, col, cap, n.pay, n.tot, cc,
                    (const float2*)phi, (float2*)b0, (float2*)b1, e_row));
    }
    return g;
  }
#define PACES_TERM(R, AMP, MIDV)                                              \
  PACES_DISPATCH_SHAPE(m.ndim, m.V,                                           \
      launch_ev(k_cheb_term<R, A, B, MIDV>, g, s, ev_a, ev_b,                 \
                m, kk, e, ctl, err, col, cap, n.pay, n.tot, cc,               \
                (const AMP*)phi, (AMP*)b0, (AMP*)b1, e_part))
  if (prec == 64) {
    if (mid) { PACES_TERM(double, double2, true); } else { PACES_TERM(double, double2, false); }
  } else {
    if (mid) { PACES_TERM(float, float2, true); } else { PACES_TERM(float, float2, false); }
  }
#undef PACES_TERM
  return g;
}

int pop_norm(int prec, int N, int R, double th2, int64_t est,
             const StepCtl* ctl, const void* psi, const uint64_t* pay,
             const uint8_t* dist,
             const double* e_row, double* n2_part, double* en_part,
             double* pop_part, uint32_t* sel_bsum, uint32_t* cnt_s, int* err,
             hipStream_t s) {
  const bool priv = R == 1 && N <= kPrivBins;
  const size_t lds = sizeof(double) * ((priv ? N * 64 : R * N) + 3 * R);
  // batched partials hold R * N populations per block: fewer blocks
  // a bounded grid: blocks stride over the tiles, so the per-block work
  // (bins cleared and folded, one count added to the total) is amortised
  const int g = std::min(tiles_for(est), 1024);
  if (prec == 64)
    k_pop_norm<double><<<g, kBlock, lds, s>>>(
        N, R, th2, ctl, (const double2*)psi, pay, dist, e_row, n2_part, en_part,
        pop_part, sel_bsum, cnt_s, err);
  else
    k_pop_norm<float><<<g, kBlock, lds, s>>>(
        N, R, th2, ctl, (const float2*)psi, pay, dist, e_row, n2_part, en_part,
        pop_part, sel_bsum, cnt_s, err);
  return g;
}

void autocorr(const DevModel& m, int Wi, int prec, const uint64_t* keys0,
              const double* amps0, int64_t n0, const uint64_t* table,
              uint64_t mask, const uint64_t* keys, const void* psi,
              double* out2, int32_t* p0map, int* err, hipStream_t s) {
  if (prec == 64) {
    PACES_DISPATCH_W(Wi, k_autocorr<WW, double2><<<m.R, kBlock, 0, s>>>(
                             m, keys0, amps0, n0, table, mask, keys,
                             (const double2*)psi, out2, p0map, err));
  } else {
    PACES_DISPATCH_W(Wi, k_autocorr<WW, float2><<<m.R, kBlock, 0, s>>>(
                             m, keys0, amps0, n0, table, mask, keys,
                             (const float2*)psi, out2, p0map, err));
  }
}

void end_step(StepCtl* ctl, int R, const double* ring, int rec_doubles,
              double* mass_tot, int* err, StepCtl* h_ctl_dev, int* h_err_dev,
              hipStream_t s) {
  static_assert(sizeof(StepCtl) % 4 == 0, "StepCtl is copied as 32-bit words");
  k_end_step<<<1, 64, 0, s>>>(ctl, R, ring, rec_doubles, mass_tot, err,
                              reinterpret_cast<uint32_t*>(h_ctl_dev),
                              h_err_dev);
}

void obs_final(int N, int R, int want_energy, double dt, int n_mass, int n_e,
               int n_pop, const double* mass_part, const double* n2_part,
               const double* e_part, const double* en_part,
               const double* pop_part, const double* a2, const ChebCoef* cc,
               const StepCtl* ctl, const uint32_t* cnt,
               const double* mass_tot, double* ring, int rec_doubles,
               int64_t ring_cap, int* err, hipStream_t s) {
  k_obs_final<<<dim3(N + 1, R), kBlock, 0, s>>>(
      N, R, want_energy, dt, n_mass, n_e, n_pop, mass_part, n2_part, e_part,
      en_part, pop_part, a2, cc, ctl, cnt, mass_tot, ring, rec_doubles,
      ring_cap, err);
}

void row_info(const DevModel& m, int Wi, const uint64_t* keys, int64_t n,
              uint64_t* pay, uint64_t* tot, hipStream_t s) {
  if (n <= 0) return;
  PACES_DISPATCH_W(Wi, k_row_info<WW><<<grid_for(n), kBlock, 0, s>>>(
                           m, keys, n, pay, tot));
}

void amps_to_f64(int prec, const void* src, double* dst, int64_t n,
                 hipStream_t s) {
  if (n <= 0) return;
  if (prec == 64)
    (void)hipMemcpyAsync(dst, src, size_t(n) * 16, hipMemcpyDeviceToDevice, s);
  else
    k_f32_to_f64<<<grid_for(n), kBlock, 0, s>>>((const float2*)src, dst, n);
}
void amps_from_f64(int prec, const double* src, void* dst, int64_t n,
                   hipStream_t s) {
  if (n <= 0) return;
  if (prec == 64)
    (void)hipMemcpyAsync(dst, src, size_t(n) * 16, hipMemcpyDeviceToDevice, s);
  else
    k_f64_to_f32<<<grid_for(n), kBlock, 0, s>>>(src, (float2*)dst, n);
}

}  // namespace paces
