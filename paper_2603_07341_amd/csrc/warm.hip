// warm.hip -- the in-place step from the previous step's graph on gfx950
// (the method and its invariants are described in warm.hpp).
//
// Rows are walked in tiles of kTile rows (one distance byte each, the
// columns of the frontier rows), so the search inside the set streams its
// arrays; only slots that leave the set, and the slots of states new to
// it, reach the hash table.  Found states are numbered by tile scans, so
// the rows a step gives them are the same in every run.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.hpp"
#include "warm.hpp"

namespace paces {

namespace {

constexpr uint64_t kTomb = 0xFFFFFFFF00000000ull;  // entry of a dropped row
constexpr uint32_t kOwnerW = 0xFFFFFFFEu;           // candidate owns its key

// Whether slot s of a row with payload pay is structurally nonzero (the
// test of slot_target without forming the key).
__device__ __forceinline__ bool slot_live(const DevModel& m, uint64_t pay,
                                          int s) {
  const int j = pay_site(pay);
  if (s < 2 * m.ndim) {
    if (!((m.hop_mask >> (s >> 1)) & 1u)) return false;
    return m.nbr[j * 2 * m.ndim + s] >= 0;
  }
  const int e = s - 2 * m.ndim, nu = e >> 1;
  if (!((m.eph_mask >> nu) & 1u)) return false;
  const int n = pay_occ(pay, nu);
  return (e & 1) == 0 ? n > 0 : n < m.cut[nu];
}

// Whether a distance byte marks a row of the new set: a live row within k,
// or a state found this step (kNewRow | r, below kHole).
__device__ __forceinline__ bool kept(uint8_t d, int k) {
  return d <= k || (d >= kNewRow && d < kHole);
}

// Row of the q-th state found this step: the q-th hole, else the next row
// past the set's range.
__device__ __forceinline__ int64_t found_row(int64_t q, const StepCtl* ctl,
                                             const uint32_t* freel) {
  const int64_t nf = ctl->nfree;
  return q < nf ? int64_t(freel[q]) : int64_t(ctl->n_old) + (q - nf);
}

// Row of key k in the table (plain or staged entry; tombstones and
// candidates passed over), or -1.
template <int W>
__device__ __forceinline__ int64_t warm_find(const uint64_t* table,
                                             uint64_t mask,
                                             const uint64_t* keys,
                                             const uint64_t (&k)[W],
                                             uint64_t h) {
  const uint32_t tag = hash_tag(h);
  uint64_t i = h & mask;
  for (uint64_t probes = 0; probes <= mask && probes < kMaxProbe; ++probes) {
    const uint64_t e = table[i];
    if (e == kEmpty) break;
    if (uint32_t(e >> 32) == tag) {
      const uint32_t v = uint32_t(e);
      if (!(v & kCand)) {
        const int64_t row = int64_t(v & ~kStaged);
        if (key_eq<W>(k, keys + row * W)) return row;
      }
    }
    i = (i + 1) & mask;
  }
  return -1;
}

// Slot of the table entry of key k whose value is `value`, or -1.
template <int W>
__device__ __forceinline__ int64_t warm_slot(const uint64_t* table,
                                             uint64_t mask,
                                             const uint64_t (&k)[W],
                                             uint64_t h, uint32_t value) {
  const uint32_t tag = hash_tag(h);
  uint64_t i = h & mask;
  for (uint64_t probes = 0; probes <= mask && probes < kMaxProbe; ++probes) {
    const uint64_t e = table[i];
    if (e == kEmpty) break;
    if (uint32_t(e >> 32) == tag && uint32_t(e) == value) return int64_t(i);
    i = (i + 1) & mask;
  }
  return -1;
}

// ---- start ------------------------------------------------------------------
// kHole stays, every other byte becomes kFar (bytes past n_old of the last
// word belong to rows past the range, which a step writes before reading).
__global__ void __launch_bounds__(kBlock)
    k_warm_fill(uint8_t* dist, const StepCtl* ctl, const int* err) {
  if (*err) return;
  uint32_t* d4 = reinterpret_cast<uint32_t*>(dist);
  const int64_t n4 = cdiv(int64_t(ctl->n_old), 4);
  for (int64_t i = gtid(); i < n4; i += gstride()) {
    const uint32_t v = d4[i];
    uint32_t o = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const uint32_t byte = (v >> (8 * b)) & 0xFFu;
      o |= (byte == kHole ? uint32_t(kHole) : uint32_t(kFar)) << (8 * b);
    }
    d4[i] = o;
  }
}

// Rows of [0, n) with a given distance byte (d >= 0) or live (d < 0),
// counted per tile of the select layout, then written in row order.
__device__ __forceinline__ bool dist_hit(uint8_t v, int d) {
  return d < 0 ? v != kHole : v == uint8_t(d);
}

__global__ void __launch_bounds__(kBlock)
    k_dist_count(const uint8_t* dist, const uint32_t* nptr, int d,
                 uint32_t* bsum) {
  const int64_t n = *nptr, ntiles = cdiv(n, kTile);
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    uint32_t v = 0;
#pragma unroll
    for (int q = 0; q < kItems; ++q) {
      const int64_t e = t * kTile + q * kBlock + threadIdx.x;
      if (e < n && dist_hit(dist[e], d)) ++v;
    }
    uint32_t tot;
    block_excl_scan(v, &tot);
    if (threadIdx.x == 0) bsum[t] = tot;
  }
}

__global__ void __launch_bounds__(kBlock)
    k_dist_write(int Wi, const uint64_t* keys, const uint8_t* dist,
                 const uint32_t* nptr, int d, const uint32_t* bsum,
                 uint64_t* out, uint32_t* rows) {
  const int64_t n = *nptr, ntiles = cdiv(n, kTile);
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    uint32_t run = bsum[t];
#pragma unroll 1
    for (int q = 0; q < kItems; ++q) {
      const int64_t e = t * kTile + q * kBlock + threadIdx.x;
      const bool hit = e < n && dist_hit(dist[e], d);
      uint32_t tot;
      const uint32_t off = block_excl_scan(hit ? 1u : 0u, &tot) + run;
      run += tot;
      if (!hit) continue;
      if (rows) rows[off] = uint32_t(e);
      if (out)
        for (int w = 0; w < Wi; ++w)
          out[int64_t(off) * Wi + w] = keys[e * Wi + w];
    }
  }
}

__global__ void __launch_bounds__(kBlock)
    k_warm_mark(DevModel m, StepCtl* ctl, const uint32_t* midx,
                const uint64_t* pay, uint8_t* dist, uint32_t* cnt_m,
                int holes, const int* err) {
  __shared__ uint32_t bins[kMaxReal];
  if (*err) return;
  const int64_t nM = ctl->nM;
  if (m.R == 1) {
    // one realization: |M| is the selection's count (cnt_m was cleared by
    // the step's start)
    for (int64_t i = gtid(); i < nM; i += gstride()) dist[midx[i]] = 0;
    if (gtid() == 0) cnt_m[0] = uint32_t(nM);
  } else {
    for (int r = threadIdx.x; r < m.R; r += blockDim.x) bins[r] = 0;
    __syncthreads();
    for (int64_t i = gtid(); i < nM; i += gstride()) {
      const uint32_t r = midx[i];
      dist[r] = 0;
      atomicAdd(&bins[pay_real(pay[r])], 1u);
    }
    count_flush(m.R, bins, cnt_m);
  }
  if (gtid() == 0) {
    if (!holes) ctl->nfree = 0;
    ctl->n_staged = 0;
    ctl->gstart[0] = 0;
    ctl->gstart[1] = 0;
    ctl->w_noc = 0;
    ctl->w_nkeep = 0;
    ctl->w_moved = 0;
    ctl->w_tomb = 0;
    ctl->n_live = 0;
  }
}

// ---- a round ----------------------------------------------------------------
// Live rows at distance r-1, in the select tile layout.  Count pass:
// columns mark their rows at distance r (unless nearer; every writer
// writes r, and no row at distance r-1 is written in round r), the slots
// whose neighbour lies outside the set go to wmask and are counted per
// tile.  Write pass: those slots as candidates, in tile order.  Holes and
// found states never match r-1.
template <bool WRITE, int D>
__global__ void __launch_bounds__(kBlock)
    k_warm_old(DevModel m, int r, const StepCtl* ctl, const uint64_t* pay,
               const int32_t* col, uint8_t* dist, uint16_t* wmask,
               uint32_t* bsum, uint64_t* wlist, int64_t cand_cap, int* err) {
  if (*err) return;
  const uint8_t front = uint8_t(r - 1);
  const int64_t n = ctl->n_old, ntiles = cdiv(n, kTile);
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    uint32_t run = WRITE ? bsum[t] : 0u, cnt = 0;
#pragma unroll 1
    for (int q = 0; q < kItems; ++q) {
      const int64_t e = t * kTile + q * kBlock + threadIdx.x;
      uint32_t msk = 0;
      if (e < n && dist[e] == front) {
        if (WRITE) {
          msk = wmask[e];
        } else {
          const uint64_t p = pay[e];
          int32_t cs[D];
          load_cols<D>(col + e * D, cs);
#pragma unroll
          for (int s = 0; s < D; ++s) {
            const int32_t c = cs[s];
            if (c >= 0) {
              if (dist[c] > r) dist[c] = uint8_t(r);
            } else if (slot_live(m, p, s)) {
              msk |= 1u << s;
            }
          }
          wmask[e] = uint16_t(msk);
        }
      }
      const uint32_t nb = __popc(msk);
      if (WRITE) {
        uint32_t tot;
        uint64_t off = uint64_t(block_excl_scan(nb, &tot)) + run;
        run += tot;
        while (msk) {
          const int s = __ffs(msk) - 1;
          msk &= msk - 1;
          if (int64_t(off) < cand_cap)
            wlist[off] = (uint64_t(e) << 8) | uint64_t(s);
          else
            atomicOr(err, kErrChunks);
          ++off;
        }
      } else {
        cnt += nb;
      }
    }
    if (!WRITE) {
      uint32_t tot;
      block_excl_scan(cnt, &tot);
      if (threadIdx.x == 0) bsum[t] = tot;
    }
  }
}

// Candidates of round r: w_noc from live rows, then every slot of the
// states found in round r-1; the round's states are numbered from
// n_staged on.
__global__ void k_warm_prep(StepCtl* ctl, int r, int D, int64_t cand_cap,
                            int* err) {
  if (*err) return;
  const int64_t noc = ctl->w_noc;
  const int64_t nf = int64_t(ctl->gstart[r]) - ctl->gstart[r - 1];
  int64_t nc = noc + nf * D;
  if (nc > cand_cap) {
    atomicOr(err, kErrChunks);
    nc = 0;
  }
  ctl->w_f0 = ctl->gstart[r - 1];
  ctl->r_ncand = uint32_t(nc);
  ctl->r_ntiles = uint32_t(cdiv(nc, kBlock));
  ctl->r_ncur = ctl->n_staged;
  ctl->r_total = 0;
}

// Key of candidate c and its parent's row: a live row (from wlist) or the
// row of a state found in the round before.  False for a structurally
// zero slot.
template <int W>
__device__ __forceinline__ bool warm_cand(const DevModel& m,
                                          const StepCtl* ctl,
                                          const uint32_t* freel, int64_t noc,
                                          int64_t f0, const uint64_t* wlist,
                                          const Side& c, int64_t cand,
                                          uint64_t (&k)[W], int64_t& p,
                                          int& s) {
  if (cand < noc) {
    const uint64_t e = wlist[cand];
    p = int64_t(e >> 8);
    s = int(e & 0xFFu);
  } else {
    const int64_t d = cand - noc;
    p = found_row(f0 + d / m.D, ctl, freel);
    s = int(d % m.D);
  }
  uint64_t par[W];
  load_key<W>(c.keys, p, par);
  return slot_target<W>(m, par, c.pay[p], s, k);
}

// Insert-if-absent of each candidate's key.  Table values: a live row, a
// found state's row (kStaged | row) or, during the round, kCand |
// candidate.  A key found as a live row marks it at distance r; a key
// found staged or claimed by another candidate needs nothing; the
// candidate whose compare-and-swap fills an empty slot owns the key (probe
// distance into c_slot), counted per tile of candidates.  Tombstones are
// passed over and never claimed, so removing the staged entries restores
// the table.
template <int W>
__global__ void __launch_bounds__(kBlock)
    k_warm_probe(DevModel m, int r, const StepCtl* ctl, Side c,
                 const uint32_t* freel, const uint64_t* wlist,
                 uint64_t* table, uint64_t mask, uint32_t* c_slot,
                 uint32_t* c_ref, uint32_t* tile_cnt, int* err) {
  if (*err) return;
  const int64_t nc = ctl->r_ncand, noc = ctl->w_noc, f0 = ctl->w_f0;
  const int64_t ntiles = cdiv(nc, kBlock);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t cand = tile * kBlock + threadIdx.x;
    uint32_t owner = 0;
    if (cand < nc) {
      uint64_t k[W];
      int64_t p;
      int s;
      uint32_t ref = kNone;
      if (warm_cand<W>(m, ctl, freel, noc, f0, wlist, c, cand, k, p, s)) {
        const uint64_t h = key_hash<W>(m, k);
        const uint32_t tag = hash_tag(h);
        const uint64_t mine =
            (uint64_t(tag) << 32) | uint64_t(kCand | uint32_t(cand));
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
              ref = kOwnerW;
              c_slot[cand] = uint32_t(probes);
              owner = 1;
              done = true;
              break;
            }
            e = old;
          }
          if (uint32_t(e >> 32) == tag) {
            const uint32_t v = uint32_t(e);
            if (v & kCand) {
              const int64_t c2 = int64_t(v & ~kCand);
              uint64_t k2[W];
              int64_t p2;
              int s2;
              warm_cand<W>(m, ctl, freel, noc, f0, wlist, c, c2, k2, p2, s2);
              bool same = true;
#pragma unroll
              for (int q = 0; q < W; ++q) same &= (k2[q] == k[q]);
              done = same;
            } else {
              const int64_t row = int64_t(v & ~kStaged);
              if (key_eq<W>(k, c.keys + row * W)) {
                // a live row is within distance r; a staged one is nearer
                if (!(v & kStaged) && c.dist[row] > r)
                  c.dist[row] = uint8_t(r);
                done = true;
              }
            }
            if (done) break;
          }
          i = (i + 1) & mask;
        }
        if (!done) atomicOr(err, kErrTableFull);
      }
      c_ref[cand] = ref;
    }
    uint32_t tot;
    block_excl_scan(owner, &tot);
    if (threadIdx.x == 0) tile_cnt[tile] = tot;
  }
}

// Owners take their rows (numbered by the tile scan): key, payload,
// totals, distance kNewRow | r, amplitude 0; their table slot points at
// the row, staged.
template <int W, typename Amp>
__global__ void __launch_bounds__(kBlock)
    k_warm_commit(DevModel m, int r, const StepCtl* ctl, int64_t cap, Side c,
                  const uint32_t* freel, const uint64_t* wlist,
                  uint64_t* table, uint64_t mask, const uint32_t* c_slot,
                  const uint32_t* c_ref, const uint32_t* tile_base, Amp* psi,
                  int* err) {
  if (*err) return;
  const int64_t nc = ctl->r_ncand, noc = ctl->w_noc, f0 = ctl->w_f0;
  const int64_t n_cur = ctl->r_ncur, ntiles = cdiv(nc, kBlock);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t cand = tile * kBlock + threadIdx.x;
    const bool own = cand < nc && c_ref[cand] == kOwnerW;
    uint32_t tot_in_tile;
    const uint32_t rank = block_excl_scan(own ? 1u : 0u, &tot_in_tile);
    if (!own) continue;
    const int64_t row = found_row(n_cur + tile_base[tile] + rank, ctl, freel);
    if (row >= cap) {
      atomicOr(err, kErrCapacity);
      continue;
    }
    uint64_t k[W];
    int64_t p;
    int s;
    warm_cand<W>(m, ctl, freel, noc, f0, wlist, c, cand, k, p, s);
    store_key<W>(c.keys, row, k);
    uint64_t np, nt;
    slot_row_info<W>(m, k, c.pay[p], c.tot[p], s, np, nt);
    c.pay[row] = np;
    c.tot[row] = nt;
    c.dist[row] = uint8_t(kNewRow | r);
    const uint64_t h = key_hash<W>(m, k);
    table[((h & mask) + c_slot[cand]) & mask] =
        (uint64_t(hash_tag(h)) << 32) | uint64_t(kStaged | uint32_t(row));
    Amp z;
    z.x = 0;
    z.y = 0;
    psi[row] = z;
  }
}

__global__ void k_warm_finish(StepCtl* ctl, int r, const int* err) {
  if (*err) return;
  const uint32_t n = ctl->r_ncur + ctl->r_total;
  ctl->n_staged = n;
  ctl->gstart[r + 1] = n;
}

// ---- sizes ------------------------------------------------------------------
__global__ void k_warm_range(StepCtl* ctl, int R, uint32_t* ball,
                             const int* err) {
  if (*err) return;
  const int64_t extra = int64_t(ctl->n_staged) - ctl->nfree;
  ctl->n_new = uint32_t(int64_t(ctl->n_old) + (extra > 0 ? extra : 0));
  ctl->n_live = 0;
  for (int r = 0; r < R; ++r) ball[r] = 0u;
}

// Live rows of the new set, in total and per realization (counted only
// when per_real).  A thread reads the distances of 16 rows at once (the
// array's allocation is a multiple of 256 bytes, so the last group stays
// inside it).
__global__ void __launch_bounds__(kBlock)
    k_warm_live(DevModel m, int k, StepCtl* ctl, const uint8_t* dist,
                const uint64_t* pay, int per_real, uint32_t* ball,
                const int* err) {
  __shared__ uint32_t bins[kMaxReal];
  if (*err) return;
  if (per_real) {
    for (int r = threadIdx.x; r < m.R; r += blockDim.x) bins[r] = 0;
    __syncthreads();
  }
  const int64_t n = ctl->n_new, n16 = cdiv(n, 16);
  const uint4* d16 = reinterpret_cast<const uint4*>(dist);
  uint32_t live = 0;
  for (int64_t g = gtid(); g < n16; g += gstride()) {
    const uint4 v = d16[g];
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int64_t e = g * 16 + q;
      if (e >= n || !kept(uint8_t(w[q >> 2] >> (8 * (q & 3))), k)) continue;
      ++live;
      if (per_real) atomicAdd(&bins[pay_real(pay[e])], 1u);
    }
  }
  uint32_t tot;
  block_excl_scan(live, &tot);
  if (threadIdx.x == 0 && tot) atomicAdd(&ctl->n_live, tot);
  if (per_real) count_flush(m.R, bins, ball);
}

__global__ void k_warm_cap_over(int R, int64_t max_states,
                                 const uint32_t* ball, int* err) {
  if (*err) return;
  for (int r = 0; r < R; ++r)
    if (int64_t(ball[r]) > max_states) atomicOr(err, kErrCap);
}

// ---- the commit -------------------------------------------------------------
// Live rows the search did not reach become holes: weight into the
// partials, amplitude 0, table entry a tombstone, columns of the row and
// of its neighbours toward it -1, distance kHole.
template <int W, typename Amp>
__global__ void __launch_bounds__(kBlock)
    k_warm_drop(DevModel m, int k, StepCtl* ctl, Side c, uint64_t* table,
                uint64_t mask, Amp* psi, double* mass_part, const int* err) {
  __shared__ double bins[kMaxReal];
  if (*err) return;
  if (gtid() == 0) ctl->w_moved = 1;
  const int R = m.R, D = m.D;
  if (R > 1) {
    for (int r = threadIdx.x; r < R; r += blockDim.x) bins[r] = 0.0;
    __syncthreads();
  }
  const int64_t nold = ctl->n_old;
  double lost = 0;
  uint32_t tombs = 0;
  for (int64_t e = gtid(); e < nold; e += gstride()) {
    if (c.dist[e] != kFar) continue;
    const Amp v = psi[e];
    if (R > 1)
      atomicAdd(&bins[pay_real(c.pay[e])], weight(v));
    else
      lost += weight(v);
    Amp z;
    z.x = 0;
    z.y = 0;
    psi[e] = z;
    uint64_t key[W];
    load_key<W>(c.keys, e, key);
    const int64_t sl =
        warm_slot<W>(table, mask, key, key_hash<W>(m, key), uint32_t(e));
    if (sl >= 0) {
      table[sl] = kTomb;
      ++tombs;
    }
    for (int s = 0; s < D; ++s) {
      const int32_t nb = c.col[e * D + s];
      // a neighbour that stays (within k) loses its column toward e; one
      // dropped too clears its own
      if (nb >= 0 && c.dist[nb] <= k) c.col[int64_t(nb) * D + (s ^ 1)] = -1;
      c.col[e * D + s] = -1;
    }
    c.dist[e] = kHole;
  }
  if (R > 1) {
    __syncthreads();
    for (int r = threadIdx.x; r < R; r += blockDim.x)
      mass_part[int64_t(blockIdx.x) * R + r] = bins[r];
  } else {
    lost = block_sum(lost);
    if (threadIdx.x == 0) mass_part[blockIdx.x] = lost;
  }
  uint32_t tot;
  block_excl_scan(tombs, &tot);
  if (threadIdx.x == 0 && tot) atomicAdd(&ctl->w_tomb, tot);
}

// States found this step: distance r, table entry plain (lane of slot 0),
// columns by lookup.  An edge is seen from both ends as slots s and s ^ 1,
// so a found state also sets the column of a live row toward it (that row
// had -1 there: the state was outside the old set); between two found
// states both ends write the same values.
template <int W>
__global__ void __launch_bounds__(kBlock)
    k_warm_fix(DevModel m, const StepCtl* ctl, Side c, const uint32_t* freel,
               uint64_t* table, uint64_t mask, const int* err) {
  if (*err) return;
  const int D = m.D;
  const int64_t ns = ctl->n_staged;
  for (int64_t t = gtid(); t < ns * D; t += gstride()) {
    const int64_t q = t / D;
    const int s = int(t % D);
    const int64_t row = found_row(q, ctl, freel);
    uint64_t par[W], k[W];
    load_key<W>(c.keys, row, par);
    if (s == 0) {
      const uint64_t h = key_hash<W>(m, par);
      const int64_t sl = warm_slot<W>(table, mask, par, h,
                                      kStaged | uint32_t(row));
      if (sl >= 0)
        table[sl] = (uint64_t(hash_tag(h)) << 32) | uint64_t(row);
      c.dist[row] = uint8_t(c.dist[row] & ~kNewRow);
    }
    int32_t out = -1;
    if (slot_target<W>(m, par, c.pay[row], s, k)) {
      const int64_t f = warm_find<W>(table, mask, c.keys, k, key_hash<W>(m, k));
      if (f >= 0) {
        out = int32_t(f);
        c.col[f * D + (s ^ 1)] = int32_t(row);
      }
    }
    c.col[row * D + s] = out;
  }
}

// ---- repeat and bookkeeping ---------------------------------------------------
__global__ void __launch_bounds__(kBlock)
    k_warm_unstage_table(uint64_t* table, uint64_t mask) {
  const int64_t P = int64_t(mask) + 1;
  for (int64_t i = gtid(); i < P; i += gstride()) {
    const uint64_t e = table[i];
    if (e == kEmpty || uint32_t(e >> 32) == 0xFFFFFFFFu) continue;
    if (uint32_t(e) & (kCand | kStaged)) table[i] = kEmpty;
  }
}

// Holes that took a found state become holes again (bytes past the range
// need nothing).
__global__ void __launch_bounds__(kBlock)
    k_warm_unstage_rows(uint8_t* dist, int64_t n) {
  for (int64_t e = gtid(); e < n; e += gstride()) {
    const uint8_t d = dist[e];
    if (d >= kNewRow && d < kHole) dist[e] = kHole;
  }
}

__global__ void __launch_bounds__(kBlock)
    k_dist_rounds(const StepCtl* ctl, int k, uint8_t* dist) {
  const int64_t n = ctl->n_new;
  for (int64_t e = gtid(); e < n; e += gstride()) {
    int r = 0;
    while (r < k && e >= int64_t(ctl->fstart[r + 1])) ++r;
    dist[e] = uint8_t(r);
  }
}

__global__ void __launch_bounds__(kBlock)
    k_dist_fill(uint8_t* dist, int64_t n, uint8_t v) {
  for (int64_t e = gtid(); e < n; e += gstride()) dist[e] = v;
}

__global__ void k_u32_set(uint32_t* out, int64_t v) { *out = uint32_t(v); }

__global__ void __launch_bounds__(kBlock)
    k_gather_rows(int Wi, int A8, const uint64_t* keys, const uint64_t* pay,
                  const uint64_t* tot, const uint64_t* psi,
                  const uint32_t* idx, int64_t n, uint64_t* okeys,
                  uint64_t* opay, uint64_t* otot, uint64_t* oamps) {
  for (int64_t i = gtid(); i < n; i += gstride()) {
    const int64_t r = idx[i];
    if (okeys)
      for (int w = 0; w < Wi; ++w) okeys[i * Wi + w] = keys[r * Wi + w];
    if (opay) opay[i] = pay[r];
    if (otot) otot[i] = tot[r];
    if (oamps)
      for (int w = 0; w < A8; ++w) oamps[i * A8 + w] = psi[r * A8 + w];
  }
}

}  // namespace

// ---- host wrappers ----------------------------------------------------------

void warm_begin(const DevModel& m, StepCtl* ctl, const uint32_t* midx,
                const Side& c, const WarmBufs& wb, uint32_t* cnt_m,
                int64_t n_old, bool holes, uint32_t* scan_tmp, int* err,
                hipStream_t s) {
  k_warm_fill<<<grid_for(cdiv(n_old, 4)), kBlock, 0, s>>>(c.dist, ctl, err);
  if (holes) {
    // holes, ascending, into the free list
    const int g = tiles_for(n_old);
    k_dist_count<<<g, kBlock, 0, s>>>(c.dist, &ctl->n_old, int(kHole),
                                      scan_tmp);
    tile_sums_scan(scan_tmp, &ctl->n_old, &ctl->nfree, err, s);
    k_dist_write<<<g, kBlock, 0, s>>>(1, nullptr, c.dist, &ctl->n_old,
                                      int(kHole), scan_tmp, nullptr, wb.freel);
  }
  k_warm_mark<<<grid_for(n_old), kBlock, 0, s>>>(m, ctl, midx, c.pay, c.dist,
                                                  cnt_m, holes ? 1 : 0, err);
}

void warm_round(const DevModel& m, int Wi, int prec, const Side& c, int r,
                StepCtl* ctl, int64_t cap, int64_t n_old, int64_t est,
                uint64_t* table, uint64_t mask, const RoundBufs& rb,
                const WarmBufs& wb, uint32_t* scan_tmp, void* psi, int* err,
                hipStream_t s) {
  const int D = m.D;
  const int go = tiles_for(n_old);
#define PACES_WARM_OLD(WRITE)                                                 \
  switch (D) {                                                                \
    case 4: k_warm_old<WRITE, 4><<<go, kBlock, 0, s>>>(PACES_WARM_OLD_ARGS); break;   \
    case 6: k_warm_old<WRITE, 6><<<go, kBlock, 0, s>>>(PACES_WARM_OLD_ARGS); break;   \
    case 8: k_warm_old<WRITE, 8><<<go, kBlock, 0, s>>>(PACES_WARM_OLD_ARGS); break;   \
    case 10: k_warm_old<WRITE, 10><<<go, kBlock, 0, s>>>(PACES_WARM_OLD_ARGS); break; \
    case 12: k_warm_old<WRITE, 12><<<go, kBlock, 0, s>>>(PACES_WARM_OLD_ARGS); break; \
    case 14: k_warm_old<WRITE, 14><<<go, kBlock, 0, s>>>(PACES_WARM_OLD_ARGS); break; \
    default: break;                                                           \
  }
#define PACES_WARM_OLD_ARGS \
  m, r, ctl, c.pay, c.col, c.dist, wb.wmask, scan_tmp, wb.wlist, rb.cand_cap, err
  PACES_WARM_OLD(false)
  tile_sums_scan(scan_tmp, &ctl->n_old, &ctl->w_noc, err, s);
  PACES_WARM_OLD(true)
#undef PACES_WARM_OLD_ARGS
#undef PACES_WARM_OLD
  k_warm_prep<<<1, 1, 0, s>>>(ctl, r, D, rb.cand_cap, err);
  // candidates: at most the set's slots plus the new states'
  const int64_t nc_bound = std::min<int64_t>(rb.cand_cap, (n_old + est) * D);
  const int g = grid_for(nc_bound);
  PACES_DISPATCH_W(Wi, k_warm_probe<WW><<<g, kBlock, 0, s>>>(
                           m, r, ctl, c, wb.freel, wb.wlist, table, mask,
                           rb.c_slot, rb.c_ref, rb.tile_cnt, err));
  tile_scan(rb.tile_cnt, &ctl->r_ntiles, cdiv(nc_bound, kBlock), rb.scan_tmp,
            rb.tile_base, &ctl->r_total, err, s);
  if (prec == 64) {
    PACES_DISPATCH_W(Wi, k_warm_commit<WW, double2><<<g, kBlock, 0, s>>>(
                             m, r, ctl, cap, c, wb.freel, wb.wlist, table,
                             mask, rb.c_slot, rb.c_ref, rb.tile_base,
                             (double2*)psi, err));
  } else {
    PACES_DISPATCH_W(Wi, k_warm_commit<WW, float2><<<g, kBlock, 0, s>>>(
                             m, r, ctl, cap, c, wb.freel, wb.wlist, table,
                             mask, rb.c_slot, rb.c_ref, rb.tile_base,
                             (float2*)psi, err));
  }
  k_warm_finish<<<1, 1, 0, s>>>(ctl, r, err);
}

void warm_sizes(const DevModel& m, const Side& c, int k, StepCtl* ctl,
                int64_t est, int64_t max_states, uint32_t* ball, int* err,
                hipStream_t s) {
  k_warm_range<<<1, 1, 0, s>>>(ctl, m.R, ball, err);
  const int per_real = (m.R > 1 || max_states > 0) ? 1 : 0;
  // 16 rows per thread and one count added to the total per block
  k_warm_live<<<std::min(grid_for(cdiv(est, 16)), 512), kBlock, 0, s>>>(
      m, k, ctl, c.dist, c.pay, per_real, ball, err);
  if (max_states > 0)
    k_warm_cap_over<<<1, 1, 0, s>>>(m.R, max_states, ball, err);
}

int warm_commit(const DevModel& m, int Wi, int prec, const Side& c, int k,
                StepCtl* ctl, int64_t n_old, int64_t est, uint64_t* table,
                uint64_t mask, const WarmBufs& wb, void* psi,
                double* mass_part, int* err, hipStream_t s) {
  const int g = std::min(grid_for(n_old), kPartBlocks);
  if (prec == 64) {
    PACES_DISPATCH_W(Wi, k_warm_drop<WW, double2><<<g, kBlock, 0, s>>>(
                             m, k, ctl, c, table, mask, (double2*)psi,
                             mass_part, err));
  } else {
    PACES_DISPATCH_W(Wi, k_warm_drop<WW, float2><<<g, kBlock, 0, s>>>(
                             m, k, ctl, c, table, mask, (float2*)psi,
                             mass_part, err));
  }
  PACES_DISPATCH_W(Wi, k_warm_fix<WW><<<grid_for(est * m.D), kBlock, 0, s>>>(
                           m, ctl, c, wb.freel, table, mask, err));
  return g;
}

void warm_unstage(const StepCtl* ctl, const Side& c, const WarmBufs& wb,
                  uint64_t* table, uint64_t mask, int64_t n_old,
                  hipStream_t s) {
  (void)ctl;
  (void)wb;
  k_warm_unstage_table<<<grid_for(int64_t(mask) + 1), kBlock, 0, s>>>(table,
                                                                      mask);
  if (n_old > 0)
    k_warm_unstage_rows<<<grid_for(n_old), kBlock, 0, s>>>(c.dist, n_old);
}

void dist_of_rounds(const StepCtl* ctl, int k, uint8_t* dist, int64_t est,
                    hipStream_t s) {
  k_dist_rounds<<<grid_for(est), kBlock, 0, s>>>(ctl, k, dist);
}

void dist_fill(uint8_t* dist, int64_t n, uint8_t v, hipStream_t s) {
  if (n > 0) k_dist_fill<<<grid_for(n), kBlock, 0, s>>>(dist, n, v);
}

void rows_at_distance(int Wi, const uint64_t* keys, const uint8_t* dist,
                      int64_t n, int d, uint64_t* out, uint32_t* rows,
                      uint32_t* count, uint32_t* tmp, hipStream_t s) {
  if (n <= 0) {
    k_u32_set<<<1, 1, 0, s>>>(count, 0);
    return;
  }
  const int g = tiles_for(n);
  // the kernels read the row count from device memory: the last word of
  // tmp, past the tile sums; the word before it is a clear latch for the
  // scan, which skips its work when its latch is set (the sim's own may
  // hold the error of a step that is being repeated)
  uint32_t* nrows = tmp + scan_tmp_words(n) - 1;
  int* clear = reinterpret_cast<int*>(tmp + scan_tmp_words(n) - 2);
  k_u32_set<<<1, 1, 0, s>>>(nrows, n);
  k_u32_set<<<1, 1, 0, s>>>(reinterpret_cast<uint32_t*>(clear), 0);
  k_dist_count<<<g, kBlock, 0, s>>>(dist, nrows, d, tmp);
  tile_sums_scan(tmp, nrows, count, clear, s);
  k_dist_write<<<g, kBlock, 0, s>>>(Wi, keys, dist, nrows, d, tmp, out, rows);
}

void gather_rows(int Wi, size_t A, const Side& c, const void* psi,
                 const uint32_t* idx, int64_t n, uint64_t* keys,
                 uint64_t* pay, uint64_t* tot, void* amps, hipStream_t s) {
  if (n <= 0) return;
  k_gather_rows<<<grid_for(n), kBlock, 0, s>>>(
      Wi, int(A / 8), c.keys, c.pay, c.tot, static_cast<const uint64_t*>(psi),
      idx, n, keys, pay, tot, static_cast<uint64_t*>(amps));
}

}  // namespace paces
