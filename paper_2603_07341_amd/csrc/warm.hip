// warm.hip -- expansion of a step from the previous step's graph on gfx950
// (the method and its invariants are described in warm.hpp).
//
// Old rows are walked in tiles of kTile rows (one u8 distance each, the
// columns of the frontier rows), so the search inside the old set streams
// its arrays; only slots that leave the old set, and the slots of states
// new to the set, reach the hash table.  New rows are numbered by tile
// scans, so the row order of a step is the same in every run.
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

// Outcome of a lookup in a table that holds old rows and staged rows.
struct Found {
  int64_t row;  // -1: absent
  bool staged;  // row of the new set (else of the old set)
};

// Key k in the table: old rows compare against keys_o, staged rows against
// keys_n; tombstones and candidates are passed over.
template <int W>
__device__ __forceinline__ Found warm_find(const uint64_t* table,
                                           uint64_t mask,
                                           const uint64_t* keys_o,
                                           const uint64_t* keys_n,
                                           const uint64_t (&k)[W],
                                           uint64_t h) {
  const uint32_t tag = hash_tag(h);
  uint64_t i = h & mask;
  for (uint64_t probes = 0; probes <= mask && probes < kMaxProbe; ++probes) {
    const uint64_t e = table[i];
    if (e == kEmpty) break;
    if (uint32_t(e >> 32) == tag) {
      const uint32_t v = uint32_t(e);
      if (v & kStaged) {
        const uint32_t q = v & ~kStaged;
        if (!(v & kCand) && key_eq<W>(k, keys_n + int64_t(q) * W))
          return Found{int64_t(q), true};
      } else if (!(v & kCand)) {
        if (key_eq<W>(k, keys_o + int64_t(v) * W)) return Found{int64_t(v), false};
      }
    }
    i = (i + 1) & mask;
  }
  return Found{-1, false};
}

// ---- start ------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
    k_warm_fill(uint8_t* dist, const StepCtl* ctl, const int* err) {
  if (*err) return;
  uint32_t* d4 = reinterpret_cast<uint32_t*>(dist);
  const int64_t n4 = cdiv(int64_t(ctl->n_old), 4);
  for (int64_t i = gtid(); i < n4; i += gstride()) d4[i] = 0xFFFFFFFFu;
}

__global__ void __launch_bounds__(kBlock)
    k_warm_mark(DevModel m, StepCtl* ctl, const uint32_t* midx,
                const uint64_t* pay_o, uint8_t* dist, uint32_t* cnt_m,
                const int* err) {
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
      atomicAdd(&bins[pay_real(pay_o[r])], 1u);
    }
    count_flush(m.R, bins, cnt_m);
  }
  if (gtid() == 0) {
    ctl->n_staged = 0;
    ctl->gstart[0] = 0;
    ctl->gstart[1] = 0;
    ctl->w_noc = 0;
    ctl->w_nkeep = 0;
    ctl->w_moved = 0;
    ctl->w_tomb = 0;
  }
}

// ---- a round ----------------------------------------------------------------
// Old rows at distance r-1, in the select tile layout.  Count pass: columns
// into the old set mark their rows at distance r (unless nearer; every
// writer writes r, and no row at distance r-1 is written in round r), the
// slots whose neighbour lies outside the old set go to wmask and are
// counted per tile.  Write pass: those slots as candidates, in tile order.
template <bool WRITE, int D>
__global__ void __launch_bounds__(kBlock)
    k_warm_old(DevModel m, int r, const StepCtl* ctl, const uint64_t* pay_o,
               const int32_t* col_o, uint8_t* dist, uint16_t* wmask,
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
          const uint64_t p = pay_o[e];
          int32_t cs[D];
          load_cols<D>(col_o + e * D, cs);
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

// Candidates of round r: w_noc from old rows, then every slot of the new
// states of round r-1; the round's rows start at n_staged.
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

// Key of candidate c: from an old row (keys_o) or a staged row (keys_n).
// Returns false for a structurally zero slot.
template <int W>
__device__ __forceinline__ bool warm_cand(const DevModel& m, int64_t noc,
                                          int64_t f0, const uint64_t* wlist,
                                          const Side& o, const Side& n,
                                          int64_t c, uint64_t (&k)[W],
                                          bool& from_old, int64_t& p,
                                          int& s) {
  uint64_t par[W];
  if (c < noc) {
    const uint64_t e = wlist[c];
    p = int64_t(e >> 8);
    s = int(e & 0xFFu);
    from_old = true;
    load_key<W>(o.keys, p, par);
    return slot_target<W>(m, par, o.pay[p], s, k);
  }
  const int64_t d = c - noc;
  p = f0 + d / m.D;
  s = int(d % m.D);
  from_old = false;
  load_key<W>(n.keys, p, par);
  return slot_target<W>(m, par, n.pay[p], s, k);
}

// Insert-if-absent of each candidate's key.  Table values: an old row, a
// staged row (kStaged | row) or, during the round, kCand | candidate.  A
// key found as an old row marks that row at distance r; a key found staged
// or claimed by another candidate needs nothing; the candidate whose
// compare-and-swap fills an empty slot owns the key (probe distance into
// c_slot), counted per tile of candidates.  Tombstones are passed over and
// never claimed, so removing the staged entries restores the old table.
template <int W>
__global__ void __launch_bounds__(kBlock)
    k_warm_probe(DevModel m, int r, const StepCtl* ctl, Side o, Side n,
                 const uint64_t* wlist, uint64_t* table, uint64_t mask,
                 uint32_t* c_slot, uint32_t* c_ref, uint32_t* tile_cnt,
                 int* err) {
  if (*err) return;
  const int64_t nc = ctl->r_ncand, noc = ctl->w_noc, f0 = ctl->w_f0;
  const int64_t ntiles = cdiv(nc, kBlock);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t c = tile * kBlock + threadIdx.x;
    uint32_t owner = 0;
    if (c < nc) {
      uint64_t k[W];
      bool from_old;
      int64_t p;
      int s;
      uint32_t ref = kNone;
      if (warm_cand<W>(m, noc, f0, wlist, o, n, c, k, from_old, p, s)) {
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
              ref = kOwnerW;
              c_slot[c] = uint32_t(probes);
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
              bool fo2;
              int64_t p2;
              int s2;
              warm_cand<W>(m, noc, f0, wlist, o, n, c2, k2, fo2, p2, s2);
              bool same = true;
#pragma unroll
              for (int q = 0; q < W; ++q) same &= (k2[q] == k[q]);
              done = same;
            } else if (v & kStaged) {
              done = key_eq<W>(k, n.keys + int64_t(v & ~kStaged) * W);
            } else if (key_eq<W>(k, o.keys + int64_t(v) * W)) {
              if (o.dist[v] > r) o.dist[v] = uint8_t(r);
              done = true;
            }
            if (done) break;
          }
          i = (i + 1) & mask;
        }
        if (!done) atomicOr(err, kErrTableFull);
      }
      c_ref[c] = ref;
    }
    uint32_t tot;
    block_excl_scan(owner, &tot);
    if (threadIdx.x == 0) tile_cnt[tile] = tot;
  }
}

// Owners append their key as a row of the new set (rows numbered by the
// tile scan), with payload, totals, distance r and phi 0, and point their
// table slot at it.
template <int W, typename Amp>
__global__ void __launch_bounds__(kBlock)
    k_warm_commit(DevModel m, int r, const StepCtl* ctl, int64_t cap, Side o,
                  Side n, const uint64_t* wlist, uint64_t* table,
                  uint64_t mask, const uint32_t* c_slot, const uint32_t* c_ref,
                  const uint32_t* tile_base, Amp* phi, int* err) {
  if (*err) return;
  const int64_t nc = ctl->r_ncand, noc = ctl->w_noc, f0 = ctl->w_f0;
  const int64_t n_cur = ctl->r_ncur, ntiles = cdiv(nc, kBlock);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t c = tile * kBlock + threadIdx.x;
    const bool own = c < nc && c_ref[c] == kOwnerW;
    uint32_t tot_in_tile;
    const uint32_t rank = block_excl_scan(own ? 1u : 0u, &tot_in_tile);
    if (!own) continue;
    const int64_t row = n_cur + tile_base[tile] + rank;
    if (row >= cap) {
      atomicOr(err, kErrCapacity);
      continue;
    }
    uint64_t k[W];
    bool from_old;
    int64_t p;
    int s;
    warm_cand<W>(m, noc, f0, wlist, o, n, c, k, from_old, p, s);
    store_key<W>(n.keys, row, k);
    const uint64_t py = from_old ? o.pay[p] : n.pay[p];
    const uint64_t tt = from_old ? o.tot[p] : n.tot[p];
    uint64_t np, nt;
    slot_row_info<W>(m, k, py, tt, s, np, nt);
    n.pay[row] = np;
    n.tot[row] = nt;
    n.dist[row] = uint8_t(r);
    const uint64_t h = key_hash<W>(m, k);
    table[((h & mask) + c_slot[c]) & mask] =
        (uint64_t(hash_tag(h)) << 32) | uint64_t(kStaged | uint32_t(row));
    Amp z;
    z.x = 0;
    z.y = 0;
    phi[row] = z;
  }
}

__global__ void k_warm_finish(StepCtl* ctl, int r, const int* err) {
  if (*err) return;
  const uint32_t n = ctl->r_ncur + ctl->r_total;
  ctl->n_staged = n;
  ctl->gstart[r + 1] = n;
}

// ---- the new set ------------------------------------------------------------
// Old rows that stay (distance <= k), counted per tile of the select layout.
__global__ void __launch_bounds__(kBlock)
    k_warm_keep_count(const uint8_t* dist, int k, const StepCtl* ctl,
                      uint32_t* bsum, const int* err) {
  if (*err) return;
  const int64_t n = ctl->n_old, ntiles = cdiv(n, kTile);
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    uint32_t v = 0;
#pragma unroll
    for (int q = 0; q < kItems; ++q) {
      const int64_t e = t * kTile + q * kBlock + threadIdx.x;
      if (e < n && dist[e] <= k) ++v;
    }
    uint32_t tot;
    block_excl_scan(v, &tot);
    if (threadIdx.x == 0) bsum[t] = tot;
  }
}

__global__ void k_warm_sizes(StepCtl* ctl, int64_t cap, int* err) {
  if (*err) return;
  const int64_t n = int64_t(ctl->n_staged) + ctl->w_nkeep;
  if (n > cap) {
    atomicOr(err, kErrCapacity);
    return;
  }
  ctl->n_new = uint32_t(n);
}

// New row of old row c from the keep map: the old rows that stay, one bit
// each in words of 64 rows, with the count of rows kept before each word
// (12 bytes per 64 rows, small enough to stay in the L2 cache where a row
// map of 4 bytes per row would not).  kNone for a dropped row.
struct KeepMap {
  const uint64_t* bits;
  const uint32_t* pre;
  uint32_t base;  // rows of the new set before the first old row
  __device__ __forceinline__ uint32_t row_of(int64_t c) const {
    const uint64_t w = bits[c >> 6];
    const int b = int(c & 63);
    if (!((w >> b) & 1ull)) return kNone;
    return base + pre[c >> 6] + uint32_t(__popcll(w & ((1ull << b) - 1ull)));
  }
};

// Old rows that stay move behind the staged rows in their old order: key,
// payload, totals (when the payload does not hold them), distance, phi =
// psi; the keep map (one ballot per wave of 64 consecutive rows); the
// weight of the dropped rows into per-block partials.
template <int W, typename Amp>
__global__ void __launch_bounds__(kBlock)
    k_warm_compact(DevModel m, int k, const StepCtl* ctl, Side o, Side n,
                   const Amp* psi_o, Amp* phi, const uint32_t* bsum,
                   uint64_t* kbits, uint32_t* kpre, double* mass_part,
                   int copy_tot, const int* err) {
  __shared__ double bins[kMaxReal];
  if (*err) return;
  const int R = m.R;
  if (R > 1) {
    for (int r = threadIdx.x; r < R; r += blockDim.x) bins[r] = 0.0;
    __syncthreads();
  }
  const int64_t nold = ctl->n_old, base = ctl->n_staged;
  const int64_t ntiles = cdiv(nold, kTile);
  const int lane = threadIdx.x & 63;
  double lost = 0;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    uint32_t run = bsum[t];
#pragma unroll 1
    for (int q = 0; q < kItems; ++q) {
      const int64_t e = t * kTile + q * kBlock + threadIdx.x;
      const uint8_t d = e < nold ? o.dist[e] : kFar;
      const bool keep = e < nold && d <= k;
      uint32_t tot;
      const uint32_t off = block_excl_scan(keep ? 1u : 0u, &tot) + run;
      run += tot;
      // lanes of a wave hold 64 consecutive rows, the first at a multiple
      // of 64: its ballot is the word of the keep map
      const uint64_t word = __ballot(keep);
      if (lane == 0 && e < nold) {
        kbits[e >> 6] = word;
        kpre[e >> 6] = off;
      }
      if (e >= nold) continue;
      const Amp v = psi_o[e];
      if (keep) {
        const int64_t row = base + off;
#pragma unroll
        for (int w = 0; w < W; ++w) n.keys[row * W + w] = o.keys[e * W + w];
        n.pay[row] = o.pay[e];
        if (copy_tot) n.tot[row] = o.tot[e];
        n.dist[row] = d;
        phi[row] = v;
      } else if (R > 1) {
        atomicAdd(&bins[pay_real(o.pay[e])], weight(v));
      } else {
        lost += weight(v);
      }
    }
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

// Columns of the old rows that stay: a column into the old set through the
// keep map (-1 if that row was dropped).  A slot without a column (its
// neighbour is outside the old set) is -1 here; if that neighbour is a new
// row, the new row's own lookup of this row sets it (k_warm_cols_new).
template <int D>
__global__ void __launch_bounds__(kBlock)
    k_warm_cols_old(const StepCtl* ctl, const int32_t* __restrict__ col_o,
                    int32_t* __restrict__ col_n, KeepMap km, const int* err) {
  if (*err) return;
  km.base = ctl->n_staged;
  const int64_t nold = ctl->n_old;
  for (int64_t e = gtid(); e < nold; e += gstride()) {
    const uint32_t row = km.row_of(e);
    if (row == kNone) continue;
    int32_t c[D];
    load_cols<D>(col_o + e * D, c);
#pragma unroll
    for (int s = 0; s < D; ++s) {
      int32_t out = -1;
      if (c[s] >= 0) {
        const uint32_t v = km.row_of(c[s]);
        out = v == kNone ? -1 : int32_t(v);
      }
      col_n[int64_t(row) * D + s] = out;
    }
  }
}

// Columns of the staged rows by lookup: an old row through the keep map, a
// staged row as it is.  An edge is found from both ends with slots s and s
// ^ 1 (a hop and the opposite hop, a lowering and the raising at the same
// site), so a staged row also sets the column of an old row that stays
// toward it, which k_warm_cols_old left at -1 (it runs first).
template <int W>
__global__ void __launch_bounds__(kBlock)
    k_warm_cols_new(DevModel m, const StepCtl* ctl, Side o, Side n,
                    const uint64_t* table, uint64_t mask, KeepMap km,
                    const int* err) {
  if (*err) return;
  km.base = ctl->n_staged;
  const int D = m.D;
  const int64_t ns = ctl->n_staged;
  for (int64_t c = gtid(); c < ns * D; c += gstride()) {
    const int64_t q = c / D;
    const int s = int(c % D);
    uint64_t par[W], k[W];
    load_key<W>(n.keys, q, par);
    int32_t out = -1;
    if (slot_target<W>(m, par, n.pay[q], s, k)) {
      const Found f =
          warm_find<W>(table, mask, o.keys, n.keys, k, key_hash<W>(m, k));
      if (f.row >= 0) {
        if (f.staged) {
          out = int32_t(f.row);
        } else {
          const uint32_t v = km.row_of(f.row);
          if (v != kNone) {
            out = int32_t(v);
            n.col[int64_t(v) * D + (s ^ 1)] = int32_t(q);
          }
        }
      }
    }
    n.col[c] = out;
  }
}

// The table in place: old rows to their new rows (tombstones for dropped
// ones), staged rows to plain rows.  Two entries per lane (16-byte loads
// and stores; the table has a power-of-two size of at least 1024).
__device__ __forceinline__ uint64_t retable_entry(uint64_t e, const KeepMap& km,
                                                  uint32_t& tombs) {
  if (e == kEmpty || uint32_t(e >> 32) == 0xFFFFFFFFu) return e;
  const uint32_t v = uint32_t(e);
  const uint64_t hi = e & 0xFFFFFFFF00000000ull;
  if (v & kCand) return e;  // none are left once every round committed
  if (v & kStaged) return hi | uint64_t(v & ~kStaged);
  const uint32_t nv = km.row_of(v);
  if (nv == kNone) {
    ++tombs;
    return kTomb;
  }
  return hi | uint64_t(nv);
}

typedef uint64_t v2u64 __attribute__((ext_vector_type(2)));

__global__ void __launch_bounds__(kBlock)
    k_warm_retable(StepCtl* ctl, uint64_t* table, uint64_t mask, KeepMap km,
                   const int* err) {
  if (*err) return;
  km.base = ctl->n_staged;
  const int64_t P2 = (int64_t(mask) + 1) / 2;
  v2u64* t2 = reinterpret_cast<v2u64*>(table);
  uint32_t tombs = 0;
  for (int64_t i = gtid(); i < P2; i += gstride()) {
    const v2u64 e = __builtin_nontemporal_load(t2 + i);
    v2u64 o;
    o.x = retable_entry(e.x, km, tombs);
    o.y = retable_entry(e.y, km, tombs);
    if (o.x != e.x || o.y != e.y) __builtin_nontemporal_store(o, t2 + i);
  }
  uint32_t tot;
  block_excl_scan(tombs, &tot);
  if (threadIdx.x == 0 && tot) atomicAdd(&ctl->w_tomb, tot);
  if (gtid() == 0) ctl->w_moved = 1;
}

__global__ void __launch_bounds__(kBlock)
    k_warm_unstage(uint64_t* table, uint64_t mask) {
  const int64_t P = int64_t(mask) + 1;
  for (int64_t i = gtid(); i < P; i += gstride()) {
    const uint64_t e = table[i];
    if (e == kEmpty || uint32_t(e >> 32) == 0xFFFFFFFFu) continue;
    if (uint32_t(e) & (kCand | kStaged)) table[i] = kEmpty;
  }
}

// ---- rows at a given distance (sets of the last step) -----------------------
__global__ void __launch_bounds__(kBlock)
    k_dist_count(const uint8_t* dist, int64_t n, int d, uint32_t* bsum) {
  const int64_t ntiles = cdiv(n, kTile);
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    uint32_t v = 0;
#pragma unroll
    for (int q = 0; q < kItems; ++q) {
      const int64_t e = t * kTile + q * kBlock + threadIdx.x;
      if (e < n && dist[e] == d) ++v;
    }
    uint32_t tot;
    block_excl_scan(v, &tot);
    if (threadIdx.x == 0) bsum[t] = tot;
  }
}

__global__ void __launch_bounds__(kBlock)
    k_dist_write(int Wi, const uint64_t* keys, const uint8_t* dist, int64_t n,
                 int d, const uint32_t* bsum, uint64_t* out) {
  const int64_t ntiles = cdiv(n, kTile);
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    uint32_t run = bsum[t];
#pragma unroll 1
    for (int q = 0; q < kItems; ++q) {
      const int64_t e = t * kTile + q * kBlock + threadIdx.x;
      const bool hit = e < n && dist[e] == d;
      uint32_t tot;
      const uint32_t off = block_excl_scan(hit ? 1u : 0u, &tot) + run;
      run += tot;
      if (hit)
        for (int w = 0; w < Wi; ++w) out[int64_t(off) * Wi + w] = keys[e * Wi + w];
    }
  }
}

__global__ void k_u32_from_i64(uint32_t* out, int64_t v) { *out = uint32_t(v); }

}  // namespace

// ---- host wrappers ----------------------------------------------------------

void warm_begin(const DevModel& m, StepCtl* ctl, const uint32_t* midx,
                const Side& o, uint32_t* cnt_m, int64_t n_old, int* err,
                hipStream_t s) {
  k_warm_fill<<<grid_for(cdiv(n_old, 4)), kBlock, 0, s>>>(o.dist, ctl, err);
  k_warm_mark<<<grid_for(n_old), kBlock, 0, s>>>(m, ctl, midx, o.pay, o.dist,
                                                  cnt_m, err);
}

void warm_round(const DevModel& m, int Wi, int prec, const Side& o,
                const Side& n, int r, StepCtl* ctl, int64_t cap,
                int64_t n_old, int64_t est, uint64_t* table, uint64_t mask,
                const RoundBufs& rb, const WarmBufs& wb, uint32_t* scan_tmp,
                void* phi, int* err, hipStream_t s) {
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
  m, r, ctl, o.pay, o.col, o.dist, wb.wmask, scan_tmp, wb.wlist, rb.cand_cap, err
  PACES_WARM_OLD(false)
  tile_sums_scan(scan_tmp, &ctl->n_old, &ctl->w_noc, err, s);
  PACES_WARM_OLD(true)
#undef PACES_WARM_OLD_ARGS
#undef PACES_WARM_OLD
  k_warm_prep<<<1, 1, 0, s>>>(ctl, r, D, rb.cand_cap, err);
  // candidates: at most the old set's slots plus the new set's
  const int64_t nc_bound = std::min<int64_t>(rb.cand_cap, (n_old + est) * D);
  const int g = grid_for(nc_bound);
  PACES_DISPATCH_W(Wi, k_warm_probe<WW><<<g, kBlock, 0, s>>>(
                           m, r, ctl, o, n, wb.wlist, table, mask, rb.c_slot,
                           rb.c_ref, rb.tile_cnt, err));
  tile_scan(rb.tile_cnt, &ctl->r_ntiles, cdiv(nc_bound, kBlock), rb.scan_tmp,
            rb.tile_base, &ctl->r_total, err, s);
  if (prec == 64) {
    PACES_DISPATCH_W(Wi, k_warm_commit<WW, double2><<<g, kBlock, 0, s>>>(
                             m, r, ctl, cap, o, n, wb.wlist, table, mask,
                             rb.c_slot, rb.c_ref, rb.tile_base,
                             (double2*)phi, err));
  } else {
    PACES_DISPATCH_W(Wi, k_warm_commit<WW, float2><<<g, kBlock, 0, s>>>(
                             m, r, ctl, cap, o, n, wb.wlist, table, mask,
                             rb.c_slot, rb.c_ref, rb.tile_base,
                             (float2*)phi, err));
  }
  k_warm_finish<<<1, 1, 0, s>>>(ctl, r, err);
}

void warm_count(const Side& o, int k, StepCtl* ctl, int64_t n_old,
                int64_t cap, uint32_t* scan_tmp, int* err, hipStream_t s) {
  k_warm_keep_count<<<tiles_for(n_old), kBlock, 0, s>>>(o.dist, k, ctl,
                                                        scan_tmp, err);
  tile_sums_scan(scan_tmp, &ctl->n_old, &ctl->w_nkeep, err, s);
  k_warm_sizes<<<1, 1, 0, s>>>(ctl, cap, err);
}

int warm_compact(const DevModel& m, int Wi, int prec, const Side& o,
                 const Side& n, int k, const StepCtl* ctl, int64_t n_old,
                 const void* psi_o, void* phi, const uint32_t* scan_tmp,
                 const WarmBufs& wb, double* mass_part, int* err,
                 hipStream_t s) {
  const int g = tiles_for(n_old);
  const int copy_tot = m.V > 2 ? 1 : 0;
  if (prec == 64) {
    PACES_DISPATCH_W(Wi, k_warm_compact<WW, double2><<<g, kBlock, 0, s>>>(
                             m, k, ctl, o, n, (const double2*)psi_o,
                             (double2*)phi, scan_tmp, wb.kbits, wb.kpre,
                             mass_part, copy_tot, err));
  } else {
    PACES_DISPATCH_W(Wi, k_warm_compact<WW, float2><<<g, kBlock, 0, s>>>(
                             m, k, ctl, o, n, (const float2*)psi_o,
                             (float2*)phi, scan_tmp, wb.kbits, wb.kpre,
                             mass_part, copy_tot, err));
  }
  return g;
}

namespace {
KeepMap keep_map(const WarmBufs& wb) { return KeepMap{wb.kbits, wb.kpre, 0u}; }
}  // namespace

void warm_columns(const DevModel& m, int Wi, const Side& o, const Side& n,
                  const StepCtl* ctl, int64_t n_old, int64_t est,
                  const uint64_t* table, uint64_t mask, const WarmBufs& wb,
                  int* err, hipStream_t s) {
  const int g = grid_for(n_old);
  switch (m.D) {
    case 2: k_warm_cols_old<2><<<g, kBlock, 0, s>>>(ctl, o.col, n.col, keep_map(wb), err); break;
    case 4: k_warm_cols_old<4><<<g, kBlock, 0, s>>>(ctl, o.col, n.col, keep_map(wb), err); break;
    case 6: k_warm_cols_old<6><<<g, kBlock, 0, s>>>(ctl, o.col, n.col, keep_map(wb), err); break;
    case 8: k_warm_cols_old<8><<<g, kBlock, 0, s>>>(ctl, o.col, n.col, keep_map(wb), err); break;
    case 10: k_warm_cols_old<10><<<g, kBlock, 0, s>>>(ctl, o.col, n.col, keep_map(wb), err); break;
    case 12: k_warm_cols_old<12><<<g, kBlock, 0, s>>>(ctl, o.col, n.col, keep_map(wb), err); break;
    case 14: k_warm_cols_old<14><<<g, kBlock, 0, s>>>(ctl, o.col, n.col, keep_map(wb), err); break;
    default: break;
  }
  PACES_DISPATCH_W(Wi, k_warm_cols_new<WW><<<grid_for(est * m.D), kBlock, 0, s>>>(
                           m, ctl, o, n, table, mask, keep_map(wb), err));
}

void warm_retable(StepCtl* ctl, uint64_t* table, uint64_t mask,
                  const WarmBufs& wb, int* err, hipStream_t s) {
  k_warm_retable<<<grid_for((int64_t(mask) + 1) / 2), kBlock, 0, s>>>(
      ctl, table, mask, keep_map(wb), err);
}

void warm_unstage(uint64_t* table, uint64_t mask, hipStream_t s) {
  k_warm_unstage<<<grid_for(int64_t(mask) + 1), kBlock, 0, s>>>(table, mask);
}

void rows_at_distance(int Wi, const uint64_t* keys, const uint8_t* dist,
                      int64_t n, int d, uint64_t* out, uint32_t* count,
                      uint32_t* tmp, int* err, hipStream_t s) {
  if (n <= 0) {
    k_u32_from_i64<<<1, 1, 0, s>>>(count, 0);
    return;
  }
  const int g = tiles_for(n);
  k_dist_count<<<g, kBlock, 0, s>>>(dist, n, d, tmp);
  // the scan reads the row count from device memory: the last word of tmp,
  // past the tile sums
  uint32_t* nrows = tmp + scan_tmp_words(n) - 1;
  k_u32_from_i64<<<1, 1, 0, s>>>(nrows, n);
  tile_sums_scan(tmp, nrows, count, err, s);
  k_dist_write<<<g, kBlock, 0, s>>>(Wi, keys, dist, n, d, tmp, out);
}

}  // namespace paces
