// runtime.cpp -- host runtime behind the C ABI of include/paces.h: model
// tables, the sim's device buffers and capacity growth, and the sequence of
// kernel launches that makes one time step.
//
// Step (paper: Sec. "Formal operator representation and notes on
// parallelization", with truncation before re-growth as in Sec.
// "Truncation & post-adaptation detruncation"):
//   select -> insert M -> k expansion rounds (+ lookup pass of the last
//   frontier) -> transfer -> bounds and coefficients -> Clenshaw terms ->
//   observables.
// The host reads back the few counts it needs to size the next launch (nM,
// new rows per chunk, the number of series terms); everything else stays on
// the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/paces.h"
#include "kernels.hpp"

using namespace paces;

namespace {

thread_local std::string g_err;

paces_status fail(paces_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIP_TRY(expr)                                                     \
  do {                                                                    \
    hipError_t e_ = (expr);                                               \
    if (e_ != hipSuccess)                                                 \
      return fail(e_ == hipErrorOutOfMemory ? PACES_E_OOM : PACES_E_HIP,  \
                  std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

#define ST_TRY(expr)                   \
  do {                                 \
    paces_status s_ = (expr);          \
    if (s_ != PACES_OK) return s_;     \
  } while (0)

int bits_for(int count) {
  int b = 0;
  while ((int64_t(1) << b) < count) ++b;
  return b;
}

template <typename T>
paces_status dalloc(T** p, int64_t count) {
  *p = nullptr;
  if (count <= 0) count = 1;
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, size_t(count) * sizeof(T));
  if (e != hipSuccess)
    return fail(PACES_E_OOM, std::string("hipMalloc failed: ") +
                                 hipGetErrorString(e));
  *p = static_cast<T*>(q);
  return PACES_OK;
}
template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

uint64_t splitmix_next(uint64_t& s) {
  s += 0x9E3779B97F4A7C15ull;
  uint64_t z = s;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

struct paces_model {
  int ndim = 1, ext[3] = {1, 1, 1}, per[3] = {0, 0, 0};
  int N = 1, V = 1, cut[4] = {0, 0, 0, 0};
  double omega[4] = {0, 0, 0, 0}, g[4] = {0, 0, 0, 0}, J[3] = {0, 0, 0};
  std::vector<double> eps;
  int bj = 1, bnu[4] = {0, 0, 0, 0}, P = 0, B = 0, W = 1, D = 0, Wi = 1;
  std::vector<int32_t> nbr;
  std::vector<double> gsq;
  int32_t* d_nbr = nullptr;
  double* d_gsq = nullptr;
  double* d_eps = nullptr;
  DevModel dm{};
};

namespace {

// Canonical <-> internal keys: internal rows carry Wi >= W words, the extra
// leading words are zero.
void to_internal(const paces_model* m, int64_t n, const uint64_t* in,
                 std::vector<uint64_t>& out) {
  out.assign(size_t(n) * m->Wi, 0);
  for (int64_t i = 0; i < n; ++i)
    for (int w = 0; w < m->W; ++w)
      out[size_t(i) * m->Wi + (m->Wi - m->W) + w] = in[size_t(i) * m->W + w];
}
void to_canonical(const paces_model* m, int64_t n, const uint64_t* in,
                  uint64_t* out) {
  for (int64_t i = 0; i < n; ++i)
    for (int w = 0; w < m->W; ++w)
      out[size_t(i) * m->W + w] = in[size_t(i) * m->Wi + (m->Wi - m->W) + w];
}

uint64_t field_get(const paces_model* m, const uint64_t* key, int off,
                   int width) {
  uint64_t v = 0;
  for (int b = 0; b < width; ++b) {
    const int pos = off + b;
    v |= ((key[m->W - 1 - pos / 64] >> (pos % 64)) & 1u) << b;
  }
  return v;
}
int field_offset(const paces_model* m, int i, int nu) {
  int sub = 0;
  for (int q = nu + 1; q < m->V; ++q) sub += m->bnu[q];
  return m->bj + (m->N - 1 - i) * m->P + sub;
}

// Host validation of canonical keys: all fields in range, no stray bits.
paces_status check_keys(const paces_model* m, int64_t n, const uint64_t* keys) {
  for (int64_t i = 0; i < n; ++i) {
    const uint64_t* k = keys + size_t(i) * m->W;
    for (int pos = m->B; pos < 64 * m->W; ++pos)
      if ((k[m->W - 1 - pos / 64] >> (pos % 64)) & 1u)
        return fail(PACES_E_ARG, "key has bits above B set");
    const uint64_t j = field_get(m, k, 0, m->bj);
    if (j >= uint64_t(m->N)) return fail(PACES_E_ARG, "exciton site out of range");
    for (int s = 0; s < m->N; ++s)
      for (int nu = 0; nu < m->V; ++nu)
        if (field_get(m, k, field_offset(m, s, nu), m->bnu[nu]) >
            uint64_t(m->cut[nu]))
          return fail(PACES_E_ARG, "occupation above cutoff");
  }
  return PACES_OK;
}

paces_status check_unique(const paces_model* m, int64_t n,
                          const uint64_t* keys) {
  std::vector<int64_t> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  const int W = m->W;
  auto less = [&](int64_t a, int64_t b) {
    return std::lexicographical_compare(keys + a * W, keys + a * W + W,
                                        keys + b * W, keys + b * W + W);
  };
  std::sort(idx.begin(), idx.end(), less);
  for (int64_t i = 1; i < n; ++i)
    if (std::equal(keys + idx[i] * W, keys + idx[i] * W + W,
                   keys + idx[i - 1] * W))
      return fail(PACES_E_ARG, "duplicate basis state in the input");
  return PACES_OK;
}

struct Side {
  uint64_t* keys = nullptr;
  uint64_t* pay = nullptr;
  uint64_t* tot = nullptr;
  double* diag = nullptr;
};

struct EventPair {
  int stage;
  hipEvent_t a, b;
  double bytes;
};

}  // namespace

struct paces_sim {
  const paces_model* m = nullptr;
  paces_run_params p{};
  int prec = 64;
  size_t A = 16;  // bytes per amplitude
  double th2 = 0;

  int64_t cap = 0;  // row capacity of every row array
  Side side[2];
  int cur = 0;      // side holding the current set S
  void* vec[4] = {nullptr, nullptr, nullptr, nullptr};
  int ipsi = 0, iphi = 1, ibA = 2, ibB = 3;
  int32_t* col = nullptr;
  uint64_t* table = nullptr;
  uint64_t tmask = 0;
  uint32_t* midx = nullptr;

  int64_t cand_rows = 0;
  RoundBufs rb{};
  uint32_t* scan_tmp = nullptr;  // for select
  uint32_t* d_u32 = nullptr;     // [4] small device counters
  double* parts = nullptr;       // partial sums
  double *mass_part = nullptr, *n2_part = nullptr, *e_part = nullptr,
         *pop_part = nullptr, *bnd_part = nullptr;
  ChebCoef* cc = nullptr;
  double* a2 = nullptr;
  double* mass_total = nullptr;
  int* err = nullptr;

  uint64_t* keys0 = nullptr;
  double* amps0 = nullptr;
  int64_t n0 = 0;

  double* ring = nullptr;
  int64_t ring_cap = 0, nrec = 0;
  int rec_doubles = 0;

  // host-side state
  int64_t nS = 0, nM = 0;
  std::vector<int64_t> fstart;  // frontier r = rows [fstart[r], fstart[r+1])
  double t = 0;
  bool fresh = true;
  int latched = 0;
  uint32_t* h_u32 = nullptr;  // pinned
  int32_t* h_i32 = nullptr;   // pinned
  std::vector<double> pop_host;

  bool prof = false;
  std::vector<EventPair> events;
  paces_profile acc{};
};

namespace {

paces_status sync_read_u32(paces_sim* s, const uint32_t* d, uint32_t* out,
                           hipStream_t st) {
  HIP_TRY(hipMemcpyAsync(s->h_u32, d, 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  *out = *s->h_u32;
  return PACES_OK;
}

paces_status check_latch(paces_sim* s, hipStream_t st) {
  HIP_TRY(hipMemcpyAsync(s->h_i32, s->err, 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const int e = *s->h_i32;
  if (!e) return PACES_OK;
  s->latched = e;
  if (e & kErrTableFull)
    return fail(PACES_E_CAPACITY, "hash table overflow");
  if (e & kErrCapacity) return fail(PACES_E_CAPACITY, "row capacity exceeded");
  if (e & kErrTerms)
    return fail(PACES_E_PROPAGATOR, "series needs more than k_max_terms terms");
  return fail(PACES_E_NONFINITE, "non-finite norm after propagation");
}

struct Stage {
  paces_sim* s;
  int stage;
  hipStream_t st;
  hipEvent_t a{}, b{};
  double bytes;
  Stage(paces_sim* s_, int stage_, hipStream_t st_, double bytes_ = 0)
      : s(s_), stage(stage_), st(st_), bytes(bytes_) {
    if (s->prof) {
      (void)hipEventCreate(&a);
      (void)hipEventCreate(&b);
      (void)hipEventRecord(a, st);
    }
  }
  ~Stage() {
    if (s->prof) {
      (void)hipEventRecord(b, st);
      s->events.push_back({stage, a, b, bytes});
    }
  }
};

void free_rows(paces_sim* s) {
  for (int q = 0; q < 2; ++q) {
    dfree(s->side[q].keys);
    dfree(s->side[q].pay);
    dfree(s->side[q].tot);
    dfree(s->side[q].diag);
  }
  for (auto& v : s->vec) {
    if (v) (void)hipFree(v);
    v = nullptr;
  }
  dfree(s->col);
  dfree(s->table);
  dfree(s->midx);
  dfree(s->scan_tmp);
}

uint64_t table_size_for(int64_t cap) {
  uint64_t P = 1024;
  while (P < uint64_t(2 * cap)) P <<= 1;
  return P;
}

// Grow every row array to new_cap, keeping rows [0, n_cur_side) of side cur
// (old set + psi) and [0, n_new) of the other side (phi, columns of parents
// before col_rows), then rebuild the table from the new side's rows.
paces_status grow(paces_sim* s, int64_t new_cap, int64_t n_new,
                  int64_t col_rows, bool table_from_new, hipStream_t st) {
  const paces_model* m = s->m;
  new_cap = (new_cap + 255) / 256 * 256;
  paces_sim old;  // holds the old pointers only
  for (int q = 0; q < 2; ++q) old.side[q] = s->side[q];
  for (int v = 0; v < 4; ++v) old.vec[v] = s->vec[v];
  old.col = s->col;
  old.table = s->table;
  old.midx = s->midx;
  old.scan_tmp = s->scan_tmp;
  const int64_t old_cap = s->cap;
  const int64_t nvalid[2] = {s->cur == 0 ? s->nS : n_new,
                             s->cur == 1 ? s->nS : n_new};

  for (int q = 0; q < 2; ++q) {
    ST_TRY(dalloc(&s->side[q].keys, new_cap * m->Wi));
    ST_TRY(dalloc(&s->side[q].pay, new_cap));
    ST_TRY(dalloc(&s->side[q].tot, new_cap));
    ST_TRY(dalloc(&s->side[q].diag, new_cap));
    const int64_t nv = old_cap ? nvalid[q] : 0;
    if (nv > 0) {
      HIP_TRY(hipMemcpyAsync(s->side[q].keys, old.side[q].keys,
                             size_t(nv) * m->Wi * 8, hipMemcpyDeviceToDevice, st));
      HIP_TRY(hipMemcpyAsync(s->side[q].pay, old.side[q].pay, size_t(nv) * 8,
                             hipMemcpyDeviceToDevice, st));
      HIP_TRY(hipMemcpyAsync(s->side[q].tot, old.side[q].tot, size_t(nv) * 8,
                             hipMemcpyDeviceToDevice, st));
      HIP_TRY(hipMemcpyAsync(s->side[q].diag, old.side[q].diag, size_t(nv) * 8,
                             hipMemcpyDeviceToDevice, st));
    }
  }
  for (int v = 0; v < 4; ++v) {
    HIP_TRY(hipMalloc(&s->vec[v], size_t(new_cap) * s->A));
    int64_t nv = 0;
    if (old_cap) {
      if (v == s->ipsi) nv = s->nS;
      if (v == s->iphi) nv = n_new;
    }
    if (nv > 0)
      HIP_TRY(hipMemcpyAsync(s->vec[v], old.vec[v], size_t(nv) * s->A,
                             hipMemcpyDeviceToDevice, st));
  }
  ST_TRY(dalloc(&s->col, new_cap * m->D));
  if (old_cap && col_rows > 0)
    HIP_TRY(hipMemcpy2DAsync(s->col, size_t(new_cap) * 4, old.col,
                             size_t(old_cap) * 4, size_t(col_rows) * 4, m->D,
                             hipMemcpyDeviceToDevice, st));
  const uint64_t P = table_size_for(new_cap);
  ST_TRY(dalloc(&s->table, int64_t(P)));
  s->tmask = P - 1;
  fill_u64(s->table, int64_t(P), kEmpty, st);
  ST_TRY(dalloc(&s->midx, new_cap));
  ST_TRY(dalloc(&s->scan_tmp, scan_tmp_words(new_cap)));
  s->cap = new_cap;
  if (table_from_new && n_new > 0) {
    // rebuild the table from the new side's rows (identity selection)
    Side& sn = s->side[1 - s->cur];
    iota_u32(s->midx, n_new, st);
    insert_rows(m->dm, m->Wi, sn.keys, sn.pay, sn.tot, sn.diag, s->midx, n_new,
                sn.keys, sn.pay, sn.tot, sn.diag, s->table, s->tmask, s->err,
                st);
  }
  HIP_TRY(hipStreamSynchronize(st));
  for (int q = 0; q < 2; ++q) {
    dfree(old.side[q].keys);
    dfree(old.side[q].pay);
    dfree(old.side[q].tot);
    dfree(old.side[q].diag);
  }
  for (auto& v : old.vec)
    if (v) (void)hipFree(v);
  dfree(old.col);
  dfree(old.table);
  dfree(old.midx);
  dfree(old.scan_tmp);
  return PACES_OK;
}

paces_status ensure_cand(paces_sim* s, int64_t rows) {
  if (rows <= s->cand_rows) return PACES_OK;
  const int D = s->m->D;
  dfree(s->rb.c_slot);
  dfree(s->rb.c_ref);
  dfree(s->rb.crow);
  dfree(s->rb.rowcnt);
  dfree(s->rb.rowbase);
  dfree(s->rb.scan_tmp);
  ST_TRY(dalloc(&s->rb.c_slot, rows * D));
  ST_TRY(dalloc(&s->rb.c_ref, rows * D));
  ST_TRY(dalloc(&s->rb.crow, rows * D));
  ST_TRY(dalloc(&s->rb.rowcnt, rows));
  ST_TRY(dalloc(&s->rb.rowbase, rows));
  ST_TRY(dalloc(&s->rb.scan_tmp, scan_tmp_words(rows)));
  s->cand_rows = rows;
  return PACES_OK;
}

paces_status ensure_ring(paces_sim* s, hipStream_t st) {
  if (s->nrec < s->ring_cap) return PACES_OK;
  const int64_t nc = std::max<int64_t>(1024, 2 * s->ring_cap);
  double* r = nullptr;
  ST_TRY(dalloc(&r, nc * s->rec_doubles));
  if (s->nrec > 0)
    HIP_TRY(hipMemcpyAsync(r, s->ring, size_t(s->nrec) * s->rec_doubles * 8,
                           hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  dfree(s->ring);
  s->ring = r;
  s->ring_cap = nc;
  return PACES_OK;
}

// Upload a state given as canonical keys + FP64 amplitudes into side cur.
paces_status upload_state(paces_sim* s, int64_t n, const uint64_t* keys,
                          const double* amps, hipStream_t st) {
  const paces_model* m = s->m;
  if (n > s->cap) {
    s->nS = 0;
    ST_TRY(grow(s, std::max<int64_t>(n, 2 * s->cap), 0, 0, false, st));
  }
  std::vector<uint64_t> ik;
  to_internal(m, n, keys, ik);
  Side& sc = s->side[s->cur];
  HIP_TRY(hipMemcpyAsync(sc.keys, ik.data(), ik.size() * 8,
                         hipMemcpyHostToDevice, st));
  double* tmp = nullptr;
  ST_TRY(dalloc(&tmp, 2 * n));
  HIP_TRY(hipMemcpyAsync(tmp, amps, size_t(n) * 16, hipMemcpyHostToDevice, st));
  amps_from_f64(s->prec, tmp, s->vec[s->ipsi], n, st);
  row_info(m->dm, m->Wi, sc.keys, n, sc.pay, sc.tot, sc.diag, st);
  HIP_TRY(hipStreamSynchronize(st));
  dfree(tmp);
  s->nS = n;
  return PACES_OK;
}

paces_status do_step(paces_sim* s, hipStream_t st) {
  const paces_model* m = s->m;
  const DevModel& dm = m->dm;
  const int D = m->D, Wi = m->Wi;
  const int64_t n_old = s->nS;
  const int old = s->cur, nw = 1 - s->cur;

  // ---- select
  int k = s->p.k;
  {
    Stage sg(s, PACES_STAGE_SELECT, st);
    if (s->fresh) {
      k = s->p.k_init;
      s->nM = n_old;
      iota_u32(s->midx, n_old, st);
    } else {
      select_rows(s->prec, s->vec[s->ipsi], n_old, s->th2, s->midx,
                  s->scan_tmp, s->d_u32, st);
    }
  }
  if (!s->fresh) {
    uint32_t nm;
    ST_TRY(sync_read_u32(s, s->d_u32, &nm, st));
    s->nM = nm;
  }

  // ---- expand: rows 0..nM-1 of the new set are M in selection order
  {
    Stage sg(s, PACES_STAGE_EXPAND, st);
    fill_u64(s->table, int64_t(s->tmask + 1), kEmpty, st);
    insert_rows(dm, Wi, s->side[old].keys, s->side[old].pay, s->side[old].tot,
                s->side[old].diag, s->midx, s->nM, s->side[nw].keys,
                s->side[nw].pay, s->side[nw].tot, s->side[nw].diag, s->table,
                s->tmask, s->err, st);
  }
  int64_t n_cur = s->nM;
  s->fstart.assign(1, 0);
  s->fstart.push_back(n_cur);
  for (int r = 1; r <= k; ++r) {
    const int64_t f0 = s->fstart[r - 1], f1 = s->fstart[r];
    int64_t p0 = f0;
    while (p0 < f1) {
      int64_t rows = std::min<int64_t>(f1 - p0, int64_t(1) << 24);
      // rows * D new states at most; shrink the chunk before growing
      int64_t room = (s->cap - n_cur) / D;
      if (room < rows && room < std::max<int64_t>(rows / 4, 65536)) {
        ST_TRY(grow(s, std::max(2 * s->cap, n_cur + rows * D), n_cur, p0,
                    true, st));
        room = (s->cap - n_cur) / D;
      }
      rows = std::min(rows, room);
      ST_TRY(ensure_cand(s, rows));
      Side& sn = s->side[nw];
      {
        Stage sg(s, PACES_STAGE_EXPAND, st);
        expand_chunk(dm, Wi, s->prec, sn.keys, sn.pay, sn.tot, sn.diag, p0,
                     rows, n_cur, s->table, s->tmask, s->rb, s->col, s->cap,
                     s->vec[s->iphi], s->err, st);
      }
      uint32_t added;
      ST_TRY(sync_read_u32(s, s->rb.total, &added, st));
      n_cur += added;
      p0 += rows;
    }
    s->fstart.push_back(n_cur);
  }
  {
    Stage sg(s, PACES_STAGE_EXPAND, st);
    const int64_t f0 = s->fstart[k], f1 = s->fstart[k + 1];
    lookup_cols(dm, Wi, s->side[nw].keys, s->side[nw].pay, f0, f1 - f0,
                s->table, s->tmask, s->col, s->cap, st);
  }
  const int64_t nS = n_cur;

  // ---- transfer
  {
    Stage sg(s, PACES_STAGE_TRANSFER, st);
    transfer(dm, Wi, s->prec, s->side[old].keys, s->vec[s->ipsi], n_old,
             s->table, s->tmask, s->side[nw].keys, s->vec[s->iphi],
             s->mass_part, st);
  }
  // ---- build: bounds and coefficients
  {
    Stage sg(s, PACES_STAGE_BUILD, st);
    bounds_and_coef(dm, s->side[nw].pay, s->side[nw].diag, s->col, s->cap, nS,
                    s->p.dt, s->p.tol, s->p.k_max_terms, s->bnd_part, s->cc,
                    s->err, st);
  }
  HIP_TRY(hipMemcpyAsync(s->h_i32, &s->cc->K, 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const int K = *s->h_i32;
  if (K < 1 || K > kMaxTerms)
    return fail(PACES_E_PROPAGATOR, "invalid number of series terms");

  // ---- propagate
  const bool want_e = (s->p.obs_mask & PACES_OBS_ENERGY) != 0;
  const Side& sn = s->side[nw];
  int result = -1;
  {
    Stage sg(s, PACES_STAGE_PROPAGATE, st);
    void* phi = s->vec[s->iphi];
    if (K == 1) {
      cheb_scale(s->prec, nS, s->cc, phi, s->vec[s->ibA], s->n2_part,
                 s->pop_part, sn.pay, m->N, st);
      if (want_e)
        energy_only(dm, s->prec, nS, s->col, s->cap, sn.pay, sn.diag, phi,
                    s->e_part, st);
      result = s->ibA;
    } else {
      int cur = -1, prv = -1;
      for (int kk = K - 2; kk >= 0; --kk) {
        TermArgs ta{};
        ta.ck = kk;
        ta.fac = kk == 0 ? 1 : 2;
        ta.final_ = kk == 0;
        ta.energy = (kk == K - 2) && want_e;
        ta.in_coef = -1;
        ta.prev_coef = -1;
        const void* in;
        const void* prev;
        int out;
        if (kk == K - 2) {
          in = phi;
          ta.in_coef = K - 1;
          prev = nullptr;
          out = s->ibA;
        } else if (kk == K - 3) {
          in = s->vec[cur];
          prev = phi;
          ta.prev_coef = K - 1;
          out = (cur == s->ibA) ? s->ibB : s->ibA;
        } else {
          in = s->vec[cur];
          prev = s->vec[prv];
          out = prv;
        }
        const bool middle = !ta.final_ && !ta.energy;
        const double A = double(s->A);
        const double bytes =
            double(nS) * ((prev ? 4.0 : 3.0) * A + 4.0 * D + 16.0);
        if (middle && s->prof) {
          Stage tsg(s, PACES_STAGE_TERM, st, bytes);
          cheb_term(dm, s->prec, nS, s->col, s->cap, sn.pay, sn.diag, s->cc,
                    ta, phi, in, prev, s->vec[out], s->e_part, s->n2_part,
                    s->pop_part, st);
        } else {
          cheb_term(dm, s->prec, nS, s->col, s->cap, sn.pay, sn.diag, s->cc,
                    ta, phi, in, prev, s->vec[out], s->e_part, s->n2_part,
                    s->pop_part, st);
        }
        prv = cur;
        cur = out;
      }
      result = cur;
    }
  }
  // result buffer becomes psi
  std::swap(s->ipsi, result == s->ibA ? s->ibA : s->ibB);
  s->cur = nw;
  s->nS = nS;
  s->t = s->t + s->p.dt;
  s->fresh = false;

  // ---- observe
  {
    Stage sg(s, PACES_STAGE_OBSERVE, st);
    ST_TRY(ensure_ring(s, st));
    autocorr(dm, Wi, s->prec, s->keys0, s->amps0, s->n0, s->table, s->tmask,
             s->side[s->cur].keys, s->vec[s->ipsi], s->a2, st);
    ObsArgs oa{};
    oa.t = s->t;
    oa.nS = double(nS);
    oa.nM = double(s->nM);
    oa.dt = s->p.dt;
    oa.N = m->N;
    oa.want_energy = want_e ? 1 : 0;
    obs_final(oa, s->mass_part, s->n2_part, s->e_part, s->pop_part, s->a2,
              s->cc, s->mass_total, s->ring + s->nrec * s->rec_doubles,
              s->err, st);
    s->nrec += 1;
  }
  s->acc.rows_steps += double(nS);
  return PACES_OK;
}

// Device copies of the model tables, made on first use so that loading a
// model and the host codec need no GPU.
paces_status ensure_device_tables(paces_model* m) {
  if (m->d_nbr) return PACES_OK;
  ST_TRY(dalloc(&m->d_nbr, int64_t(m->nbr.size())));
  ST_TRY(dalloc(&m->d_gsq, int64_t(m->gsq.size())));
  ST_TRY(dalloc(&m->d_eps, int64_t(m->N)));
  HIP_TRY(hipMemcpy(m->d_nbr, m->nbr.data(), m->nbr.size() * 4,
                    hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(m->d_gsq, m->gsq.data(), m->gsq.size() * 8,
                    hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(m->d_eps, m->eps.data(), m->eps.size() * 8,
                    hipMemcpyHostToDevice));
  m->dm.nbr = m->d_nbr;
  m->dm.gsq = m->d_gsq;
  m->dm.eps = m->d_eps;
  return PACES_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* paces_last_error(void) { return g_err.c_str(); }
int32_t paces_abi_version(void) { return PACES_ABI_VERSION; }

int32_t paces_record_doubles(const paces_model* m) {
  return m ? kObsFields + m->N : 0;
}

paces_status paces_load_model(const paces_model_desc* d, paces_model** out) {
  if (!d || !out) return fail(PACES_E_ARG, "null argument");
  *out = nullptr;
  paces_model* m = new paces_model();
  auto bad = [&](const char* msg) {
    delete m;
    return fail(PACES_E_ARG, msg);
  };
  m->ndim = d->ndim;
  if (m->ndim < 1 || m->ndim > 3) return bad("ndim must be 1..3");
  m->N = 1;
  for (int a = 0; a < 3; ++a) {
    m->ext[a] = a < m->ndim ? d->extent[a] : 1;
    m->per[a] = a < m->ndim ? (d->periodic[a] != 0) : 0;
    m->J[a] = a < m->ndim ? d->J[a] : 0.0;
    if (m->ext[a] < 1 || (m->per[a] && m->ext[a] < 3))
      return bad("extent must be >= 1, and >= 3 when periodic");
    m->N *= m->ext[a];
  }
  if (m->N > 4096) return bad("at most 4096 sites");
  m->V = d->n_modes;
  if (m->V < 1 || m->V > 4) return bad("n_modes must be 1..4");
  m->P = 0;
  for (int nu = 0; nu < m->V; ++nu) {
    m->cut[nu] = d->cutoff[nu];
    m->omega[nu] = d->omega[nu];
    m->g[nu] = d->g[nu];
    if (m->cut[nu] < 1 || m->cut[nu] > 254) return bad("cutoff must be 1..254");
    m->bnu[nu] = bits_for(m->cut[nu] + 1);
    m->P += m->bnu[nu];
  }
  if (int64_t(m->N) * m->cut[0] > 65535 ||
      (m->V > 1 && int64_t(m->N) * std::max({m->cut[1], m->cut[2], m->cut[3]}) >
                       65535))
    return bad("N * cutoff must stay below 65536");
  m->eps.assign(m->N, 0.0);
  if (d->eps)
    for (int i = 0; i < m->N; ++i) m->eps[i] = d->eps[i];
  m->bj = std::max(1, bits_for(m->N));
  m->B = m->N * m->P + m->bj;
  m->W = (m->B + 63) / 64;
  m->Wi = supported_words(m->W);
  if (!m->Wi) return bad("key wider than 1024 bits");
  m->D = 2 * m->ndim + 2 * m->V;
  m->nbr.assign(size_t(m->N) * 2 * m->ndim, -1);
  for (int i = 0; i < m->N; ++i) {
    int c[3] = {i % m->ext[0], (i / m->ext[0]) % m->ext[1],
                i / (m->ext[0] * m->ext[1])};
    for (int a = 0; a < m->ndim; ++a)
      for (int dir = 0; dir < 2; ++dir) {
        int cc[3] = {c[0], c[1], c[2]};
        cc[a] += dir == 0 ? 1 : -1;
        if (cc[a] < 0 || cc[a] >= m->ext[a]) {
          if (!m->per[a]) continue;
          cc[a] = (cc[a] + m->ext[a]) % m->ext[a];
        }
        m->nbr[size_t(i) * 2 * m->ndim + 2 * a + dir] =
            cc[0] + m->ext[0] * (cc[1] + m->ext[1] * cc[2]);
      }
  }
  // g_nu * sqrt(n): the matrix element of (a + a^dag) between n-1 and n
  m->gsq.assign(size_t(m->V) * kGsqStride, 0.0);
  for (int nu = 0; nu < m->V; ++nu)
    for (int n = 0; n < kGsqStride; ++n)
      m->gsq[size_t(nu) * kGsqStride + n] = m->g[nu] * std::sqrt(double(n));

  DevModel& dm = m->dm;
  std::memset(&dm, 0, sizeof(dm));
  dm.N = m->N;
  dm.V = m->V;
  dm.ndim = m->ndim;
  dm.D = m->D;
  dm.W = m->Wi;
  dm.B = m->B;
  dm.bj = m->bj;
  dm.P = m->P;
  for (int nu = 0; nu < m->V; ++nu) {
    dm.bnu[nu] = m->bnu[nu];
    dm.cut[nu] = m->cut[nu];
    dm.omega[nu] = m->omega[nu];
    int sub = 0;
    for (int q = nu + 1; q < m->V; ++q) sub += m->bnu[q];
    dm.sub[nu] = sub;
    if (m->g[nu] != 0.0) dm.eph_mask |= 1u << nu;
  }
  for (int a = 0; a < 3; ++a) {
    dm.J[a] = m->J[a];
    if (a < m->ndim && m->J[a] != 0.0) dm.hop_mask |= 1u << a;
  }
  uint64_t seed = 0x5eed0f6b17ull;
  for (int w = 0; w < kMaxW; ++w) dm.mul[w] = splitmix_next(seed) | 1ull;

  *out = m;
  return PACES_OK;
}

paces_status paces_free_model(paces_model* m) {
  if (!m) return PACES_OK;
  dfree(m->d_nbr);
  dfree(m->d_gsq);
  dfree(m->d_eps);
  delete m;
  return PACES_OK;
}

paces_status paces_model_info(const paces_model* m, int32_t* N, int32_t* W,
                              int32_t* D, int32_t* B) {
  if (!m) return fail(PACES_E_ARG, "null model");
  if (N) *N = m->N;
  if (W) *W = m->W;
  if (D) *D = m->D;
  if (B) *B = m->B;
  return PACES_OK;
}

paces_status paces_pack_keys(const paces_model* m, int64_t n,
                             const int32_t* exc, const uint16_t* occ,
                             uint64_t* keys) {
  if (!m || n < 0 || (n > 0 && (!exc || !occ || !keys)))
    return fail(PACES_E_ARG, "bad arguments");
  const int NV = m->N * m->V;
  for (int64_t i = 0; i < n; ++i) {
    uint64_t* k = keys + size_t(i) * m->W;
    std::fill(k, k + m->W, 0ull);
    auto put = [&](int off, int width, uint64_t v) {
      for (int b = 0; b < width; ++b)
        if ((v >> b) & 1u) {
          const int pos = off + b;
          k[m->W - 1 - pos / 64] |= uint64_t(1) << (pos % 64);
        }
    };
    if (exc[i] < 0 || exc[i] >= m->N)
      return fail(PACES_E_ARG, "exciton site out of range");
    put(0, m->bj, uint64_t(exc[i]));
    for (int s = 0; s < m->N; ++s)
      for (int nu = 0; nu < m->V; ++nu) {
        const uint16_t v = occ[size_t(i) * NV + s * m->V + nu];
        if (v > m->cut[nu]) return fail(PACES_E_ARG, "occupation above cutoff");
        put(field_offset(m, s, nu), m->bnu[nu], v);
      }
  }
  return PACES_OK;
}

paces_status paces_unpack_keys(const paces_model* m, int64_t n,
                               const uint64_t* keys, int32_t* exc,
                               uint16_t* occ) {
  if (!m || n < 0 || (n > 0 && (!exc || !occ || !keys)))
    return fail(PACES_E_ARG, "bad arguments");
  const int NV = m->N * m->V;
  for (int64_t i = 0; i < n; ++i) {
    const uint64_t* k = keys + size_t(i) * m->W;
    exc[i] = int32_t(field_get(m, k, 0, m->bj));
    for (int s = 0; s < m->N; ++s)
      for (int nu = 0; nu < m->V; ++nu)
        occ[size_t(i) * NV + s * m->V + nu] =
            uint16_t(field_get(m, k, field_offset(m, s, nu), m->bnu[nu]));
  }
  return PACES_OK;
}

paces_status paces_init_state(const paces_model* m, const paces_run_params* p,
                              int64_t n, const int32_t* exc,
                              const uint16_t* occ, const double* coef,
                              void* hip_stream, paces_sim** out) {
  if (!m || !p || !out || n < 1 || !exc || !occ || !coef)
    return fail(PACES_E_ARG, "bad arguments");
  *out = nullptr;
  if (!(p->dt > 0) || p->k < 0 || p->k_init < 0 || !(p->theta >= 0) ||
      (p->precision != 64 && p->precision != 32) || p->k_max_terms < 0 ||
      p->k_max_terms > kMaxTerms || p->tol < 0 || p->cap_states < 0)
    return fail(PACES_E_ARG, "bad run parameters");
  if (n > (int64_t(1) << 31) - 1) return fail(PACES_E_ARG, "too many states");
  ST_TRY(ensure_device_tables(const_cast<paces_model*>(m)));
  std::vector<uint64_t> keys(size_t(n) * m->W);
  ST_TRY(paces_pack_keys(m, n, exc, occ, keys.data()));
  ST_TRY(check_unique(m, n, keys.data()));
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  paces_sim* s = new paces_sim();
  s->m = m;
  s->p = *p;
  if (s->p.tol == 0) s->p.tol = 1e-16;
  if (s->p.k_max_terms == 0) s->p.k_max_terms = kMaxTerms;
  if (s->p.obs_mask == 0) s->p.obs_mask = PACES_OBS_ENERGY;
  s->prec = p->precision;
  s->A = s->prec == 64 ? 16 : 8;
  s->th2 = p->theta * p->theta;
  s->rec_doubles = kObsFields + m->N;
  s->pop_host.assign(m->N, 0.0);
  auto cleanup = [&](paces_status st_) {
    paces_free_sim(s);
    return st_;
  };
  if (hipHostMalloc(reinterpret_cast<void**>(&s->h_u32), 64) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&s->h_i32), 64) != hipSuccess)
    return cleanup(fail(PACES_E_OOM, "pinned host allocation failed"));
  const int64_t nparts = 5 * kPartBlocks + int64_t(kPartBlocks) * m->N;
  if (dalloc(&s->d_u32, 16) || dalloc(&s->parts, nparts) ||
      dalloc(&s->cc, 1) || dalloc(&s->a2, 2) || dalloc(&s->mass_total, 1) ||
      dalloc(&s->err, 1) || dalloc(&s->keys0, n * m->Wi) ||
      dalloc(&s->amps0, 2 * n))
    return cleanup(PACES_E_OOM);
  s->mass_part = s->parts;
  s->n2_part = s->parts + kPartBlocks;
  s->e_part = s->parts + 2 * kPartBlocks;
  s->bnd_part = s->parts + 3 * kPartBlocks;  // (lo, hi) per block
  s->pop_part = s->parts + 5 * kPartBlocks;  // N per block
  if (hipMemsetAsync(s->err, 0, 4, st) != hipSuccess ||
      hipMemsetAsync(s->mass_total, 0, 8, st) != hipSuccess ||
      hipMemsetAsync(s->parts, 0, size_t(nparts) * 8, st) != hipSuccess)
    return cleanup(fail(PACES_E_HIP, "memset failed"));
  const int64_t cap0 = std::max<int64_t>({p->cap_states, 4 * n, 1 << 16});
  paces_status g = grow(s, cap0, 0, 0, false, st);
  if (g) return cleanup(g);
  std::vector<uint64_t> ik;
  to_internal(m, n, keys.data(), ik);
  if (hipMemcpyAsync(s->keys0, ik.data(), ik.size() * 8, hipMemcpyHostToDevice,
                     st) != hipSuccess ||
      hipMemcpyAsync(s->amps0, coef, size_t(n) * 16, hipMemcpyHostToDevice,
                     st) != hipSuccess)
    return cleanup(fail(PACES_E_HIP, "upload failed"));
  s->n0 = n;
  g = upload_state(s, n, keys.data(), coef, st);
  if (g) return cleanup(g);
  s->fresh = true;
  s->t = 0;
  *out = s;
  return PACES_OK;
}

paces_status paces_free_sim(paces_sim* s) {
  if (!s) return PACES_OK;
  (void)hipDeviceSynchronize();
  free_rows(s);
  dfree(s->rb.c_slot);
  dfree(s->rb.c_ref);
  dfree(s->rb.crow);
  dfree(s->rb.rowcnt);
  dfree(s->rb.rowbase);
  dfree(s->rb.scan_tmp);
  dfree(s->d_u32);
  dfree(s->parts);
  dfree(s->cc);
  dfree(s->a2);
  dfree(s->mass_total);
  dfree(s->err);
  dfree(s->keys0);
  dfree(s->amps0);
  dfree(s->ring);
  for (auto& e : s->events) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  if (s->h_u32) (void)hipHostFree(s->h_u32);
  if (s->h_i32) (void)hipHostFree(s->h_i32);
  delete s;
  return PACES_OK;
}

paces_status paces_step(paces_sim* s, int64_t n_steps, void* hip_stream) {
  if (!s || n_steps < 0) return fail(PACES_E_ARG, "bad arguments");
  if (s->latched) return fail(PACES_E_STATE, "sim is in an error state");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  s->rb.total = s->d_u32 + 1;
  for (int64_t i = 0; i < n_steps; ++i) {
    paces_status r = do_step(s, st);
    if (r != PACES_OK) {
      s->latched = s->latched ? s->latched : -1;
      return r;
    }
    // the step read device counts, so the stream is synchronised often;
    // check the latch once per step at no extra cost
    ST_TRY(check_latch(s, st));
  }
  return PACES_OK;
}

paces_status paces_observe(paces_sim* s, paces_obs* out, void* hip_stream) {
  if (!s || !out) return fail(PACES_E_ARG, "bad arguments");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  ST_TRY(check_latch(s, st));
  std::memset(out, 0, sizeof(*out));
  if (s->nrec == 0) {
    out->t = s->t;
    out->n_S = s->nS;
    out->pop = s->pop_host.data();
    return PACES_OK;
  }
  std::vector<double> rec(s->rec_doubles);
  HIP_TRY(hipMemcpyAsync(rec.data(), s->ring + (s->nrec - 1) * s->rec_doubles,
                         rec.size() * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  out->t = rec[0];
  out->norm2 = rec[1];
  out->energy = rec[2];
  out->autocorr_re = rec[3];
  out->autocorr_im = rec[4];
  out->mass_step = rec[5];
  out->mass_total = rec[6];
  out->n_S = int64_t(rec[7]);
  out->n_M = int64_t(rec[8]);
  out->K = int32_t(rec[9]);
  out->E_min = rec[10];
  out->E_max = rec[11];
  for (int j = 0; j < s->m->N; ++j) s->pop_host[j] = rec[kObsFields + j];
  out->pop = s->pop_host.data();
  return PACES_OK;
}

paces_status paces_num_records(paces_sim* s, int64_t* n) {
  if (!s || !n) return fail(PACES_E_ARG, "bad arguments");
  *n = s->nrec;
  return PACES_OK;
}

paces_status paces_series(paces_sim* s, int64_t first, int64_t n, double* out,
                          void* hip_stream) {
  if (!s || first < 0 || n < 0 || first + n > s->nrec || (n && !out))
    return fail(PACES_E_ARG, "bad arguments");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (n == 0) return PACES_OK;
  HIP_TRY(hipMemcpyAsync(out, s->ring + first * s->rec_doubles,
                         size_t(n) * s->rec_doubles * 8, hipMemcpyDeviceToHost,
                         st));
  HIP_TRY(hipStreamSynchronize(st));
  return PACES_OK;
}

paces_status paces_get_state(paces_sim* s, int64_t* n, uint64_t* keys,
                             double* amps, void* hip_stream) {
  if (!s || !n) return fail(PACES_E_ARG, "bad arguments");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  ST_TRY(check_latch(s, st));
  *n = s->nS;
  const paces_model* m = s->m;
  if (keys) {
    std::vector<uint64_t> ik(size_t(s->nS) * m->Wi);
    HIP_TRY(hipMemcpyAsync(ik.data(), s->side[s->cur].keys, ik.size() * 8,
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    to_canonical(m, s->nS, ik.data(), keys);
  }
  if (amps) {
    double* tmp = nullptr;
    ST_TRY(dalloc(&tmp, 2 * s->nS));
    amps_to_f64(s->prec, s->vec[s->ipsi], tmp, s->nS, st);
    HIP_TRY(hipMemcpyAsync(amps, tmp, size_t(s->nS) * 16, hipMemcpyDeviceToHost,
                           st));
    HIP_TRY(hipStreamSynchronize(st));
    dfree(tmp);
  }
  return PACES_OK;
}

paces_status paces_set_state(paces_sim* s, int64_t n, const uint64_t* keys,
                             const double* amps, double t, void* hip_stream) {
  if (!s || n < 0 || (n > 0 && (!keys || !amps)))
    return fail(PACES_E_ARG, "bad arguments");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  ST_TRY(check_keys(s->m, n, keys));
  ST_TRY(check_unique(s->m, n, keys));
  HIP_TRY(hipStreamSynchronize(st));
  HIP_TRY(hipMemsetAsync(s->err, 0, 4, st));
  s->latched = 0;
  ST_TRY(upload_state(s, n, keys, amps, st));
  s->t = t;
  s->fresh = false;
  s->fstart.clear();
  return PACES_OK;
}

paces_status paces_get_set(paces_sim* s, int32_t which, int32_t round,
                           int64_t* n, uint64_t* keys, void* hip_stream) {
  if (!s || !n) return fail(PACES_E_ARG, "bad arguments");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  int64_t a = 0, b = 0;
  if (which == PACES_SET_S) {
    b = s->nS;
  } else if (s->fstart.empty()) {
    return fail(PACES_E_STATE, "no step has run since the state was set");
  } else if (which == PACES_SET_M) {
    b = s->nM;
  } else if (which == PACES_SET_FRONTIER) {
    if (round < 0 || round + 1 >= int(s->fstart.size()))
      return fail(PACES_E_ARG, "no such round");
    a = s->fstart[round];
    b = s->fstart[round + 1];
  } else {
    return fail(PACES_E_ARG, "unknown set");
  }
  *n = b - a;
  if (!keys) return PACES_OK;
  const paces_model* m = s->m;
  std::vector<uint64_t> ik(size_t(b - a) * m->Wi);
  HIP_TRY(hipMemcpyAsync(ik.data(), s->side[s->cur].keys + a * m->Wi,
                         ik.size() * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  to_canonical(m, b - a, ik.data(), keys);
  return PACES_OK;
}

paces_status paces_get_phi(paces_sim* s, double* amps, void* hip_stream) {
  if (!s || !amps) return fail(PACES_E_ARG, "bad arguments");
  if (s->fstart.empty())
    return fail(PACES_E_STATE, "no step has run since the state was set");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  double* tmp = nullptr;
  ST_TRY(dalloc(&tmp, 2 * s->nS));
  amps_to_f64(s->prec, s->vec[s->iphi], tmp, s->nS, st);
  HIP_TRY(hipMemcpyAsync(amps, tmp, size_t(s->nS) * 16, hipMemcpyDeviceToHost,
                         st));
  HIP_TRY(hipStreamSynchronize(st));
  dfree(tmp);
  return PACES_OK;
}

paces_status paces_profile_enable(paces_sim* s, int32_t on) {
  if (!s) return fail(PACES_E_ARG, "bad arguments");
  s->prof = on != 0;
  return PACES_OK;
}

paces_status paces_profile_get(paces_sim* s, paces_profile* out,
                               void* hip_stream) {
  if (!s || !out) return fail(PACES_E_ARG, "bad arguments");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  HIP_TRY(hipStreamSynchronize(st));
  for (auto& e : s->events) {
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, e.a, e.b));
    s->acc.ms[e.stage] += ms;
    s->acc.launches[e.stage] += 1;
    if (e.stage == PACES_STAGE_TERM) s->acc.term_bytes += e.bytes;
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  s->events.clear();
  *out = s->acc;
  return PACES_OK;
}

paces_status paces_profile_reset(paces_sim* s) {
  if (!s) return fail(PACES_E_ARG, "bad arguments");
  paces_profile z{};
  s->acc = z;
  return PACES_OK;
}

}  // extern "C"
