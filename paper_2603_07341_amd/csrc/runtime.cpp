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
// Sizes live on the device; the host enqueues a whole step, reads the
// counts and the error latch once, and repeats the step with more room if
// a capacity was exceeded.  A step's launch sequence can be captured once
// as a HIP graph and replayed (grid sizes are bucketed so consecutive steps
// share a graph).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <memory>
#include <mutex>
#include <unordered_map>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/paces.h"
#include "adjoint.hpp"
#include "cap.hpp"
#include "kernels.hpp"
#include "lanczos.hpp"
#include "taylor.hpp"
#include "warm.hpp"

using namespace paces;

namespace {

thread_local std::string g_err;

paces_status dev_alloc(void** p, size_t bytes);
void dev_free(void* p);

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
  const paces_status e = dev_alloc(&q, size_t(count) * sizeof(T));
  if (e) return e;
  *p = static_cast<T*>(q);
  return PACES_OK;
}
// Aligned sub-arrays of one device block: list the pieces, then carve.
struct Pieces {
  std::vector<std::pair<void**, size_t>> list;
  template <typename T>
  void add(T** p, int64_t count) {
    list.push_back({reinterpret_cast<void**>(p),
                    size_t(std::max<int64_t>(count, 1)) * sizeof(T)});
  }
  void add_bytes(void** p, size_t bytes) {
    list.push_back({p, std::max<size_t>(bytes, 1)});
  }
  static size_t round(size_t b) { return (b + 255) & ~size_t(255); }
  size_t total() const {
    size_t t = 0;
    for (auto& q : list) t += round(q.second);
    return t;
  }
  // One allocation for every piece; pointers are written only on success.
  paces_status carve(void** block) {
    const size_t total = this->total();
    void* b = nullptr;
    const paces_status e = dev_alloc(&b, total);
    if (e) return e;
    char* c = static_cast<char*>(b);
    for (auto& q : list) {
      *q.first = c;
      c += round(q.second);
    }
    *block = b;
    return PACES_OK;
  }
};

template <typename T>
void dfree(T*& p) {
  if (p) dev_free(p);
  p = nullptr;
}

// Device memory: the caller's allocator if one is registered, else
// hipMalloc.  Every allocation of the library goes through here, and each
// block is returned to the allocator that made it, so the allocator may
// change while blocks are alive.
struct DevAllocator {
  void* (*alloc)(size_t, void*, void*) = nullptr;
  void (*release)(void*, void*, void*) = nullptr;
  void* user = nullptr;
};
DevAllocator g_allocator;
std::mutex g_blocks_mu;
std::unordered_map<void*, DevAllocator> g_blocks;  // blocks of an allocator

paces_status dev_alloc(void** p, size_t bytes) {
  *p = nullptr;
  const DevAllocator a = g_allocator;
  if (a.alloc) {
    *p = a.alloc(bytes, nullptr, a.user);
    if (!*p) return fail(PACES_E_OOM, "registered allocator returned NULL");
    std::lock_guard<std::mutex> lk(g_blocks_mu);
    g_blocks[*p] = a;
  } else {
    const hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess)
      return fail(PACES_E_OOM, std::string("hipMalloc failed: ") +
                                   hipGetErrorString(e));
  }
  return PACES_OK;
}
void dev_free(void* p) {
  if (!p) return;
  DevAllocator a;
  {
    std::lock_guard<std::mutex> lk(g_blocks_mu);
    auto it = g_blocks.find(p);
    if (it != g_blocks.end()) {
      a = it->second;
      g_blocks.erase(it);
    }
  }
  if (a.release)
    a.release(p, nullptr, a.user);
  else
    (void)hipFree(p);
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
  int R = 1, br = 0;  // disorder realizations and bits of the id
  std::vector<int32_t> nbr;
  std::vector<double> gsq;
  int32_t* d_nbr = nullptr;
  double* d_gsq = nullptr;
  double* d_eps = nullptr;
  DevModel dm{};
};

namespace {

// Canonical <-> internal keys: internal rows carry Wi >= W words; the
// realization id sits in the br bits above the B bits of the state, the
// remaining leading bits are zero.
void set_ibit(const paces_model* m, uint64_t* key, int pos) {
  key[m->Wi - 1 - pos / 64] |= uint64_t(1) << (pos % 64);
}
int internal_real(const paces_model* m, const uint64_t* key) {
  int r = 0;
  for (int b = 0; b < m->br; ++b) {
    const int pos = m->B + b;
    r |= int((key[m->Wi - 1 - pos / 64] >> (pos % 64)) & 1u) << b;
  }
  return r;
}
// real: realization of each row (NULL: all rows in realization 0).
void to_internal(const paces_model* m, int64_t n, const uint64_t* in,
                 const int32_t* real, uint64_t* out) {
  for (int64_t i = 0; i < n; ++i) {
    uint64_t* k = out + size_t(i) * m->Wi;
    for (int w = 0; w < m->Wi; ++w) k[w] = 0;
    for (int w = 0; w < m->W; ++w) k[(m->Wi - m->W) + w] = in[size_t(i) * m->W + w];
    const int r = real ? real[i] : 0;
    for (int b = 0; b < m->br; ++b)
      if ((r >> b) & 1) set_ibit(m, k, m->B + b);
  }
}
void to_canonical(const paces_model* m, int64_t n, const uint64_t* in,
                  uint64_t* out, int32_t* real) {
  for (int64_t i = 0; i < n; ++i) {
    if (real) real[i] = internal_real(m, in + size_t(i) * m->Wi);
    uint64_t* k = out + size_t(i) * m->W;
    for (int w = 0; w < m->W; ++w) k[w] = in[size_t(i) * m->Wi + (m->Wi - m->W) + w];
    for (int pos = m->B; pos < 64 * m->W; ++pos)
      k[m->W - 1 - pos / 64] &= ~(uint64_t(1) << (pos % 64));
  }
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

paces_status check_unique(int W, int64_t n, const uint64_t* keys) {
  std::vector<int64_t> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
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

struct EventPair {
  int stage;
  int kk;  // Clenshaw launch index (series launches only)
  hipEvent_t a, b;
  double bytes;
};

}  // namespace

struct AdjRecord;  // recorded run of the adjoint gradient

struct paces_sim {
  const paces_model* m = nullptr;
  paces_run_params p{};
  int prec = 64;
  size_t A = 16;  // bytes per amplitude
  double th2 = 0;

  int64_t cap = 0;  // row capacity of every row array
  Side side[2]{};
  int cur = 0;      // side holding the current set S
  void* vec[4] = {nullptr, nullptr, nullptr, nullptr};
  int ipsi = 0, iphi = 1, ib0 = 2, ib1 = 3;
  uint64_t* table = nullptr;
  uint64_t tmask = 0;        // probe mask of the current step
  uint64_t tmask_alloc = 0;  // allocated table size - 1
  uint32_t* midx = nullptr;
  uint32_t* scan_tmp = nullptr;  // select
  RoundBufs rb{};
  int chunks = 1;  // candidate chunks per expansion round

  // expansion from the previous step's graph (warm.hpp)
  WarmBufs wb{};
  bool graph_ok = false;   // side cur holds complete columns and the table
                           // maps its keys to its rows (probed over tmask)
  bool warm_step = false;  // the step being run expands from that graph,
                           // in place on side cur
  bool last_warm = false;  // the last completed step did
  int nside = 1;           // side the step being run builds its set on
  bool swapped = false;    // the in-place step made psi its phi (ipsi and
                           // iphi exchanged at its transfer)
  int64_t tomb = 0;        // tombstones in the table since it was built
  int64_t scattered = 0;   // found states placed in holes since the set was
                           // last laid out from scratch
  int64_t warm_off_cap = -1;  // row capacity at which an in-place step ran
                              // out of rows (none from the previous graph
                              // until the capacity changes)
  int warm_np = 0;         // partial blocks of the dropped weight
  int warm_nmass = 0;      // the step's folded weight partials
  int64_t nlive = 0;       // live rows of side cur; nS is its row range
  bool has_holes = false;  // side cur has holes (nlive < nS)
  uint32_t* dcount = nullptr;  // [1] a count read back by the host

  // a step run stage by stage (paces_run_stage)
  int staged_next = 0;   // the stage expected next
  int64_t staged_est = 0;
  int staged_mass = 0, staged_e = 0;  // partial counts handed on

  StepCtl* ctl = nullptr;
  int* err = nullptr;
  double* parts = nullptr;
  double *mass_part = nullptr, *n2_part = nullptr, *e_part = nullptr,
         *en_part = nullptr, *pop_part = nullptr, *bnd_part = nullptr;
  double *mass_fold = nullptr, *e_fold = nullptr;
  double* e_row = nullptr;     // per-row energy terms (batched sims)
  ChebCoef* cc = nullptr;      // [R]
  double* a2 = nullptr;        // [R][2]
  uint32_t* cnt = nullptr;     // [2R]: |M_r| then |S_r|
  double* mass_tot = nullptr;  // [R] cumulative discarded weight

  uint64_t* keys0 = nullptr;
  double* amps0 = nullptr;
  int64_t n0 = 0;
  int32_t* p0_last = nullptr;  // [R][n0] rows of the initial states in S
  AdjRecord* adj = nullptr;

  // device blocks that hold several arrays each (one allocation and one
  // free per growth instead of one per array)
  void* rows_block = nullptr;  // row arrays except the hash table
  void* cand_block = nullptr;  // candidate buffers of the expansion rounds
  void* cap_block = nullptr;   // per-row buffers of the state cap
  size_t rows_bytes = 0, cand_bytes = 0, capb_bytes = 0;  // their sizes
  bool mem_capped = false;  // the last growth was cut to fit the device

  // Krylov propagator (krylov_order > 0)
  LanczosState* lz = nullptr;   // [R]
  double* lz_part = nullptr;    // per-block partials of the Lanczos SpMV
  double* lz_energy = nullptr;  // [R] <phi|H|phi>
  std::vector<void*> kry;       // basis vectors 2 .. order, row capacity
                                // (Taylor: the second term and two sums)
  // truncated Taylor propagator (taylor_order != 0)
  TaylorPlan* tplan = nullptr;  // [R]
  double* thetas = nullptr;     // [kTaylorMaxDeg + 1]

  // state cap (max_states per realization)
  uint32_t* ball = nullptr;       // [R] rows of the new set per realization
  bool cap_active = false;        // the step runs with a cut selection
  int64_t cap_buf = 0;            // rows the buffers below hold
  uint8_t* keep = nullptr;        // [rows] selection flags over old rows
  uint32_t* midx_full = nullptr;  // [rows] the step's full selection
  int64_t nM_full = 0;
  uint64_t *cap_w = nullptr, *cap_h = nullptr;  // [rows] sort keys
  uint8_t* cap_status = nullptr;  // [rows] 0 open, 1 kept, 2 dropped
  uint32_t* cap_hist = nullptr;   // [R][256]
  int32_t *cap_mode = nullptr, *cap_dstar = nullptr;  // [R]
  int8_t* cap_capped = nullptr;   // [R]
  std::vector<int64_t> cap_q, cap_nM;
  std::vector<int8_t> cap_on;

  double* ring = nullptr;
  int64_t ring_cap = 0;
  int rec_doubles = 0;

  // host mirror of the device state after the last completed step
  StepCtl h{};              // copy of *ctl
  int64_t nS = 0;
  bool fresh = true;
  bool have_sets = false;   // M / frontiers / phi describe the last step
  bool counts_valid = false;  // scan_tmp holds the next select's counts
  int launched = 32;        // Clenshaw launches enqueued per step
  int K_last = 0;
  int k_last = 0;           // neighbour order of the last step
  int latched = 0;
  StepCtl* h_ctl = nullptr;  // pinned, mapped
  int* h_err = nullptr;      // pinned, mapped
  StepCtl* d_hctl = nullptr;  // device addresses of h_ctl / h_err
  int* d_herr = nullptr;
  std::vector<double> pop_host;

  int prof = 0;  // 0 off, 1 stages and kernels, 2 timed kernels only
  std::vector<EventPair> pending, events;
  paces_profile acc{};

  // launch tuning and captured step graphs
  paces_tuning tune{0, 1, 1, 1};
  hipStream_t cap_stream = nullptr;  // capture only; never runs work
  uint64_t gen = 0;                  // bumped whenever a buffer moves
  // What enqueueing a step leaves on the host (buffer roles, partial
  // counts); a graph replay sets it as its capture did.
  struct HostFx {
    int ipsi, iphi, warm_np, warm_nmass;
    bool swapped;
  };
  struct GraphEntry {
    std::vector<int64_t> key;
    hipGraphExec_t exec;
    uint64_t used;
    HostFx fx;
  };
  std::vector<GraphEntry> graphs;
  uint64_t graph_clock = 0;
};

namespace {

paces_status check_latch_code(paces_sim* s, int e) {
  if (!e) return PACES_OK;
  s->latched = e;
  if (e & kErrTerms)
    return fail(PACES_E_PROPAGATOR, "series needs more than k_max_terms terms");
  if (e & kErrNonFinite)
    return fail(PACES_E_NONFINITE, "non-finite norm after propagation");
  if (e & kErrTableFull) return fail(PACES_E_CAPACITY, "hash table overflow");
  return fail(PACES_E_CAPACITY, "row capacity exceeded");
}

struct Stage {
  paces_sim* s;
  int stage, kk;
  hipStream_t st;
  hipEvent_t a{}, b{};
  Stage(paces_sim* s_, int stage_, hipStream_t st_, int kk_ = -1)
      : s(s_), stage(stage_), kk(kk_), st(st_) {
    if (s->prof == 1) {
      (void)hipEventCreate(&a);
      (void)hipEventCreate(&b);
      (void)hipEventRecord(a, st);
    }
  }
  ~Stage() {
    if (s->prof == 1) {
      (void)hipEventRecord(b, st);
      s->pending.push_back({stage, kk, a, b, 0.0});
    }
  }
};

// Start / stop events of one timed kernel, recorded by its own dispatch;
// queued for classification after the step.  Level 1 times every such
// launch, level 2 one per step (index 1: a middle Clenshaw term whenever
// the series has four or more terms, the second Lanczos SpMV), since each
// timed dispatch still costs the stream some idle time.
struct KernelTiming {
  hipEvent_t a{}, b{};
  KernelTiming(paces_sim* s, int stage, int kk) {
    if (!s->prof || (s->prof == 2 && kk != 1)) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
      if (a) (void)hipEventDestroy(a);
      a = b = nullptr;
      return;
    }
    s->pending.push_back({stage, kk, a, b, 0.0});
  }
};

void drop_pending(paces_sim* s) {
  for (auto& e : s->pending) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  s->pending.clear();
}

void free_rows(paces_sim* s) {
  if (s->rows_block) dev_free(s->rows_block);
  s->rows_block = nullptr;
  s->rows_bytes = 0;
  for (int q = 0; q < 2; ++q) s->side[q] = Side{};
  for (auto& v : s->vec) v = nullptr;
  s->wb.freel = nullptr;
  s->wb.wmask = nullptr;
  s->graph_ok = false;
  s->midx = nullptr;
  s->scan_tmp = nullptr;
  s->e_row = nullptr;
  s->kry.clear();
  dfree(s->table);
}

void free_cand(paces_sim* s) {
  if (s->cand_block) dev_free(s->cand_block);
  s->cand_block = nullptr;
  s->cand_bytes = 0;
  s->rb = RoundBufs{};
  s->wb.wlist = nullptr;
}

paces_status alloc_cand(paces_sim* s, int64_t want) {
  free_cand(s);
  const int64_t tiles = want / 256 + 2;
  Pieces pc;
  pc.add(&s->rb.c_slot, want);
  pc.add(&s->rb.c_ref, want);
  pc.add(&s->rb.crow, want);
  pc.add(&s->wb.wlist, want);
  pc.add(&s->rb.tile_cnt, tiles);
  pc.add(&s->rb.tile_base, tiles);
  pc.add(&s->rb.scan_tmp, scan_tmp_words(tiles));
  ST_TRY(pc.carve(&s->cand_block));
  s->cand_bytes = pc.total();
  s->rb.cand_cap = want;
  return PACES_OK;
}

uint64_t table_size_for(int64_t cap, int shift) {
  uint64_t P = 1024;
  while (P < (uint64_t(cap) << shift)) P <<= 1;
  return P;
}

// Round a row count up to a quarter octave (4, 5, 6 or 7 times a power of
// two): launch grids sized from bucketed counts repeat from step to step,
// so captured graphs can be replayed.
int64_t bucket(int64_t x) {
  if (x <= 64) return 64;
  int e = 0;
  while ((x >> e) > 7) ++e;
  int64_t m = (x + (int64_t(1) << e) - 1) >> e;  // 4..8
  return m << e;
}

void drop_graphs(paces_sim* s) {
  for (auto& g : s->graphs) (void)hipGraphExecDestroy(g.exec);
  s->graphs.clear();
}

// Largest candidate buffer (entries, 20 bytes each plus tile counts); a
// round with more candidates runs in chunks of this size.
constexpr int64_t kCandMax = int64_t(1) << 29;

int64_t cand_want(const paces_model* m, int64_t cap) {
  // candidate buffers: half the worst case to start with; grown on demand
  return std::min<int64_t>(std::max<int64_t>(cap * m->D / 2, int64_t(1) << 16),
                           kCandMax);
}

// Bytes per row of the state carried across a growth: keys, payload,
// totals and psi of the current side.
size_t carried_bytes(const paces_sim* s) {
  return size_t(s->m->Wi) * 8 + 16 + s->A;
}

// Pieces of the row block for cap rows: both sides' keys and row data, the
// four amplitude vectors, the ELL columns, the selection and its scan, the
// per-row energies of batched sims and the extra propagator vectors.
struct RowBlock {
  Side sd[2]{};
  void* vec[4] = {nullptr, nullptr, nullptr, nullptr};
  uint32_t *midx = nullptr, *scan = nullptr;
  uint32_t* freel = nullptr;
  uint16_t* wmask = nullptr;
  double* erow = nullptr;
  std::vector<void*> kry;
  Pieces pc;
  RowBlock(const paces_sim* s, int64_t cap) {
    const paces_model* m = s->m;
    // Krylov basis: w_0 = phi and w_1 = the second Clenshaw buffer; the
    // remaining order - 1 vectors here.  Taylor: one more term buffer and
    // the two substep sums.
    const int n_extra = s->p.krylov_order > 0 ? s->p.krylov_order - 1
                                              : (s->p.taylor_order != 0 ? 3 : 0);
    kry.assign(n_extra, nullptr);
    for (int q = 0; q < 2; ++q) {
      pc.add(&sd[q].keys, cap * m->Wi);
      pc.add(&sd[q].pay, cap);
      pc.add(&sd[q].tot, cap);
      pc.add(&sd[q].col, cap * m->D);
      pc.add(&sd[q].dist, cap);
    }
    for (int v = 0; v < 4; ++v) pc.add_bytes(&vec[v], size_t(cap) * s->A);
    pc.add(&midx, cap);
    pc.add(&freel, cap);
    pc.add(&wmask, cap);
    pc.add(&scan, scan_tmp_words(cap));
    if (m->R > 1) pc.add(&erow, cap);
    for (auto& v : kry) pc.add_bytes(&v, size_t(cap) * s->A);
  }
};

// Whether a capacity of cap rows fits the device.  A growth parks the
// current set in a compact temporary block and frees the old row block and
// table before it allocates the new ones, so the peak is the temporary plus
// the new row block, table, candidate and state-cap buffers.  Only checked
// for the library's own allocator (the caller's may cache).
bool fits_device(const paces_sim* s, int64_t cap) {
  if (g_allocator.alloc) return true;
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) return true;
  const double margin = double(size_t(2) << 30) + 0.02 * double(tot);
  const double block = double(RowBlock(s, cap).pc.total());
  const int64_t want = cand_want(s->m, cap);
  const double cand = want > s->rb.cand_cap ? 20.0 * double(want)
                                            : double(s->cand_bytes);
  const bool capbuf = s->p.q_nom > 0 || s->p.max_states > 0;
  const double temp = double(s->nS) * double(carried_bytes(s));
  const double after =
      block + 8.0 * double(table_size_for(cap, s->tune.table_shift)) + cand +
      (capbuf ? 22.0 * double(cap) : 0.0) + temp;
  const double back = double(s->rows_bytes) + double(s->cand_bytes) +
                      double(s->capb_bytes) + 8.0 * double(s->tmask_alloc + 1);
  return after <= double(fr) + back - margin;
}

// Reallocate every row array for new_cap rows, keeping the current set
// (side cur, rows [0, nS)) and its amplitudes.  Everything else is rebuilt
// by the next step.  Where new_cap rows do not fit the device the capacity
// is cut, down to min_cap (then the allocation is tried as asked).
paces_status grow(paces_sim* s, int64_t new_cap, int64_t min_cap,
                  hipStream_t st) {
  const paces_model* m = s->m;
  drop_graphs(s);
  ++s->gen;
  auto round_cap = [](int64_t c) {
    return std::min<int64_t>((c + 255) / 256 * 256, (int64_t(1) << 31) - 256);
  };
  new_cap = round_cap(new_cap);
  min_cap = std::min(round_cap(std::max(min_cap, s->cap + 1)), new_cap);
  if (new_cap <= s->cap && s->cap > 0)
    return fail(PACES_E_CAPACITY, "row capacity limit (2^31 rows) reached");
  const int64_t asked = new_cap;
  while (new_cap > min_cap && !fits_device(s, new_cap))
    new_cap = std::max(min_cap, round_cap(new_cap - new_cap / 8));
  s->mem_capped = new_cap < asked;
  // The current set and psi are parked in a compact block while the old
  // row block, table and candidate buffers are released, then copied into
  // the new row block (every row array but the table, in one block).
  // Holes of an in-place step are left out.
  const int64_t n = s->nlive;
  const size_t kb = size_t(n) * m->Wi * 8, ab = size_t(n) * s->A;
  uint8_t* park = nullptr;
  if (n > 0) {
    void* q = nullptr;
    ST_TRY(dev_alloc(&q, kb + 16 * size_t(n) + ab + 4 * size_t(n) + 1024));
    park = static_cast<uint8_t*>(q);
    const Side& o = s->side[s->cur];
    if (s->has_holes) {
      uint32_t* idx = reinterpret_cast<uint32_t*>(park + kb + 16 * size_t(n) + ab);
      rows_at_distance(m->Wi, o.keys, o.dist, s->nS, -1, nullptr, idx,
                       s->dcount, s->scan_tmp, st);
      gather_rows(m->Wi, s->A, o, s->vec[s->ipsi], idx, n,
                  reinterpret_cast<uint64_t*>(park),
                  reinterpret_cast<uint64_t*>(park + kb),
                  reinterpret_cast<uint64_t*>(park + kb + 8 * size_t(n)),
                  park + kb + 16 * size_t(n), st);
    } else {
      HIP_TRY(hipMemcpyAsync(park, o.keys, kb, hipMemcpyDeviceToDevice, st));
      HIP_TRY(hipMemcpyAsync(park + kb, o.pay, size_t(n) * 8,
                             hipMemcpyDeviceToDevice, st));
      HIP_TRY(hipMemcpyAsync(park + kb + 8 * size_t(n), o.tot, size_t(n) * 8,
                             hipMemcpyDeviceToDevice, st));
      HIP_TRY(hipMemcpyAsync(park + kb + 16 * size_t(n), s->vec[s->ipsi], ab,
                             hipMemcpyDeviceToDevice, st));
    }
  }
  HIP_TRY(hipStreamSynchronize(st));
  if (s->rows_block) dev_free(s->rows_block);
  s->rows_block = nullptr;
  s->rows_bytes = 0;
  dfree(s->table);
  const int64_t want_c = cand_want(m, new_cap);
  if (want_c > s->rb.cand_cap) free_cand(s);
  // (RowBlock holds the addresses of its own members: built in place)
  std::unique_ptr<RowBlock> nbp(new RowBlock(s, new_cap));
  void* block = nullptr;
  paces_status got = nbp->pc.carve(&block);
  if (got != PACES_OK && min_cap < new_cap) {
    new_cap = min_cap;
    s->mem_capped = true;
    nbp.reset(new RowBlock(s, new_cap));
    got = nbp->pc.carve(&block);
  }
  RowBlock& nb = *nbp;
  if (got != PACES_OK) {
    // the set is gone with the old block: the sim needs a new state
    if (park) dev_free(park);
    free_rows(s);
    s->cap = 0;
    s->nS = 0;
    s->nlive = 0;
    s->has_holes = false;
    s->latched = kErrCapacity;
    return fail(PACES_E_OOM, "row arrays do not fit the device");
  }
  if (n > 0) {
    Side& c = nb.sd[s->cur];
    HIP_TRY(hipMemcpyAsync(c.keys, park, kb, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(c.pay, park + kb, size_t(n) * 8,
                           hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(c.tot, park + kb + 8 * size_t(n), size_t(n) * 8,
                           hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(nb.vec[s->ipsi], park + kb + 16 * size_t(n), ab,
                           hipMemcpyDeviceToDevice, st));
    dist_fill(c.dist, n, 0, st);
    HIP_TRY(hipStreamSynchronize(st));
    dev_free(park);
  }
  if (n != s->nS) {
    // holes were left out: the device's row count of the set (read by the
    // selection and the transfer of the step being repeated) follows
    const uint32_t n32 = uint32_t(n);
    HIP_TRY(hipMemcpyAsync(&s->ctl->n_old, &n32, 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    s->h.n_old = n32;
    s->h.n_new = n32;
  }
  s->nS = n;
  s->has_holes = false;
  s->rows_block = block;
  s->rows_bytes = nb.pc.total();
  s->side[0] = nb.sd[0];
  s->side[1] = nb.sd[1];
  for (int v = 0; v < 4; ++v) s->vec[v] = nb.vec[v];
  s->wb.freel = nb.freel;
  s->wb.wmask = nb.wmask;
  s->graph_ok = false;  // columns and table are rebuilt by the next step
  s->midx = nb.midx;
  s->scan_tmp = nb.scan;
  s->e_row = nb.erow;
  s->kry = nb.kry;
  s->cap = new_cap;
  s->counts_valid = false;
  const uint64_t P = table_size_for(new_cap, s->tune.table_shift);
  ST_TRY(dalloc(&s->table, int64_t(P)));
  s->tmask_alloc = P - 1;
  s->tmask = P - 1;
  if (want_c > s->rb.cand_cap) ST_TRY(alloc_cand(s, want_c));
  return PACES_OK;
}

// More candidate room for a round whose frontier overflowed the chunks of
// the step: larger buffers up to kCandMax, then more chunks per round.
paces_status more_chunks(paces_sim* s, hipStream_t st) {
  drop_graphs(s);
  ++s->gen;
  if (s->rb.cand_cap < kCandMax) {
    HIP_TRY(hipStreamSynchronize(st));
    return alloc_cand(s, std::min<int64_t>(2 * s->rb.cand_cap, kCandMax));
  }
  const int need = int(std::min<uint32_t>(s->h_ctl->r_need, 1u << 16));
  s->chunks = std::max(s->chunks + 1, need);
  return PACES_OK;
}

paces_status ensure_ring(paces_sim* s, hipStream_t st) {
  if (int64_t(s->h.nrec) + 1 < s->ring_cap) return PACES_OK;
  const int64_t nc = std::max<int64_t>(1024, 2 * s->ring_cap);
  double* r = nullptr;
  const int64_t per_step = int64_t(s->m->R) * s->rec_doubles;
  ST_TRY(dalloc(&r, nc * per_step));
  if (s->h.nrec > 0)
    HIP_TRY(hipMemcpyAsync(r, s->ring, size_t(s->h.nrec) * per_step * 8,
                           hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  drop_graphs(s);
  ++s->gen;
  dfree(s->ring);
  s->ring = r;
  s->ring_cap = nc;
  return PACES_OK;
}

paces_status push_ctl(paces_sim* s, hipStream_t st) {
  *s->h_ctl = s->h;
  HIP_TRY(hipMemcpyAsync(s->ctl, s->h_ctl, sizeof(StepCtl),
                         hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  return PACES_OK;
}

// Upload a state given as internal keys + FP64 amplitudes into side cur.
paces_status upload_state(paces_sim* s, int64_t n,
                          const std::vector<uint64_t>& ik, const double* amps,
                          hipStream_t st) {
  const paces_model* m = s->m;
  if (n > s->cap) {
    s->nS = 0;
    s->nlive = 0;
    s->has_holes = false;
    ST_TRY(grow(s, std::max<int64_t>(2 * n, 2 * s->cap), n, st));
  }
  Side& sc = s->side[s->cur];
  if (n > 0) {
    HIP_TRY(hipMemcpyAsync(sc.keys, ik.data(), ik.size() * 8,
                           hipMemcpyHostToDevice, st));
    double* tmp = nullptr;
    ST_TRY(dalloc(&tmp, 2 * n));
    HIP_TRY(hipMemcpyAsync(tmp, amps, size_t(n) * 16, hipMemcpyHostToDevice, st));
    amps_from_f64(s->prec, tmp, s->vec[s->ipsi], n, st);
    row_info(m->dm, m->Wi, sc.keys, n, sc.pay, sc.tot, st);
    dist_fill(sc.dist, n, 0, st);  // every row live
    HIP_TRY(hipStreamSynchronize(st));
    dfree(tmp);
  }
  s->nS = n;
  s->nlive = n;
  s->has_holes = false;
  s->h.n_old = uint32_t(n);
  s->graph_ok = false;  // no columns yet: the next step expands from scratch
  return push_ctl(s, st);
}

// Enqueue one attempt of a step.  Nothing here waits on the GPU.  `est`
// (the host's guess of the new set's size) only sizes launch grids; every
// kernel strides over whatever the device counts say.
// A frozen step (adjoint replay) takes M from a record instead of the
// threshold, and keeps the row maps the backward pass needs.
struct FrozenStep {
  const uint64_t* mkeys;  // nM internal keys
  int64_t nM;
  int k;
  int32_t* tmap;   // [old rows] new row of every old row (may be null)
  int32_t* p0map;  // [n0] rows of the initial states (may be null)
};

// Partial results a step hands from one stage to the next.
struct StepLocals {
  int n_mass = 0, n_e = 0;
};

int step_order(const paces_sim* s, const FrozenStep* fz) {
  return fz ? fz->k : (s->fresh ? s->p.k_init : s->p.k);
}

// select: clear the step's counters and latch, then M (threshold, preset
// flags of a state cap, or a frozen record).
void stage_select(paces_sim* s, bool counted, hipStream_t st,
                  const FrozenStep* fz) {
  const int R = s->m->R;
  begin_step(s->ctl, s->err, s->cnt, R, st);
  Stage sg(s, PACES_STAGE_SELECT, st);
  if (fz)
    adj_set_frozen(s->ctl, s->cnt, uint32_t(fz->nM), s->err, st);
  else if (s->cap_active)
    select_flags(s->keep, s->ctl, s->midx, s->scan_tmp,
                 std::min(bucket(s->nS), s->cap), s->err, st);
  else
    select_rows(s->prec, s->vec[s->ipsi], s->side[s->cur].dist, s->th2,
                s->fresh, counted, s->ctl, s->midx, s->scan_tmp,
                std::min(bucket(s->nS), s->cap), s->err, st);
  if (s->warm_step)
    warm_begin(s->m->dm, s->ctl, s->midx, s->side[s->cur], s->wb, s->cnt,
               s->nS, s->has_holes, s->scan_tmp, s->err, st);
}

// expand + merge + build of the columns from the previous step's graph, in
// place: k rounds of the breadth-first search (found states take holes or
// rows past the range), the new set's sizes with the state-cap check, then
// the commit: unreached rows become holes (with the dropped weight), found
// states get their columns and their table entries.
void stage_expand_warm(paces_sim* s, int64_t est, hipStream_t st) {
  const paces_model* m = s->m;
  const DevModel& dm = m->dm;
  const int Wi = m->Wi;
  const int k = s->p.k;
  const Side c = s->side[s->cur];
  Stage sg(s, PACES_STAGE_EXPAND, st);
  for (int r = 1; r <= k; ++r)
    warm_round(dm, Wi, s->prec, c, r, s->ctl, s->cap, s->nS, est, s->table,
               s->tmask, s->rb, s->wb, s->scan_tmp, s->vec[s->ipsi], s->err,
               st);
  warm_sizes(dm, c, k, s->ctl, est, s->p.max_states, s->ball, s->err, st);
  s->warm_np = warm_commit(dm, Wi, s->prec, c, k, s->ctl, s->nS, est,
                           s->table, s->tmask, s->wb, s->vec[s->ipsi],
                           s->mass_part, s->err, st);
}

// expand + merge + build of the columns: M into the cleared table, k
// rounds, the lookup pass of the last frontier, the state-cap check.
void stage_expand(paces_sim* s, int64_t est, hipStream_t st,
                  const FrozenStep* fz) {
  if (s->warm_step && !fz) {
    stage_expand_warm(s, est, st);
    return;
  }
  const paces_model* m = s->m;
  const DevModel& dm = m->dm;
  const int Wi = m->Wi;
  const int k = step_order(s, fz);
  const Side so = s->side[s->cur], sn = s->side[1 - s->cur];
  Stage sg(s, PACES_STAGE_EXPAND, st);
  fill_u64(s->table, int64_t(s->tmask + 1), kEmpty, st);
  if (fz) {
    if (fz->nM > 0)
      (void)hipMemcpyAsync(sn.keys, fz->mkeys, size_t(fz->nM) * Wi * 8,
                           hipMemcpyDeviceToDevice, st);
    row_info(dm, Wi, sn.keys, fz->nM, sn.pay, sn.tot, st);
    rehash_rows(dm, Wi, sn, nullptr, fz->nM, s->table, s->tmask, s->err, st);
  } else {
    insert_rows(dm, Wi, s->prec, so, sn, s->midx, s->ctl, s->table, s->tmask,
                s->cnt, s->vec[s->ipsi], s->vec[s->iphi], s->err, st);
  }
  for (int r = 1; r <= k; ++r)
    expand_round(dm, Wi, s->prec, sn, r, s->ctl, s->cap, est, s->table,
                 s->tmask, s->rb, sn.col, s->vec[s->iphi], s->chunks, s->err,
                 st);
  lookup_last(dm, Wi, sn, k, s->ctl, est, s->table, s->tmask, sn.col, s->cap,
              s->err, st);
  if (s->p.max_states > 0)
    cap_check(dm, s->ctl, sn.pay, est, s->p.max_states, s->ball, s->err, st);
  dist_of_rounds(s->ctl, k, sn.dist, est, st);
}

// transfer: old amplitudes into phi, discarded weight.
void stage_transfer(paces_sim* s, hipStream_t st, const FrozenStep* fz,
                    StepLocals& L) {
  const paces_model* m = s->m;
  const int R = m->R;
  const Side so = s->side[s->cur], sn = s->side[1 - s->cur];
  Stage sg(s, PACES_STAGE_TRANSFER, st);
  if (s->warm_step && !fz) {
    // the in-place expansion left phi in psi's buffer (kept amplitudes,
    // zeros elsewhere) and the dropped weight in partials
    L.n_mass = R == 1 ? fold_sum(s->mass_part, s->warm_np, s->mass_fold,
                                 s->err, st)
                      : s->warm_np;
    s->warm_nmass = L.n_mass;
    if (!s->swapped) {
      std::swap(s->ipsi, s->iphi);
      s->swapped = true;
    }
    return;
  }
  // rows of M were placed with their amplitudes by the insert; the frozen
  // replay maps every old row
  const int skip = fz ? 0 : (s->cap_active ? 2 : (s->fresh ? 0 : 1));
  const int np = transfer(m->dm, m->Wi, s->prec, so, s->vec[s->ipsi],
                          bucket(s->nS), s->ctl, s->table, s->tmask, sn.keys,
                          s->vec[s->iphi], s->mass_part,
                          fz ? fz->tmap : nullptr, skip, s->th2, s->keep,
                          s->err, st);
  L.n_mass = R == 1 ? fold_sum(s->mass_part, np, s->mass_fold, s->err, st)
                    : np;
}

// build: spectral bounds and the propagator's coefficients or plan (the
// Krylov propagator builds its small matrix inside the propagation).
void stage_build(paces_sim* s, int64_t est, hipStream_t st) {
  const paces_model* m = s->m;
  const Side sn = s->side[s->nside];
  if (s->p.krylov_order > 0) return;
  Stage sg(s, PACES_STAGE_BUILD, st);
  if (s->p.taylor_order != 0) {
    const int nb = bounds_part(m->dm, sn, sn.col, s->cap, est, s->ctl,
                               s->bnd_part, s->err, st);
    taylor_plan(m->R, s->bnd_part, nb, s->p.dt, s->p.taylor_order, s->thetas,
                s->p.k_max_terms, s->launched, s->tplan, s->cc, s->ctl,
                s->err, st);
  } else {
    bounds_and_coef(m->dm, sn, sn.col, s->cap, est, s->ctl, s->p.dt, s->p.tol,
                    s->p.k_max_terms, s->launched, s->bnd_part, s->cc, s->err,
                    st);
  }
}

// propagate: psi' = exp(-i H dt) phi into vector ib0.
void stage_propagate(paces_sim* s, int64_t est, hipStream_t st,
                     StepLocals& L) {
  const paces_model* m = s->m;
  const DevModel& dm = m->dm;
  const int R = m->R;
  const Side sn = s->side[s->nside];
  const bool want_e = (s->p.obs_mask & PACES_OBS_ENERGY) != 0;
  Stage sg(s, PACES_STAGE_PROPAGATE, st);
  if (s->p.taylor_order != 0) {
    // truncated Taylor series: launch L is term L mod m + 1 of substep L / m
    void* bufB[2] = {s->vec[s->ib1], s->kry[0]};
    void* bufF[2] = {s->kry[1], s->kry[2]};
    int np = 0;
    // the adaptive series is exact to rounding, so the energy of phi is
    // that of the result; the fixed order needs its own pass
    const bool fixed = s->p.taylor_order > 0;
    for (int l = 0; l < s->launched; ++l) {
      KernelTiming kt(s, PACES_STAGE_TERM, l);
      const int g = taylor_term(dm, s->prec, l, want_e && !fixed, s->p.dt,
                                std::max<int64_t>(1, est / s->tune.term_rows),
                                s->ctl, sn.col, sn, s->tplan,
                                s->vec[s->iphi], bufB, bufF, s->vec[s->ib0],
                                s->e_part, s->e_row, s->err, kt.a, kt.b, st);
      if (l == 0) np = g;
    }
    if (want_e && fixed)
      np = taylor_energy(dm, s->prec, est, s->ctl, sn.col, sn, s->vec[s->ib0],
                         s->e_part, s->e_row, s->err, st);
    if (want_e && R == 1) L.n_e = fold_sum(s->e_part, np, s->e_fold, s->err, st);
  } else if (s->p.krylov_order > 0) {
    // Krylov propagator: nk SpMVs with their folds, nk - 1 recurrence
    // passes, the small exponential and the combination into b0
    const int nk = s->p.krylov_order + 1;
    KrylovVecs kv{};
    kv.w[0] = s->vec[s->iphi];
    for (int j = 1; j < nk; ++j)
      kv.w[j] = j == 1 ? s->vec[s->ib1] : s->kry[j - 2];
    const double brk = s->prec == 64 ? kLzBreak64 : kLzBreak32;
    lz_begin(s->lz, R, s->err, st);
    for (int j = 0; j < nk; ++j) {
      const bool last = j == nk - 1;
      void* out = last ? nullptr : kv.w[j + 1];
      int np = 0;
      if (!last) {
        KernelTiming kt(s, PACES_STAGE_KRYLOV, j);
        np = lz_spmv(dm, s->prec, j, est, s->ctl, sn.col, sn, s->lz, kv.w[j],
                     out, s->lz_part, s->err, kt.a, kt.b, st);
      } else {
        np = lz_spmv(dm, s->prec, j, est, s->ctl, sn.col, sn, s->lz, kv.w[j],
                     out, s->lz_part, s->err, nullptr, nullptr, st);
      }
      lz_fold(j, s->lz_part, np, R, brk * brk, s->lz, s->lz_energy, s->err,
              st);
      if (!last)
        lz_orth(dm, s->prec, j, est, s->ctl, sn.pay, s->lz, kv.w[j + 1],
                kv.w[j], j > 0 ? kv.w[j - 1] : nullptr, s->err, st);
    }
    lz_small(R, s->p.dt, s->p.tol, s->p.k_max_terms, s->lz, s->cc, s->ctl,
             s->err, st);
    lz_combine(dm, s->prec, est, s->ctl, sn.pay, s->lz, kv, nk,
               s->vec[s->ib0], s->err, st);
  } else {
    int np = 0;
    for (int kk = s->launched - 1; kk >= 0; --kk) {
      KernelTiming kt(s, PACES_STAGE_TERM, kk);
      const bool mid = s->K_last >= 4 && kk >= 1 && kk <= s->K_last - 3;
      np = cheb_term(dm, s->prec, kk, want_e, mid,
                     std::max<int64_t>(1, est / s->tune.term_rows), s->ctl,
                     sn.col, s->cap, sn, s->cc, s->vec[s->iphi],
                     s->vec[s->ib0], s->vec[s->ib1], s->e_part, s->e_row,
                     s->err, kt.a, kt.b, st);
    }
    if (want_e && R == 1) L.n_e = fold_sum(s->e_part, np, s->e_fold, s->err, st);
  }
}

// observe: norm, energy, a(t), populations into the record ring; commit
// the step's counts on the device and mirror them to the host.
void stage_observe(paces_sim* s, int64_t est, hipStream_t st,
                   const FrozenStep* fz, const StepLocals& L) {
  const paces_model* m = s->m;
  const DevModel& dm = m->dm;
  const int R = m->R;
  const Side sn = s->side[s->nside];
  const bool want_e = (s->p.obs_mask & PACES_OBS_ENERGY) != 0;
  const bool krylov = s->p.krylov_order > 0;
  Stage sg(s, PACES_STAGE_OBSERVE, st);
  const int n_pop = pop_norm(s->prec, m->N, R, s->th2, est, s->ctl,
                             s->vec[s->ib0], sn.pay, sn.dist,
                             want_e && R > 1 && !krylov ? s->e_row : nullptr,
                             s->n2_part, s->en_part, s->pop_part, s->scan_tmp,
                             s->cnt + R, s->err, st);
  autocorr(dm, m->Wi, s->prec, s->keys0, s->amps0, s->n0, s->table, s->tmask,
           sn.keys, s->vec[s->ib0], s->a2, fz ? fz->p0map : s->p0_last,
           s->err, st);
  obs_final(m->N, R, want_e && !krylov ? 1 : 0, s->p.dt, L.n_mass, L.n_e,
            n_pop, R == 1 ? s->mass_fold : s->mass_part, s->n2_part,
            s->e_fold, s->en_part, s->pop_part, s->a2, s->cc, s->ctl, s->cnt,
            s->mass_tot, s->ring, s->rec_doubles, s->ring_cap, s->err, st);
  if (want_e && krylov)
    lz_record_energy(R, s->lz_energy, s->ctl, s->ring, s->rec_doubles,
                     s->ring_cap, s->err, st);
  end_step(s->ctl, R, s->ring, s->rec_doubles, s->mass_tot, s->err, s->d_hctl,
           s->d_herr, st);
}

void enqueue_step(paces_sim* s, int64_t est, bool counted, hipStream_t st,
                  const FrozenStep* fz = nullptr) {
  StepLocals L;
  stage_select(s, counted, st, fz);
  stage_expand(s, est, st, fz);
  stage_transfer(s, st, fz, L);
  stage_build(s, est, st);
  stage_propagate(s, est, st, L);
  stage_observe(s, est, st, fz, L);
}

// Replay the captured graph of this step's launch sequence, capturing it
// first if no graph matches.  Everything a launch takes from the host is in
// the key; buffer moves bump s->gen (and drop every graph).
paces_status launch_step_graph(paces_sim* s, int64_t est, bool counted,
                               hipStream_t st) {
  const std::vector<int64_t> key = {
      int64_t(s->gen), s->cur, s->ipsi, s->iphi, s->ib0, s->ib1,
      s->fresh ? 1 : 0, counted ? 1 : 0, s->fresh ? s->p.k_init : s->p.k,
      s->launched, s->K_last, est, std::min(bucket(s->nS), s->cap),
      int64_t(s->tmask), s->tune.term_rows, s->p.krylov_order,
      s->p.taylor_order, s->chunks, s->warm_step ? 1 : 0,
      s->has_holes ? 1 : 0};
  for (auto& g : s->graphs)
    if (g.key == key) {
      g.used = ++s->graph_clock;
      HIP_TRY(hipGraphLaunch(g.exec, st));
      s->ipsi = g.fx.ipsi;
      s->iphi = g.fx.iphi;
      s->warm_np = g.fx.warm_np;
      s->warm_nmass = g.fx.warm_nmass;
      s->swapped = g.fx.swapped;
      return PACES_OK;
    }
  if (!s->cap_stream)
    HIP_TRY(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
  enqueue_step(s, est, counted, s->cap_stream);
  hipGraph_t graph = nullptr;
  HIP_TRY(hipStreamEndCapture(s->cap_stream, &graph));
  hipGraphExec_t exec = nullptr;
  const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess)
    return fail(PACES_E_HIP, std::string("graph instantiation: ") +
                                 hipGetErrorString(e));
  if (s->graphs.size() >= 32) {
    auto old = std::min_element(
        s->graphs.begin(), s->graphs.end(),
        [](const paces_sim::GraphEntry& a, const paces_sim::GraphEntry& b) {
          return a.used < b.used;
        });
    (void)hipGraphExecDestroy(old->exec);
    s->graphs.erase(old);
  }
  const paces_sim::HostFx fx{s->ipsi, s->iphi, s->warm_np, s->warm_nmass,
                             s->swapped};
  s->graphs.push_back({key, exec, ++s->graph_clock, fx});
  HIP_TRY(hipGraphLaunch(exec, st));
  return PACES_OK;
}

paces_status cap_buffers(paces_sim* s) {
  const int R = s->m->R;
  if (s->cap_buf < s->cap) {
    if (s->cap_block) dev_free(s->cap_block);
    s->cap_block = nullptr;
    s->cap_buf = 0;
    s->capb_bytes = 0;
    Pieces pc;
    pc.add(&s->keep, s->cap);
    pc.add(&s->midx_full, s->cap);
    pc.add(&s->cap_w, s->cap);
    pc.add(&s->cap_h, s->cap);
    pc.add(&s->cap_status, s->cap);
    ST_TRY(pc.carve(&s->cap_block));
    s->capb_bytes = pc.total();
    s->cap_buf = s->cap;
  }
  if (!s->cap_hist) {
    ST_TRY(dalloc(&s->cap_hist, int64_t(R) * 256));
    ST_TRY(dalloc(&s->cap_mode, R));
    ST_TRY(dalloc(&s->cap_dstar, R));
    ST_TRY(dalloc(&s->cap_capped, R));
  }
  return PACES_OK;
}

paces_status topq_cut(paces_sim* s, hipStream_t st);

// Fixed-size truncation: M = the q_nom heaviest rows of every
// realization's set, ties broken as for the state cap.
paces_status qnom_select(paces_sim* s, hipStream_t st) {
  const paces_model* m = s->m;
  const int R = m->R;
  ST_TRY(cap_buffers(s));
  // every live row of the set
  const Side& c = s->side[s->cur];
  s->nM_full = s->nlive;
  if (s->has_holes) {
    rows_at_distance(m->Wi, c.keys, c.dist, s->nS, -1, nullptr, s->midx_full,
                     s->dcount, s->scan_tmp, st);
    s->counts_valid = false;
  } else {
    iota_u32(s->midx_full, s->nS, st);
  }
  std::vector<uint32_t> cnt(R, 0);
  if (R == 1) {
    cnt[0] = uint32_t(s->nlive);
  } else {
    count_per_real(m->dm, c.pay, s->nM_full, s->ball, st,
                   s->has_holes ? s->midx_full : nullptr);
    HIP_TRY(hipMemcpyAsync(cnt.data(), s->ball, size_t(R) * 4,
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  s->cap_nM.assign(cnt.begin(), cnt.end());
  s->cap_on.assign(R, 0);
  s->cap_q.assign(R, s->p.q_nom);
  for (int r = 0; r < R; ++r) s->cap_on[r] = int64_t(cnt[r]) > s->p.q_nom;
  return topq_cut(s, st);
}

// State cap: some realization's new set exceeds max_states.  Cut its
// selection to the q heaviest rows (weight descending, splitmix64 key hash
// ascending, key ascending) with q = floor(cap |M_prev| / |S_prev|) from
// the last record (floor(cap / (D+1)) without one), and on every further
// overflow q <- floor(9 min(q, |M|) cap / (10 |ball|)); the full selection
// of the step is kept for the repeated cuts.  over: the ball outgrew the
// row capacity before it was counted (first cut of one realization only,
// whose q needs no ball count).
paces_status cap_select(paces_sim* s, hipStream_t st, bool over) {
  const paces_model* m = s->m;
  const int R = m->R;
  const int64_t cap = s->p.max_states;
  std::vector<uint32_t> ball(R), cnt(R);
  HIP_TRY(hipMemcpyAsync(ball.data(), s->ball, size_t(R) * 4,
                         hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(cnt.data(), s->cnt, size_t(R) * 4,
                         hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  // the ball outgrew the rows: it was not counted, but it is over the cap
  if (over) std::fill(ball.begin(), ball.end(), ~0u);
  if (!s->cap_active) {
    ST_TRY(cap_buffers(s));
    s->nM_full = s->h_ctl->nM;
    if (s->nM_full > 0)
      HIP_TRY(hipMemcpyAsync(s->midx_full, s->midx, size_t(s->nM_full) * 4,
                             hipMemcpyDeviceToDevice, st));
    s->cap_nM.assign(cnt.begin(), cnt.end());
    s->cap_on.assign(R, 0);
    s->cap_q.assign(R, 0);
  }
  // counts of the last recorded step per realization
  std::vector<double> prev;
  if (!s->fresh && s->h.nrec > 0) {
    prev.resize(size_t(R) * s->rec_doubles);
    HIP_TRY(hipMemcpyAsync(prev.data(),
                           s->ring + (int64_t(s->h.nrec) - 1) * R * s->rec_doubles,
                           prev.size() * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  for (int r = 0; r < R; ++r) {
    if (int64_t(ball[r]) <= cap) continue;
    if (!s->cap_on[r]) {
      s->cap_on[r] = 1;
      const int64_t nSp = prev.empty() ? 0 : int64_t(prev[size_t(r) * s->rec_doubles + 7]);
      const int64_t nMp = prev.empty() ? 0 : int64_t(prev[size_t(r) * s->rec_doubles + 8]);
      s->cap_q[r] = (nSp > 0 && nMp > 0) ? cap * nMp / nSp : cap / (m->D + 1);
    } else {
      const int64_t qe = std::min(s->cap_q[r], s->cap_nM[r]);
      s->cap_q[r] = 9 * qe * cap / (10 * int64_t(ball[r]));
    }
  }
  return topq_cut(s, st);
}

// Cut the selection midx_full of every realization r with cap_on[r] to its
// cap_q[r] heaviest rows (weight descending, splitmix64 key hash ascending,
// key ascending) by an MSD radix select, leaving the result as row flags
// for a preset-selection attempt.
paces_status topq_cut(paces_sim* s, hipStream_t st) {
  const paces_model* m = s->m;
  const int R = m->R;
  const int Wi = m->Wi, W = m->W;
  const Side& so = s->side[s->cur];
  std::vector<int8_t> capped(s->cap_on.begin(), s->cap_on.end());
  HIP_TRY(hipMemcpyAsync(s->cap_capped, capped.data(), size_t(R),
                         hipMemcpyHostToDevice, st));
  cap_prepare(m->dm, Wi, W, s->prec, s->midx_full, s->nM_full, so.keys,
              so.pay, s->vec[s->ipsi], s->cap_capped, s->cap_w, s->cap_h,
              s->cap_status, st);
  std::vector<int64_t> need(R, 0);
  std::vector<int32_t> mode(R, kCapSkip), dstar(R, 0);
  std::vector<char> open(R, 0);
  for (int r = 0; r < R; ++r) {
    if (!s->cap_on[r]) continue;
    need[r] = std::min(s->cap_q[r], s->cap_nM[r]);
    if (need[r] == 0)
      mode[r] = kCapDrop;
    else if (need[r] == s->cap_nM[r])
      mode[r] = kCapKeep;
    else
      open[r] = 1;
  }
  std::vector<uint32_t> hist(size_t(R) * 256);
  for (int pass = 0; pass <= cap_passes(W); ++pass) {
    HIP_TRY(hipMemcpyAsync(s->cap_mode, mode.data(), size_t(R) * 4,
                           hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->cap_dstar, dstar.data(), size_t(R) * 4,
                           hipMemcpyHostToDevice, st));
    cap_apply(m->dm, Wi, W, std::max(pass - 1, 0), s->midx_full, s->nM_full,
              so.keys, so.pay, s->cap_w, s->cap_h, s->cap_mode, s->cap_dstar,
              s->cap_status, st);
    std::fill(mode.begin(), mode.end(), int32_t(kCapSkip));
    if (std::find(open.begin(), open.end(), 1) == open.end()) break;
    if (pass == cap_passes(W))
      return fail(PACES_E_STATE, "state cap: rows left undecided");
    HIP_TRY(hipMemsetAsync(s->cap_hist, 0, hist.size() * 4, st));
    cap_hist(m->dm, Wi, W, pass, s->midx_full, s->nM_full, so.keys, so.pay,
             s->cap_w, s->cap_h, s->cap_status, s->cap_hist, st);
    HIP_TRY(hipMemcpyAsync(hist.data(), s->cap_hist, hist.size() * 4,
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int r = 0; r < R; ++r) {
      if (!open[r]) continue;
      const uint32_t* h = hist.data() + size_t(r) * 256;
      int64_t below = 0;
      int d = 0;
      for (; d < 255; ++d) {
        if (below + h[d] >= need[r]) break;
        below += h[d];
      }
      need[r] -= below;
      dstar[r] = d;
      if (need[r] == int64_t(h[d])) {
        mode[r] = kCapCut;
        open[r] = 0;
      } else {
        mode[r] = kCapSplit;
      }
    }
  }
  cap_flags(s->midx_full, s->nM_full, s->cap_status, s->keep, s->nS, st);
  s->cap_active = true;
  return PACES_OK;
}

// Fraction of the set placed into holes by in-place steps after which the
// next step lays the set out from scratch (tuning warm = 1).
constexpr double kRelayout = 0.1;

// An expansion from scratch probes only as much of the table as the step
// needs (load factor at most 2^-table_shift for a new set up to the
// estimate); the table clear costs with it.
void cold_table_mask(paces_sim* s, int64_t est) {
  uint64_t P = 1024;
  while (P < (uint64_t(est) << s->tune.table_shift) && P <= s->tmask_alloc)
    P <<= 1;
  s->tmask = std::min<uint64_t>(P - 1, s->tmask_alloc);
}

// Host preparation of a step: room for the new set, the record ring, the
// launch estimate and the part of the table the step probes, and the
// fixed-size truncation's selection.  Returns the estimate.
paces_status prepare_step(paces_sim* s, hipStream_t st, bool frozen,
                          int64_t* est_out) {
  // keep room for the new set: growth of the set per step stays well below
  // the factor used here in the workloads; an overflow is caught anyway.
  // Growth to 4 |S| makes the next one due only when the set has doubled.
  // A capacity cut to fit the device grows again only when the step's
  // estimate no longer fits it.  Under a state cap no set holds more than
  // R * max_states rows: that plus an eighth (holes of in-place steps) is
  // all the capacity such a run grows to; a ball beyond it is cut (or, for
  // several realizations, grows the rows when it is met).
  int64_t need = s->nS + std::max<int64_t>(s->nS / 2, 65536);
  int64_t want = 4 * s->nS;
  if (s->p.max_states > 0) {
    const int64_t top = int64_t(s->m->R) * s->p.max_states;
    const int64_t lim = top + std::max<int64_t>(top / 8, 65536);
    need = std::min(need, lim);
    want = std::min(want, lim);
  }
  if (s->nS > s->cap / 2 && s->cap < want &&
      (!s->mem_capped || need > s->cap))
    ST_TRY(grow(s, want, need, st));
  ST_TRY(ensure_ring(s, st));
  const int64_t est = std::min<int64_t>(
      s->cap, bucket(std::max<int64_t>(s->nS + s->nS / 2, s->nS + 65536)));
  // expand from the previous step's graph when it is there and its table
  // (probed over the same part, tombstones included) has room for a new
  // set up to the estimate at load factor 2^-table_shift
  // A step from scratch lays the set out in breadth-first order from M
  // (a row's neighbours sit in the same or the next layer at a matching
  // place); in-place steps put found states into holes wherever drops left
  // them, which loosens that order.  Once as many states as kRelayout of
  // the set went into holes, the next step is from scratch again.
  s->warm_step =
      s->tune.warm && s->graph_ok && !s->fresh && !frozen &&
      s->cap <= kWarmMaxRows && s->cap != s->warm_off_cap &&
      (s->tune.warm == 2 ||
       double(s->scattered) <= kRelayout * double(s->nlive)) &&
      (uint64_t(est + s->tomb) << s->tune.table_shift) <= s->tmask + 1;
  s->nside = s->warm_step ? s->cur : 1 - s->cur;
  s->swapped = false;
  if (!s->warm_step) cold_table_mask(s, est);
  s->cap_active = false;
  if (s->p.q_nom > 0 && !s->fresh && !frozen) ST_TRY(qnom_select(s, st));
  *est_out = est;
  return PACES_OK;
}

// Host side of a completed step (the device counts are in *h_ctl).
void finish_step(paces_sim* s, const FrozenStep* fz) {
  const paces_model* m = s->m;
  const StepCtl& c = *s->h_ctl;
  const int K = int(c.kmax);
  // classify the timed Clenshaw launches of this step
  const double rowb = 4.0 * double(s->A) + 4.0 * m->D + (m->V > 2 ? 16 : 8);
  // Lanczos SpMV: w_j and z once each, the columns and the payload
  const double rowk = 2.0 * double(s->A) + 4.0 * m->D + (m->V > 2 ? 16 : 8);
  for (auto& ev : s->pending) {
    if (ev.stage == PACES_STAGE_KRYLOV) ev.bytes = double(c.n_new) * rowk;
    if (ev.stage == PACES_STAGE_TERM) {
      if (ev.kk >= 1 && ev.kk <= K - 3) {
        ev.bytes = double(c.n_new) * rowb;
      } else {
        (void)hipEventDestroy(ev.a);
        (void)hipEventDestroy(ev.b);
        ev.stage = -1;
        continue;
      }
    }
    s->events.push_back(ev);
  }
  s->pending.clear();
  // the table now maps the new set (rebuilt by an expansion from scratch,
  // rewritten by one from the previous graph)
  s->tomb = s->warm_step ? s->tomb + int64_t(c.w_tomb) : 0;
  s->scattered =
      s->warm_step ? s->scattered + int64_t(std::min(c.n_staged, c.nfree)) : 0;
  s->last_warm = s->warm_step;
  s->graph_ok = true;
  s->h = c;
  s->nS = c.n_new;
  s->nlive = s->warm_step ? int64_t(c.n_live) : int64_t(c.n_new);
  s->has_holes = s->nlive < s->nS;
  s->cur = s->nside;
  std::swap(s->ipsi, s->ib0);
  s->swapped = false;
  s->k_last = step_order(s, fz);
  s->fresh = false;
  s->have_sets = true;
  s->K_last = K;
  s->launched = std::max(4, std::min(K + 2, kMaxTerms));
  s->acc.rows_steps += double(c.n_new);
  s->counts_valid = true;
  s->cap_active = false;
}

// A staged step in progress is dropped.  An in-place step whose expansion
// has run cannot be: its set is already the new one while the amplitudes
// are still phi.
paces_status abandon_staged(paces_sim* s) {
  if (s->staged_next > PACES_STAGE_EXPAND && s->warm_step)
    return fail(PACES_E_STATE,
                "a staged in-place step is half done: run its remaining "
                "stages");
  s->staged_next = 0;
  return PACES_OK;
}

// After a latched attempt of an in-place step.  Before the commit the
// table and the rows are put back as they were, and the repeated attempt
// expands from scratch unless the state cap asks for a cut selection.
// Returns true when the step has committed: then only the propagation and
// the observables can be repeated.
bool warm_after_latch(paces_sim* s, int e, hipStream_t st) {
  if (!s->warm_step) return false;
  if (s->h_ctl->w_moved) return true;
  warm_unstage(s->ctl, s->side[s->cur], s->wb, s->table, s->tmask, s->nS, st);
  if (s->swapped) {
    std::swap(s->ipsi, s->iphi);
    s->swapped = false;
  }
  if (e != kErrCap) s->graph_ok = false;
  return false;
}

// An attempt from scratch that ran out of rows under the state cap of one
// realization, before any cut: the capacity holds the cap, so the ball is
// over it, and the first cut (q from the last record) needs no ball count.
// The step is cut instead of growing the rows for a ball it will not keep.
bool overflow_over_cap(const paces_sim* s, int e, bool was_warm,
                       const FrozenStep* fz) {
  return e == kErrCapacity && !was_warm && !fz && !s->cap_active &&
         s->m->R == 1 && s->p.max_states > 0 && s->cap >= s->p.max_states;
}

// After an attempt that latched e: make the room or the selection the
// repeated attempt needs, or return the error.
paces_status handle_latch(paces_sim* s, int e, hipStream_t st) {
  if (e == kErrCap) return cap_select(s, st, false);
  if (e & (kErrTerms | kErrNonFinite)) return check_latch_code(s, e);
  if (e & kErrNeedTerms) {
    s->launched = std::min(int(s->h_ctl->kmax) + 2, kMaxTerms);
    return PACES_OK;
  }
  if (e & kErrTableFull) {
    if (s->tmask < s->tmask_alloc) {
      s->tmask = 2 * s->tmask + 1;
      return PACES_OK;
    }
    return grow(s, 2 * s->cap, s->cap + s->cap / 4, st);
  }
  if (e & kErrChunks) return more_chunks(s, st);
  if (e & kErrCapacity) return grow(s, 2 * s->cap, s->cap + s->cap / 4, st);
  return check_latch_code(s, e);
}

// One step: enqueue, read back the counts, repeat with more room when a
// capacity was exceeded.
paces_status do_step(paces_sim* s, hipStream_t st,
                     const FrozenStep* fz = nullptr) {
  int64_t est = 0;
  ST_TRY(prepare_step(s, st, fz != nullptr, &est));
  const bool graph = s->tune.graph && !s->prof && !fz && !s->cap_active;
  bool tail_only = false;  // an in-place step repeats its propagation
  StepLocals tail;
  for (int attempt = 0; attempt < 40; ++attempt) {
    const bool counted = s->counts_valid && attempt == 0 && !fz &&
                         !s->cap_active;
    if (tail_only) {
      clear_latch(s->err, st);
      stage_propagate(s, est, st, tail);
      stage_observe(s, est, st, nullptr, tail);
    } else if (graph && attempt == 0) {
      ST_TRY(launch_step_graph(s, est, counted, st));
    } else {
      enqueue_step(s, est, counted, st, fz);
    }
    // the step's last kernel mirrored the counts and the latch into h_ctl
    // and h_err
    HIP_TRY(hipStreamSynchronize(st));
    const int e = *s->h_err;
    if (e == 0) {
      finish_step(s, fz);
      return PACES_OK;
    }
    drop_pending(s);
    const bool was_warm = s->warm_step;
    if (warm_after_latch(s, e, st)) {
      // committed in place: more series launches are all it can ask for
      if (e != kErrNeedTerms) {
        s->latched = e;
        return check_latch_code(s, e);
      }
      s->launched = std::min(int(s->h_ctl->kmax) + 2, kMaxTerms);
      tail_only = true;
      tail.n_mass = s->warm_nmass;
      tail.n_e = 0;
      continue;
    }
    if (was_warm && e == kErrCapacity) {
      // in place the old rows hold their places until the commit, so the
      // new set needs more rows than from scratch (where only the new set
      // is written): repeat from scratch before growing, and stay there
      // while the capacity is this one (a state cap that cuts every step
      // would overflow it every time)
      s->warm_off_cap = s->cap;
      s->warm_step = false;
      s->nside = 1 - s->cur;
      cold_table_mask(s, est);
      continue;
    }
    if (overflow_over_cap(s, e, was_warm, fz)) {
      ST_TRY(cap_select(s, st, true));
      continue;
    }
    ST_TRY(handle_latch(s, e, st));
    if (s->warm_step && !s->graph_ok) {
      s->warm_step = false;
      cold_table_mask(s, est);
    }
    s->nside = s->warm_step ? s->cur : 1 - s->cur;
  }
  return fail(PACES_E_CAPACITY, "step did not fit after repeated growth");
}

// Counts and latch of a step in progress, read while it is incomplete.
paces_status read_latch(paces_sim* s, hipStream_t st, int* e) {
  HIP_TRY(hipMemcpyAsync(s->h_ctl, s->ctl, sizeof(StepCtl),
                         hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(s->h_err, s->err, sizeof(int), hipMemcpyDeviceToHost,
                         st));
  HIP_TRY(hipStreamSynchronize(st));
  *e = *s->h_err;
  return PACES_OK;
}

// Copy of the current state and the host mirror, for trial steps.
struct Snapshot {
  int64_t n = 0;
  uint64_t *keys = nullptr, *pay = nullptr, *tot = nullptr;
  void* psi = nullptr;
  double* mass_tot = nullptr;
  StepCtl h{};
  bool fresh = false;
  int launched = 0, K_last = 0, k_last = 0;
  ~Snapshot() {
    dfree(keys);
    dfree(pay);
    dfree(tot);
    if (psi) dev_free(psi);
    dfree(mass_tot);
  }
};

paces_status take_snapshot(paces_sim* s, Snapshot& z, hipStream_t st) {
  const paces_model* m = s->m;
  const int64_t n = std::max<int64_t>(s->nlive, 1);
  ST_TRY(dalloc(&z.keys, n * m->Wi));
  ST_TRY(dalloc(&z.pay, n));
  ST_TRY(dalloc(&z.tot, n));
  ST_TRY(dalloc(&z.mass_tot, m->R));
  ST_TRY(dev_alloc(&z.psi, size_t(n) * s->A));
  const Side& c = s->side[s->cur];
  z.n = s->nlive;
  if (s->has_holes && s->nlive > 0) {
    // the live rows only, in row order
    uint32_t* idx = nullptr;
    ST_TRY(dalloc(&idx, s->nlive));
    rows_at_distance(m->Wi, c.keys, c.dist, s->nS, -1, nullptr, idx,
                     s->dcount, s->scan_tmp, st);
    s->counts_valid = false;
    gather_rows(m->Wi, s->A, c, s->vec[s->ipsi], idx, s->nlive, z.keys,
                z.pay, z.tot, z.psi, st);
    HIP_TRY(hipStreamSynchronize(st));
    dfree(idx);
  } else if (s->nS > 0) {
    HIP_TRY(hipMemcpyAsync(z.keys, c.keys, size_t(s->nS) * m->Wi * 8,
                           hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(z.pay, c.pay, size_t(s->nS) * 8,
                           hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(z.tot, c.tot, size_t(s->nS) * 8,
                           hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(z.psi, s->vec[s->ipsi], size_t(s->nS) * s->A,
                           hipMemcpyDeviceToDevice, st));
  }
  HIP_TRY(hipMemcpyAsync(z.mass_tot, s->mass_tot, size_t(m->R) * 8,
                         hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  z.h = s->h;
  z.h.n_old = uint32_t(z.n);  // the compact rows are the set a step starts from
  z.h.n_new = uint32_t(z.n);
  z.fresh = s->fresh;
  z.launched = s->launched;
  z.K_last = s->K_last;
  z.k_last = s->k_last;
  return PACES_OK;
}

paces_status restore_snapshot(paces_sim* s, const Snapshot& z,
                              hipStream_t st) {
  const paces_model* m = s->m;
  if (z.n > s->cap) ST_TRY(grow(s, 2 * z.n, z.n, st));
  const Side& c = s->side[s->cur];
  if (z.n > 0) {
    HIP_TRY(hipMemcpyAsync(c.keys, z.keys, size_t(z.n) * m->Wi * 8,
                           hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(c.pay, z.pay, size_t(z.n) * 8,
                           hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(c.tot, z.tot, size_t(z.n) * 8,
                           hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->vec[s->ipsi], z.psi, size_t(z.n) * s->A,
                           hipMemcpyDeviceToDevice, st));
    dist_fill(c.dist, z.n, 0, st);
  }
  HIP_TRY(hipMemcpyAsync(s->mass_tot, z.mass_tot, size_t(m->R) * 8,
                         hipMemcpyDeviceToDevice, st));
  s->h = z.h;
  s->nS = z.n;
  s->nlive = z.n;
  s->has_holes = false;
  s->fresh = z.fresh;
  s->launched = z.launched;
  s->K_last = z.K_last;
  s->k_last = z.k_last;
  s->have_sets = false;
  s->counts_valid = false;
  s->graph_ok = false;
  s->latched = 0;
  return push_ctl(s, st);
}

// Resize the table for a new table_shift (keeps rows and amplitudes).
paces_status resize_table(paces_sim* s, hipStream_t st) {
  const uint64_t P = table_size_for(s->cap, s->tune.table_shift);
  if (P - 1 == s->tmask_alloc) return PACES_OK;
  HIP_TRY(hipStreamSynchronize(st));
  drop_graphs(s);
  ++s->gen;
  dfree(s->table);
  s->graph_ok = false;
  ST_TRY(dalloc(&s->table, int64_t(P)));
  s->tmask_alloc = P - 1;
  s->tmask = P - 1;
  return PACES_OK;
}

paces_status check_tuning(const paces_tuning* t) {
  if (!t || (t->graph != 0 && t->graph != 1) || (t->warm < 0 || t->warm > 2) ||
      t->table_shift < 0 ||
      t->table_shift > 3 ||
      (t->term_rows != 1 && t->term_rows != 2 && t->term_rows != 4 &&
       t->term_rows != 8))
    return fail(PACES_E_ARG, "bad tuning");
  return PACES_OK;
}


}  // namespace

// ---- adjoint gradient on a recorded run (Form (3)) -------------------------
// The forward pass runs ordinary steps and keeps, per step, the selected set
// M (so that a replay reproduces every set exactly, whatever the model
// parameters) and, every C steps, the whole state.  The backward pass
// replays one segment of C steps from its checkpoint, keeping per step the
// ELL columns, payload, phi = T_s psi_s, the row maps and the Chebyshev
// interval, then walks the segment in reverse.
struct AdjStep {
  int64_t nM = 0, n_new = 0, moff = 0;
  int k = 0, K = 0;
  double emin = 0, emax = 0;
};

struct AdjRecord {
  int C = 50;
  int64_t n = 0;
  std::vector<AdjStep> steps;
  uint64_t* mkeys = nullptr;  // M keys of every step, internal words
  int64_t mcap = 0, mused = 0;
  std::vector<Snapshot*> ck;        // state before step q*C
  std::vector<int32_t*> ck_p0;      // rows of the initial states there
  Snapshot* fin = nullptr;          // state after the last step
  std::vector<double> a;            // a_0 .. a_n, (re, im)
  ~AdjRecord() {
    dfree(mkeys);
    for (auto* c : ck) delete c;
    for (auto* p : ck_p0) dfree(p);
    delete fin;
  }
};

namespace {

paces_status adj_supported(const paces_sim* s) {
  const paces_model* m = s->m;
  if (s->p.krylov_order > 0 || s->p.taylor_order != 0)
    return fail(PACES_E_UNSUPPORTED,
                "the adjoint differentiates the series propagator");
  if (m->R != 1 || s->prec != 64)
    return fail(PACES_E_UNSUPPORTED,
                "the adjoint needs one realization and FP64 amplitudes");
  for (int a = 0; a < m->ndim; ++a)
    if (m->J[a] == 0.0)
      return fail(PACES_E_UNSUPPORTED, "the adjoint needs every J_axis != 0");
  for (int nu = 0; nu < m->V; ++nu)
    if (m->g[nu] == 0.0)
      return fail(PACES_E_UNSUPPORTED, "the adjoint needs every g_nu != 0");
  return PACES_OK;
}

bool same_shape(const paces_model* a, const paces_model* b) {
  if (a->ndim != b->ndim || a->N != b->N || a->V != b->V || a->R != b->R ||
      a->Wi != b->Wi || a->D != b->D)
    return false;
  for (int x = 0; x < 3; ++x)
    if (a->ext[x] != b->ext[x] || a->per[x] != b->per[x]) return false;
  for (int nu = 0; nu < a->V; ++nu)
    if (a->cut[nu] != b->cut[nu]) return false;
  return true;
}

// Append the nM keys of rows [0, nM) of the current side (the selected set
// of the step just made) to the record.
paces_status adj_keep_m(paces_sim* s, int64_t nM, hipStream_t st) {
  AdjRecord& R = *s->adj;
  const int Wi = s->m->Wi;
  if (R.mused + nM > R.mcap) {
    const int64_t nc = std::max<int64_t>(2 * R.mcap, R.mused + nM + 4096);
    uint64_t* q = nullptr;
    ST_TRY(dalloc(&q, nc * Wi));
    if (R.mused > 0)
      HIP_TRY(hipMemcpyAsync(q, R.mkeys, size_t(R.mused) * Wi * 8,
                             hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    dfree(R.mkeys);
    R.mkeys = q;
    R.mcap = nc;
  }
  if (nM > 0 && s->last_warm) {
    // rows of M are those at distance 0, anywhere in the set
    const Side& c = s->side[s->cur];
    uint32_t got = 0;
    rows_at_distance(Wi, c.keys, c.dist, s->nS, 0, R.mkeys + R.mused * Wi,
                     nullptr, s->dcount, s->scan_tmp, st);
    s->counts_valid = false;
    HIP_TRY(hipMemcpyAsync(&got, s->dcount, 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (int64_t(got) != nM)
      return fail(PACES_E_STATE, "selection rows do not match their count");
  } else if (nM > 0) {
    HIP_TRY(hipMemcpyAsync(R.mkeys + R.mused * Wi, s->side[s->cur].keys,
                           size_t(nM) * Wi * 8, hipMemcpyDeviceToDevice, st));
  }
  R.mused += nM;
  return PACES_OK;
}

paces_status adj_frozen_step(paces_sim* s, int64_t i, int32_t* tmap,
                             int32_t* p0map, hipStream_t st) {
  const AdjRecord& R = *s->adj;
  const AdjStep& a = R.steps[i];
  const FrozenStep fz{R.mkeys + a.moff * s->m->Wi, a.nM, a.k, tmap, p0map};
  ST_TRY(do_step(s, st, &fz));
  if (s->nS != a.n_new)
    return fail(PACES_E_STATE, "replay did not reproduce the recorded set");
  return PACES_OK;
}

// a of the records [first, first + n) into out (2 doubles per record).
paces_status adj_read_a(paces_sim* s, int64_t first, int64_t n, double* out,
                        hipStream_t st) {
  if (n <= 0) return PACES_OK;
  std::vector<double> rec(size_t(n) * s->rec_doubles);
  HIP_TRY(hipMemcpyAsync(rec.data(), s->ring + first * s->rec_doubles,
                         rec.size() * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  for (int64_t i = 0; i < n; ++i) {
    out[2 * i] = rec[size_t(i) * s->rec_doubles + 3];
    out[2 * i + 1] = rec[size_t(i) * s->rec_doubles + 4];
  }
  return PACES_OK;
}

// Gauss-Legendre nodes and weights on [0, 1] (roots of P_n by Newton's
// method from the usual cosine guesses).
void legendre(int n, double x, double& pn, double& dp) {
  double p0 = 1, p1 = x;
  for (int k = 2; k <= n; ++k) {
    const double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  pn = p1;
  dp = n * (x * p1 - p0) / (x * x - 1);
}
void gauss_legendre(int n, double* tau, double* w) {
  for (int i = 0; i < n; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (n + 0.5)), pn, dp;
    for (int it = 0; it < 100; ++it) {
      legendre(n, x, pn, dp);
      const double dx = pn / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    legendre(n, x, pn, dp);
    tau[i] = 0.5 * (1 - x);
    w[i] = 1.0 / ((1 - x * x) * dp * dp);  // 2 / (...) halved for [0, 1]
  }
}

// Nodes so that the Gauss-Legendre error bound for exp(i w tau) on [0, 1],
// w^{2n} (n!)^4 / ((2n+1) ((2n)!)^3), is below 1e-17.
int nodes_for(double wdt) {
  for (int n = 2; n <= kMaxNodes; ++n) {
    double f = 1, f2 = 1;
    for (int k = 2; k <= n; ++k) f *= k;
    for (int k = 2; k <= 2 * n; ++k) f2 *= k;
    const double b = std::pow(wdt, 2 * n) * std::pow(f, 4) /
                     ((2 * n + 1) * f2 * f2 * f2);
    if (b < 1e-17) return n;
  }
  return 0;
}

// Per-step slice of the segment store.
struct SegSlot {
  int32_t* col;
  uint64_t *pay, *tot;
  double2* phi;
  int32_t *tmap, *p0;
  ChebCoef* cc;
};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Device buffers freed together when the owner goes out of scope.
struct WorkSpace {
  std::vector<void*> p;
  ~WorkSpace() {
    for (void* q : p) dev_free(q);
  }
  template <typename T>
  paces_status get(T** out, int64_t count) {
    *out = nullptr;
    ST_TRY(dalloc(out, std::max<int64_t>(count, 1)));
    p.push_back(*out);
    return PACES_OK;
  }
};

}  // namespace

namespace {
// PACES_LOG=<file> (or 1 for paces_log.csv): append the records of every
// step as CSV lines "step,realization,<fields>,<populations>", read at the
// step's synchronisation point.
paces_status log_step(paces_sim* s, const char* where, hipStream_t st) {
  const int R = s->m->R;
  const int64_t step = int64_t(s->h.nrec) - 1;
  std::vector<double> rec(size_t(R) * s->rec_doubles);
  HIP_TRY(hipMemcpyAsync(rec.data(), s->ring + step * R * s->rec_doubles,
                         rec.size() * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const char* path = std::strcmp(where, "1") == 0 ? "paces_log.csv" : where;
  FILE* f = std::fopen(path, "a");
  if (!f) return fail(PACES_E_ARG, std::string("cannot open log ") + path);
  for (int r = 0; r < R; ++r) {
    std::fprintf(f, "%lld,%d", (long long)step, r);
    for (int q = 0; q < s->rec_doubles; ++q)
      std::fprintf(f, ",%.17g", rec[size_t(r) * s->rec_doubles + q]);
    std::fprintf(f, "\n");
  }
  std::fclose(f);
  return PACES_OK;
}

// Device copies of the model tables, made on first use so that loading a
// model and the host codec need no GPU.
paces_status ensure_device_tables(paces_model* m) {
  if (m->d_nbr) return PACES_OK;
  ST_TRY(dalloc(&m->d_nbr, int64_t(m->nbr.size())));
  ST_TRY(dalloc(&m->d_gsq, int64_t(m->gsq.size())));
  ST_TRY(dalloc(&m->d_eps, int64_t(m->R) * m->N));
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

// ---- exp(-i H_S dt) phi on a given set (paces_expmv) ------------------------
// Work memory for n rows: model tables, step control, latch, Chebyshev
// coefficients, Gershgorin partials, internal keys (when the canonical
// width needs padding), payload and totals, ELL columns, the second
// Clenshaw vector and the hash table (at least twice the rows).
struct ExpmvLayout {
  size_t nbr = 0, gsq = 0, eps = 0, ctl = 0, err = 0, cc = 0, part = 0;
  size_t keys = 0, pay = 0, tot = 0, col = 0, b1 = 0, table = 0, total = 0;
  uint64_t P = 0;
};

ExpmvLayout expmv_layout(const paces_model* m, int64_t n) {
  ExpmvLayout L;
  size_t off = 0;
  auto put = [&](size_t bytes) {
    const size_t at = off;
    off += (std::max<size_t>(bytes, 1) + 255) & ~size_t(255);
    return at;
  };
  L.nbr = put(m->nbr.size() * 4);
  L.gsq = put(m->gsq.size() * 8);
  L.eps = put(m->eps.size() * 8);
  L.ctl = put(sizeof(StepCtl));
  L.err = put(sizeof(int));
  L.cc = put(sizeof(ChebCoef));
  L.part = put(size_t(2) * kPartBlocks * 8);
  L.keys = m->Wi != m->W ? put(size_t(n) * m->Wi * 8) : 0;
  L.pay = put(size_t(n) * 8);
  L.tot = put(size_t(n) * 8);
  L.col = put(size_t(n) * m->D * 4);
  L.b1 = put(size_t(n) * 16);
  L.P = table_size_for(n, 1);
  L.table = put(size_t(L.P) * 8);
  L.total = off;
  return L;
}

// Status of a latch read back after the propagation on a given set.
paces_status expmv_latch(int e) {
  if (!e) return PACES_OK;
  if (e & kErrInput)
    return fail(PACES_E_ARG, "a key is out of range or repeated");
  if (e & kErrTerms)
    return fail(PACES_E_PROPAGATOR, "series needs more than 128 terms");
  if (e & kErrNonFinite) return fail(PACES_E_NONFINITE, "spectrum not finite");
  return fail(PACES_E_CAPACITY, "hash table overflow");
}

// The propagation of a step on a set given as n canonical keys, with the
// work memory `work` laid out by expmv_layout.  Synchronises.
paces_status expmv_run(const paces_model* m, int64_t n, const uint64_t* keys,
                       const void* phi, double dt, void* psi, uint8_t* work,
                       hipStream_t st) {
  const ExpmvLayout L = expmv_layout(m, n);
  DevModel dm = m->dm;
  dm.nbr = reinterpret_cast<const int32_t*>(work + L.nbr);
  dm.gsq = reinterpret_cast<const double*>(work + L.gsq);
  dm.eps = reinterpret_cast<const double*>(work + L.eps);
  HIP_TRY(hipMemcpyAsync(work + L.nbr, m->nbr.data(), m->nbr.size() * 4,
                         hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(work + L.gsq, m->gsq.data(), m->gsq.size() * 8,
                         hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(work + L.eps, m->eps.data(), m->eps.size() * 8,
                         hipMemcpyHostToDevice, st));
  StepCtl* ctl = reinterpret_cast<StepCtl*>(work + L.ctl);
  int* err = reinterpret_cast<int*>(work + L.err);
  ChebCoef* cc = reinterpret_cast<ChebCoef*>(work + L.cc);
  double* part = reinterpret_cast<double*>(work + L.part);
  uint64_t* table = reinterpret_cast<uint64_t*>(work + L.table);
  Side sd{};
  sd.keys = const_cast<uint64_t*>(keys);
  if (m->Wi != m->W) {
    sd.keys = reinterpret_cast<uint64_t*>(work + L.keys);
    pad_keys(m->W, m->Wi, keys, sd.keys, n, st);
  }
  sd.pay = reinterpret_cast<uint64_t*>(work + L.pay);
  sd.tot = reinterpret_cast<uint64_t*>(work + L.tot);
  int32_t* col = reinterpret_cast<int32_t*>(work + L.col);
  const uint64_t mask = L.P - 1;
  set_begin(ctl, err, n, st);
  row_info(dm, m->Wi, sd.keys, n, sd.pay, sd.tot, st);
  fill_u64(table, int64_t(L.P), kEmpty, st);
  rehash_rows(dm, m->Wi, sd, nullptr, n, table, mask, err, st);
  check_set(dm, m->Wi, sd.keys, n, table, mask, err, st);
  lookup_last(dm, m->Wi, sd, 0, ctl, n, table, mask, col, n, err, st);
  bounds_and_coef(dm, sd, col, n, n, ctl, dt, 1e-16, kMaxTerms, kMaxTerms,
                  part, cc, err, st);
  StepCtl hc{};
  int he = 0;
  HIP_TRY(hipMemcpyAsync(&hc, ctl, sizeof(StepCtl), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(&he, err, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  ST_TRY(expmv_latch(he));
  for (int kk = std::max(1, int(hc.kmax)) - 1; kk >= 0; --kk)
    cheb_term(dm, 64, kk, false, false, n, ctl, col, n, sd, cc, phi, psi,
              work + L.b1, nullptr, nullptr, err, nullptr, nullptr, st);
  HIP_TRY(hipMemcpyAsync(&he, err, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return expmv_latch(he);
}

// Work memory of paces_expmv_static: one file-scope array, which every GPU
// the library runs on holds until the process ends.  Host code never uses
// the array's name as an address: each device's copy is found once by
// hipGetSymbolAddress with that device current and kept in g_static_work.
constexpr size_t kStaticWorkBytes = size_t(64) << 20;
static __device__ __align__(256) uint8_t scratch[kStaticWorkBytes];
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_work[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`.
paces_status static_work(void** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return fail(PACES_E_UNSUPPORTED, "device index beyond the static table");
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (!g_static_work[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(PACES_E_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                   hipGetErrorString(e));
    g_static_work[dev] = p;
  }
  *out = g_static_work[dev];
  return PACES_OK;
}

// The live rows of side cur in row order (holes left out): canonical keys
// and realizations, and an amplitude vector (psi or phi) widened to FP64
// interleaved.  Synchronises.
paces_status export_rows(paces_sim* s, const void* vec, uint64_t* keys,
                         double* amps, int32_t* real, hipStream_t st) {
  const paces_model* m = s->m;
  const Side& c = s->side[s->cur];
  const int64_t n = s->nlive;
  uint32_t* idx = nullptr;
  uint64_t* gk = nullptr;
  uint8_t* ga = nullptr;
  double* tmp = nullptr;
  paces_status r = PACES_OK;
  const uint64_t* ksrc = c.keys;
  const void* asrc = vec;
  if (s->has_holes) {
    r = dalloc(&idx, n);
    if (!r) r = dalloc(&gk, n * m->Wi);
    if (!r) r = dev_alloc(reinterpret_cast<void**>(&ga), size_t(n) * s->A);
    if (!r) {
      rows_at_distance(m->Wi, c.keys, c.dist, s->nS, -1, nullptr, idx,
                       s->dcount, s->scan_tmp, st);
      s->counts_valid = false;
      gather_rows(m->Wi, s->A, c, vec, idx, n, gk, nullptr, nullptr, ga, st);
      ksrc = gk;
      asrc = ga;
    }
  }
  if (!r && (keys || real)) {
    std::vector<uint64_t> ik(size_t(n) * m->Wi), ck;
    if (hipMemcpyAsync(ik.data(), ksrc, ik.size() * 8, hipMemcpyDeviceToHost,
                       st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      r = fail(PACES_E_HIP, "copy failed");
    } else {
      if (!keys) ck.resize(size_t(n) * m->W);
      to_canonical(m, n, ik.data(), keys ? keys : ck.data(), real);
    }
  }
  if (!r && amps) {
    r = dalloc(&tmp, 2 * n);
    if (!r) {
      amps_to_f64(s->prec, asrc, tmp, n, st);
      if (hipMemcpyAsync(amps, tmp, size_t(n) * 16, hipMemcpyDeviceToHost,
                         st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        r = fail(PACES_E_HIP, "copy failed");
    }
  }
  (void)hipStreamSynchronize(st);
  dfree(tmp);
  dfree(idx);
  dfree(gk);
  if (ga) dev_free(ga);
  return r;
}

paces_status expmv_args(const paces_model* m, int64_t n, const void* keys,
                        const void* phi, double dt, const void* psi) {
  if (!m || n < 0 || (n > 0 && (!keys || !phi || !psi)) || !std::isfinite(dt))
    return fail(PACES_E_ARG, "bad arguments");
  if (n > (int64_t(1) << 31) - 256) return fail(PACES_E_ARG, "too many rows");
  if (n > 0 && phi == psi) return fail(PACES_E_ARG, "psi must not alias phi");
  if (m->R != 1)
    return fail(PACES_E_UNSUPPORTED, "a model with one realization is needed");
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

double paces_taylor_theta(int32_t m) {
  if (m < 1 || m > kTaylorMaxDeg) return -1.0;
  return taylor_thetas_host()[m];
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
  // total occupations are packed in 14 bits (two modes or fewer) or 16
  const int64_t tot_max = m->V <= 2 ? 16383 : 65535;
  for (int nu = 0; nu < m->V; ++nu)
    if (int64_t(m->N) * m->cut[nu] > tot_max)
      return bad("N * cutoff exceeds the packed total occupation");
  m->R = d->n_real == 0 ? 1 : d->n_real;
  if (m->R < 1 || m->R > kMaxReal) return bad("n_real must be 0..256");
  // per-realization populations and sums of a block live in 64 KiB of LDS
  if (int64_t(m->R) * (m->N + 3) > 8064)
    return bad("n_real * (sites + 3) must not exceed 8064");
  m->br = m->R > 1 ? bits_for(m->R) : 0;
  m->eps.assign(size_t(m->R) * m->N, 0.0);
  if (d->eps)
    for (size_t i = 0; i < m->eps.size(); ++i) m->eps[i] = d->eps[i];
  {
    bool finite = true;
    for (double v : m->eps) finite &= std::isfinite(v);
    for (int nu = 0; nu < m->V; ++nu)
      finite &= std::isfinite(m->omega[nu]) && std::isfinite(m->g[nu]);
    for (int a = 0; a < 3; ++a) finite &= std::isfinite(m->J[a]);
    if (!finite) return bad("model parameters must be finite");
  }
  m->bj = std::max(1, bits_for(m->N));
  m->B = m->N * m->P + m->bj;
  m->W = (m->B + 63) / 64;
  m->Wi = supported_words((m->B + m->br + 63) / 64);
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
  dm.R = m->R;
  dm.br = m->br;
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

paces_status paces_expmv(const paces_model* m, int64_t n, const void* dev_keys,
                         const void* dev_phi, double dt, void* dev_psi,
                         void* hip_stream) {
  ST_TRY(expmv_args(m, n, dev_keys, dev_phi, dt, dev_psi));
  if (n == 0) return PACES_OK;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  void* work = nullptr;
  ST_TRY(dev_alloc(&work, expmv_layout(m, n).total));
  const paces_status e =
      expmv_run(m, n, static_cast<const uint64_t*>(dev_keys), dev_phi, dt,
                dev_psi, static_cast<uint8_t*>(work), st);
  (void)hipStreamSynchronize(st);
  dev_free(work);
  return e;
}

paces_status paces_expmv_static(const paces_model* m, int64_t n,
                                const void* dev_keys, const void* dev_phi,
                                double dt, void* dev_psi, void* hip_stream) {
  ST_TRY(expmv_args(m, n, dev_keys, dev_phi, dt, dev_psi));
  if (n == 0) return PACES_OK;
  const size_t need = expmv_layout(m, n).total;
  if (need > kStaticWorkBytes)
    return fail(PACES_E_CAPACITY,
                std::to_string(n) + " rows need " + std::to_string(need) +
                    " bytes of work memory, above the static " +
                    std::to_string(kStaticWorkBytes) + " bytes");
  void* work = nullptr;
  ST_TRY(static_work(&work));
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  return expmv_run(m, n, static_cast<const uint64_t*>(dev_keys), dev_phi, dt,
                   dev_psi, static_cast<uint8_t*>(work), st);
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
  if (!(p->dt > 0) || p->k < 0 || p->k_init < 0 || p->k > kMaxRounds ||
      p->k_init > kMaxRounds || !(p->theta >= 0) ||
      (p->precision != 64 && p->precision != 32) || p->k_max_terms < 0 ||
      p->k_max_terms > kMaxTerms || p->tol < 0 || p->cap_states < 0 ||
      p->max_states < 0 || p->max_states >= (int64_t(1) << 31) ||
      p->q_nom < 0 || p->q_nom >= (int64_t(1) << 31) ||
      (p->q_nom > 0 && p->max_states > 0) || p->krylov_order < 0 ||
      p->krylov_order >= kMaxKrylov || p->taylor_order < -1 ||
      p->taylor_order > 60 ||
      (p->taylor_order != 0 && p->krylov_order != 0))
    return fail(PACES_E_ARG, "bad run parameters");
  const int R = m->R;
  if (n * R > (int64_t(1) << 30)) return fail(PACES_E_ARG, "too many states");
  for (int64_t i = 0; i < 2 * n; ++i)
    if (!std::isfinite(coef[i]))
      return fail(PACES_E_ARG, "coefficients must be finite");
  std::vector<uint64_t> keys(size_t(n) * m->W);
  ST_TRY(paces_pack_keys(m, n, exc, occ, keys.data()));
  ST_TRY(check_unique(m->W, n, keys.data()));
  ST_TRY(ensure_device_tables(const_cast<paces_model*>(m)));
  // every realization starts from the same state: rows r*n .. r*n+n-1
  const int64_t nt = n * R;
  std::vector<int32_t> real(nt);
  std::vector<uint64_t> rk(size_t(nt) * m->W), ik(size_t(nt) * m->Wi);
  std::vector<double> ra(size_t(nt) * 2);
  for (int r = 0; r < R; ++r)
    for (int64_t i = 0; i < n; ++i) {
      real[r * n + i] = r;
      std::memcpy(&rk[size_t(r * n + i) * m->W], &keys[size_t(i) * m->W],
                  size_t(m->W) * 8);
      ra[2 * (r * n + i)] = coef[2 * i];
      ra[2 * (r * n + i) + 1] = coef[2 * i + 1];
    }
  to_internal(m, nt, rk.data(), real.data(), ik.data());
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
  // coherent mapped host memory: the step's last kernel writes the counts
  // there directly
  const unsigned hflags = hipHostMallocMapped | hipHostMallocCoherent;
  if (hipHostMalloc(reinterpret_cast<void**>(&s->h_ctl), sizeof(StepCtl),
                    hflags) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&s->h_err), 64, hflags) !=
          hipSuccess)
    return cleanup(fail(PACES_E_OOM, "pinned host allocation failed"));
  if (hipHostGetDevicePointer(reinterpret_cast<void**>(&s->d_hctl), s->h_ctl,
                              0) != hipSuccess ||
      hipHostGetDevicePointer(reinterpret_cast<void**>(&s->d_herr), s->h_err,
                              0) != hipSuccess)
    return cleanup(fail(PACES_E_HIP, "no device address for pinned memory"));
  // per-block partials of the row kernels (layouts in kernels.hpp)
  const int64_t blk = R == 1 ? kMaxPartials : int64_t(kPartBlocks) * R;
  const int64_t sz_mass = blk, sz_e = R == 1 ? kMaxPartials : 0,
                sz_bnd = 2 * blk, sz_pop = int64_t(kPartBlocks) * R;
  const int64_t nparts = sz_mass + sz_e + sz_bnd + 2 * sz_pop +
                         sz_pop * m->N + 2 * 256;
  if (dalloc(&s->ctl, 1) || dalloc(&s->err, 1) || dalloc(&s->parts, nparts) ||
      dalloc(&s->cc, R) || dalloc(&s->a2, 2 * R) || dalloc(&s->cnt, 2 * R) ||
      dalloc(&s->mass_tot, R) || dalloc(&s->p0_last, nt) ||
      dalloc(&s->ball, R) || dalloc(&s->dcount, 1) ||
      dalloc(&s->keys0, nt * m->Wi) ||
      dalloc(&s->amps0, 2 * nt))
    return cleanup(PACES_E_OOM);
  if (p->taylor_order != 0) {
    if (dalloc(&s->tplan, R) || dalloc(&s->thetas, kTaylorMaxDeg + 1))
      return cleanup(PACES_E_OOM);
    if (hipMemcpy(s->thetas, taylor_thetas_host(),
                  sizeof(double) * (kTaylorMaxDeg + 1),
                  hipMemcpyHostToDevice) != hipSuccess)
      return cleanup(fail(PACES_E_HIP, "upload failed"));
  }
  if (p->krylov_order > 0 &&
      (dalloc(&s->lz, R) || dalloc(&s->lz_energy, R) ||
       dalloc(&s->lz_part, 3 * std::max<int64_t>(kLzGrid1,
                                                 int64_t(kPartBlocks) * R))))
    return cleanup(PACES_E_OOM);
  double* q = s->parts;
  s->mass_part = q;  q += sz_mass;
  s->e_part = q;     q += sz_e;
  s->bnd_part = q;   q += sz_bnd;
  s->n2_part = q;    q += sz_pop;
  s->en_part = q;    q += sz_pop;
  s->pop_part = q;   q += sz_pop * m->N;
  s->mass_fold = q;  q += 256;
  s->e_fold = q;
  if (hipMemsetAsync(s->err, 0, 4, st) != hipSuccess ||
      hipMemsetAsync(s->parts, 0, size_t(nparts) * 8, st) != hipSuccess ||
      hipMemsetAsync(s->mass_tot, 0, size_t(R) * 8, st) != hipSuccess ||
      hipMemsetAsync(s->cnt, 0, size_t(2 * R) * 4, st) != hipSuccess)
    return cleanup(fail(PACES_E_HIP, "memset failed"));
  const int64_t cap0 = std::max<int64_t>({p->cap_states, 4 * nt, 1 << 16});
  paces_status g =
      grow(s, cap0, std::max<int64_t>(4 * nt, int64_t(1) << 16), st);
  if (g) return cleanup(g);
  g = ensure_ring(s, st);
  if (g) return cleanup(g);
  if (hipMemcpyAsync(s->keys0, ik.data(), ik.size() * 8, hipMemcpyHostToDevice,
                     st) != hipSuccess ||
      hipMemcpyAsync(s->amps0, ra.data(), ra.size() * 8, hipMemcpyHostToDevice,
                     st) != hipSuccess)
    return cleanup(fail(PACES_E_HIP, "upload failed"));
  s->n0 = n;
  std::memset(&s->h, 0, sizeof(s->h));
  g = upload_state(s, nt, ik, ra.data(), st);
  if (g) return cleanup(g);
  s->fresh = true;
  *out = s;
  return PACES_OK;
}

paces_status paces_free_sim(paces_sim* s) {
  if (!s) return PACES_OK;
  (void)hipDeviceSynchronize();
  free_rows(s);
  free_cand(s);
  dfree(s->ctl);
  dfree(s->err);
  dfree(s->parts);
  dfree(s->cc);
  dfree(s->a2);
  dfree(s->cnt);
  dfree(s->mass_tot);
  dfree(s->p0_last);
  dfree(s->ball);
  dfree(s->dcount);
  if (s->cap_block) dev_free(s->cap_block);
  dfree(s->cap_hist);
  dfree(s->cap_mode);
  dfree(s->cap_dstar);
  dfree(s->cap_capped);
  dfree(s->keys0);
  dfree(s->amps0);
  dfree(s->ring);
  dfree(s->lz);
  dfree(s->lz_part);
  dfree(s->lz_energy);
  dfree(s->tplan);
  dfree(s->thetas);
  drop_pending(s);
  for (auto& e : s->events) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  if (s->h_ctl) (void)hipHostFree(s->h_ctl);
  if (s->h_err) (void)hipHostFree(s->h_err);
  drop_graphs(s);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  delete s->adj;
  delete s;
  return PACES_OK;
}

paces_status paces_step(paces_sim* s, int64_t n_steps, void* hip_stream) {
  if (!s || n_steps < 0) return fail(PACES_E_ARG, "bad arguments");
  if (s->latched) return fail(PACES_E_STATE, "sim is in an error state");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const char* log = std::getenv("PACES_LOG");
  ST_TRY(abandon_staged(s));
  for (int64_t i = 0; i < n_steps; ++i) {
    paces_status r = do_step(s, st);
    if (r != PACES_OK) {
      if (!s->latched) s->latched = -1;
      return r;
    }
    if (log && *log && std::strcmp(log, "0") != 0) ST_TRY(log_step(s, log, st));
  }
  return PACES_OK;
}

paces_status paces_run_stage(paces_sim* s, int32_t stage, void* hip_stream) {
  if (!s) return fail(PACES_E_ARG, "bad arguments");
  if (stage < PACES_STAGE_SELECT || stage > PACES_STAGE_OBSERVE)
    return fail(PACES_E_ARG, "stage must be select .. observe");
  if (s->latched) return fail(PACES_E_STATE, "sim is in an error state");
  static const char* names[] = {"select", "expand", "transfer", "build",
                                "propagate", "observe"};
  if (stage != PACES_STAGE_SELECT && stage != s->staged_next)
    return fail(PACES_E_STATE, std::string("stages run in order; expected ") +
                                   names[s->staged_next]);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  StepLocals L;
  L.n_mass = s->staged_mass;
  L.n_e = s->staged_e;
  switch (stage) {
    case PACES_STAGE_SELECT: {
      ST_TRY(abandon_staged(s));
      ST_TRY(prepare_step(s, st, false, &s->staged_est));
      stage_select(s, false, st, nullptr);
      break;
    }
    case PACES_STAGE_EXPAND: {
      // the sizes of the new set are known only now: repeat select +
      // expand with more room (or a cut selection) until they fit
      int e = 0;
      for (int attempt = 0;; ++attempt) {
        if (attempt > 0) stage_select(s, false, st, nullptr);
        stage_expand(s, s->staged_est, st, nullptr);
        ST_TRY(read_latch(s, st, &e));
        if (!e) break;
        drop_pending(s);
        const int retry = kErrTableFull | kErrCapacity | kErrChunks | kErrCap;
        if (attempt >= 40 || (e & ~retry)) {
          s->staged_next = 0;
          return check_latch_code(s, e);
        }
        const bool was_warm = s->warm_step;
        if (warm_after_latch(s, e, st)) {
          s->staged_next = 0;
          s->latched = e;
          return check_latch_code(s, e);
        }
        if (was_warm && e == kErrCapacity) {
          // as in paces_step: from scratch before growing
          s->warm_off_cap = s->cap;
          s->warm_step = false;
          s->nside = 1 - s->cur;
          cold_table_mask(s, s->staged_est);
          continue;
        }
        paces_status h = overflow_over_cap(s, e, was_warm, nullptr)
                             ? cap_select(s, st, true)
                             : handle_latch(s, e, st);
        if (h) {
          s->staged_next = 0;
          return h;
        }
        if (s->warm_step && !s->graph_ok) {
          s->warm_step = false;
          cold_table_mask(s, s->staged_est);
        }
        s->nside = s->warm_step ? s->cur : 1 - s->cur;
      }
      break;
    }
    case PACES_STAGE_TRANSFER:
      stage_transfer(s, st, nullptr, L);
      break;
    case PACES_STAGE_BUILD:
      // the number of series launches is set from the coefficients below
      s->launched = kMaxTerms;
      stage_build(s, s->staged_est, st);
      break;
    case PACES_STAGE_PROPAGATE: {
      int e = 0;
      ST_TRY(read_latch(s, st, &e));
      if (e) {
        s->staged_next = 0;
        drop_pending(s);
        return check_latch_code(s, e);
      }
      s->launched = std::max(1, int(s->h_ctl->kmax));
      stage_propagate(s, s->staged_est, st, L);
      break;
    }
    case PACES_STAGE_OBSERVE: {
      stage_observe(s, s->staged_est, st, nullptr, L);
      HIP_TRY(hipStreamSynchronize(st));
      s->staged_next = 0;
      const int e = *s->h_err;
      if (e) {
        drop_pending(s);
        return check_latch_code(s, e);
      }
      finish_step(s, nullptr);
      const char* log = std::getenv("PACES_LOG");
      if (log && *log && std::strcmp(log, "0") != 0)
        ST_TRY(log_step(s, log, st));
      return PACES_OK;
    }
  }
  s->staged_mass = L.n_mass;
  s->staged_e = L.n_e;
  s->staged_next = stage + 1;
  return PACES_OK;
}

paces_status paces_observe(paces_sim* s, int32_t realization, paces_obs* out,
                           void* hip_stream) {
  if (!s || !out || realization < 0 || realization >= s->m->R)
    return fail(PACES_E_ARG, "bad arguments");
  if (s->latched) return fail(PACES_E_STATE, "sim is in an error state");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  std::memset(out, 0, sizeof(*out));
  if (s->h.nrec == 0) {
    out->t = s->h.t;
    out->n_S = s->nlive;
    std::fill(s->pop_host.begin(), s->pop_host.end(), 0.0);
    out->pop = s->pop_host.data();
    return PACES_OK;
  }
  std::vector<double> rec(s->rec_doubles);
  const int64_t at = (int64_t(s->h.nrec) - 1) * s->m->R + realization;
  HIP_TRY(hipMemcpyAsync(rec.data(), s->ring + at * s->rec_doubles,
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
  *n = s->h.nrec;
  return PACES_OK;
}

paces_status paces_series(paces_sim* s, int64_t first, int64_t n, double* out,
                          void* hip_stream) {
  if (!s || first < 0 || n < 0 || first + n > int64_t(s->h.nrec) ||
      (n && !out))
    return fail(PACES_E_ARG, "bad arguments");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (n == 0) return PACES_OK;
  const int64_t per = int64_t(s->m->R) * s->rec_doubles;
  HIP_TRY(hipMemcpyAsync(out, s->ring + first * per, size_t(n * per) * 8,
                         hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return PACES_OK;
}

paces_status paces_get_state(paces_sim* s, int64_t* n, uint64_t* keys,
                             double* amps, int32_t* real, void* hip_stream) {
  if (!s || !n) return fail(PACES_E_ARG, "bad arguments");
  if (s->latched) return fail(PACES_E_STATE, "sim is in an error state");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  *n = s->nlive;
  if ((!keys && !real && !amps) || s->nlive == 0) return PACES_OK;
  return export_rows(s, s->vec[s->ipsi], keys, amps, real, st);
}

paces_status paces_set_state(paces_sim* s, int64_t n, const uint64_t* keys,
                             const double* amps, const int32_t* real, double t,
                             void* hip_stream) {
  if (!s || n < 0 || (n > 0 && (!keys || !amps)))
    return fail(PACES_E_ARG, "bad arguments");
  if (n > (int64_t(1) << 30)) return fail(PACES_E_ARG, "too many states");
  const paces_model* m = s->m;
  if (real)
    for (int64_t i = 0; i < n; ++i)
      if (real[i] < 0 || real[i] >= m->R)
        return fail(PACES_E_ARG, "realization index out of range");
  for (int64_t i = 0; i < 2 * n; ++i)
    if (!std::isfinite(amps[i]))
      return fail(PACES_E_ARG, "amplitudes must be finite");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  ST_TRY(check_keys(m, n, keys));
  std::vector<uint64_t> ik(size_t(n) * m->Wi);
  to_internal(m, n, keys, real, ik.data());
  ST_TRY(check_unique(m->Wi, n, ik.data()));
  HIP_TRY(hipStreamSynchronize(st));
  s->latched = 0;
  s->h.t = t;
  ST_TRY(upload_state(s, n, ik, amps, st));
  s->fresh = false;
  s->have_sets = false;
  s->staged_next = 0;
  s->counts_valid = false;
  return PACES_OK;
}

paces_status paces_get_set(paces_sim* s, int32_t which, int32_t round,
                           int64_t* n, uint64_t* keys, int32_t* real,
                           void* hip_stream) {
  if (!s || !n) return fail(PACES_E_ARG, "bad arguments");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  int64_t a = 0, b = 0;
  if (which == PACES_SET_S) {
    b = s->nS;
  } else if (!s->have_sets) {
    return fail(PACES_E_STATE, "no step has run since the state was set");
  } else if (which == PACES_SET_M) {
    b = s->h.nM;
  } else if (which == PACES_SET_FRONTIER) {
    if (round < 0 || round > s->k_last) return fail(PACES_E_ARG, "no such round");
    a = s->h.fstart[round];
    b = s->h.fstart[round + 1];
  } else {
    return fail(PACES_E_ARG, "unknown set");
  }
  const paces_model* m = s->m;
  const Side& c = s->side[s->cur];
  uint64_t* gathered = nullptr;
  const bool spread =
      which == PACES_SET_S ? s->has_holes : (s->last_warm || s->has_holes);
  if (spread && s->nS > 0) {
    // a step from the previous graph leaves M and the frontiers spread over
    // the row range, and holes in it: gather the rows at that distance (every
    // live row for S)
    const int d = which == PACES_SET_S ? -1 : which == PACES_SET_M ? 0 : round;
    uint32_t got = 0;
    ST_TRY(dalloc(&gathered, s->nS * m->Wi));
    rows_at_distance(m->Wi, c.keys, c.dist, s->nS, d, gathered, nullptr,
                     s->dcount, s->scan_tmp, st);
    s->counts_valid = false;
    if (hipMemcpyAsync(&got, s->dcount, 4, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      dfree(gathered);
      return fail(PACES_E_HIP, "copy failed");
    }
    a = 0;
    b = got;
  }
  *n = b - a;
  if ((!keys && !real) || b == a) {
    dfree(gathered);
    return PACES_OK;
  }
  std::vector<uint64_t> ik(size_t(b - a) * m->Wi), ck;
  const uint64_t* src = gathered ? gathered : c.keys + a * m->Wi;
  const hipError_t ce = hipMemcpyAsync(ik.data(), src, ik.size() * 8,
                                       hipMemcpyDeviceToHost, st);
  const hipError_t se = hipStreamSynchronize(st);
  dfree(gathered);
  if (ce != hipSuccess || se != hipSuccess) return fail(PACES_E_HIP, "copy failed");
  if (!keys) ck.resize(size_t(b - a) * m->W);
  to_canonical(m, b - a, ik.data(), keys ? keys : ck.data(), real);
  return PACES_OK;
}

paces_status paces_get_phi(paces_sim* s, double* amps, void* hip_stream) {
  if (!s || !amps) return fail(PACES_E_ARG, "bad arguments");
  if (!s->have_sets)
    return fail(PACES_E_STATE, "no step has run since the state was set");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (s->nlive == 0) return PACES_OK;
  return export_rows(s, s->vec[s->iphi], nullptr, amps, nullptr, st);
}

paces_status paces_profile_enable(paces_sim* s, int32_t on) {
  if (!s) return fail(PACES_E_ARG, "bad arguments");
  if (on < 0 || on > 2) return fail(PACES_E_ARG, "profiling level 0, 1 or 2");
  s->prof = on;
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
    if (e.stage == PACES_STAGE_KRYLOV) s->acc.krylov_bytes += e.bytes;
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  s->events.clear();
  *out = s->acc;
  return PACES_OK;
}

paces_status paces_profile_mark(int32_t tag, void* hip_stream) {
  paces::mark(tag, static_cast<hipStream_t>(hip_stream));
  HIP_TRY(hipGetLastError());
  return PACES_OK;
}

paces_status paces_profile_reset(paces_sim* s) {
  if (!s) return fail(PACES_E_ARG, "bad arguments");
  paces_profile z{};
  s->acc = z;
  return PACES_OK;
}

paces_status paces_set_allocator(void* (*alloc)(size_t, void*, void*),
                                 void (*release)(void*, void*, void*),
                                 void* user) {
  if ((alloc == nullptr) != (release == nullptr))
    return fail(PACES_E_ARG, "allocator needs both functions or neither");
  g_allocator.alloc = alloc;
  g_allocator.release = release;
  g_allocator.user = user;
  return PACES_OK;
}

paces_status paces_set_model(paces_sim* s, const paces_model* m) {
  if (!s || !m) return fail(PACES_E_ARG, "bad arguments");
  if (!same_shape(s->m, m))
    return fail(PACES_E_ARG, "model shape differs from the sim's");
  ST_TRY(ensure_device_tables(const_cast<paces_model*>(m)));
  if (m != s->m) {
    drop_graphs(s);  // kernels take the model's values by value
    delete s->adj;   // a recorded adjoint run assumes one model
    s->adj = nullptr;
    // a coupling that becomes zero or nonzero changes which slots exist:
    // the next step expands from scratch
    s->graph_ok = false;
  }
  s->m = m;
  return PACES_OK;
}

paces_status paces_model_key_words(const paces_model* m, int32_t* W) {
  if (!m || !W) return fail(PACES_E_ARG, "bad arguments");
  *W = m->W;
  return PACES_OK;
}

paces_status paces_series_field(paces_sim* s, int32_t field, void* dev_out,
                                int64_t first, int64_t n, void* hip_stream) {
  if (!s || !dev_out || field < 0 || field >= s->rec_doubles || first < 0 ||
      n < 0 || first + n > int64_t(s->h.nrec))
    return fail(PACES_E_ARG, "bad arguments");
  if (n == 0) return PACES_OK;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int64_t R = s->m->R, pitch = int64_t(s->rec_doubles) * 8;
  HIP_TRY(hipMemcpy2DAsync(dev_out, 8, s->ring + first * R * s->rec_doubles + field,
                           size_t(pitch), 8, size_t(n * R),
                           hipMemcpyDeviceToDevice, st));
  return PACES_OK;
}

int32_t paces_num_params(const paces_model* m) {
  return m ? m->ndim + 2 * m->V + m->N : 0;
}

paces_status paces_adjoint_forward(paces_sim* s, int64_t n_steps,
                                   int32_t ckpt_every, double* a_out,
                                   void* hip_stream) {
  if (!s || n_steps < 1 || ckpt_every < 1 || n_steps > (int64_t(1) << 24))
    return fail(PACES_E_ARG, "bad arguments");
  if (s->latched) return fail(PACES_E_STATE, "sim is in an error state");
  if (!s->fresh || s->h.nrec != 0)
    return fail(PACES_E_STATE, "the adjoint forward starts from a new sim");
  ST_TRY(adj_supported(s));
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  delete s->adj;
  s->adj = new AdjRecord();
  AdjRecord& R = *s->adj;
  R.C = ckpt_every;
  R.n = n_steps;
  R.steps.assign(n_steps, AdjStep());
  R.a.assign(2 * (n_steps + 1), 0.0);
  auto bail = [&](paces_status e) {
    delete s->adj;
    s->adj = nullptr;
    return e;
  };
  // a_0 = <psi0|psi0>
  {
    std::vector<double> a0(2 * s->n0);
    HIP_TRY(hipMemcpy(a0.data(), s->amps0, a0.size() * 8,
                      hipMemcpyDeviceToHost));
    double acc = 0;
    for (int64_t i = 0; i < s->n0; ++i)
      acc += a0[2 * i] * a0[2 * i] + a0[2 * i + 1] * a0[2 * i + 1];
    R.a[0] = acc;
  }
  for (int64_t i = 0; i < n_steps; ++i) {
    if (i % R.C == 0) {
      Snapshot* z = new Snapshot();
      R.ck.push_back(z);
      paces_status e = take_snapshot(s, *z, st);
      int32_t* p0 = nullptr;
      if (!e) e = dalloc(&p0, s->n0);
      R.ck_p0.push_back(p0);
      if (e) return bail(e);
      if (i == 0) {
        // the initial state sits in input order
        std::vector<int32_t> id(s->n0);
        std::iota(id.begin(), id.end(), 0);
        if (hipMemcpy(p0, id.data(), id.size() * 4, hipMemcpyHostToDevice) !=
            hipSuccess)
          return bail(fail(PACES_E_HIP, "upload failed"));
      } else if (hipMemcpyAsync(p0, s->p0_last, size_t(s->n0) * 4,
                                hipMemcpyDeviceToDevice, st) != hipSuccess) {
        return bail(fail(PACES_E_HIP, "copy failed"));
      }
    }
    paces_status e = do_step(s, st);
    if (e) return bail(e);
    AdjStep& a = R.steps[i];
    a.nM = s->h.nM;
    a.k = s->k_last;
    a.n_new = s->nlive;
    a.K = s->K_last;
    a.moff = R.mused;
    e = adj_keep_m(s, a.nM, st);
    if (e) return bail(e);
  }
  R.fin = new Snapshot();
  paces_status e = take_snapshot(s, *R.fin, st);
  if (e) return bail(e);
  // a_1..a_n and the spectral intervals from the records
  std::vector<double> rec(size_t(n_steps) * s->rec_doubles);
  if (hipMemcpyAsync(rec.data(), s->ring, rec.size() * 8,
                     hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return bail(fail(PACES_E_HIP, "record read failed"));
  for (int64_t i = 0; i < n_steps; ++i) {
    const double* r = rec.data() + size_t(i) * s->rec_doubles;
    R.a[2 * (i + 1)] = r[3];
    R.a[2 * (i + 1) + 1] = r[4];
    R.steps[i].emin = r[10];
    R.steps[i].emax = r[11];
  }
  if (a_out) std::copy(R.a.begin(), R.a.end(), a_out);
  return PACES_OK;
}

paces_status paces_adjoint_forward_dev(paces_sim* s, int64_t n_steps,
                                       int32_t ckpt_every, void* dev_a,
                                       void* hip_stream) {
  if (!dev_a) return fail(PACES_E_ARG, "bad arguments");
  ST_TRY(paces_adjoint_forward(s, n_steps, ckpt_every, nullptr, hip_stream));
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  // a_0 from the host record, a_1..a_n straight from the device records
  double* out = static_cast<double*>(dev_a);
  HIP_TRY(hipMemcpyAsync(out, s->adj->a.data(), 16, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpy2DAsync(out + 2, 16, s->ring + 3,
                           size_t(s->rec_doubles) * 8, 16, size_t(n_steps),
                           hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  return PACES_OK;
}

paces_status paces_adjoint_replay(paces_sim* s, const paces_model* model,
                                  double* a_out, void* hip_stream) {
  if (!s || !a_out) return fail(PACES_E_ARG, "bad arguments");
  if (!s->adj) return fail(PACES_E_STATE, "no adjoint record");
  const paces_model* own = s->m;
  if (!model) model = own;
  if (!same_shape(own, model))
    return fail(PACES_E_ARG, "model shape differs from the recorded run");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  ST_TRY(ensure_device_tables(const_cast<paces_model*>(model)));
  AdjRecord& R = *s->adj;
  paces_status e = restore_snapshot(s, *R.ck[0], st);
  s->m = model;
  const int64_t first = s->h.nrec;
  for (int64_t i = 0; i < R.n && !e; ++i)
    e = adj_frozen_step(s, i, nullptr, nullptr, st);
  if (!e) e = adj_read_a(s, first, R.n, a_out + 2, st);
  s->m = own;
  a_out[0] = R.a[0];
  a_out[1] = R.a[1];
  paces_status e2 = restore_snapshot(s, *R.fin, st);
  return e ? e : e2;
}

// Backward sweep of the adjoint gradient; gbar[2 (n + 1)] and grad[P] are
// device arrays (grad is overwritten).
paces_status adjoint_backward(paces_sim* s, const double* gbar, double* grad,
                              hipStream_t st) {
  AdjRecord& R = *s->adj;
  const paces_model* m = s->m;
  const DevModel& dm = m->dm;
  const int P = paces_num_params(m), D = m->D, V = m->V;
  const int64_t n0 = s->n0, nseg = (R.n + R.C - 1) / R.C;
  // sizes and node counts
  int64_t maxn = R.ck[0]->n;
  int nqmax = 1;
  std::vector<int> nq(R.n);
  for (int64_t i = 0; i < R.n; ++i) {
    maxn = std::max(maxn, R.steps[i].n_new);
    nq[i] = nodes_for((R.steps[i].emax - R.steps[i].emin) * s->p.dt);
    if (!nq[i])
      return fail(PACES_E_UNSUPPORTED,
                  "spectral width times dt too large for the quadrature");
    nqmax = std::max(nqmax, nq[i]);
  }
  WorkSpace buf;  // freed on return
  double2 *lamA, *lamB, *b0, *b1, *tx1, *ty1, *accx, *accy, *cn;
  double *part, *tau, *w;
  ChebCoef* ccj;
  ST_TRY(buf.get(&lamA, maxn));
  ST_TRY(buf.get(&lamB, maxn));
  ST_TRY(buf.get(&b0, maxn));
  ST_TRY(buf.get(&b1, maxn));
  ST_TRY(buf.get(&tx1, maxn));
  ST_TRY(buf.get(&ty1, maxn));
  ST_TRY(buf.get(&accx, int64_t(nqmax) * maxn));
  ST_TRY(buf.get(&accy, int64_t(nqmax) * maxn));
  ST_TRY(buf.get(&cn, int64_t(kMaxNodes) * kMaxTerms));
  ST_TRY(buf.get(&part, int64_t(1024) * P));
  ST_TRY(buf.get(&tau, int64_t(kMaxNodes + 1) * kMaxNodes));
  ST_TRY(buf.get(&w, int64_t(kMaxNodes + 1) * kMaxNodes));
  ST_TRY(buf.get(&ccj, 1));
  {
    std::vector<double> ht((kMaxNodes + 1) * kMaxNodes, 0.0), hw(ht.size(), 0.0);
    for (int q = 1; q <= kMaxNodes; ++q)
      gauss_legendre(q, &ht[q * kMaxNodes], &hw[q * kMaxNodes]);
    HIP_TRY(hipMemcpy(tau, ht.data(), ht.size() * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(w, hw.data(), hw.size() * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemsetAsync(grad, 0, size_t(P) * 8, st));
  }
  uint8_t* store = nullptr;
  size_t store_cap = 0;
  auto release_store = [&]() {
    if (store) dev_free(store);
    store = nullptr;
  };
  paces_status e = PACES_OK;
  const bool totw = V > 2;
  for (int64_t q = nseg - 1; q >= 0 && !e; --q) {
    const int64_t start = q * R.C, end = std::min(R.n, start + R.C);
    // lay out the segment store
    std::vector<SegSlot> slot(end - start);
    std::vector<size_t> off(end - start);
    size_t tot_bytes = 0;
    for (int64_t i = start; i < end; ++i) {
      const int64_t n1 = R.steps[i].n_new;
      const int64_t ns = i ? R.steps[i - 1].n_new : R.ck[0]->n;
      off[i - start] = tot_bytes;
      tot_bytes += align256(size_t(D) * n1 * 4) + align256(size_t(n1) * 8) +
                   (totw ? align256(size_t(n1) * 8) : 0) +
                   align256(size_t(n1) * 16) + align256(size_t(ns) * 4) +
                   align256(size_t(n0) * 4) + align256(sizeof(ChebCoef));
    }
    if (tot_bytes > store_cap) {
      release_store();
      void* q = nullptr;
      e = dev_alloc(&q, tot_bytes);
      if (e) break;
      store = static_cast<uint8_t*>(q);
      store_cap = tot_bytes;
    }
    for (int64_t i = start; i < end; ++i) {
      const int64_t n1 = R.steps[i].n_new;
      const int64_t ns = i ? R.steps[i - 1].n_new : R.ck[0]->n;
      uint8_t* b = store + off[i - start];
      SegSlot& z = slot[i - start];
      z.col = reinterpret_cast<int32_t*>(b);
      b += align256(size_t(D) * n1 * 4);
      z.pay = reinterpret_cast<uint64_t*>(b);
      b += align256(size_t(n1) * 8);
      z.tot = nullptr;
      if (totw) {
        z.tot = reinterpret_cast<uint64_t*>(b);
        b += align256(size_t(n1) * 8);
      }
      z.phi = reinterpret_cast<double2*>(b);
      b += align256(size_t(n1) * 16);
      z.tmap = reinterpret_cast<int32_t*>(b);
      b += align256(size_t(ns) * 4);
      z.p0 = reinterpret_cast<int32_t*>(b);
      b += align256(size_t(n0) * 4);
      z.cc = reinterpret_cast<ChebCoef*>(b);
    }
    // replay the segment from its checkpoint, keeping what the reverse
    // sweep needs
    e = restore_snapshot(s, *R.ck[q], st);
    for (int64_t i = start; i < end && !e; ++i) {
      SegSlot& z = slot[i - start];
      e = adj_frozen_step(s, i, z.tmap, z.p0, st);
      if (e) break;
      const int64_t n1 = s->nS;
      if (hipMemcpyAsync(z.col, s->side[s->cur].col, size_t(n1) * D * 4,
                         hipMemcpyDeviceToDevice, st) != hipSuccess)
        e = fail(PACES_E_HIP, "copy failed");
      const Side& c = s->side[s->cur];
      if (!e && (hipMemcpyAsync(z.pay, c.pay, size_t(n1) * 8,
                                hipMemcpyDeviceToDevice, st) != hipSuccess ||
                 (totw && hipMemcpyAsync(z.tot, c.tot, size_t(n1) * 8,
                                         hipMemcpyDeviceToDevice, st) != hipSuccess) ||
                 hipMemcpyAsync(z.phi, s->vec[s->iphi], size_t(n1) * 16,
                                hipMemcpyDeviceToDevice, st) != hipSuccess ||
                 hipMemcpyAsync(z.cc, s->cc, sizeof(ChebCoef),
                                hipMemcpyDeviceToDevice, st) != hipSuccess))
        e = fail(PACES_E_HIP, "copy failed");
    }
    if (e) break;
    // lambda at the end of the segment, in the replay's row order
    const int64_t nend = R.steps[end - 1].n_new;
    if (q == nseg - 1) {
      adj_zero(lamA, nend, st);
      adj_add_psi0(n0, slot[end - 1 - start].p0, s->amps0, gbar + 2 * R.n,
                   lamA, s->err, st);
    } else {
      // lamA holds lambda_end in the order of checkpoint q+1
      adj_permute(dm, m->Wi, R.ck[q + 1]->keys, nend, s->table, s->tmask,
                  s->side[s->cur].keys, lamA, lamB, s->err, st);
      std::swap(lamA, lamB);
    }
    // reverse sweep
    for (int64_t i = end - 1; i >= start; --i) {
      const SegSlot& z = slot[i - start];
      const AdjStep& a = R.steps[i];
      const int64_t n1 = a.n_new;
      const int64_t ns = i ? R.steps[i - 1].n_new : R.ck[0]->n;
      const Side sd{nullptr, z.pay, z.tot};
      // mu = exp(+i H dt) lambda_{i+1}
      adj_set_rows(s->ctl, uint32_t(n1), st);
      adj_conj_coef(z.cc, ccj, st);
      for (int kk = a.K - 1; kk >= 0; --kk)
        cheb_term(dm, 64, kk, false, false, n1, s->ctl, z.col, n1, sd, ccj,
                  lamA, b0, b1, nullptr, nullptr, s->err, nullptr, nullptr,
                  st);
      // lambda_i = T_i^T mu + gbar_i psi0
      adj_back(ns, z.tmap, b0, lamB, s->err, st);
      const int32_t* p0 = i == start ? R.ck_p0[q] : slot[i - 1 - start].p0;
      adj_add_psi0(n0, p0, s->amps0, gbar + 2 * i, lamB, s->err, st);
      // mu and phi at the quadrature nodes, contracted with dH/dtheta
      const int nqi = nq[i];
      adj_node_coef(z.cc, s->p.dt, tau + nqi * kMaxNodes, nqi, s->p.tol, cn,
                    s->err, st);
      for (int kk = 0; kk < a.K; ++kk)
        adj_nodes(dm, kk, a.K, n1, z.col, z.pay, z.tot, z.cc, cn, nqi, b0,
                  tx1, z.phi, ty1, accx, accy, s->err, st);
      const int nb = adj_contract(dm, n1, z.col, z.pay, z.tot, nqi,
                                  w + nqi * kMaxNodes, accx, accy, part,
                                  s->err, st);
      adj_fold(part, nb, P, 2.0 * s->p.dt, grad, s->err, st);
      std::swap(lamA, lamB);
    }
    // lamA: lambda_start in the order of checkpoint q
    HIP_TRY(hipMemcpyAsync(s->h_err, s->err, sizeof(int),
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (*s->h_err) e = fail(PACES_E_STATE, "device error in the adjoint sweep");
  }
  if (!e) HIP_TRY(hipStreamSynchronize(st));
  release_store();
  paces_status e2 = restore_snapshot(s, *R.fin, st);
  return e ? e : e2;
}

paces_status paces_adjoint_backward(paces_sim* s, const double* gbar,
                                    double* grad_out, void* hip_stream) {
  if (!s || !gbar || !grad_out) return fail(PACES_E_ARG, "bad arguments");
  if (!s->adj) return fail(PACES_E_STATE, "no adjoint record");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int P = paces_num_params(s->m);
  WorkSpace buf;  // freed on return
  double *g_dev, *grad;
  ST_TRY(buf.get(&g_dev, 2 * (s->adj->n + 1)));
  ST_TRY(buf.get(&grad, P));
  HIP_TRY(hipMemcpyAsync(g_dev, gbar, size_t(2 * (s->adj->n + 1)) * 8,
                         hipMemcpyHostToDevice, st));
  ST_TRY(adjoint_backward(s, g_dev, grad, st));
  HIP_TRY(hipMemcpyAsync(grad_out, grad, size_t(P) * 8, hipMemcpyDeviceToHost,
                         st));
  HIP_TRY(hipStreamSynchronize(st));
  return PACES_OK;
}

paces_status paces_adjoint_backward_dev(paces_sim* s, const void* dev_gbar,
                                        void* dev_grad, void* hip_stream) {
  if (!s || !dev_gbar || !dev_grad) return fail(PACES_E_ARG, "bad arguments");
  if (!s->adj) return fail(PACES_E_STATE, "no adjoint record");
  return adjoint_backward(s, static_cast<const double*>(dev_gbar),
                          static_cast<double*>(dev_grad),
                          static_cast<hipStream_t>(hip_stream));
}

paces_status paces_get_tuning(paces_sim* s, paces_tuning* out) {
  if (!s || !out) return fail(PACES_E_ARG, "bad arguments");
  *out = s->tune;
  return PACES_OK;
}

paces_status paces_set_tuning(paces_sim* s, const paces_tuning* t,
                              void* hip_stream) {
  if (!s) return fail(PACES_E_ARG, "bad arguments");
  ST_TRY(check_tuning(t));
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (t->term_rows != s->tune.term_rows || t->graph != s->tune.graph)
    drop_graphs(s);
  s->tune = *t;
  return resize_table(s, st);
}

paces_status paces_autotune(paces_sim* s, int32_t steps, paces_tuning* chosen,
                            void* hip_stream) {
  if (!s || steps < 1 || steps > 64) return fail(PACES_E_ARG, "bad arguments");
  if (s->latched) return fail(PACES_E_STATE, "sim is in an error state");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int prof = s->prof;
  s->prof = 0;
  Snapshot z;
  paces_status r = take_snapshot(s, z, st);
  const paces_tuning start = s->tune;
  paces_tuning best = start;
  float best_ms = INFINITY;
  hipEvent_t a = nullptr, b = nullptr;
  if (r == PACES_OK && (hipEventCreate(&a) != hipSuccess ||
                        hipEventCreate(&b) != hipSuccess))
    r = fail(PACES_E_HIP, "event creation failed");
  for (int g = 0; g < 2 && r == PACES_OK; ++g)
    for (int sh = 0; sh <= 2 && r == PACES_OK; ++sh)
      for (int tr : {1, 2, 4}) {
        paces_tuning t{g, sh, tr, start.warm};
        r = paces_set_tuning(s, &t, hip_stream);
        if (r == PACES_OK) r = restore_snapshot(s, z, st);
        // one untimed step (captures the graph), then the timed ones
        if (r == PACES_OK) r = do_step(s, st);
        if (r == PACES_OK && hipEventRecord(a, st) != hipSuccess)
          r = fail(PACES_E_HIP, "event record failed");
        for (int i = 0; i < steps && r == PACES_OK; ++i) r = do_step(s, st);
        if (r != PACES_OK) break;
        float ms = 0;
        if (hipEventRecord(b, st) != hipSuccess ||
            hipEventSynchronize(b) != hipSuccess ||
            hipEventElapsedTime(&ms, a, b) != hipSuccess) {
          r = fail(PACES_E_HIP, "event timing failed");
          break;
        }
        if (ms < best_ms) {
          best_ms = ms;
          best = t;
        }
      }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (r == PACES_OK) r = paces_set_tuning(s, &best, hip_stream);
  if (r == PACES_OK) r = restore_snapshot(s, z, st);
  s->prof = prof;
  if (r != PACES_OK) {
    s->tune = start;
    return r;
  }
  if (chosen) *chosen = best;
  return PACES_OK;
}

}  // extern "C"
