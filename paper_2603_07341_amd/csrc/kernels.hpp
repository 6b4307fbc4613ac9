// kernels.hpp -- host-side launch wrappers of the step's HIP kernels.
//
// Row counts of a step live in device memory (StepCtl) and every kernel
// reads them there, so a whole step is enqueued without the host waiting on
// the GPU.  Kernels run on fixed grid-stride grids and clamp every count to
// the allocated capacity; an overflow is latched and the host repeats the
// step with larger buffers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"

namespace paces {

constexpr int kMaxTerms = 128;   // Chebyshev terms per step, hard limit
constexpr int kMaxRounds = 30;   // neighbour order per step, hard limit
constexpr int kPartBlocks = 2048;  // grid of the population reduction
constexpr int kMaxPartials = 1 << 18;  // per-block partials of row kernels
constexpr int kObsFields = 12;
constexpr int kMaxReal = 256;      // disorder realizations per sim

// Chebyshev expansion of exp(-i H dt) on [E_min, E_max], computed on the
// device from the Gershgorin bounds of the step.
struct ChebCoef {
  double emin, emax;   // padded Gershgorin interval
  double a, b;         // half width and centre
  double alpha, beta;  // H~ = alpha H + beta: alpha = 1/a, beta = -b/a
  double phase[2];     // exp(-i b dt)
  int K;               // number of terms used
  int pad_;
  double c[kMaxTerms][2];  // c_k = (2 - delta_k0) (-i)^k J_k(a dt)
};

// Device-resident counts of one step.
struct StepCtl {
  uint32_t n_old;                     // rows of the set the step starts from
  uint32_t nM;                        // selected rows
  uint32_t fstart[kMaxRounds + 2];    // frontier r: [fstart[r], fstart[r+1])
  uint32_t n_new;                     // rows of the new set
  // current chunk of the current expansion round: parents [r_f0, r_f0 +
  // r_rows) of the frontier; r_ncur the rows of the set so far
  uint32_t r_f0, r_rows, r_ncand, r_ntiles, r_ncur, r_total;
  uint32_t r_need;                    // chunks the largest round needs
  uint32_t kmax;                      // largest K over realizations
  uint32_t nrec;                      // steps recorded (R records each)
  // expansion from the previous step's graph (warm.hpp): new states of
  // round r are rows [gstart[r], gstart[r+1]) of the new set; w_noc
  // candidates of the round come from old rows, the rest from the new
  // states of the round before (first row w_f0); w_nkeep old rows stay;
  // w_moved is set once the hash table holds the new rows; w_tomb counts
  // the table entries of dropped rows turned into tombstones by this step
  uint32_t gstart[kMaxRounds + 2];
  uint32_t n_staged, w_noc, w_f0, w_nkeep, w_moved, w_tomb;
  // in-place steps: holes of the set at the step's start (the free list's
  // length) and the set's live rows after the step (n_new is its row range)
  uint32_t nfree, n_live;
  double t;                           // time after the last completed step
};

// Buffers of one expansion round.
struct RoundBufs {
  uint32_t* c_slot;     // [cand] probe distance of owning candidates from
                        // the key's home slot (below kMaxProbe)
  uint32_t* c_ref;      // [cand] outcome of the probe
  uint32_t* crow;       // [cand] row of owning candidates
  uint32_t* tile_cnt;   // [cand / 256] owners per tile of candidates
  uint32_t* tile_base;  // [cand / 256] exclusive scan of tile_cnt
  uint32_t* scan_tmp;
  int64_t cand_cap;     // candidates the buffers hold
};

// Row arrays of one set.  col (ELL columns, D per row) and dist (distance
// of the row from the step's selection, 0..k) describe the set a step
// built; dist is written by steps that expand from the previous graph.
struct Side {
  uint64_t* keys;
  uint64_t* pay;
  uint64_t* tot;
  int32_t* col;
  uint8_t* dist;
};

int supported_words(int W);  // internal word count >= W, or 0
int64_t scan_tmp_words(int64_t n);

void fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s);
// One empty dispatch (kernel k_mark) on the stream.
void mark(int tag, hipStream_t s);
// The error latch cleared on the stream.
void clear_latch(int* err, hipStream_t s);
// A given set of n states as the rows of a step: keys padded from W to Wi
// words; control counts with frontier 0 = rows [0, n) and the latch
// cleared; every key valid and distinct (else kErrInput), after the rows
// are in the table.
void pad_keys(int W, int Wi, const uint64_t* in, uint64_t* out, int64_t n,
              hipStream_t s);
void set_begin(StepCtl* ctl, int* err, int64_t n, hipStream_t s);
void check_set(const DevModel& m, int Wi, const uint64_t* keys, int64_t n,
               const uint64_t* table, uint64_t mask, int* err,
               hipStream_t s);

// Start of a step: clear the latch, reset the counters (cnt: 2R
// per-realization row counts, |M_r| then |S_r|).
void begin_step(StepCtl* ctl, int* err, uint32_t* cnt, int R, hipStream_t s);
// Rows of ctl->n_old with weight >= th2 that are not holes (dist may be
// null), ascending, into midx; ctl->nM.
// select_all: the first step takes every row.
// counted: tmp already holds the per-tile counts (from pop_norm).
void select_rows(int prec, const void* psi, const uint8_t* dist, double th2,
                 bool select_all, bool counted, StepCtl* ctl, uint32_t* midx,
                 uint32_t* tmp, int64_t cap, int* err, hipStream_t s);
// Rows of ctl->n_old with keep[row] != 0, ascending, into midx; ctl->nM.
void select_flags(const uint8_t* keep, StepCtl* ctl, uint32_t* midx,
                  uint32_t* tmp, int64_t cap, int* err, hipStream_t s);
// Rows 0..nM-1 of the new side are M; inserted into the cleared table.
// phi (may be null) receives their amplitudes from psi_o.
void insert_rows(const DevModel& m, int Wi, int prec, const Side& o,
                 const Side& n, const uint32_t* midx, const StepCtl* ctl,
                 uint64_t* table, uint64_t mask, uint32_t* cnt_m,
                 const void* psi_o, void* phi, int* err, hipStream_t s);
// Rebuild the table from rows [0, n) of a side (after growth).
void rehash_rows(const DevModel& m, int Wi, const Side& n, uint32_t* midx,
                 int64_t rows, uint64_t* table, uint64_t mask, int* err,
                 hipStream_t s);
// Expansion round r (1..k): frontier r-1 emits its slots; new rows are
// appended and become frontier r.  Writes the parents' ELL columns and
// zeroes phi of the new rows.  The frontier is taken in `chunks` chunks of
// at most cand_cap / D parents each (one after another, each sees the rows
// the previous ones added); a frontier larger than that latches kErrChunks
// with the chunk count it needs in ctl->r_need.
// est: host estimate of the new set's rows, used only to size grids.
void expand_round(const DevModel& m, int Wi, int prec, const Side& n, int r,
                  StepCtl* ctl, int64_t cap, int64_t est, uint64_t* table,
                  uint64_t mask, const RoundBufs& rb, int32_t* col, void* phi,
                  int chunks, int* err, hipStream_t s);
// Exclusive scan of cnt[0, *ntiles) (at most `bound` entries) into base,
// the total into *total; tmp holds scan_tmp_words(bound) words.
void tile_scan(const uint32_t* cnt, const uint32_t* ntiles, int64_t bound,
               uint32_t* tmp, uint32_t* base, uint32_t* total, int* err,
               hipStream_t s);
// In place: bsum holds one count per tile of kTile rows over *nrows rows
// (written by a kernel of the select layout); exclusive scan, total into
// *total.
void tile_sums_scan(uint32_t* bsum, const uint32_t* nrows, uint32_t* total,
                    int* err, hipStream_t s);
// Columns of frontier k (lookup only); sets ctl->n_new.
void lookup_last(const DevModel& m, int Wi, const Side& n, int k,
                 StepCtl* ctl, int64_t est, const uint64_t* table,
                 uint64_t mask, int32_t* col, int64_t cap, int* err,
                 hipStream_t s);
// Number of per-block partials written by a kernel over `rows` rows.
int part_grid(int64_t rows);
// Returns the number of mass partials written.  tmap (may be null) gets
// the new row of every old row, -1 if dropped (then skip must be 0).
// skip: 0 every old row; 1 rows with weight < th2 only; 2 rows with
// keep[row] == 0 only -- the rows of M, placed by insert_rows.
int transfer(const DevModel& m, int Wi, int prec, const Side& o,
             const void* psi_o, int64_t n_old, const StepCtl* ctl,
             const uint64_t* table, uint64_t mask, const uint64_t* keys_n,
             void* phi, double* mass_part, int32_t* tmap, int skip, double th2,
             const uint8_t* keep, int* err, hipStream_t s);
// Gershgorin bounds + Chebyshev coefficients per realization (cc[R]);
// latches if some K_r exceeds the launches enqueued.
void bounds_and_coef(const DevModel& m, const Side& n, const int32_t* col,
                     int64_t cap, int64_t est, StepCtl* ctl, double dt,
                     double tol, int k_max, int launched, double* part,
                     ChebCoef* cc, int* err, hipStream_t s);
// Gershgorin bounds only: per-block (lo, hi) per realization into
// part[block][R][2]; returns the number of blocks.
int bounds_part(const DevModel& m, const Side& n, const int32_t* col,
                int64_t cap, int64_t est, const StepCtl* ctl, double* part,
                const int* err, hipStream_t s);
// Fold n per-block partials to at most 256 (deterministic); returns count.
int fold_sum(const double* in, int n, double* out, int* err, hipStream_t s);
// Clenshaw launch for index kk (see kernels.hip); buffers b[0], b[1].
// Returns the number of energy partials (written by the first launch).
// mid: the launch is expected to be a middle term (selects a kernel name).
// Batched sims (R > 1) leave the energy per row in e_row.  ev_a / ev_b
// (may be null): events the dispatch records at its start and stop.
int cheb_term(const DevModel& m, int prec, int kk, bool energy, bool mid,
              int64_t est, const StepCtl* ctl, const int32_t* col, int64_t cap,
              const Side& n, const ChebCoef* cc, const void* phi, void* b0,
              void* b1, double* e_part, double* e_row, int* err,
              hipEvent_t ev_a, hipEvent_t ev_b, hipStream_t s);
// |psi|^2 and exciton populations as per-block partials (returns their
// count, at most kPartBlocks), plus the next step's select counts.
int pop_norm(int prec, int N, int R, double th2, int64_t est,
             const StepCtl* ctl, const void* psi, const uint64_t* pay,
             const uint8_t* dist,
             const double* e_row, double* n2_part, double* en_part,
             double* pop_part, uint32_t* sel_bsum, uint32_t* cnt_s, int* err,
             hipStream_t s);
// <psi0|psi> per realization; p0map (may be null) gets the row of every
// initial state, -1 if absent.
void autocorr(const DevModel& m, int Wi, int prec, const uint64_t* keys0,
              const double* amps0, int64_t n0, const uint64_t* table,
              uint64_t mask, const uint64_t* keys, const void* psi,
              double* out2, int32_t* p0map, int* err, hipStream_t s);
// Commit a successful step on the device: time, discarded weight per
// realization, record count and the row count of the current set; then
// mirror *ctl and *err into mapped pinned host memory (device addresses
// h_ctl_dev, h_err_dev), also when an error is latched.
void end_step(StepCtl* ctl, int R, const double* ring, int rec_doubles,
              double* mass_tot, int* err, StepCtl* h_ctl_dev, int* h_err_dev,
              hipStream_t s);
// Reduce partials into observation record ctl->nrec (skipped when an error
// is latched, so a repeated step records once).
void obs_final(int N, int R, int want_energy, double dt, int n_mass, int n_e,
               int n_pop, const double* mass_part, const double* n2_part,
               const double* e_part, const double* en_part,
               const double* pop_part, const double* a2, const ChebCoef* cc,
               const StepCtl* ctl, const uint32_t* cnt,
               const double* mass_tot, double* ring, int rec_doubles,
               int64_t ring_cap, int* err, hipStream_t s);

void row_info(const DevModel& m, int Wi, const uint64_t* keys, int64_t n,
              uint64_t* pay, uint64_t* tot, hipStream_t s);
void amps_to_f64(int prec, const void* src, double* dst, int64_t n,
                 hipStream_t s);
void amps_from_f64(int prec, const double* src, void* dst, int64_t n,
                   hipStream_t s);

}  // namespace paces
