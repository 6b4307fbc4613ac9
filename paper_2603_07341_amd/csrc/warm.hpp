// warm.hpp -- a step that expands from the previous step's graph, in place.
//
// S' = B_k(M) with M a subset of the previous set S (Eq. (def_neighbor_k);
// Sec. "Truncation & post-adaptation detruncation").  The previous step
// left the ELL columns of every row of S: a column is -1 exactly where the
// slot is structurally zero or its neighbour lies outside S.  A breadth-
// first search from M therefore walks edges inside S through those columns
// (no hashing), and only a slot whose neighbour lies outside S, and every
// slot of a state found outside S, goes through the hash table, which maps
// the keys of S to their rows and persists across steps.
//
// Rows keep their index from step to step.  A state found outside S takes
// a hole of the set (a row left by a dropped state) or a new row past the
// set's row range; a dropped state leaves a hole: amplitude 0, no columns,
// no table entry (a tombstone), and the columns of its neighbours toward
// it set to -1 (an edge is seen from both ends as slots s and s ^ 1).  So
// a step writes only the rows that change; the propagator runs over the
// row range, where holes contribute nothing.  The amplitude of the old
// state becomes phi in place (Sec. "Truncation & post-adaptation
// detruncation": kept amplitudes carried, new ones 0).
//
// One byte per row (dist) holds the row's distance from M during the
// search: kFar for a live row not reached (yet), kHole for a hole, and
// kNewRow | r for a state found in round r of this step.  After the step
// it is the distance (0..k) of every live row, or kHole.
//
// Until the commit (the drop pass) the step changes nothing of the
// previous set: found states fill holes and rows past the range, and their
// table entries fill empty slots only, so warm_unstage restores the table
// exactly and the step can be repeated (the state cap does so with a cut
// selection).  After the commit only the propagation and the observables
// remain; a repeat of those needs nothing from before.
#pragma once
#include "kernels.hpp"

namespace paces {

constexpr uint32_t kStaged = 0x40000000u;  // table value names a new row
constexpr uint8_t kFar = 0xFF;             // live row not reached
constexpr uint8_t kNewRow = 0x80;          // | r: found in round r
// Row values of a table that these steps use stay below kStaged.
constexpr int64_t kWarmMaxRows = int64_t(kStaged) - 256;

// Buffers of the in-place step.
struct WarmBufs {
  uint64_t* wlist;  // [cand_cap] old row << 8 | slot: candidates of a round
                    // that come from old rows
  uint16_t* wmask;  // [rows] slots of an old frontier row whose neighbour
                    // is outside the old set
  uint32_t* freel;  // [rows] holes of the set, ascending
};

// Distances of the rows in [0, n_old): kHole kept, 0 on M (midx[0, nM)),
// kFar elsewhere; the holes into freel (ctl->nfree; holes false: the set
// has none, and the free list is not built); |M| per realization into
// cnt_m; the step's other counts cleared.
void warm_begin(const DevModel& m, StepCtl* ctl, const uint32_t* midx,
                const Side& c, const WarmBufs& wb, uint32_t* cnt_m,
                int64_t n_old, bool holes, uint32_t* scan_tmp, int* err,
                hipStream_t s);
// Round r (1..k): live rows at distance r-1 mark their neighbours inside
// the set at distance r and hand the slots whose neighbour is outside it
// on as candidates; states found in round r-1 hand on every slot.
// Candidates already in the set mark it, others are inserted into the
// table; the first of each new key becomes the state's row (the next hole,
// else the next row past the range): key, payload, distance kNewRow | r,
// amplitude 0.  A row past cap latches kErrCapacity; more candidates than
// the buffers hold latch kErrChunks.
void warm_round(const DevModel& m, int Wi, int prec, const Side& c, int r,
                StepCtl* ctl, int64_t cap, int64_t n_old, int64_t est,
                uint64_t* table, uint64_t mask, const RoundBufs& rb,
                const WarmBufs& wb, uint32_t* scan_tmp, void* psi, int* err,
                hipStream_t s);
// Sizes after the search: the row range n_new and the live rows n_live;
// live rows per realization into ball (with max_states > 0, a realization
// above it latches kErrCap).
void warm_sizes(const DevModel& m, const Side& c, int k, StepCtl* ctl,
                int64_t est, int64_t max_states, uint32_t* ball, int* err,
                hipStream_t s);
// The commit.  Drop pass: every live row the search did not reach (kFar)
// becomes a hole (its weight into per-block partials, one double per
// block or R per block; amplitude 0; table entry a tombstone; its own and
// its neighbours' columns toward it -1).  Then the found states: distance
// r, table entry plain, columns by lookup (also the column of a live
// neighbour toward them).  Returns the number of partial blocks.
int warm_commit(const DevModel& m, int Wi, int prec, const Side& c, int k,
                StepCtl* ctl, int64_t n_old, int64_t est, uint64_t* table,
                uint64_t mask, const WarmBufs& wb, void* psi,
                double* mass_part, int* err, hipStream_t s);
// Before a repeated search: staged and candidate entries of the table back
// to empty slots, and holes that took a found state back to holes,
// whatever the latch.
void warm_unstage(const StepCtl* ctl, const Side& c, const WarmBufs& wb,
                  uint64_t* table, uint64_t mask, int64_t n_old,
                  hipStream_t s);
// Distance bytes of a set built from scratch: round r of rows [fstart[r],
// fstart[r+1]) (r = 0..k), so that the set has no holes and its frontiers
// read like those of an in-place step.
void dist_of_rounds(const StepCtl* ctl, int k, uint8_t* dist, int64_t est,
                    hipStream_t s);
// dist[0, n) = v.
void dist_fill(uint8_t* dist, int64_t n, uint8_t v, hipStream_t s);
// Keys of the rows [0, n) whose distance is d (d < 0: every live row), in
// row order, into out (Wi words each; null: none); their rows into rows
// (may be null); their count into *count (device).  tmp: scan space of
// scan_tmp_words(n) words.  Works whatever the sim's latch holds.
void rows_at_distance(int Wi, const uint64_t* keys, const uint8_t* dist,
                      int64_t n, int d, uint64_t* out, uint32_t* rows,
                      uint32_t* count, uint32_t* tmp, hipStream_t s);
// Gather rows idx[0, n) of a set (keys, payload, totals and the amplitude,
// A bytes each) into dense arrays (any output may be null).
void gather_rows(int Wi, size_t A, const Side& c, const void* psi,
                 const uint32_t* idx, int64_t n, uint64_t* keys,
                 uint64_t* pay, uint64_t* tot, void* amps, hipStream_t s);

}  // namespace paces
