// warm.hpp -- expansion of a step from the previous step's graph.
//
// S' = B_k(M) with M a subset of the previous set S (Eq. (def_neighbor_k);
// Sec. "Truncation & post-adaptation detruncation").  The previous step
// left the ELL columns of every row of S: a column is -1 exactly where the
// slot is structurally zero or its neighbour lies outside S.  A breadth-
// first search from M therefore walks edges inside S through those columns
// (no hashing), and only a slot whose neighbour lies outside S, and every
// slot of a state found outside S, goes through the hash table.  The
// distances of old rows live in dist (one byte per row); states found
// outside S are appended as rows [0, n_staged) of the new set, and their
// keys enter the hash table, which still maps every key of S to its old
// row, marked as staged (kStaged | row).  Then the old rows at distance
// <= k are compacted behind them in their old order (keys, payload, the
// amplitude as phi of the transfer, distance), columns are remapped, and
// the table is rewritten in place to the new rows (entries of dropped rows
// become tombstones).  The result is the same set, the same columns and
// the same phi as the expansion from scratch, in another row order.
//
// Until the table is rewritten the step leaves the previous set, its
// columns and its table as they were (staged entries are removed by
// warm_unstage), so a step that latched an error before that point can be
// repeated from the same graph.
#pragma once
#include "kernels.hpp"

namespace paces {

constexpr uint32_t kStaged = 0x40000000u;  // table value names a new row
constexpr uint8_t kFar = 0xFF;             // distance beyond the ball
// Row values of a table that warm steps use stay below kStaged.
constexpr int64_t kWarmMaxRows = int64_t(kStaged) - 256;

// Buffers of the expansion from the previous graph.
struct WarmBufs {
  uint64_t* wlist;  // [cand_cap] old row << 8 | slot: candidates of a round
                    // that come from old rows
  uint16_t* wmask;  // [rows] slots of an old frontier row whose neighbour
                    // is outside the old set
  uint64_t* kbits;  // [rows / 64] old rows that stay, one bit each
  uint32_t* kpre;   // [rows / 64] old rows that stay before each word
};

// Distances of the old rows: 0 on M (midx[0, nM)), kFar elsewhere; |M| per
// realization into cnt_m; the staged-row counts cleared.
void warm_begin(const DevModel& m, StepCtl* ctl, const uint32_t* midx,
                const Side& o, uint32_t* cnt_m, int64_t n_old, int* err,
                hipStream_t s);
// Round r (1..k): old rows at distance r-1 mark their neighbours inside
// the old set at distance r and hand the slots whose neighbour is outside
// it on as candidates; new states of round r-1 hand on every slot.
// Candidates already in the old set mark it, others are inserted into the
// table; the first of each new key appends a row to the new set (key,
// payload, distance r, phi 0).  More candidates than the buffers hold
// latch kErrChunks.
void warm_round(const DevModel& m, int Wi, int prec, const Side& o,
                const Side& n, int r, StepCtl* ctl, int64_t cap,
                int64_t n_old, int64_t est, uint64_t* table, uint64_t mask,
                const RoundBufs& rb, const WarmBufs& wb, uint32_t* scan_tmp,
                void* phi, int* err, hipStream_t s);
// Rows of the new set: old rows at distance <= k behind the staged rows;
// n_new, with kErrCapacity when they exceed cap.
void warm_count(const Side& o, int k, StepCtl* ctl, int64_t n_old,
                int64_t cap, uint32_t* scan_tmp, int* err, hipStream_t s);
// Old rows into the new set: keys, payload (and totals when the payload
// does not hold them), distance, phi = psi, the keep map; weight of the
// dropped rows into per-block partials (one double per block, or R per
// block for several realizations).  Returns the number of partial blocks.
int warm_compact(const DevModel& m, int Wi, int prec, const Side& o,
                 const Side& n, int k, const StepCtl* ctl, int64_t n_old,
                 const void* psi_o, void* phi, const uint32_t* scan_tmp,
                 const WarmBufs& wb, double* mass_part, int* err,
                 hipStream_t s);
// Columns of the new set: old rows by remapping theirs through the keep
// map, staged rows by table lookup (which also sets the columns of old
// rows toward staged rows).
void warm_columns(const DevModel& m, int Wi, const Side& o, const Side& n,
                  const StepCtl* ctl, int64_t n_old, int64_t est,
                  const uint64_t* table, uint64_t mask, const WarmBufs& wb,
                  int* err, hipStream_t s);
// The table rewritten in place to rows of the new set (sets w_moved and
// counts new tombstones into w_tomb).
void warm_retable(StepCtl* ctl, uint64_t* table, uint64_t mask,
                  const WarmBufs& wb, int* err, hipStream_t s);
// Staged and candidate entries back to empty slots, whatever the latch:
// the table of the previous set as it was before the step.
void warm_unstage(uint64_t* table, uint64_t mask, hipStream_t s);
// Keys of the rows [0, n) whose distance is d, in row order, into out
// (Wi words each); their count into *count (device).  tmp: scan space of
// scan_tmp_words(n) words; err: the sim's latch (clear).
void rows_at_distance(int Wi, const uint64_t* keys, const uint8_t* dist,
                      int64_t n, int d, uint64_t* out, uint32_t* count,
                      uint32_t* tmp, int* err, hipStream_t s);

}  // namespace paces
