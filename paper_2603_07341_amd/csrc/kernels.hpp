// kernels.hpp -- host-side launch wrappers of the step's HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"

namespace paces {

constexpr int kMaxTerms = 128;  // Chebyshev terms per step, hard limit

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

// Scalar results of one step, reduced on the device.
struct StepScalars {
  double mass;      // discarded weight of the transfer
  double norm2;     // |psi|^2 after propagation
  double energy;    // <phi|H|phi> = <psi|H|psi> up to the series error
  double a[2];      // <psi0|psi(t)>
};

// Per-step observation record in the device ring buffer (doubles):
// [t, norm2, energy, a_re, a_im, mass_step, mass_total, nS, nM, K,
//  E_min, E_max, pop[0..N-1]].
constexpr int kObsFields = 12;

// Launch geometry of grid-stride kernels that write per-block partials.
constexpr int kPartBlocks = 1024;

int supported_words(int W);  // internal word count >= W, or 0

void fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s);
void fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);
void iota_u32(uint32_t* p, int64_t n, hipStream_t s);

// Exclusive scan of n u32 values; tmp needs scan_tmp_words(n) u32.
int64_t scan_tmp_words(int64_t n);
void exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n,
                    uint32_t* tmp, uint32_t* total, hipStream_t s);

// Compaction of rows whose weight clears theta^2 (ascending row order).
void select_rows(int prec, const void* psi, int64_t n, double th2,
                 uint32_t* midx, uint32_t* tmp, uint32_t* count,
                 hipStream_t s);

void row_info(const DevModel& m, int Wi, const uint64_t* keys, int64_t n,
              uint64_t* pay, uint64_t* tot, double* diag, hipStream_t s);

void insert_rows(const DevModel& m, int Wi, const uint64_t* keys_o,
                 const uint64_t* pay_o, const uint64_t* tot_o,
                 const double* diag_o, const uint32_t* midx, int64_t nM,
                 uint64_t* keys_n, uint64_t* pay_n, uint64_t* tot_n,
                 double* diag_n, uint64_t* table, uint64_t mask, int* err,
                 hipStream_t s);

struct RoundBufs {
  uint32_t* c_slot;  // [rows*D] table slot of each candidate
  uint32_t* c_ref;   // [rows*D] resolved reference
  uint32_t* crow;    // [rows*D] row of owning candidates
  uint32_t* rowcnt;  // [rows] new rows per parent
  uint32_t* rowbase; // [rows] exclusive scan of rowcnt
  uint32_t* scan_tmp;
  uint32_t* total;   // [1] device
};

// One chunk of an expansion round: parents [f0, f0+rows) emit their slots;
// new states are appended from row n_cur.  Writes the ELL columns of the
// parents and zeroes phi of the new rows.
void expand_chunk(const DevModel& m, int Wi, int prec, uint64_t* keys,
                  uint64_t* pay, uint64_t* tot, double* diag, int64_t f0,
                  int64_t rows, int64_t n_cur, uint64_t* table, uint64_t mask,
                  const RoundBufs& rb, int32_t* col, int64_t stride, void* phi,
                  int* err, hipStream_t s);

// Columns of parents [f0, f0+rows) by lookup only (last frontier).
void lookup_cols(const DevModel& m, int Wi, const uint64_t* keys,
                 const uint64_t* pay, int64_t f0, int64_t rows,
                 const uint64_t* table, uint64_t mask, int32_t* col,
                 int64_t stride, hipStream_t s);

// phi[row of key in new set] = psi_old; discarded weight to mass_part.
void transfer(const DevModel& m, int Wi, int prec, const uint64_t* keys_o,
              const void* psi_o, int64_t n_old, const uint64_t* table,
              uint64_t mask, const uint64_t* keys_n, void* phi,
              double* mass_part, hipStream_t s);

// Gershgorin bounds + Chebyshev coefficients (device only).
void bounds_and_coef(const DevModel& m, const uint64_t* pay,
                     const double* diag, const int32_t* col, int64_t stride,
                     int64_t n, double dt, double tol, int k_max,
                     double* part, ChebCoef* cc, int* err, hipStream_t s);

// One Clenshaw step of the Chebyshev series (see kernels.hip).
struct TermArgs {
  int in_coef;    // -1: SpMV input unscaled, else scaled by c[in_coef]
  int prev_coef;  // -1: prev unscaled, else scaled by c[prev_coef]
  int ck;         // coefficient index applied to phi
  int fac;        // 1 or 2
  int final_;     // multiply by exp(-i b dt), reduce norm and populations
  int energy;     // reduce Re <in|H|in>
};
void cheb_term(const DevModel& m, int prec, int64_t n, const int32_t* col,
               int64_t stride, const uint64_t* pay, const double* diag,
               const ChebCoef* cc, const TermArgs& ta, const void* phi,
               const void* in, const void* prev, void* out, double* e_part,
               double* n2_part, double* pop_part, hipStream_t s);
// out = c[0] * phase * phi (a one-term series).
void cheb_scale(int prec, int64_t n, const ChebCoef* cc, const void* phi,
                void* out, double* n2_part, double* pop_part,
                const uint64_t* pay, int N, hipStream_t s);
// Energy <x|H|x> partials when no series term computed it.
void energy_only(const DevModel& m, int prec, int64_t n, const int32_t* col,
                 int64_t stride, const uint64_t* pay, const double* diag,
                 const void* x, double* e_part, hipStream_t s);

void autocorr(const DevModel& m, int Wi, int prec, const uint64_t* keys0,
              const double* amps0, int64_t n0, const uint64_t* table,
              uint64_t mask, const uint64_t* keys, const void* psi,
              double* out2, hipStream_t s);

// Final reductions of a step into an observation record.
struct ObsArgs {
  double t, nS, nM, dt;
  int N, want_energy;
};
void obs_final(const ObsArgs& oa, const double* mass_part,
               const double* n2_part, const double* e_part,
               const double* pop_part, const double* a2, const ChebCoef* cc,
               double* mass_total, double* rec, int* err, hipStream_t s);

// Widen / narrow amplitudes between the boundary's interleaved FP64 and the
// internal precision.
void amps_to_f64(int prec, const void* src, double* dst, int64_t n,
                 hipStream_t s);
void amps_from_f64(int prec, const double* src, void* dst, int64_t n,
                   hipStream_t s);

}  // namespace paces
