// lanczos.hpp -- Krylov (Lanczos) propagator, the alternative to the
// Chebyshev series inside H_eff (paper: App. "Series-based exponentiation
// compared to a Lanczos algorithm").
//
// Order p works in span{phi, H phi, .., H^p phi} (dimension n = p + 1).  Per
// realization, with unnormalised basis vectors w_j = beta_j v_j (w_0 = phi,
// beta_0 = |phi|):
//   SpMV j:  z = H w_j, partial sums of <w_j, z>, |w_j|^2 and |z|^2;
//   fold j:  beta_j = |w_j|, alpha_j = <w_j, H w_j> / |w_j|^2,
//            |H v_j|^2 = |z|^2 / |w_j|^2 (breakdown test of step j + 1);
//   orth j:  w_{j+1} = (z - alpha_j w_j) / beta_j - (beta_j / beta_{j-1}) w_{j-1}
//            (in place over z).
// A realization whose |w_j| falls to brk * |H v_{j-1}| stops with j vectors
// (invariant space).  Then u = exp(-i T dt) e_1 for the tridiagonal T
// (alpha on the diagonal, beta_1.. beside it) by a Chebyshev series on T,
// and psi' = sum_j (beta_0 u_j / beta_j) w_j.
// Storage: n - 1 vectors beyond phi (the last SpMV writes none).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace paces {

constexpr int kMaxKrylov = 64;  // Krylov dimension limit: order <= 63
constexpr int kLzGrid1 = 8192;  // SpMV blocks with one realization
// |w_j| below this fraction of |H v_{j-1}| ends the basis (FP64, FP32)
constexpr double kLzBreak64 = 1e-11, kLzBreak32 = 1e-6;

struct LanczosState {
  double alpha[kMaxKrylov];
  double beta[kMaxKrylov];   // beta[0] = |phi|; beta[j] couples v_{j-1}, v_j
  double hn2[kMaxKrylov];    // |H v_j|^2
  double s[kMaxKrylov][2];   // combination weights beta_0 u_j / beta_j
  int dim;                   // basis vectors accepted so far
  int done;                  // no further vectors (breakdown or zero start)
};

// Basis vector pointers by value: w[0] = phi, w[j] for j >= 1 the buffers of
// the recurrence.
struct KrylovVecs {
  void* w[kMaxKrylov];
};

// Reset the states of R realizations.
void lz_begin(LanczosState* st, int R, const int* err, hipStream_t s);
// SpMV j over the rows of realizations still building their basis;
// out = H w_j (null for the last iteration).  part: per-block partials
// [grid][R][3]; returns the grid used.  ev_a / ev_b (may be null): events
// the dispatch records at its start and stop.
int lz_spmv(const DevModel& m, int prec, int j, int64_t est,
            const StepCtl* ctl, const int32_t* col, const Side& n,
            const LanczosState* st, const void* in, void* out, double* part,
            const int* err, hipEvent_t ev_a, hipEvent_t ev_b,
            hipStream_t s);
// Fold the partials of SpMV j into alpha_j, beta_j, |H v_j|^2 per
// realization (energy[r] = <phi|H|phi> from j = 0).  brk2 = brk^2.
void lz_fold(int j, const double* part, int nparts, int R, double brk2,
             LanczosState* st, double* energy, const int* err, hipStream_t s);
// w_{j+1} from z (in place), w_j and w_{j-1}.
void lz_orth(const DevModel& m, int prec, int j, int64_t est,
             const StepCtl* ctl, const uint64_t* pay, const LanczosState* st,
             void* z, const void* wj, const void* wjm1, const int* err,
             hipStream_t s);
// u = exp(-i T dt) e_1 and the combination weights; cc[r] gets K = the
// dimension and the padded Gershgorin interval of T; kmax the largest
// dimension.  Latches kErrTerms when the series on T needs more than
// k_max terms.
void lz_small(int R, double dt, double tol, int k_max, LanczosState* st,
              ChebCoef* cc, StepCtl* ctl, int* err, hipStream_t s);
// out = sum_j s_j w_j over the nv vectors.
void lz_combine(const DevModel& m, int prec, int64_t est, const StepCtl* ctl,
                const uint64_t* pay, const LanczosState* st,
                const KrylovVecs& w, int nv, void* out, const int* err,
                hipStream_t s);

// Energy field of the record being written (after obs_final).
void lz_record_energy(int R, const double* energy, const StepCtl* ctl,
                      double* ring, int rec_doubles, int64_t ring_cap,
                      const int* err, hipStream_t s);

}  // namespace paces
