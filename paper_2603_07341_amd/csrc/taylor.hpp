// taylor.hpp -- truncated Taylor propagator: the method the paper names for
// exp(-i H dt) phi (App. "The action of the exponential of a sparse
// matrix": the degree and substep choice of Al-Mohy & Higham, SIAM J. Sci.
// Comput. 33, 2011) and its fixed-order variant (App. "An effective Hilbert
// space up to neighbor order m = 2 is not equivalent to a second-order
// Taylor expansion").
//
// With b, a the centre and half width of the padded Gershgorin interval and
// A = -i (H - b) dt, each of s substeps applies the degree-m polynomial
// sum_j (A/s)^j / j! by m SpMV launches, b_j = (A/s) b_(j-1) / j, f += b_j;
// the result carries exp(-i b dt).  (m, s) minimises m max(1, ceil(a dt /
// theta_m)) over m = 1..55, theta_m the degree-m backward-error threshold
// at unit roundoff 2^-53; or a fixed order N with s = 1.  Launch L of a
// step is term j = L mod m + 1 of substep L / m; the host enqueues a fixed
// number of launches and latches a retry when m s exceeds it.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace paces {

constexpr int kTaylorMaxDeg = 55;

struct TaylorPlan {
  int m, s;         // degree and substeps
  double b;         // shift (centre of the Gershgorin interval)
  double phase[2];  // exp(-i b dt)
};

// theta_m for m = 1..kTaylorMaxDeg (host computation, cached); index 0 is 0.
const double* taylor_thetas_host();

// Fold the bound partials (bounds_part) into plan[r] and the record's
// interval and step count (cc[r].emin / emax / K = m s); order < 0 chooses
// (m, s) with thetas_dev, order > 0 fixes m = order, s = 1.  Latches
// kErrTerms beyond k_max products, kErrNeedTerms beyond `launched`.
void taylor_plan(int R, const double* part, int nparts, double dt, int order,
                 const double* thetas_dev, int k_max, int launched,
                 TaylorPlan* plan, ChebCoef* cc, StepCtl* ctl, int* err,
                 hipStream_t s);
// Launch L (see above).  Buffers: phi in, bufB[2] terms, bufF[2] substep
// sums,
// out the result.  Launch 0 leaves <phi|H|phi> in e_part (one realization,
// per-block partials; returns their count) or e_row (batched, per row).
// ev_a / ev_b (may be null): events the dispatch records.
int taylor_term(const DevModel& m, int prec, int L, bool energy, double dt,
                int64_t est, const StepCtl* ctl, const int32_t* col,
                const Side& n, const TaylorPlan* plan, const void* phi,
                void* const* bufB, void* const* bufF, void* out, double* e_part,
                double* e_row, const int* err, hipEvent_t ev_a,
                hipEvent_t ev_b, hipStream_t s);

// <psi|H|psi> of the result psi (fixed order): partials as for launch 0.
int taylor_energy(const DevModel& m, int prec, int64_t est,
                  const StepCtl* ctl, const int32_t* col, const Side& n,
                  const void* psi, double* e_part, double* e_row,
                  const int* err, hipStream_t s);

}  // namespace paces
