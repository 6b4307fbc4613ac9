// adjoint.hpp -- launch wrappers of the adjoint-gradient kernels (Form (3)).
//
// With the sets of a recorded run held fixed, each step is the linear map
// psi_{s+1} = U_s T_s psi_s (U_s = exp(-i H_{s+1} dt), T_s the restriction
// to the new set).  For a real loss L of a_s = <psi0|psi_s> and
// gbar_s = dL/d conj(a_s) the backward pass runs
//   lambda_n = gbar_n psi0,  mu = U_s^dag lambda_{s+1},
//   lambda_s = T_s^T mu + gbar_s psi0,
//   dL/dtheta_p += 2 Re <lambda_{s+1}| dU_s/dtheta_p |T_s psi_s>
//               = 2 dt Im int_0^1 <e^{-i tau H dt} mu | dH/dtheta_p |
//                                  e^{-i tau H dt} T_s psi_s> dtau,
// the integral by Gauss-Legendre quadrature; both propagations to every
// node share one Chebyshev recurrence per vector.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace paces {

constexpr int kMaxNodes = 12;  // Gauss-Legendre nodes per step

// Frozen step: rows 0..nM-1 of the new side hold M already; set the
// counts a select would have produced.
void adj_set_frozen(StepCtl* ctl, uint32_t* cnt, uint32_t nM, int* err,
                    hipStream_t s);
// ctl->n_new = n for the backward kernels that read it.
void adj_set_rows(StepCtl* ctl, uint32_t n, hipStream_t s);
// out = in with conjugated coefficients and phase: exp(+i H dt).
void adj_conj_coef(const ChebCoef* in, ChebCoef* out, hipStream_t s);
// Coefficients of exp(-i tau_q H dt) on the interval of cc for nq nodes,
// the phase exp(-i b tau_q dt) folded in: cn[q][k], k < kMaxTerms.
void adj_node_coef(const ChebCoef* cc, double dt, const double* tau, int nq,
                   double tol, double2* cn, int* err, hipStream_t s);
// Launch kk (0..K-1) of the shared three-term recurrence of the chains
// x (from t[0][0]) and y (from t[1][0]) on n rows; acc_c[q*n + i] collects
// sum_k cn[q][k] T_k.  K = number of launches.
void adj_nodes(const DevModel& m, int kk, int K, int64_t n,
               const int32_t* col, const uint64_t* pay, const uint64_t* tot,
               const ChebCoef* cc, const double2* cn, int nq,
               double2* tx0, double2* tx1, double2* ty0, double2* ty1,
               double2* accx, double2* accy, int* err, hipStream_t s);
// Per-block partials of sum_q w_q Im <x_q| dH/dtheta_p |y_q> for all
// parameters; returns the number of blocks.  P = ndim + 2V + N.
int adj_contract(const DevModel& m, int64_t n, const int32_t* col,
                 const uint64_t* pay, const uint64_t* tot, int nq,
                 const double* w, const double2* accx, const double2* accy,
                 double* part, int* err, hipStream_t s);
// grad[p] += scale * sum over nb partials part[b][p] (fixed order).
void adj_fold(const double* part, int nb, int P, double scale, double* grad,
              int* err, hipStream_t s);
// lam[i] = tmap[i] >= 0 ? mu[tmap[i]] : 0 for i < n.
void adj_back(int64_t n, const int32_t* tmap, const double2* mu,
              double2* lam, int* err, hipStream_t s);
// lam[p0[q]] += g * psi0_q for q < n0 (rows -1 skipped).
void adj_add_psi0(int64_t n0, const int32_t* p0, const double* amps0,
                  const double* g, double2* lam, int* err, hipStream_t s);
// out[row of key i in the table] = in[i] for the n keys of `keys_in`.
void adj_permute(const DevModel& m, int Wi, const uint64_t* keys_in,
                 int64_t n, const uint64_t* table, uint64_t mask,
                 const uint64_t* keys_tab, const double2* in, double2* out,
                 int* err, hipStream_t s);
void adj_zero(double2* v, int64_t n, hipStream_t s);

}  // namespace paces
