/*
 * paces_oracle.h -- plain FP64 CPU reference of one co-evolving-subspace
 * step for single-exciton Holstein lattices.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that tests, the smoke
 * check and the CPU-baseline leg of the benchmark can compare the GPU path
 * against an obviously correct implementation.  The product path never
 * links, loads or calls it, and it shares no source, header, table or
 * helper with the GPU library.
 *
 * What it computes (paper: Sec. "Co-evolving subspaces", Eqs. (tb),
 * (holstein), (def_neighbor_k), (H_eff); Sec. "Truncation & post-adaptation
 * detruncation"; Sec. "Generating the effective Hamiltonian from the
 * effective Hilbert space"; Sec. "Formal operator representation and notes on
 * parallelization"; App. "The action of the exponential of a sparse matrix";
 * App. "Lossless bit-level compression of state information"):
 *
 *   step:  M  = rows of S whose amplitude clears the threshold
 *          S' = all basis states within graph distance k of M
 *          phi = psi projected onto S'   (post-adaptation detruncation)
 *          psi' = exp(-i H_S' dt) phi    (H restricted to S')
 *
 * All functions return 0 on success and a nonzero code on error; the
 * message is available from orc_last_error().
 */
#ifndef PACES_ORACLE_H
#define PACES_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t ndim;          /* 1, 2 or 3 lattice axes                          */
  int32_t extent[3];     /* sites along each axis (unused axes: 1)          */
  int32_t periodic[3];   /* 1 = wrap; a periodic extent must be >= 3        */
  int32_t n_modes;       /* vibrational modes per site, 1..4                */
  int32_t cutoff[4];     /* max occupation per mode (local dim = cutoff+1)  */
  double omega[4];       /* mode frequency, uniform over sites              */
  double g[4];           /* exciton-phonon coupling, uniform over sites     */
  double J[3];           /* hopping per axis                                */
  const double* eps;     /* [N] site energies (copied)                      */
} orc_model_desc;

typedef struct {
  double dt;             /* time step                                       */
  int32_t k;             /* neighbour order for steps after the first       */
  int32_t k_init;        /* neighbour order of the first step               */
  double theta;          /* keep a row iff |c| >= theta                     */
  int32_t max_terms;     /* error when the series needs more terms          */
  int64_t max_states;    /* cap on |S|: when the ball of M exceeds it, M is
                            cut to its heaviest rows (see the source); 0 =
                            no cap                                          */
  int64_t q_nom;         /* > 0: after the first step M is the q_nom
                            heaviest rows (same order as the cap) instead
                            of the threshold; exclusive with max_states     */
  int32_t krylov_order;  /* 0: series propagator; p in 1..63: Lanczos
                            propagator in the (p+1)-dimensional Krylov
                            space (see orc_lanczos)                          */
  int32_t taylor_order;  /* 0: off; -1: truncated Taylor series with the
                            degree and substeps of Al-Mohy & Higham; N in
                            1..60: N terms in one step (see orc_taylor);
                            exclusive with krylov_order                      */
} orc_params;

/* Observables recorded after each step (field order of orc_sim_obs). */
enum {
  ORC_OBS_T = 0, ORC_OBS_NORM2, ORC_OBS_ENERGY, ORC_OBS_A_RE, ORC_OBS_A_IM,
  ORC_OBS_MASS_STEP, ORC_OBS_MASS_TOTAL, ORC_OBS_NS, ORC_OBS_NM,
  ORC_OBS_TERMS, ORC_OBS_EMIN, ORC_OBS_EMAX, ORC_OBS_NFIELDS
};

/* Sets kept from the last step (orc_sim_get_set). */
enum { ORC_SET_M = 0, ORC_SET_S = 1, ORC_SET_FRONTIER = 2 };

const char* orc_last_error(void);

/* Generic bit-field packer of the compression appendix: fields given most
 * significant first, packed without gaps and right-aligned in W 64-bit
 * words, word 0 most significant. */
/* Threads of the row loops (timing only; results do not depend on it). */
int orc_set_threads(int32_t n);
int32_t orc_threads(void);

int orc_pack_fields(int32_t nfields, const int32_t* widths,
                    const uint64_t* values, int32_t W, uint64_t* out);

int orc_model_create(const orc_model_desc* d, void** out);
void orc_model_destroy(void* m);
/* N sites, W key words, D slots per row, B key bits. */
int orc_model_info(const void* m, int32_t* N, int32_t* W, int32_t* D,
                   int32_t* B);
/* exc[n] exciton sites, occ[n*N*V] occupations (site-major) -> keys[n*W]. */
int orc_pack(const void* m, int64_t n, const int32_t* exc,
             const uint16_t* occ, uint64_t* keys);
int orc_unpack(const void* m, int64_t n, const uint64_t* keys, int32_t* exc,
               uint16_t* occ);
/* Matrix elements of H between basis states: for each key, its D slot
 * neighbours (keys_out[n*D*W]; a slot that does not exist is flagged 0 in
 * exists[n*D]) and values vals[n*D], plus the diagonal diag[n]. */
int orc_neighbors(const void* m, int64_t n, const uint64_t* keys,
                  uint64_t* keys_out, uint8_t* exists, double* vals,
                  double* diag);

int orc_sim_create(const void* m, const orc_params* p, int64_t n,
                   const int32_t* exc, const uint16_t* occ,
                   const double* coef, void** out);
void orc_sim_destroy(void* s);
int orc_sim_step(void* s, int64_t n_steps);
/* Later steps use model m (same lattice, modes and cutoffs): a
 * piecewise-constant Hamiltonian.  The caller keeps m alive. */
int orc_sim_set_model(void* s, const void* m);
/* Replace the current state: sorted or not, duplicates are an error.  The
 * next step selects from it with the threshold and neighbour order k. */
int orc_sim_set_state(void* s, int64_t n, const uint64_t* keys,
                      const double* amps, double t);
/* Counts |S|, |M| of the step that led to the loaded state, used by the
 * state cap's q rule as if that step had been run here. */
int orc_sim_set_prev_counts(void* sim, int64_t nS, int64_t nM);
int orc_sim_size(const void* s, int64_t* nS);
/* Current state as sorted keys and interleaved (re, im) amplitudes. */
int orc_sim_get_state(const void* s, uint64_t* keys, double* amps);
/* Projected vector phi of the last step, aligned with the sorted S. */
int orc_sim_get_phi(const void* s, double* amps);
/* Sets of the last step.  Pass keys = NULL to query the size. */
int orc_sim_get_set(const void* s, int32_t which, int32_t round, int64_t* n,
                    uint64_t* keys);
int orc_sim_num_obs(const void* s, int64_t* n);
/* fields[ORC_OBS_NFIELDS] and pop[N] of observation i (0 = first step). */
int orc_sim_obs(const void* s, int64_t i, double* fields, double* pop);
/* CSR of the last step's effective Hamiltonian over the sorted S.
 * Pass NULL arrays to query nnz. */
int orc_sim_csr(const void* s, int64_t* nrows, int64_t* nnz, int64_t* rowptr,
                int64_t* cols, double* vals);

/* Action of exp(-i H dt) on a vector, for an arbitrary CSR matrix H given by
 * the caller (used to pin the series against a dense exponential). */
int orc_expmv(int64_t n, const int64_t* rowptr, const int64_t* cols,
              const double* vals, double dt, double emin, double emax,
              int32_t max_terms, const double* v_in, double* v_out,
              int32_t* terms);

/* Krylov (Lanczos) propagator of order p for a caller-given CSR H:
 * v_out ~ V exp(-i T dt) V^dag v_in in span{v, Hv, .., H^p v} (App.
 * "Series-based exponentiation compared to a Lanczos algorithm").
 * basis[dim][n] receives the orthonormal Lanczos vectors (interleaved
 * complex; room for p+1 vectors), alpha[dim] the diagonal of T,
 * beta[dim] the norms (beta[0] = |v_in|, beta[j] couples v_{j-1} and v_j),
 * dim the dimension reached (smaller than p+1 after a breakdown) and
 * e_range[2] the padded Gershgorin interval of T.  Output pointers other
 * than v_out may be NULL. */
int orc_lanczos(int64_t n, const int64_t* rowptr, const int64_t* cols,
                const double* vals, double dt, int32_t order,
                const double* v_in, double* v_out, double* basis,
                double* alpha, double* beta, int32_t* dim, double* e_range);

/* Truncated Taylor propagator (the source states the method): the
 * backward-error threshold theta_m of the degree-m series at unit
 * roundoff 2^-53 (m in 1..55, else -1), the (degree, substeps) choice for
 * a given bound of ||A||, and the propagator itself for a caller-given CSR
 * H with Gershgorin interval [emin, emax]: order -1 chooses (m, s), order
 * N > 0 takes N terms in one step; mvs = matrix-vector products used. */
double orc_taylor_theta(int32_t m);
int orc_taylor_select(double norm, int32_t* m, int32_t* s);
int orc_taylor(int64_t n, const int64_t* rowptr, const int64_t* cols,
               const double* vals, double dt, double emin, double emax,
               int32_t order, const double* v_in, double* v_out,
               int32_t* mvs);

/* Adjoint gradient on a frozen sequence of sets (Form (3)).
 * orc_frozen_record runs n_steps ordinary steps from the initial state and
 * keeps S_0 (the support of psi0) and the set of every step.  With those
 * sets held fixed, orc_frozen_eval replays the run with any model of the
 * same shape and returns a[s] = <psi0|psi_s>, s = 0..n_steps, interleaved
 * (re, im); orc_frozen_grad also returns, for gbar[s] = dL/d conj(a_s) of a
 * real loss L, grad[p] = dL/dtheta_p with theta = (J per axis, g per mode,
 * omega per mode, eps per site). */
int orc_frozen_record(const void* m, const orc_params* p, int64_t n,
                      const int32_t* exc, const uint16_t* occ,
                      const double* coef, int64_t n_steps, void** out);
void orc_frozen_destroy(void* f);
/* sizes[n_steps + 1]: |S_0| .. |S_n| (may be NULL). */
int orc_frozen_info(const void* f, int64_t* n_steps, int32_t* n_params,
                    int64_t* sizes);
/* Sorted keys of S_step. */
int orc_frozen_get_set(const void* f, int64_t step, uint64_t* keys);
int orc_frozen_eval(const void* f, const void* m, double* a);
int orc_frozen_grad(const void* f, const void* m, const double* gbar,
                    double* a, double* grad);

#ifdef __cplusplus
}
#endif
#endif
