/*
 * paces.h -- C ABI of the MI355X co-evolving-subspace propagator.
 *
 * One time step of the method (paper: Sec. "Formal operator representation
 * and notes on parallelization") maps a sparse state psi on a set S of basis
 * states of a single-exciton Holstein lattice (Eqs. (tb), (holstein)) to
 *
 *     M    = { n in S : |psi_n| >= theta }             truncation
 *     S'   = { states within graph distance k of M }   Eqs. (def_neighbor_k),
 *                                                      (H_eff)
 *     phi  = psi restricted to S'                       post-adaptation
 *                                                      detruncation
 *     psi' = exp(-i H_S' dt) phi                        exact in S'
 *
 * and records observables.  Every stage runs in hand-written HIP kernels on
 * the GPU; nothing in this library falls back to the CPU.
 *
 * Conventions
 *  - Every function returns paces_status; PACES_OK is 0.  The message of
 *    the last failure on the calling thread is paces_last_error().
 *  - Host arrays passed in are copied before the call returns; the library
 *    keeps no caller pointer.  Host output arrays are sized by the caller.
 *  - hip_stream is a hipStream_t passed as void* (NULL = default stream).
 *    All device work of a sim is ordered on the stream given to each call.
 *  - Keys at the boundary are canonical: W uint64 words per basis state,
 *    word 0 most significant, fields most significant first
 *    n_{0,0} .. n_{0,V-1}, n_{1,0}, .., n_{N-1,V-1}, then the exciton site
 *    j; widths ceil(log2(cutoff+1)) per mode and max(1, ceil(log2 N)) for j
 *    (App. "Lossless bit-level compression of state information").
 *  - Amplitudes at the boundary are interleaved FP64 (re, im) pairs; in
 *    FP32 mode they are widened on export and rounded on import.
 *  - Row order of states returned by the library is unspecified and may
 *    differ between runs (hash-table races decide it); compare sets after
 *    sorting.  Amplitudes per basis state are reproduced bit for bit with
 *    the series propagator; the Krylov propagator's inner products are
 *    sums over rows in that order, so its amplitudes repeat only within
 *    rounding.
 *  - Device errors (hash-table or capacity overflow, non-finite norm,
 *    series longer than k_max_terms) are latched and reported by the next
 *    call that synchronises; the sim then refuses further steps
 *    (PACES_E_STATE) until paces_set_state.
 *  - A sim is not thread-safe; distinct sims are independent.
 *
 * Batched disorder
 *  A model may carry R independent realizations of the site energies
 *  (paper: Sec. "Application to vibronic nanoaggregates", disorder
 *  averages).  One sim then propagates R states in one set: every row
 *  belongs to one realization, rows of different realizations never
 *  couple, and each realization gets its own Gershgorin interval,
 *  Chebyshev series and observation record.  The results of realization r
 *  equal those of a sim of that realization alone (same sets, amplitudes
 *  within rounding of the reductions).  Functions that return or accept
 *  rows pair them with realization indices.
 */
#ifndef PACES_H
#define PACES_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PACES_ABI_VERSION 12

typedef enum {
  PACES_OK = 0,
  PACES_E_ARG = 1,         /* invalid argument (synchronous)              */
  PACES_E_OOM = 2,         /* device allocation failed                    */
  PACES_E_CAPACITY = 3,    /* state or table capacity exceeded            */
  PACES_E_NONFINITE = 4,   /* non-finite norm after propagation           */
  PACES_E_PROPAGATOR = 5,  /* series needs more than k_max_terms terms    */
  PACES_E_HIP = 6,         /* HIP runtime error                           */
  PACES_E_STATE = 7,       /* sim is in an error state                    */
  PACES_E_UNSUPPORTED = 8  /* valid request this build does not support   */
} paces_status;

const char* paces_last_error(void);
int32_t paces_abi_version(void);
/* theta_m of the truncated Taylor propagator (taylor_order): the largest
 * theta for which the degree-m series of exp on ||A|| <= theta has relative
 * backward error at most 2^-53; m in 1..55, else -1.  Host only. */
double paces_taylor_theta(int32_t m);

typedef struct paces_model paces_model; /* immutable after load */
typedef struct paces_sim paces_sim;     /* owns the device state of a run */

/* Holstein lattice, Eq. (holstein) on 1D/2D/3D nearest-neighbour lattices
 * with V modes per site (Sec. "Application to vibronic nanoaggregates"). */
typedef struct {
  int32_t ndim;        /* 1, 2 or 3                                        */
  int32_t extent[3];   /* sites per axis; unused axes 1                    */
  int32_t periodic[3]; /* wrap the axis; a periodic extent must be >= 3    */
  int32_t n_modes;     /* V, 1..4                                          */
  int32_t cutoff[4];   /* max occupation per mode, 1..254                  */
  double omega[4];     /* mode frequencies                                 */
  double g[4];         /* exciton-phonon couplings                         */
  double J[3];         /* hopping per axis                                 */
  int32_t n_real;      /* R realizations of eps, 1..256 (0 = 1);
                          R * (N + 3) <= 8064                              */
  const double* eps;   /* [R][N] site energies (host, copied);
                          NULL = zeros                                     */
} paces_model_desc;

typedef struct {
  double dt;           /* time step                                        */
  int32_t k;           /* neighbour order of steps after the first (m)     */
  int32_t k_init;      /* neighbour order of the first step (m_init)       */
  double theta;        /* keep a row iff |c| >= theta, tested as
                          re*re + im*im >= theta*theta in FP64, no FMA    */
  int64_t cap_states;  /* initial row capacity hint (0 = automatic)        */
  int32_t precision;   /* 64: complex128 amplitudes; 32: complex64 with
                          FP64 scalars and reductions                      */
  double tol;          /* series tail tolerance, 0 = 1e-16                 */
  int32_t k_max_terms; /* limit on series terms, 0 = 128                   */
  uint32_t obs_mask;   /* PACES_OBS_* bits; 0 = all                        */
  int64_t max_states;  /* cap on |S| per realization, 0 = none.  When the
                          new set of a realization would exceed it, its
                          selection M is cut to the q heaviest rows
                          (weight descending, then a splitmix64 hash of
                          the canonical key, then the key), q =
                          floor(cap |M_prev| / |S_prev|) from its last
                          record (floor(cap / (D+1)) without one), and
                          while the set still exceeds the cap
                          q <- floor(9 min(q, |M|) cap / (10 |S|))       */
  int64_t q_nom;       /* fixed-size truncation (the paper's q_nom), 0 =
                          off: after the first step M is the q_nom
                          heaviest rows of each realization's set in the
                          same order as the state cap, and theta is not
                          used.  Exclusive with max_states.               */
  int32_t krylov_order;/* 0: Chebyshev series propagator.  p in 1..63:
                          Krylov (Lanczos) propagator of order p (paper:
                          App. "Series-based exponentiation compared to a
                          Lanczos algorithm"), psi' = V exp(-i T dt) V^dag
                          phi in span{phi, H phi, .., H^p phi}, built by
                          the three-term recurrence without
                          re-orthogonalisation; the basis stops early
                          when |w_j| <= 1e-11 |H v_{j-1}| (1e-6 in FP32).
                          Holds p extra vectors of the row capacity; the
                          record's K is the dimension used and E_min /
                          E_max the padded Gershgorin interval of T.  Not
                          with the adjoint entry points.                  */
  int32_t taylor_order;/* 0: off.  -1: truncated Taylor series (paper: App.
                          "The action of the exponential of a sparse
                          matrix"), psi' = exp(-i b dt) [T_m(A/s)]^s phi,
                          A = -i (H - b) dt, b the centre of the padded
                          Gershgorin interval; degree m and substeps s
                          minimise m s subject to s >= a dt / theta_m (a
                          the half width, theta_m the degree-m backward
                          error threshold at 2^-53, paces_taylor_theta)
                          (Al-Mohy & Higham 2011).  N in 1..60: N terms in
                          one step (App. "An effective Hilbert space up to
                          neighbor order m = 2 is not equivalent to a
                          second-order Taylor expansion"; not unitary).
                          The record's K is m s.  Holds three extra vectors
                          of the row capacity.  Exclusive with
                          krylov_order; not with the adjoint entry points. */
} paces_run_params;

#define PACES_OBS_ENERGY 1u /* <psi|H_eff|psi> per step (one extra SpMV
                               only when the series has a single term)    */

typedef struct {
  double t, norm2, energy, autocorr_re, autocorr_im, mass_step, mass_total;
  int64_t n_S, n_M;
  int32_t K;           /* Chebyshev terms used by the step (Krylov
                          propagator: dimension of the Krylov space)       */
  double E_min, E_max; /* padded Gershgorin bounds of H_eff (Krylov: of
                          the tridiagonal T)                               */
  const double* pop;   /* [N] exciton populations; owned by the sim,
                          valid until the next call on it                  */
} paces_obs;

/* Number of doubles per record of paces_series (one record per
 * realization and step): 12 scalars
 * (t, norm2, energy, a_re, a_im, mass_step, mass_total, n_S, n_M, K,
 * E_min, E_max) followed by the N populations. */
int32_t paces_record_doubles(const paces_model* m);

/* Device memory of the library (set tables, vectors, hash table,
 * records) from the caller's allocator: alloc(bytes, stream, user) returns
 * device memory or NULL, release(ptr, stream, user) frees it; stream is
 * passed as NULL (the library synchronises its stream before it frees).
 * Both NULL restores hipMalloc / hipFree.  Applies to later allocations;
 * every block goes back to the allocator that made it, so the functions
 * must stay valid while blocks they made are alive. */
paces_status paces_set_allocator(void* (*alloc)(size_t bytes, void* stream,
                                                void* user),
                                 void (*release)(void* ptr, void* stream,
                                                 void* user),
                                 void* user);

/* Load a model: validates the description and builds the neighbour table,
 * the key layout and the g*sqrt(n) table on the host.  The tables are copied
 * to the current device by the first paces_init_state on the model, so the
 * host codec below works without a GPU. */
paces_status paces_load_model(const paces_model_desc* desc, paces_model** out);
paces_status paces_free_model(paces_model* m);
/* N sites, W words per key, D slots per row, B key bits. */
paces_status paces_model_info(const paces_model* m, int32_t* N, int32_t* W,
                              int32_t* D, int32_t* B);
/* W: 64-bit words per canonical key. */
paces_status paces_model_key_words(const paces_model* m, int32_t* W);
/* Host codec: exc[n], occ[n*N*V] (site-major) <-> keys[n*W]. */
paces_status paces_pack_keys(const paces_model* m, int64_t n,
                             const int32_t* exc, const uint16_t* occ,
                             uint64_t* keys);
paces_status paces_unpack_keys(const paces_model* m, int64_t n,
                               const uint64_t* keys, int32_t* exc,
                               uint16_t* occ);

/* Create a sim from an initial state given as an uncompressed occupation
 * table (the paper's table A) plus coefficients coef[2*n] (re, im).
 * Duplicate states are an error.  The first step uses every input state
 * as M and grows it with k_init.  With R realizations every realization
 * starts from this state (R*n rows). */
paces_status paces_init_state(const paces_model* m, const paces_run_params* p,
                              int64_t n, const int32_t* exc,
                              const uint16_t* occ, const double* coef,
                              void* hip_stream, paces_sim** out);
paces_status paces_free_sim(paces_sim* s);

/* Advance n_steps time steps on the stream.  Each step ends with one host
 * synchronisation: its last kernel mirrors the step's counts and error
 * latch into mapped host memory, and the host reads them because a row,
 * table or state-cap overflow is resolved on the host (more room, or a cut
 * selection) and the step repeated before the next one is enqueued.  The
 * call returns when the last step is complete; the records stay on the
 * device (paces_series copies them).  With the
 * environment variable PACES_LOG set to a file name (1: paces_log.csv),
 * every step's records are appended to it as CSV lines
 * "step,realization,<12 fields>,<N populations>". */
paces_status paces_step(paces_sim* s, int64_t n_steps, void* hip_stream);
/* One stage of a step, for callers that drive or inspect the stages
 * separately (paper: Sec. "Formal operator representation and notes on
 * parallelization" splits the step into these operations).  stage is
 * PACES_STAGE_SELECT .. PACES_STAGE_OBSERVE; a step is the six stages in
 * that order, and running them gives exactly what paces_step(s, 1) gives
 * (same sets, amplitudes and record).  SELECT starts a new staged step
 * (abandoning one in progress); any other stage out of order is
 * PACES_E_STATE.  The current state is replaced only when OBSERVE completes,
 * so an abandoned staged step leaves it intact; paces_step and
 * paces_set_state abandon it too.
 *   SELECT     M from the current state (threshold, state cap or q_nom)
 *   EXPAND     the new set: k rounds of neighbour generation merged in the
 *              hash table, the ELL columns of H_eff; synchronises, and
 *              repeats SELECT + EXPAND with more room (or a cut selection
 *              under a state cap) until the set fits
 *   TRANSFER   phi = psi restricted to the new set, the discarded weight
 *   BUILD      Gershgorin bounds and the propagator's coefficients or plan
 *   PROPAGATE  psi' = exp(-i H_eff dt) phi; synchronises first to size the
 *              series from the coefficients
 *   OBSERVE    observables into the record; synchronises and completes the
 *              step
 * With theta = 0 and k = 0, a state loaded by paces_set_state is propagated
 * on exactly its own set (M = S, no new states): exp(-i H_S dt) applied to
 * the given amplitudes.  Device errors are returned by the stage that
 * synchronises after them. */
paces_status paces_run_stage(paces_sim* s, int32_t stage, void* hip_stream);

/* Propagation of a state given on its own set, without a sim: psi =
 * exp(-i H_S dt) phi, H_S the Hamiltonian of Eq. (holstein) restricted to
 * the n states of dev_keys (Eq. (H_eff) with S the given set), computed as
 * a step's PROPAGATE stage does: ELL columns by hash lookup, padded
 * Gershgorin bounds, Chebyshev series by Clenshaw's recurrence with the
 * step's default tail tolerance (App. "The action of the exponential of a
 * sparse matrix" for the series approach).
 *   dev_keys  device uint64 [n][W], canonical keys (as paces_pack_keys
 *             makes them); distinct, every field in range
 *   dev_phi   device complex128 [n] (interleaved re, im), row order of
 *             dev_keys
 *   dev_psi   device complex128 [n] output, same order; must not alias
 *             dev_phi
 * Models with one realization only (else PACES_E_UNSUPPORTED).  A key out
 * of range or repeated is found on the device and returns PACES_E_ARG.
 * Work memory (about 60-120 bytes per row) comes from the library's
 * allocator for the call.  Runs on hip_stream and synchronises it before
 * returning. */
paces_status paces_expmv(const paces_model* m, int64_t n, const void* dev_keys,
                         const void* dev_phi, double dt, void* dev_psi,
                         void* hip_stream);

/* paces_expmv without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, result and checks as
 * paces_expmv; the work memory is a static device array of 64 MiB
 * (67108864 bytes) per GPU, held until the process ends, instead of the
 * allocator.  A set whose work memory (64-128 bytes per row plus a hash
 * table of at least two slots of 8 bytes per row; about 600 000 rows of
 * ring16 keys) exceeds it returns PACES_E_CAPACITY before any device work.
 * Calls on one GPU share that array: calls that overlap in time on the same
 * GPU (other host threads, other streams) race and give wrong results;
 * serialise them.  Every call clears what it reads back (control block,
 * error latch, hash table) itself.  Runs on hip_stream and synchronises it
 * before returning. */
paces_status paces_expmv_static(const paces_model* m, int64_t n,
                                const void* dev_keys, const void* dev_phi,
                                double dt, void* dev_psi, void* hip_stream);

/* Piecewise-constant H(t): later steps of the sim use model m, which must
 * have the sim's shape (lattice, modes, cutoffs, realizations); only J,
 * g, omega and eps may differ.  The caller keeps m alive while the sim
 * uses it.  Drops a recorded adjoint run. */
paces_status paces_set_model(paces_sim* s, const paces_model* m);

/* Latest observation of one realization (0..R-1); synchronises the
 * stream.  n_S and n_M of a record count the rows of that realization. */
paces_status paces_observe(paces_sim* s, int32_t realization, paces_obs* out,
                           void* hip_stream);
/* Number of recorded steps. */
paces_status paces_num_records(paces_sim* s, int64_t* n);
/* Copy the records of steps first..first+n-1 to host
 * out[n][R][paces_record_doubles]; synchronises. */
paces_status paces_series(paces_sim* s, int64_t first, int64_t n,
                          double* out, void* hip_stream);

/* One field (0 .. paces_record_doubles - 1) of the records of steps
 * first..first+n-1 into device memory dev_out[n][R] (f64), asynchronous
 * on the stream (e.g. straight into a torch tensor). */
paces_status paces_series_field(paces_sim* s, int32_t field, void* dev_out,
                                int64_t first, int64_t n, void* hip_stream);

/* Current state: *n states in row order (rows that in-place steps left
 * empty are skipped); keys[n*W], amps[2n], real[n] the realization of
 * each state (host; each may be NULL, all NULL to query the size).
 * Synchronises. */
paces_status paces_get_state(paces_sim* s, int64_t* n, uint64_t* keys,
                             double* amps, int32_t* real, void* hip_stream);
/* Replace the current state (time t); real[n] gives each row's realization
 * (NULL: realization 0).  A (realization, key) pair may appear once.  The
 * next step selects from it with theta and grows M with k. */
paces_status paces_set_state(paces_sim* s, int64_t n, const uint64_t* keys,
                             const double* amps, const int32_t* real, double t,
                             void* hip_stream);

typedef enum {
  PACES_SET_M = 0,        /* selected states of the last step            */
  PACES_SET_S = 1,        /* current set                                 */
  PACES_SET_FRONTIER = 2  /* states first reached in round r            */
} paces_set;
/* Keys (and realizations, real may be NULL) of a set of the last step
 * (keys and real NULL: size query).  Synchronises. */
paces_status paces_get_set(paces_sim* s, int32_t which, int32_t round,
                           int64_t* n, uint64_t* keys, int32_t* real,
                           void* hip_stream);
/* phi of the last step (psi projected onto the new set), rows in the order
 * of paces_get_set(PACES_SET_S); amps[2*nS].  Synchronises. */
paces_status paces_get_phi(paces_sim* s, double* amps, void* hip_stream);

/* Timing with HIP events on the step's stream.  Level 1: events around
 * every stage launch group plus every timed kernel (each Clenshaw launch,
 * each Lanczos SpMV but the last), whose events their own dispatch
 * records; level 2: one timed kernel per step (launch index 1: a middle
 * Clenshaw term whenever K >= 4, the second Lanczos SpMV).  Every event
 * costs the stream a few microseconds of idle time, hence level 2 for
 * timing whole runs.  Level 0: off.  Profiling turns graph replay off. */
typedef enum {
  PACES_STAGE_SELECT = 0,
  PACES_STAGE_EXPAND = 1,   /* expansion rounds incl. the lookup pass     */
  PACES_STAGE_TRANSFER = 2,
  PACES_STAGE_BUILD = 3,    /* bounds + coefficients                      */
  PACES_STAGE_PROPAGATE = 4,/* all Clenshaw launches                      */
  PACES_STAGE_OBSERVE = 5,
  PACES_STAGE_TERM = 6,     /* middle Clenshaw launches only              */
  PACES_STAGE_KRYLOV = 7,   /* Lanczos SpMV launches except the last      */
  PACES_NUM_STAGES = 8
} paces_stage;
typedef struct {
  double ms[PACES_NUM_STAGES];      /* summed event time                  */
  int64_t launches[PACES_NUM_STAGES];
  double term_bytes;                /* algorithmic bytes of the timed
                                       middle Clenshaw launches          */
  double krylov_bytes;              /* algorithmic bytes of the timed
                                       Lanczos SpMV launches             */
  double rows_steps;                /* sum over steps of |S|              */
} paces_profile;
paces_status paces_profile_enable(paces_sim* s, int32_t level);
/* Resolves pending events (synchronises) and returns the totals. */
paces_status paces_profile_get(paces_sim* s, paces_profile* out,
                               void* hip_stream);
paces_status paces_profile_reset(paces_sim* s);
/* Enqueue one empty kernel dispatch (k_mark) on the stream: in kernel
 * traces and hardware-counter runs, where event markers are not recorded,
 * a pair of marks brackets a region of interest in dispatch order.  tag is
 * not recorded.  Asynchronous. */
paces_status paces_profile_mark(int32_t tag, void* hip_stream);

/* Form (3): adjoint gradient.  For a real loss L of the autocorrelation
 * a_s = <psi0|psi_s>, s = 0..n (s = 0 the initial state), the gradient
 * dL/dtheta with theta = (J per axis, g per mode, omega per mode, eps per
 * site), paces_num_params entries in that order.  The sets of the recorded
 * run are held fixed (each step is then linear in psi); the gradient is
 * the discrete adjoint of that frozen-set propagation.  Needs one
 * realization, FP64 amplitudes, the series propagator and every J_axis,
 * g_nu nonzero (so that the ELL holds every lattice edge); otherwise
 * PACES_E_UNSUPPORTED. */
int32_t paces_num_params(const paces_model* m);
/* Run n_steps steps from a new sim (no step taken yet), keeping the
 * selected set of every step and the state every ckpt_every steps (device
 * memory: about |M| key words per step plus one state per checkpoint).
 * a[2*(n_steps+1)]: a_s as (re, im), host, may be NULL.  Synchronises. */
paces_status paces_adjoint_forward(paces_sim* s, int64_t n_steps,
                                   int32_t ckpt_every, double* a,
                                   void* hip_stream);
/* As paces_adjoint_forward, with a_s written to device memory dev_a
 * (complex128 [n_steps + 1], interleaved re, im) on the stream, e.g. a
 * torch tensor; the host never sees the series.  Synchronises. */
paces_status paces_adjoint_forward_dev(paces_sim* s, int64_t n_steps,
                                       int32_t ckpt_every, void* dev_a,
                                       void* hip_stream);
/* Replay the recorded run on its frozen sets with model m (NULL: the
 * sim's own; otherwise a model of the same shape, e.g. with perturbed
 * parameters) and return a[2*(n+1)].  The sim's state is left as after the
 * forward run.  Synchronises. */
paces_status paces_adjoint_replay(paces_sim* s, const paces_model* m,
                                  double* a, void* hip_stream);
/* gbar[2*(n+1)]: dL/d conj(a_s) as (re, im) (half of what torch passes
 * as the gradient of a complex output); grad[paces_num_params]: dL/dtheta.
 * Replays each checkpoint segment once, then sweeps it in reverse; the
 * Frechet derivative of each step's exponential is integrated with
 * Gauss-Legendre nodes.  The sim's state is left as after the forward run.
 * Synchronises. */
paces_status paces_adjoint_backward(paces_sim* s, const double* gbar,
                                    double* grad, void* hip_stream);

/* As paces_adjoint_backward, with gbar (complex128 [n + 1]) read from and
 * the gradient (f64 [paces_num_params]) written to device memory.
 * Synchronises. */
paces_status paces_adjoint_backward_dev(paces_sim* s, const void* dev_gbar,
                                        void* dev_grad, void* hip_stream);

/* Launch tuning.  Results do not depend on it: per-key amplitudes, sets
 * and counts are identical for every setting (sums only to rounding of
 * their reduction order). */
typedef struct {
  int32_t graph;       /* 1: capture each step's launch sequence once as a
                          HIP graph and replay it (graphs are keyed by
                          bucketed sizes and rebuilt when buffers move);
                          ignored while profiling is enabled              */
  int32_t table_shift; /* hash table probed over >= est * 2^shift entries
                          (0..3), est = 1.5 x the current set: a smaller
                          table stays in the last-level cache, a larger
                          one shortens probe chains                       */
  int32_t term_rows;   /* rows per thread of the Clenshaw grid: 1,2,4,8  */
  int32_t warm;        /* 1: a step expands from the previous step's graph
                          (its ELL columns and hash table) in place where
                          one is there, and from scratch again once the
                          states placed into holes since the last such
                          step reach a tenth of the set (which restores
                          the breadth-first row order the SpMV gathers
                          favour); 2: in place without that relayout;
                          0: every step expands from scratch             */
} paces_tuning;
/* Default {0, 1, 1, 1}. */
paces_status paces_get_tuning(paces_sim* s, paces_tuning* out);
/* May reallocate the hash table (synchronises). */
paces_status paces_set_tuning(paces_sim* s, const paces_tuning* t,
                              void* hip_stream);
/* Time 1 + steps trial steps from the current state for each setting of
 * {graph 0/1} x {table_shift 0, 1, 2} x {term_rows 1, 2, 4}, keep the fastest,
 * and restore the state as it was (records of the trials are discarded;
 * the sets of the last step are no longer available).  steps 1..64. */
paces_status paces_autotune(paces_sim* s, int32_t steps, paces_tuning* chosen,
                            void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif
