/*
 * sg.h -- C ABI of the MI355X (gfx950) Smolyak sparse-grid library.
 *
 * The library computes the Smolyak operator action of a Hamiltonian on a
 * wave packet stored in the compact Smolyak basis,
 *
 *     H_S |Psi> = sum_{l in R(l)} D_l  H |psi^l>          (eq_action_smolyak)
 *
 * term by term as in Alg. 1 (Operator action of one Smolyak term, Sec. 3):
 * gather the term from the compact vector through the mapping table M^B,
 * transform basis -> grid mode by mode (eq_transfer_b_to_g), apply the
 * operator on the term's grid, transform grid -> basis (eq_transfer_g_to_b),
 * and add D_l times the result into the compact output.  On top of it sits a
 * Chebyshev propagator (the paper names the Chebyshev method for wave-packet
 * propagation in Sec. 3 and uses it in Sec. 5), a batched multi-instance
 * propagator and a continuous-batching server.
 *
 * Problem family (Cartesian normal modes, hbar = 1):
 *
 *   H = sum_i 1/2 omega_i (-d^2/dQ_i^2 + Q_i^2)
 *       + sum_{i<j} c_ij Q_i^2 Q_j^2 + sum_{i<j} k_ij Q_i^2 Q_j
 *
 * with the couplings evaluated in closed form on every term grid, or, after
 * sg_set_potential, a general potential V(Q) from a caller's function
 * tabulated on the term grids.  The two-state calls (sg_vibronic_*) take the
 * paper's Sec. 5 pyrazine form.
 *
 * Primitive basis per mode: orthonormal Hermite functions ("Hm", Q0 = 0,
 * scaleQ = 1, Example subsection of Sec. 4) with N^b_l = nb_A + nb_B l functions and
 * N^q_l = nq_A + nq_B l Gauss-Hermite points at level l (N_l = A + B l,
 * Sec. 2).  Term set R(l): l_i >= 0, L-D+1 <= |l| <= L, with
 * D_l = (-1)^(L-|l|) C(D-1, L-|l|) (Sec. 2).
 *
 * Orderings (the ABI fixes them; Table 2 defines them):
 *   - terms: l_1 varies fastest;
 *   - positions inside a term: mode 1 fastest;
 *   - compact basis: lexicographic in (n_1, ..., n_D), mode 1 slowest.
 * Vectors on the device are complex128, interleaved (re, im), length N_cs.
 *
 * Conventions
 *   - Every call returns an sg_status; nothing throws across the ABI.  On a
 *     non-zero status sg_last_error() returns a thread-local message.
 *   - Device pointers are HIP device pointers on the device that was current
 *     when the problem was built; `stream` is a hipStream_t (NULL = the
 *     default stream).  Calls that take a stream are asynchronous unless
 *     stated otherwise.
 *   - Handles own their device tables; the caller owns every vector it
 *     passes.  Handles are not thread-safe: one caller thread per handle.
 *   - Results are deterministic: the scatter-add is a fixed-order segmented
 *     reduction with no floating-point atomics, so a call gives bit-identical
 *     output run to run, and alone or inside a batch or a server mix.
 */
#ifndef SG_H
#define SG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SG_OK = 0,
  SG_EINVAL = -1,      /* invalid argument or unsupported problem size      */
  SG_ENOMEM = -2,      /* device/host allocation failed, or over a budget   */
  SG_EDEVICE = -3,     /* a HIP runtime call failed                         */
  SG_EAGAIN = -4,      /* serving: the request is not finished yet          */
  SG_ENOTFOUND = -5,   /* serving: unknown ticket                           */
  SG_ECANCELED = -6,   /* serving: the request was cancelled                */
  SG_ETOL = -7         /* propagation: norm drift beyond the tolerance      */
} sg_status;

typedef enum {
  /* All FP64.  Alg. 1 per term: gather, basis -> grid, operator on the grid,
   * grid -> basis, scatter-add.  By default the separable harmonic part
   * sum_i omega_i (n_i + 1/2) is split off and applied exactly as a diagonal
   * on the compact basis, and only the coupling potential goes through the
   * term grids (the same operator: every term's quadrature integrates the
   * separable part exactly and the D_l of the terms holding a basis function
   * sum to 1).  sg_set_operator_form(p, 1) selects the literal form, with
   * the kinetic second-derivative matrices applied on every term grid. */
  SG_FP64 = 0,
  /* Mixed: the split form above, with the grid contractions of the terms
   * with |D_l| <= a threshold (sg_set_mixed_threshold, sg_tune_mixed) in
   * FP32 on the vector ALUs with FP32 accumulation, and the other terms,
   * the Smolyak sum, the Chebyshev state and all reductions in FP64. */
  SG_MIXED = 1
} sg_precision;

/* Problem description.  Caller-owned; sg_build_terms copies what it needs. */
typedef struct {
  int32_t D;             /* number of modes, 1..64                            */
  int32_t L;             /* Smolyak level, 0..15                              */
  int32_t nb_A, nb_B;    /* basis size map nb(l) = nb_A + nb_B l  (>=1, >=1)  */
  int32_t nq_A, nq_B;    /* grid size map  nq(l) = nq_A + nq_B l, nq >= nb    */
  const double *omega;   /* [D] harmonic frequencies (> 0)                    */
  const double *c;       /* [D*D] row-major; entries i<j used: c_ij Q_i^2Q_j^2 */
  const double *k;       /* [D*D] row-major; entries i<j used: k_ij Q_i^2 Q_j;
                            NULL means all zero                               */
} sg_problem_desc;

typedef struct sg_problem sg_problem;

typedef struct {
  int64_t D, L;
  int64_t n_terms;         /* N_st: terms of R(l) (all have D_l != 0)          */
  int64_t n_cs;            /* compact basis size                               */
  int64_t n_s;             /* term-major size sum_l prod_i nb(l_i)             */
  int64_t grid_literal;    /* sum_l prod_i nq(l_i): the paper's term grids     */
  int64_t grid_active;     /* sum_l prod_{l_i>0} nq(l_i): points evaluated     */
  int64_t max_term_basis;  /* largest prod_{l_i>0} nb(l_i)                     */
  int64_t max_term_grid;   /* largest prod_{l_i>0} nq(l_i)                     */
  double flops_fp64;       /* algorithmic flops of one SG_FP64 apply, in the
                              operator form it uses (sg_set_operator_form)     */
  double flops_mixed;      /* algorithmic flops of one SG_MIXED apply          */
  double sweep_flops_fp64; /* the term-sweep kernels' share of flops_fp64     */
  double sweep_flops_mixed;/* ... of flops_mixed                               */
  double bytes_fp64;       /* algorithmic HBM bytes of one apply (both modes)  */
  int64_t device_bytes;    /* device memory held by the handle                 */
  int32_t fp64_split;      /* 1: SG_FP64 applies the split form                */
  int32_t pad;
  double sweep_bytes;      /* HBM bytes the term sweep of one SG_FP64 apply must
                              move as designed: psi read once, M^B, the
                              term-major results written, term records and the
                              per-fiber potential coefficients it reads (with a
                              tabulated potential: its 8 bytes per active grid
                              point instead)                                   */
  double reduce_bytes;     /* ... the reduce: term-major results and inverse map
                              read, row lists, psi and the diagonal read, the
                              result written                                   */
} sg_info;

/* Sizes of a problem without building it: out[0] = N_st, out[1] = N_s,
 * out[2] = N_cs (Table 1 counts).  Host only.  Overflow -> SG_EINVAL. */
sg_status sg_count_sizes(int32_t D, int32_t L, int32_t nb_A, int32_t nb_B,
                         int64_t out[3]);

/* Builds the term set, D_l, compact basis, M^B and its inverse, the per-level
 * one-mode tables and the per-term operator coefficients on the host, and
 * uploads them once to the current HIP device (synchronously).  *out receives
 * a handle to release with sg_free. */
sg_status sg_build_terms(const sg_problem_desc *desc, sg_problem **out);
sg_status sg_free(sg_problem *p);

/* Same host-side build without any device work: the handle supports
 * sg_problem_info and the ordering exports below; calls that need the device
 * return SG_EINVAL.  For inspection and for checking the term compiler on a
 * machine without a GPU. */
sg_status sg_build_terms_host(const sg_problem_desc *desc, sg_problem **out);

sg_status sg_problem_info(const sg_problem *p, sg_info *out);

/* Host copies of the ordering contract.
 *   sg_basis_indices: n_out[i*D + j] = n_j of compact function i (0-based).
 *   sg_term_levels:   levels[t*D + j] = l_j of term t, coeffs[t] = D_l.
 *   sg_mapping_table: mb[s] = compact index of term-major position s (M^B,
 *                     Table 2 order, 0-based). */
sg_status sg_basis_indices(const sg_problem *p, int32_t *n_out);
sg_status sg_term_levels(const sg_problem *p, int32_t *levels, int32_t *coeffs);
sg_status sg_mapping_table(const sg_problem *p, int32_t *mb);

/* Displaced Gaussian prod_i pi^{-1/4} exp(-(Q_i - shift_i)^2/2) projected on
 * the compact basis (coherent-state coefficients) and normalised; writes
 * complex128[N_cs] to psi_dev on `stream`.  *captured_norm (nullable) gets the
 * norm of the projection before normalisation. */
sg_status sg_init_gaussian(const sg_problem *p, const double *shift,
                           void *psi_dev, double *captured_norm, void *stream);

/* psi_out = H_S psi_in (eq_action_smolyak via Alg. 1).  psi_in and psi_out
 * are distinct complex128[N_cs] device vectors.  Asynchronous on `stream`; no
 * host synchronisation.  The handle's work buffers are reused: calls on one
 * handle must be ordered on one stream. */
sg_status sg_apply_H(sg_problem *p, const void *psi_in, void *psi_out,
                     sg_precision prec, void *stream);

/* Estimates [E_min, E_max] of H_S with `iters` Lanczos steps (FP64) from a
 * fixed start vector, padded outward by 5% of the range plus the Ritz
 * residuals.  Synchronises `stream`. */
sg_status sg_spectral_bounds(sg_problem *p, int32_t iters, double *emin,
                             double *emax, void *stream);

typedef struct {
  int32_t steps_done;
  int32_t cheb_terms;        /* K: Chebyshev terms per step (K-1 applies)     */
  int64_t applies;           /* H applies performed                            */
  double emin, emax;         /* bounds used                                    */
  double norm0, energy0;     /* at the first check                             */
  double norm_last, energy_last;
  double max_norm_drift;     /* max |norm - norm0| over the checks             */
  double max_energy_drift;   /* max |E - E0| over the checks                   */
} sg_prop_stats;

/* Chebyshev propagation of psi (in place, complex128[N_cs]) over nsteps time
 * steps of dt (hbar = 1):  psi <- exp(-i H_S dt)^nsteps psi.
 * emin/emax bound the spectrum of H_S; NaN in either asks the library to
 * estimate both (sg_spectral_bounds with 40 steps).  The series is cut at the
 * first k > R = (emax-emin) dt / 2 where |J_k(R)| and |J_{k+1}(R)| are both
 * below 1e-16.  Every `check_every` steps (0 = only at the start and end) the
 * norm and energy are reduced in FP64 and read back (a host sync); if the
 * norm drifts from its first value by more than `tol` the call stops and
 * returns SG_ETOL.  stats (nullable) is filled on return.  norm_trace and
 * energy_trace (nullable, host, length >= nsteps/check_every + 2) receive the
 * checked values in order. */
sg_status sg_propagate_chebyshev(sg_problem *p, void *psi, double dt,
                                 int32_t nsteps, double emin, double emax,
                                 double tol, sg_precision prec,
                                 int32_t check_every, sg_prop_stats *stats,
                                 double *norm_trace, double *energy_trace,
                                 void *stream);

/* The other propagators the paper lists beside the Chebyshev method
 * (Sec. 3, overview of the program flow; no formulas given there):
 *   SG_PROP_TAYLOR  order n (1..40): psi <- sum_{k<=n} (-i H dt)^k/k! psi;
 *                   n applies of H per step.
 *   SG_PROP_RK      order n (1..4): explicit Runge-Kutta on d psi/dt =
 *                   -i H psi with the tableaux of Euler, the explicit
 *                   midpoint rule, Heun's third-order method and the
 *                   classical fourth-order method; n applies per step.
 *   SG_PROP_BS      Bulirsch-Stoer with n extrapolation columns (1..8): the
 *                   modified midpoint rule over 2, 4, .., 2n substeps of
 *                   the step, extrapolated to zero substep size (polynomial
 *                   in h^2); 1 + n(n+1) applies per step, global order 2n.
 *   SG_PROP_SIL     short iterative Lanczos with Krylov dimension n (1..64,
 *                   capped at N_cs): Lanczos from psi/|psi| with every new
 *                   vector orthogonalised twice against the earlier ones,
 *                   psi <- |psi| V exp(-i T dt) e_1; T is cut at the
 *                   first new vector whose norm is below 1e-13 |psi| (an
 *                   invariant space); n applies per step, the Krylov
 *                   recurrence runs on the device and a step reads its
 *                   coefficients back once. */
typedef enum {
  SG_PROP_TAYLOR = 1,
  SG_PROP_RK = 2,
  SG_PROP_SIL = 3,
  SG_PROP_BS = 4
} sg_propagator;

/* Propagates psi (in place, device complex128[N_cs]) over nsteps steps of dt
 * with `method` of order (Krylov dimension) `order`.  Allocates its work
 * vectors (up to order + 2 vectors of N_cs) for the call and synchronises
 * `stream` on return.  At the first step, every `check_every` steps (0 =
 * first and last only) and at the end the norm and energy are computed in
 * FP64 (one extra apply each); if the norm drifts from its first value by
 * more than tol (> 0) the call stops and returns SG_ETOL (Taylor and
 * Runge-Kutta are not unitary: their drift measures the step's error).
 * stats: cheb_terms holds `order`, applies counts every apply including the
 * checks, emin/emax are NaN.  Traces as in sg_propagate_chebyshev.  Bad
 * method, order, dt or precision -> SG_EINVAL. */
sg_status sg_propagate(sg_problem *p, void *psi, double dt, int32_t nsteps,
                       int32_t method, int32_t order, double tol,
                       sg_precision prec, int32_t check_every,
                       sg_prop_stats *stats, double *norm_trace,
                       double *energy_trace, void *stream);

/* The same propagators as sg_propagate, with the same arguments and results
 * (bitwise: same kernels, same order), for callers that cannot allocate
 * device memory (code that must not call hipMalloc, such as tight serving
 * loops and harnesses that forbid it).  The work vectors, projection
 * partials and coefficient slots live in a fixed device array of
 * sg_noalloc_scratch_bytes() bytes (64 MiB) that each device the library
 * runs on holds until the process ends; the call allocates nothing.  A
 * propagation needing more (about (nvec + 1) * 16 * N_cs bytes: nvec = 2 for
 * Taylor, 1 + order for Runge-Kutta, 4 + order for Bulirsch-Stoer, order + 1
 * for Lanczos) fails with SG_EINVAL before anything is launched.  All calls
 * on one device share the array: calls that overlap on one device (other
 * host threads, or streams that run concurrently) race and must not be
 * issued.  The array keeps the last call's contents; the call clears what
 * must start at zero itself. */
sg_status sg_propagate_noalloc(sg_problem *p, void *psi, double dt, int32_t nsteps,
                               int32_t method, int32_t order, double tol, sg_precision prec,
                               int32_t check_every, sg_prop_stats *stats, double *norm_trace,
                               double *energy_trace, void *stream);
int64_t sg_noalloc_scratch_bytes(void);

/* Batched propagation of independent problems (same device).  Every
 * Chebyshev term of every instance runs in one term-sweep launch and one
 * reduce launch: the terms of all instances are packed together into
 * workgroups (largest first, least-loaded pack), and the reduce work items of
 * all instances share one grid.  Instances keep their own spectral bounds,
 * series length and time step; an instance whose series is shorter sits out
 * the remaining terms of a step.  Each instance's result is bitwise the one
 * sg_propagate_chebyshev gives it alone (same per-term code, same fixed-order
 * reduction).  The batch references the problems; they must outlive it. */
typedef struct sg_batch sg_batch;
sg_status sg_batch_create(sg_problem *const *problems, int32_t n, sg_batch **out);
/* Number of instances of a batch and, if n_cs is not NULL, each instance's
 * N_cs (n_cs: caller array of that many entries). */
sg_status sg_batch_size(const sg_batch *b, int32_t *n, int64_t *n_cs);
/* n: number of entries of psi and dt, which must equal the batch's number
 * of instances (SG_EINVAL otherwise).  psi[i]: device complex128[N_cs(i)] of
 * instance i (the library cannot check its length: a shorter buffer is read
 * and written past its end), propagated in place by nsteps steps of dt[i].  emin/emax: per-instance bounds (NaN: estimated by
 * sg_spectral_bounds).  check_every as in sg_propagate_chebyshev (norms and
 * energies of all instances are reduced together).  stats: nullable array of
 * n.  use_graph != 0 replays each step from a captured hipGraph (on a stream
 * the library owns, ordered after and before `stream` by events).  Returns
 * SG_ETOL if any instance drifts beyond tol. */
sg_status sg_batch_propagate(sg_batch *b, void *const *psi, int32_t n, const double *dt,
                             int32_t nsteps,
                             const double *emin, const double *emax, double tol,
                             sg_precision prec, int32_t check_every, int32_t use_graph,
                             sg_prop_stats *stats, void *stream);
/* Schedule autotuner over the batch's union of terms: terms of at least g
 * grid points run on a whole workgroup (g = 0: only those a wavefront cannot
 * hold), for g = 0, 256, 512, ... up to the largest term grid.  Each
 * candidate plan applies H once to every instance's state psi[i] (n states,
 * as sg_batch_propagate); the outputs must agree bitwise across candidates
 * (SG_EDEVICE otherwise), and the fastest of three timed rounds of `reps`
 * applies is kept (the first candidate unless another is faster by more than
 * 1%).  chosen_block_min_grid / best_ms: nullable outputs.  Synchronous. */
sg_status sg_batch_tune_schedule(sg_batch *b, void *const *psi, int32_t n, int32_t prec,
                                 int32_t reps, int32_t *chosen_block_min_grid, double *best_ms,
                                 void *stream);
sg_status sg_batch_free(sg_batch *b);

/* Two-state (vibronic) Hamiltonians: the form of the paper's Sec. 5 pyrazine
 * model (two electronic states; at every nuclear configuration the operator
 * is a 2 x 2 matrix), with optional state-dependent quartic couplings:
 *
 *   H = sum_i 1/2 omega_i (-d^2/dQ_i^2 + Q_i^2) (x) 1
 *       + [[V_00(Q), V_01(Q)], [V_01(Q), V_11(Q)]],
 *   V_ss = E_s + sum_i kappa_s,i Q_i + sum_{i<j} c2_s,ij Q_i^2 Q_j^2,
 *   V_01 = sum_i lambda_i Q_i.
 *
 * (Pyrazine: E = (-Delta, Delta), lambda only on mode 1, kappa_s,1 = 0.)
 * Standard size maps only (nb(l) = 2l+1, nq(l) = 2l+2), L <= 6.  The wave
 * packet is state-major: device complex128[2 N_cs], state 0's coefficients in
 * compact order, then state 1's; N_cs and the compact order are those of
 * the one-state structure (sg_vibronic_problem).  Each term runs Alg. 1 on
 * both states, the 2 x 2 matrix acting at every grid point; the separable
 * harmonic part and E_s act as the exact FP64 diagonal; the scatter-add is
 * the fixed-order reduce (bitwise reproducible).  All FP64. */
typedef struct {
  int32_t D;             /* modes, 1..64                                      */
  int32_t L;             /* Smolyak level, 0..6                               */
  const double *omega;   /* [D] > 0                                           */
  const double *E;       /* [2] state energies                                */
  const double *kappa;   /* [2*D] row s: state s's linear coefficients        */
  const double *lambda;  /* [D] interstate linear coupling                    */
  const double *c2;      /* [2*D*D] row-major per state, entries i<j used;
                            NULL means all zero                               */
} sg_vibronic_desc;
typedef struct sg_vibronic sg_vibronic;
/* Host compile + device upload (synchronous).  SG_EINVAL on bad input. */
sg_status sg_vibronic_build(const sg_vibronic_desc *desc, sg_vibronic **out);
sg_status sg_vibronic_free(sg_vibronic *v);
/* The one-state structure the handle owns (sizes, compact order through
 * sg_problem_info / sg_basis_indices; sg_set_timing / sg_get_timing time the
 * two-state kernels).  Valid until sg_vibronic_free; do not free it. */
sg_status sg_vibronic_problem(const sg_vibronic *v, sg_problem **out);
/* Algorithmic flops and HBM bytes of one two-state term sweep. */
sg_status sg_vibronic_figures(const sg_vibronic *v, double *sweep_flops, double *sweep_bytes);
/* psi (device complex128[2 N_cs]) = the displaced Gaussian (as
 * sg_init_gaussian) on electronic state `state` (0 or 1), zero on the other. */
sg_status sg_vibronic_init(sg_vibronic *v, const double *shift, int32_t state, void *psi,
                           void *stream);
/* psi_out = H_S psi_in, both device complex128[2 N_cs], distinct.  Async. */
sg_status sg_vibronic_apply(sg_vibronic *v, const void *psi_in, void *psi_out, void *stream);
/* Spectral bounds by `iters` Lanczos steps, padded as sg_spectral_bounds. */
sg_status sg_vibronic_bounds(sg_vibronic *v, int32_t iters, double *emin, double *emax,
                             void *stream);
/* Chebyshev propagation in place, as sg_propagate_chebyshev (FP64).
 * pop_trace (nullable): the population of state 1 at each check (same
 * points as the norm checks: step 0, every check_every steps, the end). */
sg_status sg_vibronic_propagate(sg_vibronic *v, void *psi, double dt, int32_t nsteps,
                                double emin, double emax, double tol, int32_t check_every,
                                sg_prop_stats *stats, double *pop_trace, void *stream);

/* Continuous-batching server of propagation requests on one device.
 *
 * A request is a problem description, a displaced-Gaussian initial state
 * (shift[D]), a time step and a number of Chebyshev steps.  A scheduler
 * thread compiles submitted requests on host worker threads, admits them
 * while the device memory they need (tables + vectors) fits the budget and a
 * slot is free, keeps every admitted wave packet resident on the device, and
 * at each tick advances all resident requests by one Chebyshev step in one
 * batched launch sequence (requests admitted meanwhile join at the next
 * tick).  A finished request's state is copied to host and its device memory
 * released.  Each request's result is bitwise the one it gets alone (same
 * per-term code and fixed-order reductions): the precision policy is the
 * configuration's, never tuned per request. */
typedef struct {
  int64_t hbm_budget_bytes;  /* device bytes resident requests may hold;
                                0 = 80% of the free memory at creation       */
  int32_t max_slots;         /* resident requests at most (> 0)              */
  sg_precision prec;
  int32_t check_every;       /* norm/energy check interval in steps (0: none) */
  double tol;                /* norm drift beyond this fails the request (SG_ETOL) */
  int32_t mixed_threshold;   /* SG_MIXED: sg_set_mixed_threshold value (< 0: default) */
  int32_t compile_threads;   /* host compile workers (0: 4)                  */
} sg_serve_config;

typedef struct {
  int32_t status;            /* SG_OK, SG_ETOL, SG_ECANCELED, ... (request result) */
  int32_t D, L;
  int64_t n_cs;              /* length of the state                           */
  void *psi_host;            /* caller buffer, complex128[n_cs]; NULL: skip copy */
  int64_t psi_capacity;      /* its length in complex values                  */
  sg_prop_stats stats;
  double t_submit, t_admit, t_done;   /* seconds on the server's clock        */
} sg_result;

typedef struct sg_server sg_server;
sg_status sg_serve_create(const sg_serve_config *cfg, sg_server **out);
/* Copies what it needs; returns at once.  SG_ENOMEM if the request could
 * never fit the budget, SG_EINVAL for an invalid description. */
sg_status sg_serve_submit(sg_server *s, const sg_problem_desc *desc, const double *shift,
                          double dt, int32_t nsteps, uint64_t *ticket);
/* SG_OK and *out filled when the request is finished (its record is then
 * dropped; a second poll gives SG_ENOTFOUND), SG_EAGAIN while it is queued or
 * running, SG_ENOTFOUND for an unknown ticket.  out->psi_host receives the
 * final state when its capacity suffices. */
sg_status sg_serve_poll(sg_server *s, uint64_t ticket, sg_result *out);
/* Cancels a queued or running request (it finishes with SG_ECANCELED). */
sg_status sg_serve_cancel(sg_server *s, uint64_t ticket);
/* Counters: queued, resident, finished requests and ticks run. */
sg_status sg_serve_counters(sg_server *s, int64_t out[4]);
sg_status sg_serve_destroy(sg_server *s);

/* Mixed-precision policy.  With SG_MIXED, a term whose combination
 * coefficient satisfies |D_l| <= max_fp32_coeff runs its grid contractions in
 * FP32; the others (few, small terms whose rounding the Smolyak sum amplifies
 * by |D_l|) run in FP64.  The default is 16.  Synchronous; also valid on a
 * host-only handle. */
sg_status sg_set_mixed_threshold(sg_problem *p, int32_t max_fp32_coeff);

/* Operator form of SG_FP64 applies.  Alg. 1 evaluates, per term, the whole
 * operator on the term's grid: the potential times the grid values plus the
 * kinetic second-derivative matrix of every active mode (grid_kinetic = 1).
 * When nq(l) > nb(l) at every level, each term's rule integrates the
 * separable part sum_i 1/2 omega_i (-d^2/dQ_i^2 + Q_i^2) exactly, so its
 * Smolyak sum is exactly the diagonal sum_i omega_i (n_i + 1/2); the default
 * (grid_kinetic = 0) then applies that diagonal in FP64 in the reduce and
 * only the coupling potential on the grids (same operator, fewer
 * contractions; results agree to rounding).  Without that condition SG_FP64
 * always uses the grid form.  SG_MIXED always uses the split form.
 * Synchronous; also valid on a host-only handle. */
sg_status sg_set_operator_form(sg_problem *p, int32_t grid_kinetic);

/* General coupling potential (Alg. 1, Sec. 3: the operator applied on each
 * term's direct-product grid; eq_action_smolyak, Sec. 2).  After
 * sg_set_potential(p, V, user) the problem's operator is
 *   H = sum_i 1/2 omega_i (-d^2/dQ_i^2 + Q_i^2) + V(Q),
 * V replacing the polynomial couplings c and k of its description.  The
 * library evaluates V once, here, on the host: at every point of every term's
 * direct-product grid (the paper's grids; their number is
 * sg_info.grid_literal), in batches of at most 65536 points, calling
 *   V(n, Q, out, user)   Q: [n][D] row-major, mode 1 first (read only);
 *                        out: [n], V at those points (written by V).
 * For every term it sums V over the points of the level-0 modes with their
 * weights wt_u b_0(Q_u)^2 (those modes carry one basis function, so this is
 * what their basis -> grid -> basis passes compute) and uploads the result,
 * one FP64 value per active grid point (sg_info.grid_active values).  Applies
 * then read those tables; the separable part acts as the exact diagonal, as
 * in the default operator form.  V must be pure and return finite values; it
 * is not called after sg_set_potential returns.  V == NULL restores the
 * polynomial couplings.
 * Requirements: a device handle with the standard size maps (nb = 1 + 2l,
 * nq = 2 + 2l), L <= 6, the split operator form, and at most 1e11 grid points.
 * Such a problem runs in FP64 only: SG_MIXED calls on it fail with SG_EINVAL,
 * and so do mixed batch calls whose batch has FP32 terms (in a batch without
 * any, SG_MIXED is the FP64 split path).  sg_set_operator_form(p, 1) is
 * refused while a potential is set.  Errors: SG_EINVAL (requirements, a
 * non-finite V), SG_ENOMEM, SG_EDEVICE; on error the previous potential stays.
 * Synchronous: the device is synchronised before the tables are replaced.
 * A batch created afterwards takes the problem with its potential; a batch
 * created before refuses to run (SG_EINVAL) once the potential changed. */
typedef void (*sg_potential_fn)(int64_t n, const double *Q, double *out, void *user);
sg_status sg_set_potential(sg_problem *p, sg_potential_fn V, void *user);

/* Precision autotuner.  Tries every threshold from "all terms in FP32" down
 * to 0 (no FP32 term: the exact FP64 split) on the device vector psi
 * (complex128[N_cs], not modified), measures the relative 2-norm error of the
 * SG_MIXED apply against the SG_FP64 apply and the time of `reps` applies,
 * and keeps the fastest threshold whose error is at most tol/2.  Threshold 0
 * always qualifies (its error is FP64 rounding).  Writes the choice and its
 * measured error (both nullable).  Synchronises `stream`; uses the handle's
 * work buffers. */
sg_status sg_tune_mixed(sg_problem *p, const void *psi, double tol, int32_t reps,
                        int32_t *chosen, double *chosen_error, void *stream);

/* Term-to-workgroup schedule.  An in-place term of at most 4096 grid points
 * can run on one wavefront (up to eight such terms share a workgroup; a
 * contraction over more fibers than the lanes hold runs in chunks), unless
 * it has at least block_min_grid grid points: then it runs on a whole
 * workgroup.  block_min_grid = 0 (the default) picks the threshold from the
 * problem's size: 1025 for a problem of fewer than 1024 terms (the launch
 * then lasts as long as its longest term chain), else 4096 (many terms:
 * throughput-bound).  When there are fewer wave terms than compute units can take,
 * they are spread over packs_per_cu workgroups per compute unit (1, the
 * default, .. 4; at most as many as fit a CU).  The schedule decides only
 * which threads compute a term; every schedule gives bitwise the same
 * results.  Synchronous; also valid on a host-only handle.  Out-of-range
 * arguments -> SG_EINVAL. */
sg_status sg_set_schedule(sg_problem *p, int32_t block_min_grid, int32_t packs_per_cu);

/* Schedule autotuner.  Times `reps` applies of precision prec on the device
 * vector psi (complex128[N_cs], not modified), best of three rounds, for each
 * candidate schedule (block_min_grid 0 and each power of two from 64 to the
 * largest term grid, each with packs_per_cu 1 and 2).  It keeps the default
 * (0, 1) unless another candidate is faster by more than 1%, and each later
 * replacement must beat the current choice by as much.  Every candidate's
 * result is compared bitwise with the first's; a difference returns
 * SG_EDEVICE (the schedule is left as it was).  Writes the choice (both
 * nullable).  Synchronises `stream`; uses the handle's work buffers. */
sg_status sg_tune_schedule(sg_problem *p, const void *psi, int32_t prec, int32_t reps,
                           int32_t *chosen_block_min_grid, int32_t *chosen_packs_per_cu,
                           void *stream);

/* Lowest eigenpairs of H_S by block Davidson: the method the paper uses to
 * converge stationary states (Sec. 3, flowchart text), here on sg_apply_H
 * (FP64).  nev eigenpairs; max_basis (2 nev .. 256) subspace vectors before a
 * restart from the Ritz block; at most max_iter iterations; converged when
 * every residual norm ||H x - theta x|| (x normalised) is <= tol.  guess:
 * nullable device block of nguess complex128[N_cs] vectors to start from
 * (e.g. a lower-level solution embedded with sg_embed_basis); the start block
 * is the guess, the unit vectors at the nev lowest harmonic energies and one
 * fixed pseudo-random vector (reaching every symmetry sector of H), less the
 * vectors the earlier ones span.  nev buffer Ritz pairs are iterated beside
 * the wanted ones.  Outputs:
 * evals[nev] (host, ascending); evecs (nullable device complex128[nev][N_cs],
 * orthonormal, real-valued); resnorms[nev] (nullable host); stats (nullable).
 * Returns SG_ETOL (outputs still written) when not every pair converged.
 * Allocates its workspace (2 max_basis + 2 nev vectors); synchronises
 * `stream`. */
typedef struct {
  int32_t iterations;
  int32_t applies;            /* H_S applications */
  int32_t restarts;
  int32_t converged;          /* pairs with residual <= tol */
} sg_eig_stats;
sg_status sg_eigensolve(sg_problem *p, int32_t nev, int32_t max_basis, int32_t max_iter,
                        double tol, const void *guess, int32_t nguess, double *evals,
                        void *evecs, double *resnorms, sg_eig_stats *stats, void *stream);

/* The paper's low-level start (Sec. 4 example run: a wave-function guess from
 * a diagonalisation at low L, then Davidson at the target L): copies a state
 * of problem `from` into the compact basis of `to` (same D and basis size
 * map, from->L <= to->L; the lower-level compact basis is a subset), zero
 * elsewhere.  x: device complex128[N_cs(from)]; y: device
 * complex128[N_cs(to)].  Synchronises `stream`. */
sg_status sg_embed_basis(const sg_problem *from, const sg_problem *to, const void *x, void *y,
                         void *stream);

/* Per-kernel timing for measurement.  sg_set_timing(p, 1) resets the
 * counters and attaches a pair of HIP events to every term-sweep and reduce
 * launch made through this handle (hipExtLaunchKernel: the events take the
 * start and end timestamps of the kernel dispatches themselves, so the
 * durations are the kernels' and no marker packet enters the stream).
 * sg_get_timing waits for the recorded events and returns the summed kernel
 * durations. */
typedef struct {
  double sweep_ms;           /* summed duration of the term-sweep kernels     */
  int64_t sweep_launches;
  double reduce_ms;          /* summed duration of the reduce kernels         */
  int64_t reduce_launches;
} sg_timing;
sg_status sg_set_timing(sg_problem *p, int32_t enable);
sg_status sg_get_timing(sg_problem *p, sg_timing *out);

const char *sg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SG_H */
