/*
 * rttda.h -- C ABI of the MI355X (gfx950) RT-TDA propagation library.
 *
 * The library evaluates the Hamiltonian-amplitude product of real-time
 * Tamm-Dancoff (RT-TDA) electron dynamics and integrates the time-dependent
 * Schroedinger equation with it (Knoll & Levine, arxiv 2601.16949):
 *
 *   i dX/dt = H(t) X,   H(t) = diag(0, A) - E(t) M_d                 (eqs. ode_rt_tda, e_field)
 *
 * on the extended amplitude space X = (c0, C): c0 is the Kohn-Sham ground-state
 * coefficient (Real-Time TDA subsection: A_{0,ia} = 0, A_00 taken as 0) and
 * C[i][a] the singles amplitudes in virtuals-run-fastest order (text after eq.
 * A_matrix_element2).  A is given in density-fitted form:
 *
 *   (A C)_ia = (e_a - e_i) C_ia + 2 sum_Q B^Q_ia sum_jb B^Q_jb C_jb
 *              - c_x sum_Q (B^Q_oo C B^Q_vv)_ia                       (eq. A_matrix_element2, DF form)
 *
 * and M_d is the CSF-basis dipole along the unit vector d, mapped from the MO
 * basis by the Slater-Condon rules (eqs. sc1-sc6), without the constant
 * <Phi0|mu|Phi0>:
 *
 *   (M_d X)_0  = sqrt2 sum_ia mu_ia C_ia
 *   (M_d X)_ia = (C mu_vv - mu_oo C)_ia + sqrt2 mu_ia c0.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array arguments are DEVICE pointers owned by the caller (host pointers
 *    are marked "host").  Device arrays must be 16-byte aligned, except the
 *    per-step outputs of the propagators (trace, norms, correlation, populations,
 *    energy), which are written one double at a time and need 8-byte alignment;
 *    inputs stay alive for as long as a context that refers to them.
 *  - Complex amplitudes are stored as separate real planes:
 *        c0 : f64 [nrhs][2]           (re, im)
 *        c  : f64 [nrhs][2][o][v]     (plane 0 = Re C, plane 1 = Im C)
 *  - Every call is asynchronous on the context's stream (hipStream_t, NULL =
 *    the null stream).  Device faults surface at the next synchronisation.
 *  - The library never allocates device memory: all scratch space lives in
 *    the caller-supplied workspace (size from rttda_workspace_bytes()).
 *  - Errors: a negative rttda_status; rttda_last_error() returns a
 *    thread-local message describing the last failure on the calling thread.
 *    Arguments are validated before anything is enqueued, so a failed call
 *    leaves all device arrays untouched.
 *  - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef RTTDA_H
#define RTTDA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rttda_ctx rttda_ctx;

typedef enum {
  RTTDA_OK = 0,
  RTTDA_E_INVAL = -1,       /* bad argument (null/misaligned pointer, bad size, bad dtype)  */
  RTTDA_E_NOMEM = -2,       /* workspace too small                                          */
  RTTDA_E_DEVICE = -3,      /* a HIP runtime call failed                                    */
  RTTDA_E_STATE = -4,       /* context in the wrong state (e.g. destroyed, no kernel)      */
  RTTDA_E_UNSTABLE = -5,    /* norm guard tripped: non-finite or growing amplitudes        */
  RTTDA_E_UNSUPPORTED = -6  /* shape or option this library does not support             */
} rttda_status;

typedef enum { RTTDA_F64 = 0, RTTDA_F32 = 1, RTTDA_BF16 = 2 } rttda_dtype;

typedef enum {
  RTTDA_PREC_FP32 = 1,       /* FP32 factors, FP32 MFMA Coulomb/exchange, FP64 state        */
  RTTDA_PREC_MIXED_BF16 = 2  /* BF16 factors, split BF16 (hi+lo) exchange products with     */
                             /* FP32 accumulation, FP32 Coulomb, FP64 state                  */
} rttda_precision;

/* Pulse shapes: eqs. delta_pulse, continuous wave, transform_limited, chirped_pulse. */
typedef enum {
  RTTDA_PULSE_NONE = 0,
  RTTDA_PULSE_DELTA = 1,  /* first-order kick X <- X + i e0 M_d X applied when step0 == 0   */
  RTTDA_PULSE_CW = 2,     /* E(t) = e0 sin(omega t + phase)                                  */
  RTTDA_PULSE_GAUSS = 3,  /* E(t) = e0 exp(-(t-t0)^2 / 2 s^2) sin(omega (t-t0) + phase)      */
  RTTDA_PULSE_CHIRP = 4,  /* E(t) = e0 exp(-(t-t0)^2 / 2 s^2)                                */
                          /*        sin((omega + beta (t-t0)/2)(t-t0) + phase)               */
  RTTDA_PULSE_DELTA_EXACT = 5 /* unitary kick X <- exp(i e0 M_d) X applied when step0 == 0, */
                          /* by a Taylor series whose length follows from a bound on        */
                          /* e0 |M_d|; RTTDA_E_UNSUPPORTED if e0 |M_d| exceeds about 12      */
} rttda_pulse_kind;       /* s = fwhm / 2.35482; phase = pi/2 turns sin into cos             */

typedef struct rttda_pulse {
  int32_t kind;     /* rttda_pulse_kind                                          */
  int32_t reserved; /* must be 0                                                 */
  double e0;        /* peak field (au); kick strength kappa for DELTA            */
  double omega;     /* carrier angular frequency (Ha)                            */
  double t0;        /* envelope centre (au)                                      */
  double fwhm;      /* envelope full width at half maximum (au), > 0            */
  double beta;      /* chirp rate (Ha/au)                                        */
  double phase;     /* carrier phase (rad)                                       */
  double dir[3];    /* polarisation, unit vector (|dir| = 1 within 1e-12)        */
} rttda_pulse;

/* One molecule (operator).  All pointers are device pointers. */
typedef struct rttda_desc {
  int32_t n_occ;      /* o >= 1                                                          */
  int32_t n_virt;     /* v >= 1                                                          */
  int32_t n_aux;      /* N_Q >= 0                                                        */
  int32_t precision;  /* rttda_precision                                                 */
  int32_t b_dtype;    /* RTTDA_F32 with PREC_FP32, RTTDA_BF16 with PREC_MIXED_BF16       */
  int32_t max_rhs;    /* largest nrhs any call will pass (1..4096)                       */
  double cx;          /* fraction of exact exchange c_x                                  */
  const double *e_occ;  /* f64 [o]   occupied orbital energies (Ha)                      */
  const double *e_virt; /* f64 [v]   virtual orbital energies (Ha)                       */
  const void *b_ov;     /* b_dtype [N_Q][o][v]  factors B^Q_ia                           */
  const void *b_oo;     /* b_dtype [N_Q][o][o]  factors B^Q_ij, symmetric in (i, j)      */
  const void *b_vv;     /* b_dtype [N_Q][v][v]  factors B^Q_ab, symmetric in (a, b)      */
  const double *mu;     /* f64 [3][o+v][o+v]    MO dipole matrices (x, y, z), symmetric  */
  void *workspace;      /* >= rttda_workspace_bytes(desc) bytes, 256-byte aligned        */
  size_t workspace_bytes;
  void *stream;         /* hipStream_t for every call on this context (NULL allowed)     */
} rttda_desc;

/* Bytes of workspace a context with this descriptor needs (pointers may be NULL here). */
rttda_status rttda_workspace_bytes(const rttda_desc *desc, size_t *bytes);

/* Validate the descriptor, carve the workspace and precompute the orbital-gap
 * diagonal.  The context keeps the descriptor's pointers (not copies of the
 * arrays).  Enqueues work on desc->stream. */
rttda_status rttda_create(const rttda_desc *desc, rttda_ctx **out);

/* Release the host-side context (and its cached HIP graphs).  Synchronises the stream. */
rttda_status rttda_destroy(rttda_ctx *ctx);

/* Change the stream of later calls. */
rttda_status rttda_set_stream(rttda_ctx *ctx, void *stream);

/* s = H X for nrhs independent states (no factor -i), with field strengths
 * field[r] (host, au) along the unit vectors dir[r] (host, [nrhs][3]):
 *   s0[r] = -field[r] (M_dr X_r)_0,  s[r] = A C_r - field[r] (M_dr X_r)_C.
 * c0, c: inputs as described above; s0 (f64 [nrhs][2]) and s (f64
 * [nrhs][2][o][v]) are outputs and may not alias the inputs. */
rttda_status rttda_sigma(rttda_ctx *ctx, int32_t nrhs, const double *field, const double *dir,
                         const double *c0, const double *c, double *s0, double *s);

/* Advance nrhs states by n_steps classic RK4 steps of size dt, in place.
 * pulses (host, [nrhs]) gives each state's field; step0 is the index of the
 * current time (t = step0 * dt), so a run split into several calls gives the
 * same result as one call.  Delta pulses kick their state before the first
 * step when step0 == 0.  If trace is not NULL it receives the dipole trace
 *   trace[k][r] = Re <X_r | M_dr | X_r> at step step0 + k, k = 0..n_steps
 * (f64 [n_steps+1][nrhs]); norms likewise receives |c0|^2 + |C|^2 if not NULL.
 * The norm guard records the first step at which a norm is non-finite or more
 * than twice its value at the start of the call; read it with rttda_guard().
 * A call that fails its argument checks (including RTTDA_E_UNSUPPORTED for an
 * exact kick beyond the series' reach) leaves c0 and c untouched. */
rttda_status rttda_propagate(rttda_ctx *ctx, int32_t nrhs, const rttda_pulse *pulses, double dt,
                             int64_t step0, int64_t n_steps, double *c0, double *c, double *trace,
                             double *norms);

/* As rttda_propagate with the paper's integrator instead of RK4: the second-order
 * symplectic split operator on X = q + i p (Propagation Algorithm subsection,
 * eq. x_real_imagiary and the symplectic form dq/dt = H p, dp/dt = -H q), one
 * step being  p <- p - dt/2 H(t) q;  q <- q + dt H(t + dt/2) p;  p <- p - dt/2 H(t + dt) q.
 * Two real sigma per step (the two half kicks of consecutive steps share one),
 * against four complex sigma for RK4; the norm oscillates at O(dt^2) without
 * drift.  Same arguments, kick, trace, norms and guard as rttda_propagate. */
rttda_status rttda_propagate_sso(rttda_ctx *ctx, int32_t nrhs, const rttda_pulse *pulses, double dt,
                                 int64_t step0, int64_t n_steps, double *c0, double *c, double *trace,
                                 double *norms);

/* Time-correlation output for the next rttda_propagate or rttda_propagate_sso call on ctx (that
 * call only; NULL clears it): corr (device [n_steps+1][nrhs][2] FP64, 16-byte aligned, caller-
 * owned) receives R_r(t_n) = <X_r(start) | X_r(t_n)> (eq. time_correlation_function) as (real,
 * imaginary) pairs for n = 0..n_steps, where X_r(start) is the state at the start of the call
 * after its delta kicks (the paper's epsilon just after the pulse) and the inner product runs over
 * the ground amplitude and both planes. */
rttda_status rttda_set_correlation(rttda_ctx *ctx, double *corr);

/* Energy output for the next rttda_propagate call on ctx (that call only; NULL clears it): energy
 * (device [n_steps+1][nrhs] FP64, caller-owned) receives E_r(t_n) = <X_r | diag(0, A) | X_r> =
 * sum over both planes of C . (A C), the expectation of the field-free Hamiltonian of eqs.
 * ode_rt_tda and A_matrix_element2 (A_00 = 0), at steps step0..step0+n_steps.  Computed from the
 * products A C that the first RK4 stage of each step forms anyway (partial sums per block of the
 * FP64 epilogue, added in a fixed order); the last sample costs one more product.  Field-free RK4
 * moves it by the per-mode factor |R(-i w dt)|^2 per step (no drift beyond that).  The split-
 * operator route does not produce it: rttda_propagate_sso returns RTTDA_E_UNSUPPORTED while an
 * energy output is pending. */
rttda_status rttda_set_energy(rttda_ctx *ctx, double *energy);

/* Eigenstate populations as an output of the next rttda_propagate or rttda_propagate_sso call
 * on ctx (that call only; pops NULL clears it): pops (device [n_steps+1][nrhs][k] FP64, 16-byte
 * aligned) receives P_rI(t_n) = |<U_I, X_r(t_n)>|^2 (eq. populations) for the k real unit
 * vectors evecs (device [k][o][v] FP64, e.g. from rttda_eigen_lowest; 1 <= k <= 64), at every
 * step of the call, alongside the trace.  Both arrays must stay valid until the call's work ends. */
rttda_status rttda_set_populations(rttda_ctx *ctx, int32_t k, const double *evecs, double *pops);

/* Spectra on the frequency grid omega_j = omega0 + j domega (j < n_omega, Ha), from device signals
 * of n_t samples spaced dt (eq. fourier_transform; the paper's Hann window with mirroring is the
 * half-Hann window h_n = (1 + cos(pi n / (n_t-1))) / 2 on the record):
 *   kind 0, signal = dipole traces [n_t][nsig]:  S_s = omega sum_n h_n (mu_n - mu_0) sin(omega t_n) dt / kappa
 *   kind 1, signal = time correlations [n_t][nsig][2]:  S_s = omega Re sum_n h_n R_n exp(i omega t_n) dt
 * out (device): [nsig][n_omega], or with average != 0 the mean over the signals [n_omega] (the
 * x/y/z average, eq. spectrum_average).  Asynchronous on stream (hipStream_t, NULL = default). */
rttda_status rttda_spectrum(void *stream, int32_t kind, const double *signal, int32_t n_t, int32_t nsig, double dt,
                            double kappa, int32_t n_omega, double omega0, double domega, int32_t average,
                            double *out);

/* out[r] = Re <X_r | M_dr | X_r> (f64 [nrhs]) for states c0, c and host unit
 * vectors dir ([nrhs][3]): the expectation value of the field-coupling operator of
 * eq. e_field (built by eqs. sc1-sc6), the observable behind every trace sample. */
rttda_status rttda_dipole_trace(rttda_ctx *ctx, int32_t nrhs, const double *dir, const double *c0,
                                const double *c, double *out);

/* rttda_sigma without a context or workspace, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  desc
 * describes the operator as for rttda_create, except that its workspace fields are ignored: the
 * scratch is a static device array of 64 MiB that every device this entry point runs on keeps
 * until the process ends.  Arguments and outputs are those of rttda_sigma, with 1 <= nrhs <= 64.
 * RTTDA_E_NOMEM when the shape and nrhs need more scratch than the array holds (its partial slabs
 * of the exchange are capped at 16 MiB, so larger problems use fewer Q splits than a context
 * would).  Calls on one device share the array: overlapping calls race, so serialise them (one
 * stream, or wait between streams); each call rewrites whatever it reads.  The device current on
 * the calling thread must be desc->stream's.  Synchronises desc->stream once (after its small
 * host-to-device copies) and returns with the sigma work queued on it.  Calls no allocator. */
rttda_status rttda_sigma_noalloc(const rttda_desc *desc, int32_t nrhs, const double *field, const double *dir,
                                 const double *c0, const double *c, double *s0, double *s);

/* Synchronise the context's stream and report the norm guard of the last
 * rttda_propagate: *first_bad_step = -1 if it never tripped, else the absolute
 * step index; returns RTTDA_E_UNSTABLE in the latter case.  Covers
 * rttda_propagate_sso alike. */
rttda_status rttda_guard(rttda_ctx *ctx, int64_t *first_bad_step);

/* ---------------------------------------------------------------------------------------
 * Serving pool: continuous batching of propagation requests on one GPU (the paper runs
 * each polarisation as a job of its own, Absorption spectrum subsection; here many
 * molecules and pulses share the device).
 *
 * A request is a context (its operator, workspace and stream) plus states, pulses, dt and
 * a step count.  The pool admits a request when its declared HBM footprint fits the
 * budget, advances every admitted request in chunks of steps (each on its own context's
 * stream, so the work of different requests overlaps on the device; at most one chunk per
 * request is in flight), and frees the budget when the request is released.  A request's
 * result is the same as that of one rttda_propagate(_sso) call over all its steps: the
 * chunks resume at the request's own step counter, and the norm guard keeps its reference
 * norm and first bad step across them.  A request whose chunk fails (for instance an exact
 * kick beyond the series' reach) stops; the others carry on, and rttda_pool_poll and
 * rttda_pool_result report its status.  The pool owns no device memory and is not
 * thread-safe; contexts admitted to a pool must not be used elsewhere until released.
 * --------------------------------------------------------------------------------------- */
typedef struct rttda_pool rttda_pool;
typedef enum { RTTDA_INTEG_RK4 = 0, RTTDA_INTEG_SSO = 1 } rttda_integrator;
rttda_status rttda_pool_create(size_t budget_bytes, rttda_pool **out);
rttda_status rttda_pool_destroy(rttda_pool *pool); /* waits for in-flight chunks */
/* Admit a request; *slot receives its id.  pulses (host, [nrhs]) are copied; c0, c
 * (device, updated in place) and trace (device [n_steps+1][nrhs] or NULL) must outlive the
 * slot.  The pulses, dt and pointers are checked as rttda_propagate checks them
 * (RTTDA_E_INVAL).  RTTDA_E_NOMEM when footprint_bytes does not fit the remaining budget. */
rttda_status rttda_pool_admit(rttda_pool *pool, rttda_ctx *ctx, int32_t nrhs, const rttda_pulse *pulses,
                              double dt, int64_t n_steps, int32_t integrator, double *c0, double *c,
                              double *trace, size_t footprint_bytes, int32_t *slot);
/* For every admitted request whose previous chunk has finished and that has steps left,
 * enqueue its next chunk of up to chunk_steps steps.  Does not block; *issued receives
 * the number of chunks enqueued (may be NULL). */
rttda_status rttda_pool_step(rttda_pool *pool, int64_t chunk_steps, int32_t *issued);
/* Non-blocking progress of a slot: steps enqueued so far and whether all its steps have
 * finished on the device.  Returns the status of a failed chunk (the slot then counts as
 * finished) after filling both outputs. */
rttda_status rttda_pool_poll(rttda_pool *pool, int32_t slot, int64_t *steps_enqueued, int32_t *finished);
/* Wait for a slot's work and report its outcome: the status of a failed chunk, else the norm
 * guard over all its chunks (RTTDA_E_UNSTABLE, with the first bad step in *first_bad_step,
 * may be NULL; -1 when it never tripped). */
rttda_status rttda_pool_result(rttda_pool *pool, int32_t slot, int64_t *first_bad_step);
/* Wait for a slot's work, return its footprint to the budget and retire the slot. */
rttda_status rttda_pool_release(rttda_pool *pool, int32_t slot);
/* Budget in use and number of admitted (unreleased) requests. */
rttda_status rttda_pool_usage(const rttda_pool *pool, size_t *used_bytes, int32_t *active);

/* Time-step guard for the integrators of the Propagation Algorithm subsection.
 * Estimate the spectral radius of A (Lanczos on the sigma product with a fixed start
 * vector, n_iter steps, 2 <= n_iter <= 500): *rho is the largest |Ritz value| and
 * *rho_bound adds the Ritz residual of the extreme pairs, so that rho(A) <= rho_bound up
 * to the rounding of the sigma product.  Classic RK4 is stable for rho(A) dt up to about
 * 2.83 (the split operator for rho(A) dt < 2); callers check rho_bound * dt before a run.
 * Synchronises the context's stream; uses the workspace's stage buffers (no effect on
 * the state of later rttda_propagate calls). */
rttda_status rttda_spectral_radius(rttda_ctx *ctx, int32_t n_iter, double *rho, double *rho_bound);

/* The k lowest eigenpairs of A: the TI-TDA eigenproblem A X = omega X (eq. casida_tda), by block
 * Davidson on the sigma product (Coulomb and exchange kernels of the context's precision plus the
 * diagonal e_a - e_i; FP64 vectors, Rayleigh-Ritz on the host).  The search space starts from unit
 * vectors at the smallest entries of diag(A), holds at most m_max vectors (3k <= m_max <= 64, at
 * most o*v) and restarts from the 2k lowest Ritz vectors when full; corrections use diag(A) as the
 * preconditioner (D + 2 sum_Q B_ia^2 - c_x sum_Q B_ii B_aa, formed on the device).
 * work: device buffer of at least rttda_eigen_workspace_bytes (256-byte aligned, caller-owned);
 * evals, resid: host [k], the Ritz values (ascending) and residual norms |A x - w x| of the unit
 * Ritz vectors; evecs: device [k][o][v] FP64 Ritz vectors, or NULL.  Stops when every residual is
 * at most tol, after max_iter iterations, or when the space stops growing; *iters (may be NULL)
 * receives the iterations used; callers compare resid with tol.  Synchronises the context's stream
 * and uses its stage buffers (no effect on the state of later rttda_propagate calls). */
rttda_status rttda_eigen_workspace_bytes(const rttda_ctx *ctx, int32_t k, int32_t m_max, size_t *bytes);
rttda_status rttda_eigen_lowest(rttda_ctx *ctx, int32_t k, int32_t m_max, int32_t max_iter, double tol, void *work,
                                size_t work_bytes, double *evals, double *resid, double *evecs, int32_t *iters);

/* Eigenstate populations (eq. populations): out[r][I] = |<U_I, c_r>|^2 for the k real unit
 * vectors U (device [k][o][v] FP64, e.g. from rttda_eigen_lowest) and the states c (device
 * [nrhs][2][o][v] FP64 planes), 1 <= k <= 64, 1 <= nrhs <= 32.  work: device buffer of at least
 * k*2*nrhs doubles; out: host [nrhs][k].  Synchronises the context's stream. */
rttda_status rttda_populations(rttda_ctx *ctx, int32_t k, const double *evecs, int32_t nrhs, const double *c,
                               void *work, size_t work_bytes, double *out);

/* Launch configuration knobs (for the autotuner).  Zero fields keep the
 * library's choice.  Returns RTTDA_E_UNSUPPORTED for a tile variant the library
 * does not have, RTTDA_E_NOMEM when the splits do not fit the workspace. */
typedef struct rttda_tuning {
  int32_t exchange_variant; /* index into the exchange tile table (1-based), 0 = auto      */
  int32_t exchange_splits;  /* number of Q ranges the exchange is split into               */
  int32_t coulomb_splits;   /* number of Q ranges the second Coulomb product is split into */
  int32_t use_graph;        /* 1 = replay RK4 steps from a captured HIP graph, 2 = direct  */
  int32_t steps_per_graph;  /* RK4 steps captured in one graph                              */
  int32_t exchange_chunk;   /* Q values per chunk of the large-o GEMM exchange path (its W
                               scratch holds W hi/lo for one chunk, so at most what fits);
                               -1 = as many as fit (the default)                           */
  int32_t overlap;          /* 1 = the Coulomb pair runs on a second stream alongside the
                               exchange, 2 = both in order on the context's stream; the
                               default is 1 when the exchange has at least 5e10 flops per
                               stage at max_rhs, else 2                                     */
  int32_t small_path;       /* 1 = small-problem path: per RK4 stage one launch for the
                               Coulomb and exchange partial sums and one single-workgroup
                               launch for the whole stage epilogue (o*v <= 2048,
                               2 o v + v^2 + o^2 <= 12288, max_rhs <= 64, n_aux > 0);
                               2 = the general kernels.  The default is 1 where the shape fits
                               and the exchange has at most 2e7 flops per stage at max_rhs
                               (4 n_aux o v (o + v) max_rhs), else 2                           */
  int32_t coulomb_path;     /* 1 = the Coulomb pair as vector-unit GEMVs, 2 = as skinny GEMMs
                               on the FP32 matrix cores; the default is 2 from 16 RHS
                               (max_rhs), else 1                                              */
} rttda_tuning;
rttda_status rttda_set_tuning(rttda_ctx *ctx, const rttda_tuning *t);
rttda_status rttda_get_tuning(const rttda_ctx *ctx, rttda_tuning *t);
/* Largest exchange_splits the context's workspace holds: min(768, N_Q, the number of
 * partial K slabs of 2*max_rhs*o*v floats that fit 256 MiB, but at least 32). */
rttda_status rttda_exchange_splits_max(const rttda_ctx *ctx, int32_t *out);

/* Per-kernel-class timing with HIP events on the context's stream.  While profiling is
 * on, rttda_propagate launches kernels directly (no graph replay) and brackets each
 * launch group with an event pair; rttda_get_profile synchronises and returns the
 * launch counts and summed durations since profiling was last switched on.
 * Classes: 0 exchange, 1 Coulomb pair, 2 field/trace, 3 RK4 epilogue + stage scalars. */
typedef struct rttda_profile {
  int64_t launches[4];
  double ms[4];
} rttda_profile;
rttda_status rttda_set_profiling(rttda_ctx *ctx, int32_t on);
rttda_status rttda_get_profile(rttda_ctx *ctx, rttda_profile *out);

/* Number of exchange tile variants and a description of variant k (1-based). */
int32_t rttda_exchange_variants(int32_t precision);
const char *rttda_exchange_variant_name(int32_t precision, int32_t k);

/* Thread-local message for the last failed call on this thread ("" if none). */
const char *rttda_last_error(void);

/* Library version string. */
const char *rttda_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RTTDA_H */
