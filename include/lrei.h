/*
 * lrei.h - C ABI of the MI355X LREI library (liblrei.so).
 *
 * LREI (Low-Rank Eigenmode Integration, arXiv 2508.21200) advances the
 * quantum Landau-Lifshitz (q-LL, eq. 1.1) or Landau-Lifshitz-Gilbert (q-LLG,
 * eq. 1.2) equation for an n-spin density matrix rho = V Lambda_0 V* of rank r
 * (Sec. 3.1, eq. 3.1).  Only the N x r factor V is stored (N = 2^n, Sec. 3.2);
 * the spectrum Lambda_0 is fixed for all time (Sec. 2, Sec. 3.7).
 *
 * Conventions for every entry point:
 *  - Status codes are returned; no exception or abort crosses the ABI.  The
 *    message of the last failure on a context is lrei_last_error().
 *  - Host buffers passed in are copied before the call returns; device
 *    buffers (flag *_is_device = 1) are read/written on the context's stream
 *    and the call returns after that stream has drained them.  The caller
 *    keeps ownership of every buffer it passes.
 *  - A failing setter leaves the previous state unchanged.
 *  - Complex arrays are interleaved (re, im) IEEE doubles, row-major N x r:
 *    the r columns of basis state x are contiguous.  Basis state x has site i
 *    in bit i; bit value 0 is spin up (s^z = +1).
 *  - One context is used by one host thread at a time.
 */
#ifndef LREI_H
#define LREI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define LREI_API __attribute__((visibility("default")))
#else
#define LREI_API
#endif

typedef struct lrei_ctx lrei_ctx;

typedef enum {
  LREI_OK = 0,
  LREI_E_INVALID = 1,       /* bad argument; nothing changed                     */
  LREI_E_NOMEM = 2,         /* device allocation failed or problem too large      */
  LREI_E_NOTCONVERGED = 3,  /* eigensolve did not converge; state rolled back      */
  LREI_E_DEVICE = 4,        /* HIP runtime error                                   */
  LREI_E_STATE = 5,         /* call out of order (e.g. step before set_rho)        */
  LREI_E_NUMERIC = 6        /* non-finite values produced; state rolled back       */
} lrei_status;

typedef enum { LREI_QLL = 0, LREI_QLLG = 1 } lrei_model;

/* Time integrators (Sec. 3.7, 3.8).  RK2 is the paper's Heun tableau; RK3 is
 * Kutta's; RK4 is the classical method.  ABm use the standard Adams-Bashforth
 * weights with an RK start-up (see lrei_options.ab_bootstrap). */
typedef enum {
  LREI_RK1 = 1, LREI_RK2 = 2, LREI_RK3 = 3, LREI_RK4 = 4,
  LREI_AB2 = 12, LREI_AB3 = 13, LREI_AB4 = 14
} lrei_scheme;

/* Embedded Runge-Kutta pairs for adaptive stepping (lrei_evolve_adaptive).
 * HE21: Heun's method (order 2) with Euler embedded (order 1).
 * BS32: Bogacki-Shampine 3(2), order 3 with an order-2 solution that also
 * weights the right-hand side at the new state; costs the same four H.V
 * passes per attempt as an RK4 step and three stage eigensolves.
 * RK43: the classical RK4 step with the order-3 solution
 * b_hat = (1, 2, 2, 0, 1) / 6 (its last weight on the right-hand side at the
 * new state): five H.V passes and four stage eigensolves per attempt. */
typedef enum { LREI_PAIR_HE21 = 21, LREI_PAIR_BS32 = 32, LREI_PAIR_RK43 = 43 } lrei_pair;

/* LREI_FP64: every N-space pass in complex FP64.
 * LREI_MIXED: N-space passes (H.V, Gram products, basis combination) in
 * complex FP32 with per-tile FP32 MFMA products accumulated across tiles in
 * FP64; the projected problem (Cholesky, Householder, stage algebra, partial
 * eigensolve) always runs in FP64. */
typedef enum { LREI_FP64 = 0, LREI_MIXED = 1 } lrei_precision;

/* How each stage's partial eigensolve (Sec. 3.7: the r largest eigenpairs of
 * the stage matrix) is computed in the projected coordinates.
 *  LREI_WARM_PLAIN: direct solve (Householder tridiagonalisation, multisection,
 *    inverse iteration), exact to FP64 rounding whatever the start.
 *  LREI_WARM_ANALYTIC: subspace iteration started from the stage's input basis
 *    u (the predicted eigenvectors), accepted only with a certificate that its
 *    r Ritz values are the r largest eigenvalues, else the direct solve.
 *  LREI_WARM_PREDICT_IDENTITY, LREI_WARM_PREDICT_CAYLEY, LREI_WARM_LEARNED:
 *    the same iteration and judge, started from the first-order predictor
 *    Y0 = u R + (I - u u*) K u R Lambda^-1 built from an r x r rotation R:
 *    R = I; R = Cayley(-i s G) with G = u* H u and s the stage's step over
 *    hbar; or R from the network attached with lrei_attach_net (features G,
 *    s, kappa).  Only R's effect through Lambda^-1 changes the start's span.
 *    The three need r <= 16; the batch context accepts PLAIN and ANALYTIC. */
typedef enum {
  LREI_WARM_PLAIN = 0,
  LREI_WARM_ANALYTIC = 1,
  LREI_WARM_LEARNED = 2,
  LREI_WARM_PREDICT_IDENTITY = 3,
  LREI_WARM_PREDICT_CAYLEY = 4
} lrei_warm;

typedef struct {
  int precision;          /* lrei_precision, default LREI_FP64                           */
  double eig_tol;         /* Jacobi tolerance (relative to max|diag|) of the r x r Lowdin
                             re-orthonormalisation of the projected basis, used when its
                             deviation from orthonormality exceeds 1e-6 (smaller ones
                             use a series for S^-1/2), default 1e-15                    */
  int eig_max_sweeps;     /* Jacobi sweep limit of that step, default 40                 */
  int warm;               /* lrei_warm, default LREI_WARM_ANALYTIC (RK steps; the AB
                             step always uses the direct solve)                     */
  int ab_bootstrap;       /* RK scheme for the first m-1 ABm steps, default LREI_RK4     */
  int householder_mode;   /* complement action W = V^ X12* (Sec. 3.4) in the projected
                             coordinates: 0 (default) as (I - u u*) y diag(conj c),
                             1 through the Householder reflectors of u (eq. 3.3);
                             equal to rounding, 0 is faster on this GPU            */
  int use_graph;          /* 1: capture one step as a hipGraph and replay it (default)  */
  int deterministic;      /* ignored: every reduction runs in a fixed order, so results
                             are bitwise reproducible for a given launch shape        */
  const char *autotune_cache; /* path of the autotuner's text cache file, or NULL     */
  double mixed_pivot_floor; /* LREI_MIXED: the FP32-stored Krylov blocks resolve a new
                             direction only while its Cholesky pivot stays well above
                             their rounding; when the smallest pivot ratio of an RK
                             step (lrei_stats.min_pivot_ratio) falls below this floor
                             the context moves to FP64 storage for the rest of its
                             life (checked every 16 steps and at the end of a call;
                             lrei_stats.precision_promoted reports it).  Default 2e-6;
                             0 disables the check                                    */
  int fail_after_steps;   /* for tests of the failure path: k > 0 makes every lrei_step
                             call with n_steps >= k run its steps and then fail as a
                             non-finite step does (LREI_E_NUMERIC, state restored to
                             the start of the call).  Default 0 (off)                */
  int site_order;         /* the site -> row-bit order of the internal storage:
                             0 (default) the order that keeps the bonds of the three
                             top-bit sites (which pick the XCD a row block runs on)
                             few and puts their neighbours in the low bits; 1 the
                             10-site cluster with the most bonds inside it in the low
                             bits, for the tiled H.V pass (LDS tiles of up to 2^10
                             rows).  Results are unaffected; only speed changes    */
} lrei_options;

typedef struct {
  int64_t steps_done;            /* time steps completed on this context               */
  int64_t eigensolves;           /* projected eigensolves performed                    */
  int64_t warm_accepted;         /* eigensolves done by the warm-started subspace
                                    iteration (every mode but LREI_WARM_PLAIN)         */
  int64_t warm_rejected;         /* of those, the ones that fell back to the direct
                                    solver (no convergence or no certificate)          */
  int64_t warm_iterations;       /* stage-matrix block products of the warm start
                                    (subspace iterations, plus one per predictor)      */
  int32_t dropped_directions;    /* Krylov directions dropped as dependent (last step)  */
  int32_t precision_promoted;    /* 1 once a LREI_MIXED context has moved to FP64
                                    storage (lrei_options.mixed_pivot_floor)           */
  double min_pivot_ratio;        /* smallest Cholesky pivot / Gram diagonal (last step) */
  double ortho_error;            /* max |V*V - I| at the start of the last step         */
  double energy;                 /* Tr(Lambda_0 V* H V) at the start of the last step   */
  double last_step_ms;           /* wall time of the last lrei_step call                */
  double phase_ms[8];            /* projected-step kernel time by phase over the last
                                    call: Gram/Cholesky setup, Cholesky, R^-1, H u,
                                    Householder, stage matrix, eigensolve, tail      */
  double eig_phase_ms[6];        /* eigensolver time over the last call by part:
                                    the direct solver's tridiagonalisation,
                                    multisection, inverse iteration and
                                    back-transform; the warm-started solver's
                                    whole time (accepted or not) and its Ritz
                                    step                                            */
} lrei_stats;

/* Fills *opt with the defaults listed above. */
LREI_API void lrei_default_options(lrei_options *opt);

/* Creates a context on HIP device `hip_device`.  `hip_stream` is a hipStream_t
 * to run on (e.g. torch.cuda.current_stream().cuda_stream) or NULL for a
 * stream owned by the context.  `opt` may be NULL for defaults.  The context
 * owns all device memory it allocates; lrei_destroy frees it. */
LREI_API lrei_status lrei_create(lrei_ctx **out, int hip_device, void *hip_stream, const lrei_options *opt);
LREI_API void lrei_destroy(lrei_ctx *ctx);
LREI_API const char *lrei_last_error(const lrei_ctx *ctx);

/* The spin Hamiltonian of Sec. 5, eq. (5.1), in Pauli form:
 *   H = sum_b 1/2 sum_{a,c} J_b[a][c] s^a_{i_b} s^c_{j_b} + 1/2 sum_i h_i . s_i,
 * which equals eq. (5.1) with S = (hbar/2) s, J^{ac} = J delta_ac + eps_acd d_d
 * and h = g mu_B b.  `bond_ij` is [n_bonds][2] site pairs (0 <= i < j < n),
 * `bond_J` is [n_bonds][3][3] row-major (x, y, z), `site_h` is [n][3] or NULL.
 * `hbar` enters only the equations of motion.  1 <= n <= 30.
 * Invalidates the rank-r state's Adams-Bashforth history. */
LREI_API lrei_status lrei_set_hamiltonian(lrei_ctx *ctx, int n_spins, int n_bonds, const int32_t *bond_ij,
                                 const double *bond_J, const double *site_h, double hbar);

/* Sets rho = V diag(lambda) V* (Sec. 3.1, eq. 3.1).  lambda: r finite values,
 * strictly positive, non-increasing.  V: N x r complex128 with orthonormal
 * columns (max |V*V - I| <= 1e-10 on a LREI_FP64 context, <= 1e-5 on a
 * LREI_MIXED one, whose check runs on the FP32-rounded copy), host or device
 * pointer.  1 <= r <= 32,
 * r <= N.  Requires a Hamiltonian. */
LREI_API lrei_status lrei_set_rho(lrei_ctx *ctx, int r, const double *lambda, const void *V, int v_is_device);

/* Advances n_steps >= 0 time steps of size dt > 0 with damping kappa >= 0
 * (q-LL: eq. 1.1 through eq. 4.1; q-LLG: eq. 1.2 through eq. 3.2), using the
 * LREI-RK (Sec. 3.7) or LREI-AB (Sec. 3.8) scheme.  Adams-Bashforth history
 * carries over between calls with the same model, scheme, dt and kappa; any
 * change restarts it with the bootstrap scheme.  On a numerical failure
 * (LREI_E_NUMERIC, LREI_E_NOTCONVERGED) the state is restored to that at the
 * start of the call and the Adams-Bashforth history is dropped. */
LREI_API lrei_status lrei_step(lrei_ctx *ctx, int model, int scheme, double dt, double kappa, int n_steps);

/* Outcome of lrei_evolve_adaptive. */
typedef struct {
  double t;          /* time advanced by the accepted steps (t_span when reached) */
  double h_next;     /* step the controller proposes next                         */
  double err_last;   /* error estimate of the last attempt (NaN: non-finite)      */
  double err_max;    /* largest estimate among the accepted steps                 */
  int accepted;      /* accepted steps                                            */
  int rejected;      /* rejected attempts                                         */
  int attempts;      /* attempts that ran                                         */
  int reached;       /* 1: t_span reached                                         */
} lrei_adapt_result;

/* Advances the state by t_span > 0 with step-size control from local error
 * estimates (the paper's outlook, Sec. 6), using the embedded pair `pair`
 * (lrei_pair) in LREI form: each attempt is an LREI-RK step (Sec. 3.7) with
 * the pair's higher-order weights; the two candidate matrices of eq. 3.9
 * (weights b and b_hat) differ by E = h sum_l (b_l - b_hat_l) f(rho_l), and
 * the estimate is the Frobenius norm of the part of E tangent to the
 * fixed-spectrum manifold at the new state (the distance of the two projected
 * candidates to first order).  An attempt is accepted when the estimate is
 * <= tol (an absolute bound on the local error of rho in the Frobenius norm);
 * the next step is h min(5, max(0.2, 0.9 (tol / err)^(1 / (q + 1)))), q the
 * embedded order, without growth right after a rejection, clamped to
 * [h_min, h_max] and to the time left; the last step ends on t_span exactly.
 * The controller runs on the GPU between attempts (no host round trip per
 * attempt); the host checks its state after each batch of attempts.
 * Arguments: 0 < h_min <= h_init, h_min <= h_max, tol > 0, max_attempts >= 1;
 * kappa >= 0.  `out` (may be NULL) receives the outcome in every case.
 * Returns LREI_OK when t_span is reached; LREI_E_NOTCONVERGED when an attempt
 * at h <= h_min is rejected or max_attempts attempts ran first: the state is
 * then that of the last accepted step and out->t says how far it got.  A
 * non-finite attempt counts as a rejection.  Invalidates the Adams-Bashforth
 * history.  Mixed precision: tol should stay well above the FP32 storage
 * rounding of the state (about 1e-6 relative). */
LREI_API lrei_status lrei_evolve_adaptive(lrei_ctx *ctx, int model, int pair, double kappa, double t_span,
                                          double tol, double h_init, double h_min, double h_max, int max_attempts,
                                          lrei_adapt_result *out);

/* Copies the current state out: lambda (r values, always Lambda_0, Sec. 3.7)
 * and V (N x r complex128, host or device pointer).  Either may be NULL. */
LREI_API lrei_status lrei_get_rho(lrei_ctx *ctx, double *lambda, void *V, int v_is_device);

/* Energy Tr(Lambda_0 V* H V) and magnetisation M_v = (1/n) sum_i <S_i^v>
 * with S = (hbar/2) s (Sec. 3.6, eq. 3.6) for the current state.  Either
 * output may be NULL. */
LREI_API lrei_status lrei_observables(lrei_ctx *ctx, double *energy, double magnetization[3]);

LREI_API lrei_status lrei_get_stats(lrei_ctx *ctx, lrei_stats *stats);

/* Y = H X for an N x r block X (r <= 32) in the context's Hamiltonian,
 * complex128, host or device pointers (both the same kind).  This runs the
 * same matrix-free kernel the step uses (Sec. 3.3: "inexpensive due to the
 * sparsity of H"), in FP64. */
LREI_API lrei_status lrei_apply_hamiltonian(lrei_ctx *ctx, int r, const void *X, void *Y, int is_device);

/* Y = H X as lrei_apply_hamiltonian with device pointers, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): it allocates nothing and does not
 * synchronise.  X and Y are device arrays of the caller (N x r complex128,
 * natural site order, Y != X); the work is enqueued on the context's stream
 * and Y is complete when that stream reaches this point (lrei_synchronize).
 * The site-order copies of X and H X live in a static device array of
 * 64 MiB per GPU, held until the process ends: 2 N r complex128 values must
 * fit (N r <= 2^21), else LREI_E_INVALID.  Every call on one GPU uses the
 * same array, so calls that overlap on one GPU (other streams, other
 * contexts, other host threads) race; calls on one stream are ordered.
 * Errors: LREI_E_STATE without a Hamiltonian, LREI_E_INVALID (r outside
 * 1..32, null pointers, too large), LREI_E_DEVICE. */
LREI_API lrei_status lrei_apply_hamiltonian_noalloc(lrei_ctx *ctx, int r, const void *X, void *Y);

/* Checkpoint: the state (n, r, lambda, V, step counter, AB history) as an
 * opaque byte string.  With buf == NULL, *len receives the size needed. */
LREI_API lrei_status lrei_get_state(lrei_ctx *ctx, void *buf, size_t *len);
LREI_API lrei_status lrei_set_state(lrei_ctx *ctx, const void *buf, size_t len);

/* Measurement: times each kernel of one step of the given configuration with
 * HIP events on the context's stream, averaged over `iters` launches of the
 * same kernel with the same arguments and launch shape the step uses:
 *   ms[0] Chebyshev H.V pass with fused Gram products (recurrence form),
 *   ms[1] partial-sum reduction, ms[2] projected step kernel,
 *   ms[3] basis combination.
 * Needs one completed lrei_step with this configuration (the projected
 * kernel reads that step's Gram products).  The state is not modified: the
 * combination writes to a scratch block. */
LREI_API lrei_status lrei_profile_kernels(lrei_ctx *ctx, int model, int scheme, double dt, double kappa,
                                          int iters, double ms[4]);

/* Blocks until all work queued by this context has finished. */
LREI_API lrei_status lrei_synchronize(lrei_ctx *ctx);

/* Result of lrei_autotune. */
#define LREI_TUNE_MAX 128
typedef struct {
  int epl;                 /* complex columns per lane chosen for the H.V pass          */
  int grid;                /* workgroups per H.V launch chosen                           */
  int win_bits;            /* row-bit window of the H.V sweeps (0: one sweep)            */
  int n_sweeps;            /* sweeps per H.V pass for that window                        */
  double ms;               /* time of one H.V pass (all sweeps) of the chosen variant    */
  int from_cache;          /* 1: read from opt.autotune_cache without timing             */
  int n_tried;             /* variants timed (at most LREI_TUNE_MAX)                     */
  int tried_epl[LREI_TUNE_MAX], tried_grid[LREI_TUNE_MAX], tried_win[LREI_TUNE_MAX];
  double tried_ms[LREI_TUNE_MAX];
  int tile_bits;           /* tiled pass: 2^tile_bits rows of P held in LDS per workgroup
                              (0: an untiled pass)                                       */
  int tile_waves;          /* tiled pass: waves per workgroup (8 or 16)                  */
  int tried_tile[LREI_TUNE_MAX]; /* per variant: 100 tile_bits + tile_waves for the tiled
                              pass, 1 for the untiled pass with compacted gathers, 0 for
                              the untiled pass                                            */
  int compact;             /* 1: the untiled pass with compacted gathers (each row walks
                              only the terms whose coefficient is non-zero for it; r <= 16,
                              at most 64 off-diagonal terms)                              */
  int overlap_grid;        /* workgroups of the passes of a step after the first, which
                              run beside the one-workgroup stage kernels: grid less the
                              workgroups of two CUs per XCD when grid fills every CU and
                              the pass takes the dynamic chunk schedule, else grid        */
} lrei_tune_result;

/* Chooses the launch shape of the matrix-free H.V pass (eq. 5.1 applied in
 * the Krylov passes) for the current Hamiltonian, rank and precision:
 * every valid (columns per lane, workgroups, row-bit window, tiled / untiled /
 * compacted gathers) choice is timed on
 * the device with the current state as input (5 passes each) and the fastest
 * is kept for this context.  A window of w row bits splits the pass into
 * sweeps, each applying the terms whose flip masks fit one window, so that one
 * XCD's L2 holds the rows a sweep gathers from.  With opt.autotune_cache set, a matching line of that text
 * file (device, n, r, precision, term count) is used instead of timing, and a
 * new result is appended to it.  Results are unaffected; only speed changes.
 * Requires lrei_set_rho; overwrites the scratch Krylov blocks (not the state).
 * out may be NULL.  Errors: LREI_E_STATE without a state, LREI_E_DEVICE. */
LREI_API lrei_status lrei_autotune(lrei_ctx *ctx, lrei_tune_result *out);

/* ---- Batched trajectories ---------------------------------------------------
 * Many independent LREI trajectories (each its own Hamiltonian, rank, model
 * and damping) advanced together: every kernel of a step runs once for the
 * whole batch (one launch per kernel and launch shape, the trajectories'
 * work concatenated in the grid), so small problems do not each pay for
 * their own launches.  Each trajectory computes exactly what a single
 * context would (Sec. 3.7 steps with the same stage algebra); only the
 * launch packing differs.  Sites are stored in their natural order (site i in
 * bit i). */
typedef struct lrei_batch lrei_batch;

/* One trajectory: Hamiltonian as for lrei_set_hamiltonian (eq. 5.1, Pauli
 * form; site_h may be NULL), initial state as for lrei_set_rho (host
 * complex128 V, N x r, orthonormal columns; lambda positive, non-increasing),
 * model (lrei_model) and damping kappa >= 0.  The arrays are copied by
 * lrei_batch_create. */
typedef struct {
  int n_spins;             /* 1 <= n <= 30                                      */
  int n_bonds;
  const int32_t *bond_ij;  /* [n_bonds][2], 0 <= i < j < n                      */
  const double *bond_J;    /* [n_bonds][3][3]                                   */
  const double *site_h;    /* [n][3] or NULL                                    */
  int r;                   /* 1 <= r <= 32, r <= 2^n                            */
  const double *lambda;    /* [r]                                               */
  const void *V;           /* host [2^n][r] complex128                           */
  int model;               /* LREI_QLL or LREI_QLLG                              */
  double kappa;
} lrei_traj_desc;

/* Creates a batch of n_traj (1..1024) trajectories on HIP device hip_device
 * (stream as for lrei_create; opt may be NULL; opt->precision applies to all
 * trajectories).  Validates every trajectory (LREI_E_INVALID names the first
 * bad one; nothing is created) and uploads the states.  hbar > 0 is shared. */
LREI_API lrei_status lrei_batch_create(lrei_batch **out, int hip_device, void *hip_stream, const lrei_options *opt,
                                       int n_traj, const lrei_traj_desc *traj, double hbar);
LREI_API void lrei_batch_destroy(lrei_batch *b);
/* Message of the last failure on b (or of the last failed lrei_batch_create
 * when b is NULL). */
LREI_API const char *lrei_batch_last_error(const lrei_batch *b);

/* Advances every trajectory by n_steps >= 0 steps of size dt > 0 with the
 * LREI-RK scheme `scheme` (RK1..RK4; Adams-Bashforth is not batched).  One
 * step is captured as a hipGraph on first use of a (scheme, dt) pair and
 * replayed (opt->use_graph).  If any trajectory produces non-finite values,
 * every trajectory is restored to its state at the start of the call and
 * LREI_E_NUMERIC names the first failing trajectory. */
LREI_API lrei_status lrei_batch_step(lrei_batch *b, int scheme, double dt, int n_steps);

/* Copies trajectory traj's state out (as lrei_get_rho); lambda or V may be NULL. */
LREI_API lrei_status lrei_batch_get_rho(lrei_batch *b, int traj, double *lambda, void *V, int v_is_device);

/* Energy Tr(Lambda_0 V* H V) of every trajectory's current state (Sec. 3.6),
 * energy[n_traj]. */
LREI_API lrei_status lrei_batch_energies(lrei_batch *b, double *energy);

/* Measurement: average per-launch-set times (ms) over `iters` repetitions,
 * with HIP events on the batch's stream, of the kernels of one step of the
 * whole batch:  ms[0] one Krylov H.V pass (recurrence form) with fused
 * Grams, all launch classes; ms[1] its reduction; ms[2] the s stages of the
 * projected step run back to back; ms[3] the basis combinations (written to
 * the rollback copies, so the state is unchanged).  Needs a completed
 * lrei_batch_step with the same scheme and dt (LREI_E_STATE otherwise). */
LREI_API lrei_status lrei_batch_profile_kernels(lrei_batch *b, int scheme, double dt, int iters, double ms[4]);

/* Blocks until all work queued by the batch has finished. */
LREI_API lrei_status lrei_batch_synchronize(lrei_batch *b);

#define LREI_BATCH_TUNE_CLASSES 32

typedef struct {
  int n_classes;                       /* distinct ranks r in the batch                */
  int rank[LREI_BATCH_TUNE_CLASSES];   /* class k's rank, ascending                    */
  int epl[LREI_BATCH_TUNE_CLASSES];    /* chosen complex columns per lane (0: default) */
  int wg_cap[LREI_BATCH_TUNE_CLASSES]; /* chosen cap on workgroups per trajectory and
                                          pass (one per 64-row tile up to the cap; 256
                                          by default)                                  */
  double ms_default;                   /* one batched Krylov pass of every trajectory
                                          and its Gram reduction, shapes as on entry   */
  double ms;                           /* the same with the chosen shapes              */
  int n_tried;                         /* candidates timed (records kept for at most
                                          LREI_TUNE_MAX)                               */
  int tried_rank[LREI_TUNE_MAX], tried_epl[LREI_TUNE_MAX], tried_cap[LREI_TUNE_MAX];
  double tried_ms[LREI_TUNE_MAX];
} lrei_batch_tune_result;

/* Chooses the launch shape of the batched H.V pass (eq. 5.1 in the Krylov
 * passes of Sec. 3.7) per rank class: for each distinct r in turn, every
 * valid columns-per-lane value and workgroup cap (16 .. 1024 per trajectory)
 * is set for all trajectories of that rank, and one pass of the whole batch
 * plus its reduction is timed on the device (`iters` >= 1 repetitions after
 * one warm-up, HIP events on the batch stream); the fastest is kept, then the
 * next class is tuned with it in place.  Overwrites only the scratch Krylov
 * blocks; the state is untouched.  Results change at rounding level (the
 * Gram partial sums are split over a different number of workgroups); the
 * captured step graph is rebuilt on the next lrei_batch_step.  out may be
 * NULL.  On failure the shapes from before the call are restored; should
 * that rebuild fail too, every later call on b returns LREI_E_STATE.
 * Errors: LREI_E_INVALID, LREI_E_NOMEM, LREI_E_DEVICE, LREI_E_STATE. */
LREI_API lrei_status lrei_batch_autotune(lrei_batch *b, int iters, lrei_batch_tune_result *out);

/* Rank r of the current state (LREI_E_STATE before a state is set). */
LREI_API lrei_status lrei_get_rank(lrei_ctx *ctx, int *r);

/* Sets rho = A A* / Tr(A A*) from a factor A (N x m complex128, row-major,
 * natural basis order, host or device; columns need not be orthonormal),
 * 1 <= m <= min(32, N): the partial eigendecomposition the run starts from
 * (Sec. 3.7), computed on the GPU from the Gram matrix A* A; eigenvalues at or
 * below 1e-14 of the largest are dropped, so r = rank rho (read it with
 * lrei_get_rho).  Requires a Hamiltonian; errors as lrei_set_rho, plus
 * LREI_E_INVALID for a zero factor. */
LREI_API lrei_status lrei_set_rho_factor(lrei_ctx *ctx, int m, const void *A, int a_is_device);

/* Maximally mixed admixture (Sec. 5, a full-rank state): from this call on
 * the context's state is rho = p I / N + (1 - p) V Lambda V*, p in [0, 1)
 * (0 by default).  lrei_step evolves the low-rank part V Lambda V* with
 * damping (1 - p) kappa, which the paper shows gives the solution from
 * rho; lrei_observables and lrei_pair_density report rho's values
 * (Tr(A rho) = p Tr(A) / N + (1 - p) Tr(A V Lambda V*), with Tr(A) = 0 for
 * the energy and the magnetisation; R_kl gains p I / 4); lrei_get_rho,
 * lrei_set_rho and checkpoints hold the low-rank part only.  Resets an AB
 * history.  LREI_E_INVALID if p is outside [0, 1). */
LREI_API lrei_status lrei_set_mixing(lrei_ctx *ctx, double p);

/* Two-spin reduced density matrices R_kl = Tr_rest(rho) of the current state
 * (Sec. 3.6: the partial trace over every spin but k and l) for n_pairs
 * (1..4096) site pairs.  pairs (host): 2 n_pairs site indices, k != l, both
 * < n.  out (host, 32 n_pairs doubles): per pair a 4 x 4 complex matrix,
 * row-major, (re, im) pairs; row and column index q = 2 b_k + b_l, b the
 * site's spin bit (0 = up).  One fused pass over the state per pair, FP64
 * accumulation.  Errors: LREI_E_STATE (no state), LREI_E_INVALID (sites),
 * LREI_E_NOMEM, LREI_E_DEVICE. */
LREI_API lrei_status lrei_pair_density(lrei_ctx *ctx, int n_pairs, const int *pairs, double *out);

/* Entanglement of a two-spin density matrix R (32 doubles laid out as
 * above), computed on the host (Sec. 3.6 names these measures):
 * concurrence max(0, l1 - l2 - l3 - l4) with l_i the square roots of the
 * eigenvalues of R (sy x sy) conj(R) (sy x sy), descending (Wootters);
 * negativity, the sum of |negative eigenvalues| of the partial transpose on
 * the second spin (Vidal and Werner); chsh, the largest CHSH expectation
 * 2 sqrt(m1 + m2) with m1 >= m2 the two largest eigenvalues of T^T T,
 * T_ij = Tr(R s_i x s_j) (Horodecki).  Any output may be NULL.
 * LREI_E_INVALID if R is NULL or not finite. */
LREI_API lrei_status lrei_pair_entanglement(const double *R, double *concurrence, double *negativity,
                                            double *chsh);

/* ---- Learned start rotation (production form on top of the stage
 * eigensolve of Sec. 3.7; the paper has no such component) ----------------
 *
 * A network (lrei_net) is a multilayer perceptron for one rank r (1..16): 2 r^2 + 2 inputs
 * (Re, Im of G / |G|_F with G = u* H u the stage input basis' projected
 * generator, s |G|_F with s the stage's step over hbar, kappa), three hidden
 * layers of width 256 with SiLU, r^2 outputs o that correct the analytic
 * generator -i s G: A is unpacked from o + o_an (A_aa = i o_a, then the
 * upper off-diagonal entries row by row as (re, im) pairs; o_an the same
 * parametrisation of -i s G read off the features), and
 * R = (I - A/2)^{-1} (I + A/2).  Parameters: one FP32 vector, W1 [in x 256]
 * row-major, b1, W2, b2, W3, b3, W4 [256 x r^2], b4.
 *
 * A training sample (net_sample_floats(r) = 2 r^2 + 2 + 2 r^2 floats) is the
 * features of one RK stage followed by T = u* u_next, r x r row-major (re, im)
 * pairs, u_next the stage's output eigenvectors.  The loss of a sample is
 * sum_a (1 - |(R* T)_aa|^2).  Sample buffers are device memory of the
 * caller; every call below is synchronous. */
typedef struct lrei_net lrei_net;

/* Number of parameters of a network of rank r, or -1 if r is out of range. */
LREI_API long long lrei_net_param_count(int r);

/* New network on HIP device hip_device.  init: host array of
 * lrei_net_param_count(r) floats, or NULL for a seeded initialisation
 * (hidden-layer weights uniform in +-1/sqrt(fan_in), splitmix64 from seed;
 * output layer and biases zero, so the new network gives the analytic
 * rotation).  Errors: LREI_E_INVALID (r), LREI_E_DEVICE,
 * LREI_E_NOMEM; *out is NULL then. */
LREI_API lrei_status lrei_net_create(lrei_net **out, int hip_device, int r, const float *init, uint64_t seed);
LREI_API void lrei_net_destroy(lrei_net *m);
LREI_API const char *lrei_net_last_error(const lrei_net *m);
LREI_API int lrei_net_rank(const lrei_net *m);

/* Copies of the parameters to / from host memory (set also resets Adam). */
LREI_API lrei_status lrei_net_get_params(lrei_net *m, float *host);
LREI_API lrei_status lrei_net_set_params(lrei_net *m, const float *host);

/* Mean loss over the n (1..65536) samples at device address samples and, if
 * grad_host is not NULL, its gradient with respect to the parameters. */
LREI_API lrei_status lrei_net_loss_grad(lrei_net *m, const float *samples, int n, double *loss_out,
                                          float *grad_host);

/* The network's rotations for the features of n samples: R_host receives
 * n r x r complex matrices, row-major, as (re, im) doubles. */
LREI_API lrei_status lrei_net_rotations(lrei_net *m, const float *samples, int n, double *R_host);

/* Adam (beta 0.9, 0.999, eps 1e-8, step size lr) over `epochs` passes of the
 * n samples in batches of `batch` (1..4096; a last partial batch is skipped),
 * reshuffled per epoch from shuffle_seed.  epoch_loss (host, `epochs`
 * doubles, or NULL) receives each epoch's mean loss before its updates. */
LREI_API lrei_status lrei_net_train(lrei_net *m, const float *samples, int n, int batch, int epochs, float lr,
                                      uint64_t shuffle_seed, double *epoch_loss);

/* Recording of training samples by a context's RK steps: every stage whose
 * rank is <= 16 appends one sample to `samples` (device memory, room for
 * `capacity` samples of the context's rank) until it is full; capacity 0
 * stops recording.  The count restarts at 0 with each call. */
LREI_API lrei_status lrei_record(lrei_ctx *ctx, float *samples, int capacity);
/* Samples written so far (at most the capacity). */
LREI_API lrei_status lrei_record_count(lrei_ctx *ctx, int *count);

/* Attaches a network (its rank must equal the context's) for LREI_WARM_LEARNED;
 * NULL detaches.  The context reads the network's parameters while stepping,
 * so the network must outlive the attachment; training it in between changes
 * what the next steps use. */
LREI_API lrei_status lrei_attach_net(lrei_ctx *ctx, const lrei_net *m);

#ifdef __cplusplus
}
#endif

#endif /* LREI_H */
