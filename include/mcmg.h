/*
 * mcmg.h -- C ABI of the MI355X (gfx950) McMg solver library, libmcmg.so.
 *
 * McMg (arXiv 2606.30495) is a learned multi-channel multigrid
 * preconditioner for the heterogeneous Helmholtz equation
 *     -Lap u - k(x)^2 u = f,   k = omega / c          (Sec. 2.1, Eq. helm)
 * discretised with the 5-point (2D) / 7-point (3D) finite-difference stencil
 * (Eq. FDM_stencil) and a perfectly matched layer (App. A.1.1).  A setup
 * phase turns c(x) into cached per-level features (Alg. 1); the V-cycle
 * MG(r) ~ A^{-1} r (Sec. 3.2, Alg. 2) then preconditions a restarted,
 * right-preconditioned flexible GMRES (Sec. 3.3: McMg as a GMRES
 * preconditioner; Sec. 4.1: relative tolerance 1e-6, preconditioner in
 * reduced precision, residual in FP64).
 *
 * Conventions shared by every entry point
 *  - Grids: the caller gives the INTERIOR grid (n[0] x n[1] (x n[2]) nodes,
 *    spacing h, row-major, last axis fastest).  The library adds a PML of
 *    `pml.ncells` cells on every side; the EXTENDED grid has
 *    n_ext[a] = n[a] + 2 * ncells nodes per axis.  Right-hand sides,
 *    solutions and residuals live on the extended grid.
 *  - Complex fields are interleaved complex128 (double re, double im),
 *    row-major over the extended grid, in DEVICE memory, unless stated.
 *  - All work is issued on the handle's stream (mcmg_opts.stream); apply and
 *    matvec return without synchronising, solve returns when done.
 *  - No entry point throws; every failure returns a negative mcmg_status
 *    and mcmg_last_error() (thread-local) describes it.
 *  - A handle is not thread safe; distinct handles are independent.
 */
#ifndef MCMG_H
#define MCMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MCMG_OK = 0,
  MCMG_NOT_CONVERGED = 1,     /* maxit reached; u holds the best iterate   */
  MCMG_E_ARG = -1,            /* invalid argument or shape                 */
  MCMG_E_OOM = -2,            /* device allocation failed                  */
  MCMG_E_HIP = -3,            /* a HIP runtime call failed                 */
  MCMG_E_WEIGHTS = -4,        /* weight blob malformed or not matching     */
  MCMG_E_NONFINITE = -5,      /* NaN/Inf in the input or the iteration     */
  MCMG_E_BREAKDOWN = -6,      /* Krylov breakdown without convergence      */
  MCMG_E_BUDGET = -7          /* request exceeds the server's HBM budget   */
} mcmg_status;

typedef enum { MCMG_FP32 = 0, MCMG_BF16 = 1 } mcmg_precision;

typedef struct { int dim; int n[3]; } mcmg_grid;           /* interior nodes */

/* Absorbing layer of ncells cells on every side of the interior grid.
 * kind MCMG_ABL_PML (App. A.1.1): complex stretching s = 1 + i sigma,
 *   sigma = sigma_max (d / ncells)^2 (d = cells into the layer), operator in
 *   divergence form; sigma_max <= 0 selects 3 ln(1e6) / (2 (omega / max c)
 *   ncells h) (round-trip factor 1e-6).
 * kind MCMG_ABL_SPONGE (Sec. 2.1): -Lap u - k^2 (1 + i gamma) u with
 *   gamma = sigma_max min(1, sum_a (d_a / ncells)^2) (d_a = cells into the
 *   layer along axis a); sigma_max <= 0 selects 3 ln(1e6) / ((omega / max c)
 *   ncells h).  The damping sign is the one that absorbs waves leaving the
 *   domain under the radiation condition of Eq. helm (outgoing e^{+ikr}). */
enum { MCMG_ABL_PML = 0, MCMG_ABL_SPONGE = 1 };
typedef struct { int ncells; double sigma_max; int kind; } mcmg_pml;

/* Self-describing weight blob (host memory; copied by mcmg_setup).
 * Header: magic "MCMGWB01", version 1, dim, levels L <= 8, ksize 3,
 * channels[8], nu1[8], nu2[8], tensor count; then a tensor table and
 * float32 tensors [d0][d1][3^dim].  Tensor set (Sec. 3.1-3.2): f_lift,
 * g_lift, g_proj; per level f_s, W, KA, KS, Wsm^(1..nu1+nu2) (nu1 at the
 * coarsest level); per level l < L also f_a, R, P.  C_1 must be 2. */
typedef struct { const void* blob; size_t bytes; } mcmg_weights;

typedef struct {
  int precision;   /* mcmg_precision of the V-cycle convolutions           */
  int restart;     /* FGMRES restart length m (1..1024; 0 selects 30);
                      batched solves and the server take m <= 64          */
  void* stream;    /* hipStream_t for all work; NULL = default stream      */
  int ortho;       /* 0: classical Gram-Schmidt with re-orthogonalisation
                      when the norm drops below 1/sqrt(2) (default);
                      1: always two passes                                 */
} mcmg_opts;

typedef struct {
  int iters;            /* preconditioner applications (all restarts)      */
  int restarts;         /* completed cycles                                */
  double relres_true;   /* |f - A u|_2 / |f|_2 in FP64 at exit             */
  double relres_est;    /* last least-squares residual estimate / |f|      */
  int status;           /* mcmg_status of the solve                        */
  double* hist;         /* optional host array (caller-owned): estimate
                           |g_{j+1}| / |f| after every iteration           */
  int hist_cap;         /* capacity of hist                                */
  int hist_len;         /* entries written                                 */
} mcmg_info;

typedef struct mcmg_ctx* mcmg_handle;

/* Setup phase (Alg. 1, once per medium).  c: HOST float64 interior wave
 * speed (all > 0, finite).  omega > 0: angular frequency; h > 0: grid
 * spacing.  The handle copies everything it needs (speed, PML tables,
 * weights, per-level features a_l, s_l, V-cycle and Krylov workspace), so
 * the caller may free its inputs on return.  Errors: E_ARG (shape, values),
 * E_WEIGHTS (blob/dim/level mismatch, a level side < 2), E_OOM, E_HIP. */
mcmg_status mcmg_setup(const double* c, mcmg_grid grid, double omega, double h,
                       mcmg_pml pml, mcmg_weights w, const mcmg_opts* opt,
                       mcmg_handle* out);

/* z = MG(r): one V-cycle (Alg. 2).  r, z: device complex128 on the extended
 * grid; may not alias.  Asynchronous on the handle's stream. */
mcmg_status mcmg_apply(mcmg_handle h, const double* r, double* z);

/* z = MG(r) like mcmg_apply, for callers that cannot allocate device memory
 * (code under stream capture, serving loops that forbid hipMalloc): the
 * V-cycle's level state lives in a static device array of the library
 * (64 MiB on every GPU the library runs on, held until the process ends)
 * instead of the handle's buffers.  Same kernels and summation order as
 * mcmg_apply, so the same bits.  Allocates nothing (device or host); the
 * array's device address is looked up once per device.  A grid whose level
 * state needs more than 64 MiB is refused with MCMG_E_ARG.  Every call on
 * one GPU shares that GPU's array: calls that overlap on one GPU (several
 * streams or threads) race.  Asynchronous on the handle's stream. */
mcmg_status mcmg_apply_noalloc(mcmg_handle h, const double* r, double* z);

/* Au = A u in FP64 (Eq. FDM_stencil with the PML of App. A.1.1).  u, Au:
 * device complex128 on the extended grid; may not alias.  Asynchronous. */
mcmg_status mcmg_matvec(mcmg_handle h, const double* u, double* Au);

/* Restarted right-preconditioned FGMRES(m) with MG as the preconditioner.
 * f: device rhs; u: device in/out (initial guess in, solution out).  Stops
 * when the FP64 true residual |f - A u| <= tol |f|, or after maxit
 * preconditioner applications (returns MCMG_NOT_CONVERGED with the best u).
 * A Hessenberg column that is zero after the earlier rotations (for example
 * MG(v_j) = 0) is left out of the cycle's triangular solve; when it is the
 * first column of a cycle the solve returns MCMG_NOT_CONVERGED with u
 * unchanged, since a restart would repeat the same cycle.
 * info may be NULL.  Blocks until done. */
mcmg_status mcmg_solve(mcmg_handle h, const double* f, double* u, double tol,
                       int maxit, mcmg_info* info);

/* Stationary McMg iteration u <- u + MG(f - A u) (Sec. 3.3,
 * Eq. mcmg_iteration), same arguments and stopping rule as mcmg_solve. */
mcmg_status mcmg_stationary(mcmg_handle h, const double* f, double* u,
                            double tol, int maxit, mcmg_info* info);

/* ---- Training (training section, Eq. loss_fun; Sec. llpf) ----------------
 *
 * The loss of a batch of B samples (handle i: medium k_i, device residual
 * r_i, complex128 on that handle's extended grid) is
 *   L_H = (1/B) sum_i |A_i MG(k_i, r_i) - r_i| / |r_i|.
 * A is applied in FP64 and MG in float32 with the VALU convolutions of
 * Alg. 1 and Alg. 2.  The gradient comes from reverse accumulation through
 * the setup network and the V-cycle, with A^H for the loss.
 *
 * Parameters use the canonical tensor order and layout of the weight blob,
 * as one float32 vector.  hs[0] owns them, together with the Adam moments;
 * the other handles of a batch must hold the same model (dim, levels,
 * channels, smoothing counts; any media and grid sizes) and get the master's
 * parameters at the start of each step.  After training, mcmg_train_commit
 * refreshes the forms the fast solve path derives from the weights
 * (matrix-core packs, level-1 sweep weights, cached features).  Until then,
 * apply and solve on a trained handle see stale matrix-core weights.
 * Training state is allocated on first use and owned by the handle.  The
 * handles' streams are synchronised; every call blocks. */
typedef struct {
  double lr;       /* > 0 */
  double beta1;    /* [0, 1), 0.9 */
  double beta2;    /* [0, 1), 0.999 */
  double eps;      /* > 0, 1e-8 */
} mcmg_adam;

/* One Adam step on hs[0]'s parameters from the gradient of L_H over the nh
 * samples (hs[i], r[i]); *loss (may be NULL) receives L_H before the
 * update.  Frozen tensors keep their values and moments.  Errors: E_ARG
 * (models differ, bad Adam parameters), E_NONFINITE (|r_i| = 0 or a
 * non-finite loss), E_OOM, E_HIP. */
mcmg_status mcmg_train_step(mcmg_handle* hs, int nh, const double* const* r,
                            const mcmg_adam* opt, double* loss);

/* L_H and its gradient (host float32 vector of ngrad = the model's float
 * count, canonical order) without an update. */
mcmg_status mcmg_train_loss_grad(mcmg_handle* hs, int nh, const double* const* r,
                                 double* loss, float* grad, size_t ngrad);

/* LLPF: mask[i] != 0 makes canonical tensor i trainable, 0 freezes it
 * (ntensors = the model's tensor count). */
mcmg_status mcmg_train_set_trainable(mcmg_handle h, const int* mask, int ntensors);

/* Re-derive the fast-path weight forms and the cached features from the
 * trained parameters. */
mcmg_status mcmg_train_commit(mcmg_handle h);

/* Tensor and float counts of the handle's model. */
mcmg_status mcmg_weights_size(mcmg_handle h, int* ntensors, size_t* nfloats);

/* The current parameters (trained, if training ran), canonical order,
 * nfloats = mcmg_weights_size's float count, into host memory. */
mcmg_status mcmg_get_weights(mcmg_handle h, float* out, size_t nfloats);

/* ---- Born-series form (appendix on the Born-series variant; appendix on
 * the discrete Green operator, Eq. discrete_symbol) ----------------------
 *
 * The Born solvers act on the PERIODIC operator of the extended grid,
 *   A_per u = -Lap_h^per u - k^2 (1 + i gamma) u,
 * which the FFT diagonalises exactly.  They need the sponge layer
 * (MCMG_ABL_SPONGE) or npml = 0; a PML stretches the Laplacian and is
 * rejected with MCMG_E_ARG.  Each extended side must lie in [2, 5120].
 *
 * The background uses the CBS parameters (Eq. cbs_gamma):
 *   k0^2 = (min k^2 + max k^2) / 2,
 *   V    = k^2 (1 + i gamma) - k0^2,
 *   eps  = max |V|.
 * The Green operator carries the same absorption:
 *   G = (-Lap_h^per - k0^2 - i eps)^{-1}.
 * The Born-series residual is G (f - A_per u). */
enum { MCMG_BORN_MCMG = 0, MCMG_BORN_CBS = 1 };

/* Fix the background (k0sq > 0, eps > 0), or take the defaults above for
 * a value <= 0 (found by device reductions).  The first Born call on a
 * handle without this call uses the defaults.  Builds the per-axis FFT
 * tables once (a few n_a-long device arrays owned by the handle).  Blocks.
 * Errors: E_ARG (a PML, a side out of range, eps = 0 for a constant medium
 * with no sponge), E_OOM, E_HIP. */
mcmg_status mcmg_born_setup(mcmg_handle h, double k0sq, double eps);

/* The background in use (sets up the defaults first if needed). */
mcmg_status mcmg_born_params(mcmg_handle h, double* k0sq, double* eps);

/* y = G x: FFT, divide by sum_a (4/h^2) sin^2(pi m_a / n_a) - k0^2 - i eps,
 * then the inverse FFT, all in FP64.  x, y: device complex128 on the
 * extended grid; they may alias.  Asynchronous on the handle's stream. */
mcmg_status mcmg_born_green(mcmg_handle h, const double* x, double* y);

/* Au = A_per u in FP64.  u, Au: device complex128; may not alias.
 * Asynchronous. */
mcmg_status mcmg_born_matvec(mcmg_handle h, const double* u, double* Au);

/* Born-series iteration u <- u + P(G (f - A_per u)):
 *   method MCMG_BORN_MCMG: P = MG, one V-cycle in the handle's precision
 *     (Born+McMg);
 *   method MCMG_BORN_CBS: P = gamma (.), gamma = 1 + i V / eps
 *     (Eq. cbs_eq).
 * It stops when the FP64 true residual |f - A_per u| <= tol |f|, or after
 * maxit updates (MCMG_NOT_CONVERGED).  f, u: device complex128 (u in/out).
 * info (iters, relres_true, hist) may be NULL.  Blocks until done. */
mcmg_status mcmg_born_solve(mcmg_handle h, int method, const double* f, double* u,
                            double tol, int maxit, mcmg_info* info);

/* Batched FGMRES (many media and right-hand sides, uneven sizes, advanced
 * together, one launch per operation for the whole batch).  hs[i] is the
 * handle of problem i (the same handle may appear several times); f[i],
 * u[i] are device arrays on that handle's extended grid.  All handles must
 * share dim, level count, channels, smoothing counts, precision and restart
 * length (MCMG_E_ARG otherwise).  Every problem restarts on its own schedule
 * and gets exactly the iterates mcmg_solve gives it alone.  The handles'
 * streams are drained first; the batch runs on a stream of its own and the
 * call blocks until all problems are done.  A handle that appears k times
 * holds k workspaces afterwards (kept for later batches, freed with the
 * handle).  infos: nb entries or NULL.  Returns the first negative status
 * of any problem, else MCMG_NOT_CONVERGED if any stopped at maxit. */
mcmg_status mcmg_solve_batch(mcmg_handle* hs, const double* const* f,
                             double* const* u, int nb, double tol, int maxit,
                             mcmg_info* infos);

/* Extended-grid query: dim, n_ext[0..dim-1], PML cells per side. */
mcmg_status mcmg_grid_shape(mcmg_handle h, int* dim, int n_ext[3], int* npml);

/* Bytes of device memory the handle holds. */
size_t mcmg_device_bytes(mcmg_handle h);

void mcmg_destroy(mcmg_handle h);
const char* mcmg_last_error(void);

/* Per-launch timing (measurement hook).  mcmg_prof_enable(h, 1) makes the
 * handle record a HIP event pair around every kernel launch it issues on its
 * stream, together with the launch's algorithmic flops and bytes (from the
 * shapes, not counters); mcmg_prof_report() synchronises, aggregates the
 * records per kernel symbol into a JSON array of {name, launches, total_ms,
 * avg_ms, flops_per_launch, bytes_per_launch} written to buf (host, cap
 * bytes).  E_ARG if buf is too small.  mcmg_prof_enable() (on or off)
 * clears the records.  mcmg_prof_replay() re-issues the recorded launches of
 * the kernel `name`, reps times, back to back between ONE event pair on the
 * handle's stream and returns the average duration per launch (without the
 * per-launch event overhead of the records); the replayed launches write the
 * handle's work buffers and the caller's buffers they name, so call it
 * between solves. */
mcmg_status mcmg_prof_enable(mcmg_handle h, int on);
mcmg_status mcmg_prof_report(mcmg_handle h, char* buf, size_t cap);
mcmg_status mcmg_prof_replay(mcmg_handle h, const char* name, int reps, double* avg_ms,
                             int* launches);

/* Test hooks: replace / read level l's (1-based) cached features a_l, s_l
 * (device float32 [nodes][C_l], row-major nodes, channel fastest).  Used to
 * reduce the V-cycle to a textbook multigrid with hand-set features. */
mcmg_status mcmg_debug_set_features(mcmg_handle h, int level, const float* a,
                                    const float* s);
mcmg_status mcmg_debug_get_features(mcmg_handle h, int level, float* a, float* s);
mcmg_status mcmg_debug_level_shape(mcmg_handle h, int level, int n[3], int* channels);

/* ---- Serving loop -----------------------------------------------------------
 * A server owns media (handles after their setup phase: features, operator
 * tables, weights stay resident) and solves requests of 1..n right-hand
 * sides on them with continuous batching: a worker thread advances every
 * right-hand side in flight by one FGMRES step per tick (the batch engine of
 * mcmg_solve_batch: one launch per operation for all of them, captured in a
 * HIP graph while the set is unchanged), admits queued requests between
 * ticks as workspace slots and HBM budget free up, and retires right-hand
 * sides as they converge.  Media of different families (2D / 3D, level
 * structures, precision) advance on separate streams, so their work
 * overlaps on the device.  Every result is bitwise the one mcmg_solve gives
 * the same handle, right-hand side and initial guess alone.
 *
 * Memory: the budget covers every medium's handle (mcmg_device_bytes at
 * admission, which includes one workspace) plus every extra workspace slot
 * (Krylov basis V in FP64, Z in FP32, V-cycle level state).  Requests are
 * admitted in arrival order; a request waits until all of its right-hand
 * sides fit (idle slots of other media are released to make room).  */
typedef struct mcmg_server_s* mcmg_server;

typedef struct {
  size_t hbm_budget;   /* bytes the server may hold on the device (> 0)     */
  int max_inflight;    /* cap on right-hand sides in flight; 0 = no cap     */
  int graphs;          /* 1: replay captured ticks (default); 0: launches   */
} mcmg_server_opts;

typedef struct {
  uint64_t req_id;
  int status;          /* worst mcmg_status of its right-hand sides         */
  int nrhs;
  int iters_total;     /* preconditioner applications over its rhs          */
  int iters_max;
  double relres_max;   /* largest FP64 true relative residual at exit       */
  double queue_s;      /* submit -> admitted (seconds)                      */
  double latency_s;    /* submit -> every solution written (seconds)        */
} mcmg_completion;

typedef struct {
  size_t bytes_in_use;     /* media + slots now allocated                   */
  size_t bytes_peak;
  int media, slots, inflight, queued, completed;
  int inflight_peak;       /* most right-hand sides in flight at once       */
  long long ticks;         /* engine ticks issued                           */
  long long rebuilds;      /* composition changes (tables rebuilt)          */
} mcmg_server_stats;

/* E_ARG for a null or zero budget.  The worker thread starts at once. */
mcmg_status mcmg_server_create(const mcmg_server_opts* opts, mcmg_server* out);

/* Adds a medium: runs mcmg_setup with these arguments (opt->stream is
 * ignored).  E_BUDGET when its handle does not fit next to the media
 * already held; *medium_id is the medium's index (0, 1, ...). */
mcmg_status mcmg_server_add_medium(mcmg_server s, const double* c, mcmg_grid grid,
                                   double omega, double h, mcmg_pml pml, mcmg_weights w,
                                   const mcmg_opts* opt, int* medium_id);

/* Adds an existing handle as a medium; the server takes ownership (the
 * caller must not use or destroy it afterwards, also on error). */
mcmg_status mcmg_server_add_handle(mcmg_server s, mcmg_handle h, int* medium_id);

/* Queues a request of nrhs right-hand sides on medium_id.  f[i], u[i]:
 * device complex128 on the medium's extended grid; u[i] is the initial
 * guess in and the solution out.  The caller keeps all of them alive and
 * untouched until the request's completion is polled, and f[i], u[i] must
 * be fully written when this is called (the server's streams do not wait
 * for the caller's).  Returns at once.  E_BUDGET if the request could
 * never fit the budget (or max_inflight); E_ARG for bad arguments. */
mcmg_status mcmg_server_submit(mcmg_server s, int medium_id, const double* const* f,
                               double* const* u, int nrhs, double tol, int maxit,
                               uint64_t* req_id);

/* Moves up to max finished requests into out (oldest first), waiting up to
 * wait_ms milliseconds for the first one (0: no wait).  Returns the
 * worker's error (negative) if it stopped on one; the requests it held are
 * then completed with that status. */
mcmg_status mcmg_server_poll(mcmg_server s, mcmg_completion* out, int max, int* n,
                             int wait_ms);

mcmg_status mcmg_server_get_stats(mcmg_server s, mcmg_server_stats* out);

/* Stops the worker (requests still queued or in flight are abandoned; their
 * buffers are no longer touched once this returns) and frees every medium. */
void mcmg_server_destroy(mcmg_server s);

#ifdef __cplusplus
}
#endif
#endif /* MCMG_H */
