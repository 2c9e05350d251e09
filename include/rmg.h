/*
 * rmg.h - C ABI of the batched Picard-multigrid sampler for the stochastic
 * Richards equation (gfx950 / MI355X).
 *
 * Method: Kumar, Rodrigo, Gaspar, Oosterlee, "A parametric acceleration of
 * multilevel Monte Carlo convergence for nonlinear variably saturated flow".
 *   - random fields: Section 3, eqs. RandK and KLexp (lognormal Ks from a
 *     truncated Karhunen-Loeve expansion);
 *   - time stepping: Section 4.1, eqs. Mixed_based .. Mixed_based_3 (backward
 *     Euler on the mixed form, modified Picard iteration, ||dp||_inf stop);
 *   - linear solver: Section 4.2, eq. five_stencil and eq. transfer (cell-centred
 *     multigrid, harmonic-mean faces, arithmetic-mean face upscaling,
 *     piecewise-constant prolongation, restriction = prolongation^T / 4);
 *   - estimator: Section 5.1, eqs. telescope, MLMCestimator, SMC, ML_var.
 *
 * Conventions shared by every entry point
 *   Domain (0,1)^2, n x n cells, h = 1/n, n a power of two (range per entry point).
 *   Cell c = j*n + i, x (index i) fastest, j = 0 the bottom row, z up.
 *   Top (z = 1) and bottom (z = 0) faces are Dirichlet, the sides are no-flux.
 *   Pointers named d_* are device memory, h_* host memory; all are owned by the
 *   caller and must stay valid until the work enqueued on `stream` completes.
 *   The context owns only its workspace (grown on demand, reused across calls,
 *   freed by rmg_ctx_destroy).  A context is not thread safe: calls on one context
 *   must not overlap.  Separate contexts share no host state (beyond each kernel's
 *   dynamic-LDS limit, only ever raised and under a lock, and a tune-cache file given
 *   to several of them, which each rewrites whole), so calls on different
 *   contexts may run at the same time from different host threads; their GPU work
 *   then overlaps (each context has its own streams and workspace) and the results
 *   are those of the calls made one at a time.  Such calls should not confine their
 *   classes (mlmc_level_estimate flag bit 8): the confined classes of every context
 *   run on compute-unit-masked queues with the same masks, and two confined contexts
 *   were measured not to overlap.  A context holds 8 streams, and 8 more with
 *   compute-unit masks (each on a hardware queue of its own) from its first confined
 *   call on.  Two contexts in flight on one device measured best: with three, every
 *   context's streams share the same few hardware queues and the calls slowed down.
 *   (The allocation-free entry point is the exception to all of this: every call on
 *   one GPU shares its scratch array.)
 *   Every call returns an rmg_status; on failure rmg_last_error() explains it.
 *   No C++ exception crosses this interface.
 */
#ifndef RMG_H_
#define RMG_H_

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rmg_ctx rmg_ctx;

typedef enum {
  RMG_OK = 0,
  RMG_EINVAL = -1,    /* invalid argument (shape, pointer, option) */
  RMG_ENOMEM = -2,    /* workspace allocation failed */
  RMG_EHIP = -3,      /* a HIP runtime call failed */
  RMG_ENOTCONV = -4   /* outputs valid, but at least one sample did not converge */
} rmg_status;

/* Per-sample outcome (Section 4.3: a sample fails when the Picard iteration
 * exceeds its iteration limit at some time step).  NONFINITE: a correction was not
 * finite, or the sample's fields hold a non-finite value (such a sample is not solved). */
typedef enum {
  RMG_SAMPLE_OK = 0,
  RMG_SAMPLE_MAXITER = 1,
  RMG_SAMPLE_NONFINITE = 2
} rmg_sample_status;

typedef enum { RMG_GARDNER = 0, RMG_VGM = 1, RMG_LINEAR = 2 } rmg_model;
typedef enum { RMG_QOI_MEAN_SATURATION = 0, RMG_QOI_BOTTOM_OUTFLUX = 1 } rmg_qoi;
typedef enum { RMG_FP64 = 0, RMG_MIXED = 1 } rmg_precision;
typedef enum { RMG_CYCLE_V = 1, RMG_CYCLE_W = 2 } rmg_cycle;

/* Pointwise marginal of a random field built from the Gaussian KL sum G:
 * value = shift + exp(log_mean + scale * G)  (eq. RandK with Ks_bl = exp(log_mean)). */
typedef struct {
  double shift, log_mean, scale;
} rmg_marginal;

/* One deterministic problem (closure model, boundary and initial data, time grid).
 * qoi must be RMG_QOI_MEAN_SATURATION for the forward entry points; the bottom
 * outflux (RMG_QOI_BOTTOM_OUTFLUX) is the quantity of picard_mg_adjoint;
 * theta_s > theta_r, dt > 0, n_steps >= 1 and init_profile 0 or 1 (with init_rate > 0)
 * are required.
 * Fields per cell: Gardner and linear use field 0 = Ks; van Genuchten-Mualem uses
 * field 0 = Ks, 1 = alpha, 2 = n (so n_fields = 1 or 3).
 *   Gardner: K = Ks e^{a h}, theta = theta_r + (theta_s - theta_r) e^{a h} (h < 0);
 *            saturated (h >= 0): K = Ks, theta = theta_s, C = 0.
 *   vG-Mualem: eqs. Sw, sc_van, Krw with m = 1 - 1/n.
 *   Linear (test only): K = Ks, theta = theta_r + linear_c0 * h. */
typedef struct {
  int32_t model;          /* rmg_model */
  int32_t n_steps;        /* number of backward-Euler steps */
  int32_t qoi;            /* rmg_qoi */
  int32_t init_profile;   /* 0: uniform initial head h_init; 1: h_init (1 - exp(-init_rate z)) at
                             the cell centre's height z (the infiltration problem of Section 4.3,
                             eq. travellingwave: h_init = -0.4, init_rate = 80) */
  double theta_r, theta_s;
  double gardner_a;       /* Gardner exponent a */
  double linear_c0;       /* linear-law capacity */
  double vg_alpha_shift;  /* added to the alpha field (parametric continuation offset) */
  double vg_n_shift;      /* added to the n field */
  double h_top, h_bottom; /* Dirichlet pressure head on z = 1 and z = 0 */
  double h_init;          /* uniform initial pressure head */
  double dt;              /* time step */
  double init_rate;       /* > 0 when init_profile = 1 */
} rmg_problem;

/* Solver options.  Defaults for the benchmark workloads: MIXED, V, 2, 2, 1,
 * eps_mg 1e-5 (used when cycles_per_picard = 0), eps_picard 1e-8, max_picard 100
 * (500 in the MLMC benchmark), coarsest_n 4.  The paper's own setting is W, 2, 2,
 * cycles_per_picard 0, eps_mg 1e-5. */
typedef struct {
  int32_t precision;          /* rmg_precision: FP64 everywhere, or FP32 multigrid inside FP64 Picard */
  int32_t cycle;              /* rmg_cycle: V (one coarse cycle per level visit) or W (two) */
  int32_t nu1, nu2;           /* pre/post red-black Gauss-Seidel sweeps, each 0..4, not both 0 */
  int32_t cycles_per_picard;  /* fixed number of cycles per Picard step, 1..16; 0: cycle until
                                 max_c |f - A dp| < eps_mg (Section 4.2; at most 200 cycles; the residual
                                 on the finest level in the smoother precision, checked after every
                                 cycle) */
  int32_t max_picard;         /* Picard iterations allowed per time step, >= 1 */
  int32_t coarsest_n;         /* coarsest grid size, 2 or 4, solved exactly in FP64 */
  int32_t flags;              /* bit 0: force the level-streaming path (no whole-sample-in-LDS kernel);
                                 bit 1: launch the streaming Picard iterations eagerly instead of
                                 replaying a captured HIP graph (results are identical);
                                 bit 2: whole-sample kernel keeps the FP64 state in global memory
                                 even where it would fit in LDS (results are identical);
                                 bit 3: no autotuning of the streaming tile shapes (32 x 32
                                 tiles on every level; results are identical);
                                 bit 4: 16 x 16 streaming tiles on every level, no autotuning;
                                 bit 5: use the whole-sample kernel on every grid whose levels fit in
                                 LDS (64 x 64 in FP32), not only up to 32 x 32;
                                 bit 6: start the one-workgroup coarse V-cycle at 32 x 32 in FP32
                                 too (more level-streaming levels; results are identical);
                                 bit 7: mlmc_level_estimate: while level-streaming classes run, confine
                                 the whole-sample classes to a quarter of the compute units and the
                                 streaming classes other than the largest grid to three quarters, so
                                 that the largest grid's chain of short launches finds free units
                                 (helps when that chain is the critical path; results are identical);
                                 bit 8: mlmc_level_estimate: never confine (overrides bit 7 and the
                                 context's schedule tuning) */
  int32_t fallback_cycles;    /* 0: none.  1..16: a sample that fails (iteration limit or non-finite
                                 correction) restarts from its initial state with this many cycles per
                                 Picard step and fallback_max_picard iterations per step; it fails only
                                 if that attempt fails too.  Needs cycles_per_picard >= 1.  The
                                 one-V-cycle modified Picard iteration stalls or oscillates on some
                                 draws where two cycles per step converge; without a fallback such
                                 samples are excluded from the level sums, which biases them. */
  int32_t fallback_max_picard;/* Picard iterations per step of the fallback attempt, >= 1 */
  double eps_mg;              /* residual tolerance of cycles_per_picard = 0 (Section 4.2: 1e-5) */
  double eps_picard;          /* stop when ||dp||_inf < eps_picard (strict) */
} rmg_solver_opts;

/* Per-sample statistics written by picard_mg_solve (device memory). */
typedef struct {
  int32_t picard_its;   /* Picard iterations summed over all time steps */
  int32_t mg_cycles;    /* multigrid cycles summed over all time steps */
  int32_t steps_done;   /* time steps completed */
  int32_t status;       /* rmg_sample_status */
  double final_dp_inf;  /* ||dp||_inf of the last Picard iteration */
  int32_t attempts;     /* 1, or 2 when the sample restarted with the fallback setting (the
                           counts above then cover both attempts) */
  int32_t reserved;
} rmg_sample_stats;

/* Compensated (Neumaier) double-double sum: value = hi + lo. */
typedef struct {
  double hi, lo;
} rmg_dd;

/* Sums over the successful pairs of one MLMC level (Section 5.1, eqs. SMC, MC_var):
 * Y = Q_fine - Q_coarse (Q_coarse = 0 on a base level, one with n_coarse = 0). */
typedef struct {
  int64_t n, n_failed;          /* successful pairs (the sums run over these), failed pairs */
  int64_t picard_its;           /* Picard iterations of both members of every pair, failed included */
  int64_t mg_cycles;            /* multigrid cycles, likewise */
  int64_t mg_cycles_coarse;     /* the part of mg_cycles spent by the coarse members */
  int64_t n_retried;            /* pairs with a member that needed the fallback attempt (failed or not) */
  rmg_dd sY, sY2, sQf, sQf2, sQc, sQc2;
} rmg_level_sums;

/* One MLMC level: fine grid n_fine, coarse partner n_coarse = n_fine / 2 for a
 * correction level or 0 for a base level (the coarsest level of the hierarchy;
 * any entry of a call may be either, so samples can be added to one correction
 * level alone), n_samples pairs sharing their KL draws (Section 5.1: the two
 * members of a correction use the same random input). */
typedef struct {
  int32_t n_fine, n_coarse;
  int64_t n_samples;
  rmg_problem fine, coarse;       /* per-level problems (continuation may differ) */
  const double* d_basis_fine;     /* [n_modes][n_fine^2] */
  const double* d_basis_coarse;   /* [n_modes][n_coarse^2], NULL when n_coarse = 0 */
  const double* d_xi;             /* [n_samples][n_fields][n_modes] standard normals */
} rmg_level;

/* Size in bytes of the named ABI struct ("rmg_problem", "rmg_solver_opts", "rmg_kernel_timing",
 * "rmg_sample_stats", "rmg_level_sums", "rmg_level", "rmg_marginal", "rmg_pc_level",
 * "rmg_pc_opts", "rmg_pc_level_out", "rmg_pc_result"), or -1 if
 * unknown; lets bindings check their struct layouts against the compiled library. */
int64_t rmg_struct_size(const char* name);

/* Kernel timing (diagnostics; used by the benchmark to price the kernels against the
 * hardware).  The selected kinds of level-streaming launches are timed with an event
 * pair that the kernel's dispatch itself records (hipExtLaunchKernelGGL), so a pair
 * brackets the kernel's execution on the device, not the queue time before it; the
 * library also counts the work those launches did.  The streaming solver advances in
 * batches of G passes (a replayed HIP graph; G = 8 or 16, chosen by the schedule
 * tuning of a batched call); the first pass of a timed batch is launched eagerly and
 * timed (events of graph nodes cannot be timed).  Grid-size classes with fewer than
 * 2^22 cells per pass time every eighth batch, larger ones every batch, so the totals
 * cover a uniform one-in-8G (one-in-G) sample of the launches.  Results do not depend
 * on timing.
 *   RMG_TIME_SMOOTHER_DOWN: the down leg (nu1 fused red-black sweeps + residual +
 *     restriction, Section 4.2).  units = fine cells processed; algorithmic bytes per
 *     cell (each array touched once): read f, the two face coefficients and C/dt, write
 *     the iterate and a quarter of a coarse right-hand side (5.25 elements), plus one
 *     element when the initial iterate is loaded rather than zero.
 *   RMG_TIME_COARSE: the one-workgroup-per-sample coarse cycle in LDS (and the fused
 *     fine + coarse launch of a 64 x 64 class).  units = level cells the launches
 *     visited (every level of the in-LDS hierarchy, W-cycles counting repeated visits);
 *     algorithmic bytes = HBM bytes: the top level's f, faces, C/dt in and the
 *     correction out (5 elements per top-level cell).
 *   RMG_TIME_FINE: the fine kernel (FP64 outer residual, closure, fine and in-tile
 *     coarse coefficients, Section 4.1).  units = fine cells; algorithmic bytes per cell:
 *     read p, theta^n and the fields (8 (2 + F) bytes), write f, two faces and C/dt of
 *     the finest level and of the coarser levels formed in the tile (4 elements x 4/3). */
typedef enum {
  RMG_TIME_NONE = 0,
  RMG_TIME_SMOOTHER_DOWN = 1,
  RMG_TIME_COARSE = 2,
  RMG_TIME_FINE = 4
} rmg_timed_kernel;
typedef struct {
  int64_t launches;     /* timed launches */
  int64_t cells;        /* work units of those launches (see rmg_timed_kernel) */
  double total_ms;      /* summed durations of those launches on the device */
  double algo_bytes;    /* algorithmic HBM bytes of those launches */
} rmg_kernel_timing;
/* Select the timed kinds (a bit mask of rmg_timed_kernel; 0 disables timing) and reset
 * the totals. */
int rmg_set_kernel_timing(rmg_ctx* ctx, int which);
/* Totals of one kind (a single rmg_timed_kernel bit) since the last
 * rmg_set_kernel_timing (synchronises the device). */
int rmg_get_kernel_timing(rmg_ctx* ctx, int kind, rmg_kernel_timing* out);

/* Create a context on HIP device `hip_device`; *out receives it.
 * tune_cache_path (nullable): a text file holding the autotuner's choices (streaming
 * tile edges per grid-size class signature, the schedule per batched-call signature),
 * keyed also by the device's architecture and compute-unit count.  It is read here if
 * it exists and rewritten whenever the context makes a new choice, so a later process
 * starts tuned; choices never change results.  NULL: tune in memory only. */
int rmg_ctx_create(rmg_ctx** out, int hip_device, const char* tune_cache_path);
/* Cap the context's workspace at `bytes` (0: no cap).  A call whose workspace would
 * exceed the cap returns RMG_ENOMEM without allocating (a workspace already held above
 * a new cap is released by the next call that needs to grow it). */
int rmg_ctx_set_workspace_limit(rmg_ctx* ctx, int64_t bytes);
/* The context's tuning choices as text, one per line: "<device key> <signature>\t<choice>"
 * (the tune-cache file's format; signatures "tiles ..." map to the two streaming tile
 * edges, "sched ..." to "<confine 0|1> <passes per graph batch>").  Writes at most
 * cap - 1 bytes and a terminating NUL into buf (buf may be NULL when cap is 0); returns
 * the full length in bytes (excluding the NUL), or a negative rmg error code. */
int64_t rmg_ctx_tune_dump(rmg_ctx* ctx, char* buf, int64_t cap);
/* Release the context and its workspace (waits for its device to be idle). */
void rmg_ctx_destroy(rmg_ctx* ctx);
/* Text of the last error on this context ("" if none); valid until the next call. */
const char* rmg_last_error(const rmg_ctx* ctx);

/*
 * sample_fields - KL random fields, Section 3 eqs. KLexp and RandK.
 *   G[s][f][c] = sum_j d_xi[s][f][j] * d_basis[j][c]   (dense product on FP64 matrix cores)
 *   d_fields[s][f][c] = h_marg[f].shift + exp(h_marg[f].log_mean + h_marg[f].scale * G[s][f][c])
 * d_basis [n_modes][n*n] holds sqrt(lambda_j) Psi_j(x_c); d_xi [S][n_fields][n_modes];
 * d_fields [S][n_fields][n*n].  All FP64.  Asynchronous on `stream`.
 * EINVAL: n not a power of two in 4..4096, S < 1, n_fields not in 1..4, n_modes not in
 * 1..1024, NULL pointer.
 */
int sample_fields(rmg_ctx* ctx, int n, int n_fields, int n_modes,
                  const double* d_basis, const double* d_xi, const rmg_marginal* h_marg,
                  int64_t S, double* d_fields, hipStream_t stream);

/*
 * picard_mg_solve - S independent samples on one n x n grid, Sections 4.1-4.2.
 * Each sample integrates problem->n_steps backward-Euler steps from h_init; each
 * step runs modified Picard iterations, each solving its correction equation
 * with opts->cycles_per_picard multigrid cycles, until ||dp||_inf < eps_picard.
 *   d_fields  [S][n_fields][n*n] FP64 (n_fields = 1 for Gardner/linear, 3 for vG)
 *   d_h_out   [S][n*n] FP64: pressure head at the final time (last iterate for a failed sample)
 *   d_qoi     [S] FP64: the problem's QoI (NaN for a failed sample)
 *   d_status  [S] int32: rmg_sample_status
 *   d_stats   [S] rmg_sample_stats, may be NULL
 * Synchronises with `stream` once per poll of the active-sample count.
 * Returns RMG_ENOTCONV if some sample failed (its outputs are flagged).
 * EINVAL: n not a power of two in 2..1024 or below coarsest_n, S not in 1..65535,
 * NULL d_fields/d_h_out/d_qoi/d_status, any problem or option outside the ranges
 * documented on rmg_problem and rmg_solver_opts.
 * EHIP: a HIP call failed (the stream's work may be incomplete); ENOMEM: workspace.
 */
int picard_mg_solve(rmg_ctx* ctx, int n, const rmg_problem* problem, const rmg_solver_opts* opts,
                    const double* d_fields, int64_t S,
                    double* d_h_out, double* d_qoi, int32_t* d_status,
                    rmg_sample_stats* d_stats, hipStream_t stream);

/*
 * picard_mg_solve_noalloc - picard_mg_solve for callers that cannot allocate device
 * memory (code that must not call hipMalloc: under stream capture, in tight serving
 * loops, in harnesses that forbid it).  Same arguments, results and errors as
 * picard_mg_solve, computed by the same kernels; the workspace is a fixed device array
 * of 64 MiB that each GPU holds from the library's first use until the process ends,
 * and the Picard passes are launched eagerly (no graph is instantiated).  A solve whose
 * workspace would exceed the array returns RMG_EINVAL with the bytes it needs (the
 * whole-sample grids up to 32 x 32 need about 8 n^2 bytes per sample, the streaming
 * grids about 8 n^2 + 6 n^2 sizeof(smoother element) x 4/3).  Every call on one GPU
 * shares that array: calls that overlap in time on one GPU (several host threads or
 * streams) race and give wrong results; serialise them.  The array keeps the last
 * call's contents; every value a call reads from it is written by that call first.
 */
int picard_mg_solve_noalloc(rmg_ctx* ctx, int n, const rmg_problem* problem, const rmg_solver_opts* opts,
                            const double* d_fields, int64_t S,
                            double* d_h_out, double* d_qoi, int32_t* d_status,
                            rmg_sample_stats* d_stats, hipStream_t stream);

/*
 * mlmc_level_estimate - one batched evaluation of n_levels MLMC levels
 * (Section 5.1 eqs. MLMCestimator, SMC, ML_var).  For level l and pair i the
 * fine solve (n_fine, fine problem) and the coarse solve (n_coarse, coarse
 * problem) draw their fields from the same d_xi row through their own basis
 * tables; Y_i = Q_fine - Q_coarse.  All solves of all levels run in one batch
 * (grouped by grid size).  Failed pairs are excluded from the sums and counted.
 *   h_levels [n_levels], h_marg [n_fields], h_out [n_levels] (host).
 *   d_qoi_out: optional device array [sum_l 2*n_samples_l] receiving, level by
 *   level, the fine QoIs then the coarse QoIs (NaN marks failure); may be NULL.
 * Synchronises with `stream` before returning.  Returns RMG_ENOTCONV if some
 * sample failed.  EINVAL as for picard_mg_solve, plus: n_levels not in 1..16,
 * n_fine not a power of two in 4..1024, n_coarse neither 0 nor n_fine / 2,
 * a grid size used by more than one fine and one coarse segment,
 * more than 65535 solves on one grid size, NULL basis/xi pointers.
 */
int mlmc_level_estimate(rmg_ctx* ctx, int n_levels, const rmg_level* h_levels,
                        int n_fields, int n_modes, const rmg_marginal* h_marg,
                        const rmg_solver_opts* opts, rmg_level_sums* h_out,
                        double* d_qoi_out, hipStream_t stream);

/*
 * picard_mg_adjoint - per-sample quantity of interest and its gradient with respect
 * to the KL coefficients by the discrete adjoint of the backward-Euler /
 * modified-Picard solve (the derivative of the discrete model of Sections 4.1-4.2;
 * the paper itself has no adjoint).
 *   Q = sum_{k=1}^{n_steps} dt F(p^k),  F(p) = h sum_i K_i0 ((p_i0 - h_bottom) / (h/2) + 1),
 * the time-integrated downward flux through the bottom Dirichlet face (problem->qoi
 * must be RMG_QOI_BOTTOM_OUTFLUX).  Ks = h_marg->shift + exp(h_marg->log_mean +
 * h_marg->scale * G), G = sum_j d_xi[s][j] d_basis[j][c] (eqs. KLexp, RandK).
 * Backward in time, step k solves J_k^T lambda_k = dt dF/dp(p^k) - diag(C(p^k)/dt)
 * lambda_{k+1} with J_k the exact Jacobian of the step residual at p^k (the
 * modified-Picard operator plus the dK/dp terms) by the fixed-point iteration
 * preconditioned with the forward multigrid cycle on the Picard operator; it stops
 * when the correction's max norm is below eps_adjoint (absolute: choose it relative
 * to the multipliers' size, about dt times dF/dp; at most opts->max_picard
 * iterations per step).  The forward pass stores p every ckpt_every steps; the
 * backward pass recomputes each segment of ckpt_every steps from its checkpoint
 * (ckpt_every = 1: every step is stored, nothing is recomputed).
 *   d_basis [n_modes][n*n], d_xi [S][n_modes] FP64 (device);
 *   d_q [S], d_grad [S][n_modes] FP64: Q and dQ/dxi (NaN for a failed sample);
 *   d_status [S] int32: rmg_sample_status of the forward solve, or of the adjoint
 *   iteration if the forward converged;
 *   d_stats: NULL or [2][S]: the forward solves' statistics, then the adjoint's
 *   (picard_its = fixed-point iterations, mg_cycles = their cycles).
 * Gardner and linear closures only (n_fields = 1).  The adjoint iteration runs on
 * the level-streaming kernels with max(1, cycles_per_picard) cycles per iteration
 * in the precision of opts (the residual of the adjoint system is FP64 in both).
 * Synchronises with `stream`; RMG_ENOTCONV if some sample failed.  EINVAL: n not a
 * power of two in 4..1024, S not in 1..65535, n_modes not in 1..1024, another
 * closure or QoI, ckpt_every not dividing n_steps, eps_adjoint <= 0, NULL pointers,
 * and the problem / option ranges of picard_mg_solve.
 */
int picard_mg_adjoint(rmg_ctx* ctx, int n, const rmg_problem* problem, const rmg_solver_opts* opts,
                      int n_modes, const double* d_basis, const rmg_marginal* h_marg, const double* d_xi,
                      int64_t S, int ckpt_every, double eps_adjoint, double* d_q, double* d_grad,
                      int32_t* d_status, rmg_sample_stats* d_stats, hipStream_t stream);

/*
 * picard_mg_outflux - the quantity of picard_mg_adjoint without its gradient: the forward
 * solve of the same samples (fields from d_xi through eqs. KLexp, RandK), keeping every
 * step's pressure head in the workspace (S (n_steps + 1) n^2 doubles), and
 *   Q = sum_{k=1}^{n_steps} dt F(p^k),  F(p) = h sum_i K_i0 ((p_i0 - h_bottom) / (h/2) + 1),
 * reduced in the same order as picard_mg_adjoint, so for the same inputs and options the
 * two return the same Q bit for bit.  d_q [S] (NaN for a failed sample), d_status [S],
 * d_stats [S] or NULL.  Arguments, ranges and errors as picard_mg_adjoint (without the
 * checkpoint and adjoint tolerance arguments).  This is the forward pass of the
 * differentiable outflux in the Python binding; its backward pass calls picard_mg_adjoint.
 */
int picard_mg_outflux(rmg_ctx* ctx, int n, const rmg_problem* problem, const rmg_solver_opts* opts,
                      int n_modes, const double* d_basis, const rmg_marginal* h_marg, const double* d_xi,
                      int64_t S, double* d_q, int32_t* d_status, rmg_sample_stats* d_stats,
                      hipStream_t stream);

/*
 * Adaptive multilevel estimator with parametric continuation (PC_MLMC,
 * Section 5.1: Algorithm 1, eqs. errMLMC, MLMCopt and MLMCSAMP; bias estimate
 * eq. discErr of Section 6).
 *
 * Level l of the hierarchy has a grid D_l (n_fine), a time grid and a
 * nonlinearity parameter set Theta_l (its rmg_problem).  Level 0 is the base
 * level (n_coarse = 0); level l >= 1 pairs its fine solve with a coarse solve on
 * n_coarse = n_fine / 2 under the problem of level l - 1, which must equal level
 * l - 1's fine problem byte for byte (the telescoping sum, eq. telescope).
 */
typedef struct {
  int32_t n_fine, n_coarse;     /* as rmg_level */
  int64_t n_warmup;             /* warm-up pairs N*_l, >= 2 */
  rmg_problem fine, coarse;     /* Theta_l, and Theta_{l-1} (ignored on level 0) */
  const double* d_basis_fine;   /* [n_modes][n_fine^2] */
  const double* d_basis_coarse; /* [n_modes][n_coarse^2], NULL on level 0 */
} rmg_pc_level;

/* Cost per pair W_l (Algorithm 1 lets it be estimated from the warm-up):
 *   RMG_COST_WORK: multigrid cycles times cells per pair (fine and coarse member),
 *     the paper's own cost unit (Section 4.3 counts cycles), scaled by grid size;
 *   RMG_COST_TIME: wall milliseconds per pair of the level's warm-up batch, run
 *     alone (on a batched GPU a small batch measures latency more than cost). */
typedef enum { RMG_COST_WORK = 0, RMG_COST_TIME = 1 } rmg_cost_model;

typedef struct {
  double eps;                   /* sampling tolerance: stop once sum_l V_l / N_l <= eps^2 */
  double bias_rate;             /* a of eq. numErr, > 0, for the eq. discErr bias estimate */
  int32_t cost_model;           /* rmg_cost_model */
  int32_t max_rounds;           /* updates of N_l (Algorithm 1 steps 3-4) allowed, 1..10000 */
  int64_t max_pairs;            /* pairs that may be drawn on one level in total, >= n_warmup */
  int64_t max_pairs_per_call;   /* pairs of one level per batched solve, 0..32767 (0: sized
                                   from the device's free memory) */
} rmg_pc_opts;

/* Source of the random input: write the standard normals of pairs first ..
 * first + count - 1 of level `level` to h_xi [count][n_fields][n_modes] (host
 * memory owned by the library).  Pairs are numbered per level from 0 and never
 * reused; a failed pair's number is not drawn again.  Return 0, or nonzero to
 * abort the run (pc_mlmc then returns RMG_EINVAL). */
typedef int (*rmg_xi_source)(void* user, int level, int64_t first, int64_t count, double* h_xi);

typedef struct {
  int64_t drawn;                /* pairs drawn: numbers 0 .. drawn - 1 */
  int64_t target;               /* N_l from the last update of eq. MLMCSAMP (N*_l before it) */
  double W;                     /* cost per drawn pair (unit of the cost model) */
  double V;                     /* sample variance of Y_l over the successful pairs (eq. level_var) */
  double mean;                  /* E^MC_{N_l}[Y_l] (eq. SMC) */
  rmg_level_sums sums;          /* accumulated over every batch of the run */
} rmg_pc_level_out;

typedef struct {
  double mean;                  /* multilevel estimate of E[Q_L] (eq. MLMCestimator) */
  double var;                   /* multilevel estimate of V[Q_L] (eq. ML_var) */
  double sampling_err2;         /* sum_l V_l / N_l with N_l the successful pairs (eq. MLMCVar) */
  double bias;                  /* eq. discErr with s = 2: sqrt(mean of (Q_{h_L} - Q_{h_{L-1}})^2) / (2^a - 1),
                                   both grids under the finest level's parameter set Theta_L (eq.
                                   numErr); when level L's coarse member uses Theta_{L-1}
                                   (continuation), from bias_pairs further pairs of level L */
  double total_cost;            /* sum_l drawn_l W_l */
  double wall_ms;               /* wall time of the whole call */
  int32_t rounds;               /* updates of N_l performed */
  int32_t converged;            /* 1 if sampling_err2 <= eps^2 with no pair left to draw */
  int64_t calls;                /* batched mlmc_level_estimate calls made */
  int64_t bias_pairs;           /* pairs of level L drawn for the bias (numbers drawn_L, ...), or 0 */
} rmg_pc_result;

/*
 * pc_mlmc - Algorithm 1 on the device: warm-up N*_l pairs on every level, then
 * repeatedly set N_l by eq. MLMCSAMP from the current V_l and the warm-up W_l,
 * draw the missing pairs of every level in one batched mlmc_level_estimate call
 * (several if a level needs more than max_pairs_per_call), and update the sums,
 * until no level needs more pairs.  Failed pairs are excluded from the sums and
 * replaced by new draws.  The random input comes from `xi`, in host memory; the
 * library copies it to the device (it allocates a staging buffer of
 * max_pairs_per_call pairs per level for the call and frees it on return).
 *   h_levels, h_level_out [n_levels], h_marg [n_fields], h_result: host.
 * Returns RMG_OK once converged; RMG_ENOTCONV if max_rounds or max_pairs ended
 * the run first (outputs hold the state reached) or a level's warm-up left fewer
 * than two successful pairs within max_pairs (outputs not filled); EINVAL for
 * arguments outside the ranges above or those of mlmc_level_estimate, a
 * hierarchy whose level l coarse member differs from level l - 1's fine member,
 * or a nonzero return of `xi`.  Other errors of mlmc_level_estimate pass through.
 */
int pc_mlmc(rmg_ctx* ctx, int n_levels, const rmg_pc_level* h_levels, int n_fields, int n_modes,
            const rmg_marginal* h_marg, const rmg_solver_opts* opts, const rmg_pc_opts* pc,
            rmg_xi_source xi, void* user, rmg_pc_level_out* h_level_out, rmg_pc_result* h_result,
            hipStream_t stream);

/*
 * Eq. MLMCSAMP: N_l = ceil(eps^-2 (sum_k sqrt(V_k W_k)) sqrt(V_l / W_l)), the
 * sample counts minimising sum_l N_l W_l subject to sum_l V_l / N_l = eps^2
 * (eq. MLMCopt).  Host arithmetic only (no device needed).  V_l >= 0, W_l > 0,
 * eps > 0, 1..16 levels, else RMG_EINVAL; a count above 2^62 is RMG_EINVAL too.
 */
int rmg_mlmc_optimal_samples(int n_levels, const double* V, const double* W, double eps, int64_t* N_out);

#ifdef __cplusplus
}
#endif

#endif /* RMG_H_ */
