/*
 * libmpcpcg -- Schur-complement + preconditioned-conjugate-gradient solve of the
 * linear-quadratic subproblem of one nonlinear MPC step, on AMD Instinct MI355X (gfx950).
 *
 * The problem (MPCGPU, Section III-A, the QP of "Step 1" and the KKT system of
 * "Step 2") has N state knots x_0..x_{N-1} and N-1 controls u_0..u_{N-2}:
 *
 *   min  sum_k 1/2 dx_k^T Q_k dx_k + q_k^T dx_k  +  sum_k 1/2 du_k^T R_k du_k + r_k^T du_k
 *   s.t. dx_0 = x0,   dx_{k+1} = A_k dx_k + B_k du_k - e_k      (k = 0..N-2)
 *
 * whose KKT system [G C^T; C 0][-dZ; lambda] = [g; c] is solved by the Schur complement
 * method (Section III-B): S lambda = gamma, then dZ = -G^-1 (g - C^T lambda).  The
 * library forms S = C G^-1 C^T (block tridiagonal, nx x nx blocks; the paper writes
 * -C G^-1 C^T with gamma negated as well, which is the same equation) and
 * gamma = C G^-1 g - c, the symmetric stair preconditioner Phi^-1 (Section IV-A,
 * Phi^-1 = D^-1 - D^-1 E D^-1 with D the block diagonal of S and E = S - D), and runs
 * PCG (Algorithm 1) until sqrt(eta / eta_ref) < eps, where eta = r^T Phi^-1 r and
 * eta_ref = gamma^T Phi^-1 gamma.
 *
 * Conventions shared by every entry point
 *  - All array arguments are DEVICE pointers owned by the caller (e.g. torch tensors),
 *    FP32, row-major, contiguous.  The library never frees or retains caller memory.
 *    The context owns only its workspace, schedules and captured graphs.
 *  - Every call is asynchronous on the given hipStream_t (0 = the null stream).  The
 *    return value reports synchronous errors only (argument validation, a failed
 *    launch).  Per-problem outcomes are written to a device array of mpcpcg_stats.
 *  - Supported (nx, nu): (14, 7), on a register-resident fused kernel, and (28, 14), on a
 *    workspace-staged path (formation, preconditioner and PCG launches; horizons up to
 *    292 knots).  Others return MPCPCG_EUNSUPPORTED.  Schedule control (knots per group,
 *    graphs, autotune) applies to the (14, 7) path; on (28, 14) it is accepted and ignored.
 *  - A context is not thread safe; calls that share a context must be serialised by
 *    the caller and must not overlap on different streams.
 *  - Calls never abort or throw across the ABI.  mpcpcg_last_error() describes the
 *    last synchronous failure.
 */
#ifndef MPCPCG_H
#define MPCPCG_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes (negative) and per-problem statuses (non-negative, in mpcpcg_stats). */
enum {
  MPCPCG_OK = 0,             /* converged: sqrt(eta/eta_ref) < eps                      */
  MPCPCG_NOT_CONVERGED = 1,  /* stats only: max_iter reached; lambda/dZ still written    */
  MPCPCG_BREAKDOWN = 2,      /* stats only: p^T S p <= 0 or a non-finite value (input   *
                              * not positive definite, NaN/Inf in the data)              */
  MPCPCG_TIMEOUT = 3,        /* stats only: workgroups of one problem could not meet;   *
                              * outputs of that problem are undefined                    */
  MPCPCG_EINVAL = -1,        /* bad argument (null pointer, N < 1, size beyond limits)  */
  MPCPCG_EUNSUPPORTED = -2,  /* (nx, nu) not compiled into this library                 */
  MPCPCG_ENOMEM = -3,        /* workspace allocation failed                             */
  MPCPCG_EHIP = -4           /* a HIP runtime call failed (message in last_error)       */
};

typedef struct mpcpcg_ctx mpcpcg_ctx;

/* One LQ subproblem (or, for the batched calls, many packed back to back).
 *   Q  [N][nx][nx]  state cost Hessians (symmetric positive definite)
 *   R  [N-1][nu][nu] control cost Hessians (symmetric positive definite)
 *   A  [N-1][nx][nx], B [N-1][nx][nu]  dynamics Jacobians
 *   q  [N][nx], r [N-1][nu]            cost gradients
 *   x0 [nx]                             required value of dx_0 (c_0 = -x0)
 *   e  [N-1][nx] dynamics defects, or NULL for zero.
 * For packed batches, knot-indexed arrays (Q, q) of problem b start at row
 * knot_off[b], control-indexed arrays (R, A, B, r, e) at row knot_off[b] - b, and x0 is
 * [batch][nx]; N is ignored (knot_off defines every horizon). */
typedef struct {
  int32_t nx, nu, N;
  const float *Q, *R, *A, *B, *q, *r, *x0, *e;
} mpcpcg_problem;

/* Stopping rules (mpcpcg_opts.stop_rule), tested after initialisation and after every
 * main-loop iteration (Algorithm 1, the "eta' < eps" test), eta = r^T Phi^-1 r:
 *   RELATIVE: sqrt(eta / eta_ref) < eps with eta_ref = gamma^T Phi^-1 gamma, i.e. the
 *             preconditioned residual relative to that of lambda = 0 (scale free);
 *   ABSOLUTE: eta < eps, the test exactly as Algorithm 1 prints it (depends on the
 *             problem's scale; the paper sweeps eps over 1e-4 .. 1e-5). */
enum { MPCPCG_STOP_RELATIVE = 0, MPCPCG_STOP_ABSOLUTE = 1 };

typedef struct {
  float eps;          /* stopping tolerance (see stop_rule); e.g. 1e-6 relative         */
  int32_t max_iter;   /* main-loop iteration cap; 0 means N*nx                         */
  int32_t warm_start; /* non-zero: lambda (in/out) holds the start iterate on entry     */
  int32_t stop_rule;  /* MPCPCG_STOP_RELATIVE (0) or MPCPCG_STOP_ABSOLUTE (1)           */
} mpcpcg_opts;

typedef struct {
  int32_t iters;      /* main-loop iterations executed (0 if the start already passed) */
  int32_t status;     /* MPCPCG_OK / NOT_CONVERGED / BREAKDOWN / TIMEOUT                */
  float final_ratio;  /* sqrt(eta/eta_ref) at exit, whichever stop_rule ran             */
  int32_t reserved;
} mpcpcg_stats;

/* Output of mpcpcg_form_schur: S and Phi^-1 as [N][3][nx][nx] with slot 0 = block
 * (b, b-1), slot 1 = (b, b), slot 2 = (b, b+1) (blocks outside the matrix are zero), and
 * gamma [N][nx].  Any of the three pointers may be NULL to skip it. */
typedef struct {
  float *S, *Pinv, *gamma;
} mpcpcg_schur;

/* Create a context for problems of dimension (nx, nu).  max_total_knots bounds the
 * knots of one call (sum of N over a batch); max_batch bounds the problems of one call.
 * Allocates device workspace proportional to both on the current device.  The parts'
 * exchange records must fit 2 GiB: max_total_knots / 4 + max_batch <= 195,652 at (14, 7)
 * and <= 1,016,800 at (28, 14); larger sizes return MPCPCG_EINVAL before any device call. */
int mpcpcg_create(mpcpcg_ctx **ctx, int32_t nx, int32_t nu, int64_t max_total_knots,
                  int32_t max_batch);

/* Release the context's workspace and graphs.  NULL is accepted. */
int mpcpcg_destroy(mpcpcg_ctx *ctx);

/* Text of the last synchronous error on this context ("" if none; never NULL). */
const char *mpcpcg_last_error(const mpcpcg_ctx *ctx);

/* Form S, gamma and Phi^-1 of one problem (Section III-B, eq. for theta_k, phi_k,
 * zeta_k; Section IV-A for Phi^-1).  S and gamma use the positive-definite sign
 * convention stated at the top of this header. */
int mpcpcg_form_schur(mpcpcg_ctx *ctx, const mpcpcg_problem *prob, mpcpcg_schur *out,
                      hipStream_t stream);

/* Solve one problem: formation, PCG (Algorithm 1) and the primal step
 * dZ = -G^-1 (g - C^T lambda), fused in one launch.
 *   lambda [N][nx] (out; in as well when opts->warm_start), dx [N][nx], du [N-1][nu],
 *   stats: device pointer to one mpcpcg_stats. */
int mpcpcg_solve(mpcpcg_ctx *ctx, const mpcpcg_problem *prob, const mpcpcg_opts *opts,
                 float *lambda, float *dx, float *du, mpcpcg_stats *stats, hipStream_t stream);

/* Solve `batch` independent problems packed as described for mpcpcg_problem, in one
 * persistent launch (replayed from a captured hipGraph when the same pointers and
 * horizons are seen again).  knot_off is a HOST array [batch+1] of prefix sums of the
 * horizons (knot_off[0] = 0).  lambda/dx use knot rows, du control rows, stats [batch]. */
int mpcpcg_solve_batched(mpcpcg_ctx *ctx, int32_t batch, const int64_t *knot_off,
                         const mpcpcg_problem *packed, const mpcpcg_opts *opts, float *lambda,
                         float *dx, float *du, mpcpcg_stats *stats, hipStream_t stream);

/* Adjoint (reverse-mode) solve of the batched forward solve for a scalar loss
 * L(lambda, dx, du).  Given the saved forward outputs and dL/dlambda (and optionally
 * dL/ddx, dL/ddu, NULL = 0), solves S mu = dL/dlambda + C G^-1 dL/ddZ with the same PCG
 * and stopping rule, forms nu_1 = -G^-1 (dL/ddZ - C^T mu), and writes the gradients
 * restricted to the block sparsity of the inputs:
 *   dQ_k = sym(nu1x_k dx_k^T), dR_k = sym(nu1u_k du_k^T),
 *   dA_k = lambda_{k+1} nu1x_k^T + mu_{k+1} dx_k^T, dB_k = lambda_{k+1} nu1u_k^T + mu_{k+1} du_k^T,
 *   dq_k = nu1x_k, dr_k = nu1u_k, dx0 = mu_0, de_k = -mu_{k+1}, dgamma = mu.
 * Layouts equal those of the corresponding inputs; de and dgamma may be NULL.
 * stats [batch] report the adjoint PCG. */
int mpcpcg_backward(mpcpcg_ctx *ctx, int32_t batch, const int64_t *knot_off,
                    const mpcpcg_problem *packed, const mpcpcg_opts *opts, const float *lambda,
                    const float *dx, const float *du, const float *dL_dlambda,
                    const float *dL_ddx, const float *dL_ddu, float *dQ, float *dR, float *dA,
                    float *dB, float *dq, float *dr, float *dx0, float *de, float *dgamma,
                    mpcpcg_stats *stats, hipStream_t stream);

/* Forward solve that keeps its preconditioner for the adjoint, and the adjoint that reads
 * it.  The adjoint system S mu = y has the forward's matrix (S is symmetric, Section III-B)
 * and therefore its preconditioner Phi^-1 (Section IV-A).
 * mpcpcg_solve_batched_keep is mpcpcg_solve_batched with PCG (Algorithm 1), whatever the
 * context's method, that also writes to the record `factors` Phi^-1 of every knot (FP32)
 * and the inverses of Q and R it forms (FP64).  mpcpcg_backward_reuse is mpcpcg_backward
 * with PCG that forms S from those inverses and reads Phi^-1 from the record instead of
 * inverting Q, R and the diagonal blocks of S, exchanging the latter between workgroups
 * and forming the off-diagonal blocks again; its results equal mpcpcg_backward's bit for
 * bit.  `factors` is a device buffer owned by the caller, 256-byte aligned, of
 * mpcpcg_factor_bytes(ctx, knot_off[batch]) bytes (5,824 per knot);
 * the caller keeps it and the packed problem unchanged between the two calls (the record
 * is not checked against the problem).  The record of a problem whose forward solve
 * reported MPCPCG_TIMEOUT is undefined (other statuses leave it whole: Phi^-1 does not
 * depend on the iteration).  Both calls return EINVAL on an (28, 14) context,
 * for a NULL or misaligned record, and for the argument errors of the plain calls.
 * mpcpcg_factor_bytes returns -1 for a NULL or (28, 14) context or total_knots < 1. */
int64_t mpcpcg_factor_bytes(const mpcpcg_ctx *ctx, int64_t total_knots);
int mpcpcg_solve_batched_keep(mpcpcg_ctx *ctx, int32_t batch, const int64_t *knot_off,
                              const mpcpcg_problem *packed, const mpcpcg_opts *opts, float *lambda,
                              float *dx, float *du, mpcpcg_stats *stats, void *factors,
                              hipStream_t stream);
int mpcpcg_backward_reuse(mpcpcg_ctx *ctx, int32_t batch, const int64_t *knot_off,
                          const mpcpcg_problem *packed, const mpcpcg_opts *opts, const float *lambda,
                          const float *dx, const float *du, const float *dL_dlambda,
                          const float *dL_ddx, const float *dL_ddu, float *dQ, float *dR, float *dA,
                          float *dB, float *dq, float *dr, float *dx0, float *de, float *dgamma,
                          mpcpcg_stats *stats, const void *factors, hipStream_t stream);

/* Schedule control for the batched calls.
 * mpcpcg_set_knots_per_group fixes the knots handled by one workgroup (one of 4, 8, 16,
 * 24, 32, 48; 0 restores the automatic choice).  mpcpcg_autotune times every
 * candidate shape on the given batch (running real solves, outputs overwritten) and
 * caches the fastest for that batch signature; it synchronises the stream.  The chosen
 * value is returned in *knots_per_group (may be NULL). */
int mpcpcg_set_knots_per_group(mpcpcg_ctx *ctx, int32_t knots_per_group);
int mpcpcg_autotune(mpcpcg_ctx *ctx, int32_t batch, const int64_t *knot_off,
                    const mpcpcg_problem *packed, const mpcpcg_opts *opts, float *lambda,
                    float *dx, float *du, mpcpcg_stats *stats, hipStream_t stream,
                    int32_t *knots_per_group);

/* The schedule the next batched PCG solve of this horizon signature uses: knots per
 * workgroup and whether each problem's workgroups run on one XCD (per-XCD task lists).
 * After mpcpcg_autotune this is the tuned choice.  Builds (and caches) the schedule. */
int mpcpcg_tuned_schedule(mpcpcg_ctx *ctx, int32_t batch, const int64_t *knot_off,
                          int32_t *knots_per_group, int32_t *xcd_pinned);

/* Default placement of batched PCG gangs when no tuned choice exists: 1 (default) runs all
 * workgroups of a problem on one XCD when the device reports eight XCDs and every problem's
 * workgroups fit one XCD's share of the co-resident grid (any batch size; a batch of fewer
 * than eight problems leaves XCDs idle); 0 uses one global task queue.  mpcpcg_autotune
 * times both placements and keeps the faster per signature. */
int mpcpcg_set_xcd_pinning(mpcpcg_ctx *ctx, int32_t enable);

/* Enable (1, default) or disable (0) hipGraph capture/replay in mpcpcg_solve_batched. */
int mpcpcg_set_graph(mpcpcg_ctx *ctx, int32_t enable);

/* Per-signature caches (schedules, tuned choices, captured graphs, chunk lists) hold at
 * most max_signatures entries each (default 32); the least recently used entry is evicted,
 * its device arrays freed and its graphs destroyed (the device is synchronised first).
 * mpcpcg_cache_info reports the entries held over all caches and the device bytes of the
 * cached schedules (either pointer may be NULL). */
int mpcpcg_set_cache_limit(mpcpcg_ctx *ctx, int32_t max_signatures);
int mpcpcg_cache_info(const mpcpcg_ctx *ctx, int32_t *entries, int64_t *device_bytes);

/* Failure handling of problems that span several workgroups.  Every wait of one
 * workgroup for another gives up after limit_us microseconds of wall-clock time (default
 * 2 s); the problem then reports MPCPCG_TIMEOUT and every workgroup leaves normally.
 * inject_stall = 1 is a test hook: the first such wait of every launch of the (14, 7)
 * path waits for a signal that is never sent, so each multi-workgroup problem times out
 * (on the factorisation path, in its primal-step launch). */
int mpcpcg_debug_set_wait(mpcpcg_ctx *ctx, int64_t limit_us, int32_t inject_stall);

/* Solution method of mpcpcg_solve, mpcpcg_solve_batched and mpcpcg_backward.
 *   MPCPCG_METHOD_PCG (default): PCG as above (Algorithm 1).
 *   MPCPCG_METHOD_FACTOR: direct solve of the same Schur system, the alternative to the
 *     iterative solve that the paper names as future work (Section VI), by block cyclic
 *     reduction of the block-tridiagonal S (log2 N levels of parallel block eliminations,
 *     then back substitution).  At (14, 7) one workgroup per problem, except that a lone
 *     problem (a single solve or a batch of one) runs its levels with many block tasks
 *     spread over the device; at (28, 14) every level is spread over the device, one wave
 *     per block task.  FP64 throughout, exact up to rounding;
 *     eps, max_iter, warm_start and stop_rule are ignored; stats report iters = 0, status
 *     OK or BREAKDOWN (a non-positive pivot, i.e. S not positive definite, or a non-finite
 *     result), final_ratio = 0.  Its cost does not depend on the conditioning of S.  At
 *     (14, 7) it needs ~6.5 KB of extra device workspace per knot of max_total_knots,
 *     allocated on first use.
 *   MPCPCG_METHOD_AUTO: per call, at (14, 7) the faster of the two by a cost model
 *     measured on MI355X, which prices PCG at ~100 iterations for cold starts and ~45 for
 *     warm starts (opts->warm_start; the adjoint counts as cold).  On the Kuka-shaped
 *     problems this takes the factorisation for cold solves, lone problems and large
 *     batches, and PCG for warm-started small batches.  At (28, 14) always the
 *     factorisation, which is faster there at every measured size. */
enum { MPCPCG_METHOD_PCG = 0, MPCPCG_METHOD_FACTOR = 1, MPCPCG_METHOD_AUTO = 2 };
int mpcpcg_set_method(mpcpcg_ctx *ctx, int32_t method);

/* ---- The control step around the solve ---------------------------------------------
 * One iteration of the paper's controller linearises the nonlinear problem at the
 * current guess (Section III-A, Step 1), solves the LQ problem (the calls above), and
 * picks the step length by a parallel line search on the L1 merit (Section III-A, Step 3;
 * Section IV-C).  The robot model of the paper is not part of this library; these calls
 * evaluate a fixed model family that stands in for it:
 *
 * Pendulum chain: nq = nx / 2 joints (so nu = nq: one torque per joint), state
 * x = [q; v], explicit Euler step with timestep h:
 *   q+ = q + h v,  v+ = v + h acc,
 *   acc_i = u_i - g_i sin(q_i) - d v_i + kappa (sin(q_{i+1} - q_i) - sin(q_i - q_{i-1})),
 * where the spring terms past either end of the chain are absent.
 * Tracking cost J = sum_k 1/2 (x_k - xref_k)^T Q_k (x_k - xref_k) + sum_k 1/2 u_k^T R_k u_k.
 * Constraints c = [x_0 - x_s, x_1 - f(x_0, u_0), ..., x_{N-1} - f(x_{N-2}, u_{N-2})].
 *
 * Layouts follow the batched solve: knot-indexed arrays are packed over knots, control-
 * indexed arrays over controls (problem b's rows start at knot_off[b] - b), per-problem
 * arrays are [batch][...].  All arrays are device memory owned by the caller, FP32 unless
 * stated; calls are asynchronous on `stream`; arithmetic is FP64 inside. */
typedef struct {
  float h;               /* Euler timestep */
  float damping;         /* d */
  float coupling;        /* kappa */
  const float *gravity;  /* [nx/2] gains g_i, shared by the batch */
} mpcpcg_chain_model;

typedef struct {
  int32_t nx, nu, N;     /* N = total knots (knot_off[batch]); must match the context */
  const float *X;        /* [N][nx] state guess */
  const float *U;        /* [N-batch][nu] control guess (NULL if every N_b = 1) */
  const float *x_init;   /* [batch][nx] measured initial states x_s */
  const float *xref;     /* [N][nx] tracking targets */
  const float *Q;        /* [N][nx][nx] state weights (symmetric) */
  const float *R;        /* [N-batch][nu][nu] control weights (symmetric; NULL if every N_b = 1) */
} mpcpcg_trajectory;

/* Step 1: the LQ problem of the solve at the guess (X, U).  The cost is quadratic, so its
 * expansion is exact: the problem's Q, R are the trajectory's weights (pass the same
 * pointers), q_k = Q_k (x_k - xref_k), r_k = R_k u_k; A_k = df/dx, B_k = df/du at
 * (x_k, u_k); e_k = x_{k+1} - f(x_k, u_k); x0 = x_s - x_0 (the required dx_0).
 * Outputs q [N][nx], x0 [batch][nx], and (NULL allowed only if every N_b = 1)
 * A [N-batch][nx][nx], B [N-batch][nx][nu], r [N-batch][nu], e [N-batch][nx].
 * Returns OK or EINVAL (argument errors; message in mpcpcg_last_error). */
int mpcpcg_linearize(mpcpcg_ctx *ctx, int32_t batch, const int64_t *knot_off,
                     const mpcpcg_chain_model *model, const mpcpcg_trajectory *traj, float *A,
                     float *B, float *q, float *r, float *x0, float *e, hipStream_t stream);

/* Step 3: evaluate the trial iterates (X + a dX, U + a dU) for a in {1, 1/2, ..., 1/256}
 * in parallel, score each by the L1 merit phi(a) = J + mu_b ||c||_1, and write the iterate
 * with the smallest merit (the largest a among equal merits) to X_out, U_out.
 * Penalty: mu_b = mu + max |lambda_b| when lambda ([N][nx], the solve's multipliers) is
 * given, else mu; mu must be finite and >= 0.
 * Outputs: merit [batch][MPCPCG_LS_STEPS] (FP64, in the order of a), choice [batch]
 * (index j of a = 2^-j), X_out [N][nx], U_out [N-batch][nu].  X_out may be X and U_out
 * may be U (in-place update); no other output may overlap an input.
 * Uses ~150 B of context workspace per 8 knots (allocated on first use).  Calls that
 * overlap on one context race on that workspace.  Returns OK, EINVAL (argument errors;
 * message in mpcpcg_last_error) or EHIP. */
#define MPCPCG_LS_STEPS 9
int mpcpcg_line_search(mpcpcg_ctx *ctx, int32_t batch, const int64_t *knot_off,
                       const mpcpcg_chain_model *model, const mpcpcg_trajectory *traj,
                       const float *dX, const float *dU, const float *lambda, float mu,
                       float *X_out, float *U_out, double *merit, int32_t *choice,
                       hipStream_t stream);

/* One control step as a single call (the paper's goal of one host-device synchronisation
 * per control step, Section IV): sqp_iters (1..16) iterations of
 *   mpcpcg_linearize -> mpcpcg_solve_batched (with *opts and the context's method)
 *   -> mpcpcg_line_search (penalty mu + max |lambda_b|),
 * each iteration starting from the previous one's iterate.  The first iteration reads the
 * guess from traj->X / traj->U; the updated iterate goes to X_out / U_out, which may be
 * traj->X / traj->U (in-place update, the usual receding-horizon use).  lambda [N][nx]
 * receives the multipliers and is the warm start of every solve when opts->warm_start
 * is set; merit, choice and stats are those of the last iteration.
 * The LQ problem and the step live in context workspace (~1.4 KB per knot of
 * max_total_knots at (14, 7), allocated on first use).  With graphs enabled
 * (mpcpcg_set_graph), the first call with a given batch signature and argument set runs
 * the launches directly, the second captures them into one hipGraph, and later calls
 * replay it on `stream`: the whole step is then one graph launch.  The graph reads the
 * arrays at replay time, so new values in the same buffers need no new capture; other
 * pointers or scalars start the sequence again.  Calls that overlap on one context race
 * on the workspace.  Returns OK, EINVAL (argument errors; message in mpcpcg_last_error),
 * ENOMEM (workspace) or EHIP (a launch or the capture failed); convergence of each solve
 * is in stats as for mpcpcg_solve_batched. */
int mpcpcg_control_step(mpcpcg_ctx *ctx, int32_t batch, const int64_t *knot_off,
                        const mpcpcg_chain_model *model, const mpcpcg_trajectory *traj,
                        const mpcpcg_opts *opts, int32_t sqp_iters, float mu, float *lambda,
                        float *X_out, float *U_out, double *merit, int32_t *choice,
                        mpcpcg_stats *stats, hipStream_t stream);

/* ---- For callers that cannot allocate device memory ----------------------------------
 * mpcpcg_solve_noalloc is mpcpcg_solve for callers that may not call hipMalloc: code that
 * runs under HIP graph capture, tight serving loops, harnesses that forbid allocation.  It
 * takes no context and allocates nothing (no hipMalloc, hipFree, graph or allocating
 * library call).  Its scratch (Q^-1 and (R^-1 | R^-1 B^T) per knot, the exchange words of
 * the workgroups, the gang and queue counters) is one static device array of 7.86 MB that
 * each GPU the library runs on holds until the process ends; the first call on a device
 * resolves that device's copy.  Every call clears the counters and exchange words it uses
 * with a small fill kernel on `stream` (no memset), so calls may be captured into a graph.
 * Every call on one GPU shares the array: calls that overlap on one GPU (other streams,
 * other threads) race and must be serialised by the caller.
 * Problem, options and outputs are those of mpcpcg_solve (device pointers, FP32, row-major)
 * for (nx, nu) = (14, 7) and 1 <= N <= 2048; N beyond 2048 returns MPCPCG_EINVAL and other
 * shapes MPCPCG_EUNSUPPORTED, before any launch.  It always solves by PCG with the workgroup
 * shape mpcpcg_solve takes on a context with default settings, and gives the same results.
 * mpcpcg_noalloc_last_error() describes this thread's last failed call ("" if none). */
int mpcpcg_solve_noalloc(const mpcpcg_problem *prob, const mpcpcg_opts *opts, float *lambda,
                         float *dx, float *du, mpcpcg_stats *stats, hipStream_t stream);
const char *mpcpcg_noalloc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MPCPCG_H */
