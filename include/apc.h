/*
 * apc.h -- C ABI of the MI355X (gfx950) Accelerated Projection-based Consensus
 * solver (Azizan-Ruhi, Lahouti, Avestimehr, Hassibi, arXiv 1708.01413).
 *
 * Problem (Sec. 2, eq. (1)): solve A x = b, A in R^{N x n}, N >= n, with a
 * unique solution.  The rows are split into m contiguous blocks
 * [A_i, b_i] = rows off[i] .. off[i+1]-1 ("machines", Sec. 2); all m blocks
 * live on one GPU and are processed as a batch.
 *
 * Method (Sec. 3.1, eq. (2a)-(2b), Alg. 1):
 *     x_i   <- x_i + gamma * P_i (x_bar - x_i),        i = 1..m
 *     x_bar <- (eta/m) * sum_i x_i + (1 - eta) * x_bar
 * with P_i = I - A_i^T (A_i A_i^T)^{-1} A_i applied as v - Q_i (Q_i^T v)
 * from a thin QR A_i^T = Q_i R_i computed once at setup (Sec. 3.3).
 *
 * Conventions for every entry point:
 *   - Matrices are row-major.  "device" pointers point to GPU memory, "host"
 *     pointers to CPU memory.
 *   - The library never allocates device memory.  The caller owns A, B, the
 *     outputs and the workspace; sizes come from apc_workspace_bytes.
 *   - All GPU work is enqueued on the stream given to apc_setup (a
 *     hipStream_t passed as void*, NULL = default stream).  Entry points that
 *     return host values synchronise that stream; they say so below.  Device
 *     buffers a call reads must be ready in that stream's order, and buffers
 *     it writes are valid in that stream's order only: a caller producing or
 *     consuming them on another stream orders the two streams (events), as
 *     the Python binding does around every call.
 *   - No C++ exception crosses this boundary.  A non-OK status leaves a
 *     message for apc_last_error() (thread-local).  Argument errors are
 *     detected on the host before any GPU work is enqueued.
 *   - k right-hand sides (1 <= k <= 1024) are solved together: B is N x k
 *     row-major, entry (r, c) at B[r*ldb + c] (ldb >= k; for k = 1, ldb is the
 *     stride between consecutive entries), and x_bar is returned as n x k
 *     row-major with row stride ldx (>= k; for k = 1, the entry stride).
 */
#ifndef APC_H
#define APC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct apc_plan_s* apc_plan; /* opaque, host-side, owned by the library */

typedef enum {
  APC_F64 = 0,    /* Q_i and all arithmetic in FP64                                 */
  APC_F32 = 1,    /* Q_i stored in FP32, projections in FP32 with FP32             */
                  /* accumulation, iterates and update arithmetic in FP64          */
  APC_BF16_IR = 2, /* iterative refinement: inner APC on a bf16 Q_i (matrix cores, */
                   /* FP32 accumulation, FP64 state), FP64 residual B - A X and    */
                   /* FP32 inner starts x_bar(0) on matrix cores; setup QR in      */
                   /* FP64, the eigenvalue estimate's recurrence in FP64 (see      */
                   /* apc_setup)                                                   */
  APC_REDUCED_FORM = 16 /* flag, OR'ed into APC_F64 / APC_F32: use the (y, x_bar)    */
                        /* form below also for k = 1 (needed by apc_backward)      */
} apc_precision;

/* Two forms of the same iteration:
 *  - k = 1 with APC_F64 / APC_F32 keeps every local iterate x_i, as eq. (2a)
 *    states it (the m n-vectors are <1% of the bytes an update moves);
 *  - k > 1, and APC_BF16_IR for any k, keeps the exact reduced state
 *    (y, x_bar): with x_i(0) = Q_i c_i every iterate of eq. (2a) is
 *    x_i(t) = x_i(0) + P_i y(t), y(0) = 0, y(t+1) = (1-gamma) y(t) +
 *    gamma x_bar(t), hence (1/m) sum_i x_i(t+1) = x_bar(0) + y(t+1) -
 *    X y(t+1) with X = (1/m) sum_i Q_i Q_i^T (eq. (3)).  Per update it forms
 *    W = C y and Z = C^T W, C = [Q_1^T; ...; Q_m^T], as two matrix-core
 *    products; the x_i are reconstructed on request (apc_get_local). */

typedef enum {
  APC_OK = 0,
  APC_EINVAL = 1,       /* invalid argument (sizes, offsets, strides, pointers)     */
  APC_ERANK = 2,        /* some A_i is not of full row rank (setup QR)              */
  APC_ESINGULAR = 3,    /* mu_min(X) ~ 0: no unique solution (App. A)               */
  APC_EDIVERGED = 4,    /* residual became non-finite or grew without bound        */
  APC_ENOCONV = 5,      /* tolerance not reached within the iteration budget       */
  APC_ENODEV = 6,       /* no usable GPU                                            */
  APC_EHIP = 7,         /* a HIP runtime call failed                                */
  APC_EUNSUPPORTED = 8  /* valid request this version does not implement           */
} apc_status;

/* Bytes of device workspace apc_setup needs for this problem.
 * off: host array of m+1 increasing row offsets, off[0] = 0, off[m] = N,
 * 1 <= off[i+1]-off[i] <= min(n, 2048).  Returns 0 for invalid arguments. */
size_t apc_workspace_bytes(int64_t N, int64_t n, const int64_t* off, int32_t m, int32_t k,
                           int32_t precision);

/* Factor every block, initialise the iterates and choose (gamma, eta).
 *
 *   A      device, N x n FP64, row stride lda >= n.  Read during setup, and
 *          again by apc_residual / apc_solve: keep it alive and unchanged
 *          until apc_destroy.
 *   B      device, FP64 right-hand sides, N x k, entry (r, c) at B[r*ldb + c].
 *          Read during setup and by apc_residual / apc_solve (keep alive).
 *   off    host, m+1 block offsets as in apc_workspace_bytes (copied).
 *   gamma, eta  the parameters of eq. (2).  If either is NaN, both are set to
 *          Theorem 1's optimum from the extreme eigenvalues of
 *          X = (1/m) sum_i A_i^T (A_i A_i^T)^{-1} A_i (eq. (3)), estimated on
 *          the GPU by Lanczos on X v = (1/m) sum_i Q_i Q_i^T v (recurrence,
 *          reorthogonalisation and Ritz values in FP64; the product X v reads
 *          the FP64 factor in APC_F64 plans and an FP32 copy of it otherwise,
 *          with FP64 sums: relative error ~1e-7, far below the stopping
 *          tolerances) and widened to an interval that encloses the spectrum:
 *          mu_max by the top Ritz value's residual bound, mu_min by a margin
 *          of up to 20 times the bottom Ritz value's last change.
 *   workspace  device, >= apc_workspace_bytes(...) bytes, 256-byte aligned,
 *          owned by the caller, used exclusively by this plan until destroy.
 *
 * Setup steps (Sec. 3.1, Sec. 3.3, Alg. 1 initialisation): thin QR of each
 * A_i^T in FP64 (CholeskyQR2), c_i = R_i^{-T} b_i, the minimum-norm local
 * solutions x_i(0) = Q_i c_i and x_bar(0) = (1/m) sum_i x_i(0).
 * Synchronises the stream (rank check, eigenvalue estimate).
 * Errors: APC_EINVAL, APC_ERANK, APC_ESINGULAR, APC_ENOCONV (eigenvalue
 * estimate did not converge), APC_ENODEV, APC_EHIP.  *out is NULL on error. */
apc_status apc_setup(apc_plan* out, const double* A, int64_t lda, const double* B, int64_t ldb,
                     int64_t N, int64_t n, const int64_t* off, int32_t m, int32_t k,
                     int32_t precision, double gamma, double eta, void* workspace,
                     size_t ws_bytes, void* stream);

/* Apply T updates of eq. (2a)-(2b) (T >= 0).  Asynchronous.  k = 1 FP64 with
 * every block of at most 64 rows and n <= 1024 (32 rows when n > 512), and m
 * no larger than the device's CU count (unless APC_RESIDENT=0 in the
 * environment at setup): ONE launch for all T updates, in which workgroup i
 * holds block i's rows of the factor in registers, and the m workgroups meet
 * at a device-wide barrier once per update to form x_bar (the updates of
 * eq. (2a)-(2b) unchanged; only sums are ordered differently from the
 * per-update kernels).  Its wait is bounded: if the device cannot hold all m
 * workgroups at once for seconds, the launch stops, x_bar becomes NaN and the
 * next apc_residual (and so apc_solve) returns APC_EHIP.  Otherwise per update
 * it enqueues, k = 1 with n <= 16384 (FP32) or 8192 (FP64): one pass over the
 * factor that forms w_i = Q_i^T (x_bar - x_i) row by row and adds each row's
 * share of Q_i w_i while the row is in registers, then one launch for
 * x_i += gamma (x_bar - x_i - Q_i w_i), the momentum average
 * x_bar <- (eta/m) sum_i x_i + (1 - eta) x_bar and the next differences;
 * other k = 1 plans (or APC_FUSED=0 in the environment at setup): for each
 * group of blocks, projection pass A (w_i = Q_i^T (x_bar - x_i)) and pass B
 * (x_i += gamma (x_bar - x_i - Q_i w_i)), then the average;
 * k-RHS form: pass A (W = C y), its split sum, pass B (Z = C^T W) and the
 * elementwise step y <- (1-gamma) y + gamma x_bar,
 * x_bar <- eta (x_bar(0) + y - Z/m) + (1 - eta) x_bar.  Returns at once. */
apc_status apc_iterate(apc_plan p, int32_t T);

/* As apc_iterate, replayed from a captured HIP graph: the first call for a
 * given T (and, in the k-RHS form with anchor updates, a given position in
 * the anchor cycle) captures the T updates' launches on the plan's stream;
 * later calls replay the graph, which removes the host's per-launch cost.
 * Results are those of apc_iterate, bit for bit.  The plan's stream must not
 * be the default (NULL) stream, and must not be under capture by the caller.
 * apc_set_params and apc_set_anchor drop the cached graphs (their launches
 * carry gamma and eta by value).  Asynchronous, like apc_iterate.
 * Errors: APC_EINVAL (NULL plan, T < 0, default stream), APC_EHIP. */
apc_status apc_iterate_graph(apc_plan p, int32_t T);

/* As apc_iterate, and also times every launch with a pair of HIP events that
 * the launch itself records at its start and end: *ms_total receives the span
 * of the T updates; *ms_pass_a, *ms_pass_b and *ms_average the summed
 * durations of the pass-A, pass-B and averaging launches (the single-pass
 * update counts its pass over C as pass A and its second launch as the
 * average).  Host pointers, any may be NULL.  Synchronises the stream once,
 * at the end. */
apc_status apc_iterate_timed(apc_plan p, int32_t T, float* ms_total, float* ms_pass_a,
                             float* ms_pass_b, float* ms_average);

/* Relative residual ||B - A X_bar||_F / ||B||_F in FP64 on the GPU (the
 * solver's convergence monitor).  *relres is host.  Synchronises. */
apc_status apc_residual(apc_plan p, double* relres);

/* Iterate until apc_residual <= rtol, checking every 8 updates, for at most
 * max_iters updates; then copy x_bar (device, n x k, as apc_get_xbar) to
 * Xbar.  In APC_BF16_IR mode each check is one refinement step: the inner
 * solve runs ~log(1e-3)/log(rho) updates, its result is added to the FP64
 * solution X, R = B - A X is formed in FP64 and the next inner solve starts on
 * R.  *iters_out (updates) and *relres_out are host (may be NULL).
 * Returns APC_ENOCONV if rtol was not reached (Xbar is still written),
 * APC_EDIVERGED if the residual became non-finite.  Synchronises. */
apc_status apc_solve(apc_plan p, double rtol, int32_t max_iters, double* Xbar, int64_t ldx,
                     int32_t* iters_out, double* relres_out);

/* Copy the master estimate x_bar (n x k) to device memory: entry (j, c) at
 * Xbar[j*ldx + c] (ldx >= k; for k = 1 the stride between entries, >= 1).
 * Asynchronous (stream-ordered). */
apc_status apc_get_xbar(apc_plan p, double* Xbar, int64_t ldx);

/* Copy every local solution x_i to device memory.  k = 1: m rows of n
 * doubles, row i at X + i*ldx (ldx >= n).  k > 1: m blocks of n x k, entry
 * (i, j, c) at X[(i*n + j)*ldx + c] (ldx >= k).  Not available in APC_BF16_IR
 * mode (APC_EUNSUPPORTED).  Asynchronous. */
apc_status apc_get_local(apc_plan p, double* X, int64_t ldx);

/* Apply every block's FP64 projector to its own row: out_i = P_i v_i =
 * v_i - Q_i (Q_i^T v_i) (Sec. 3.1), for m device rows of n doubles (stride
 * ldv >= n for both V and Out; V and Out must not overlap).  Uses the FP64
 * factor in every precision mode.  Needs a plan with k = 1 (else
 * APC_EUNSUPPORTED).  Asynchronous. */
apc_status apc_project(apc_plan p, const double* V, double* Out, int64_t ldv);

/* Host copies of the parameters in use and of the eigenvalue estimate
 * (mu_min, mu_max, rho are NaN when gamma and eta were given by the caller).
 * Any pointer may be NULL. */
apc_status apc_get_params(apc_plan p, double* gamma, double* eta, double* mu_min, double* mu_max,
                          double* rho);

/* Host-only helper (no GPU needed): Theorem 1's optimal parameters for a
 * spectrum of X enclosed in [mu_min, mu_max], 0 < mu_min <= mu_max <= 1.
 * gamma* is the smaller of the two roots (it must satisfy |1 - gamma| <= rho
 * because of the (m-1)n eigenvalues 1 - gamma of the error recursion, App. A);
 * rho* = (sqrt(kappa) - 1)/(sqrt(kappa) + 1), eq. (7).  Outputs are host
 * pointers (any may be NULL).  APC_EINVAL for an invalid interval. */
apc_status apc_optimal_params(double mu_min, double mu_max, double* gamma, double* eta,
                              double* rho);

/* Host-only helper used by the eigenvalue estimate: extreme eigenvalues of
 * the k x k symmetric tridiagonal matrix with diagonal alpha[0..k-1] and
 * off-diagonal beta[0..k-2] (bisection on Sturm counts), and the Lanczos
 * residual bounds |beta[k-1] * s_k| of the two extreme Ritz pairs (s = unit
 * eigenvector; beta[k-1] is read only when with_bounds != 0).  Host pointers.
 * APC_EINVAL when k < 1 or a pointer is NULL. */
apc_status apc_tridiag_extremes(const double* alpha, const double* beta, int32_t k,
                                int32_t with_bounds, double* lo, double* hi, double* bound_lo,
                                double* bound_hi);

/* Host copies of diagnostics: the number of Lanczos steps the eigenvalue
 * estimate took (0 when gamma and eta were given); the launch shape chosen for
 * this problem (pass-A rows per workgroup and column splits, block groups per
 * update); and the refinement steps apc_solve has taken (APC_BF16_IR).  Any
 * pointer may be NULL. */
apc_status apc_get_info(apc_plan p, int32_t* lanczos_steps, int32_t* rows_per_tile,
                        int32_t* column_splits, int32_t* block_groups, int32_t* refinements);

/* Host copies of what setup did for the thin QR of Sec. 3.1 (CholeskyQR):
 * *qr_passes = 2, or 1 when an APC_F32 / APC_BF16_IR plan (k = 1 with the
 * single-pass update, or the k-RHS form) skipped the second pass because the
 * rows' measured departure from orthonormality after the first,
 * max_i ||C_i C_i^T - I|| estimated with a random vector, was at most
 * 1e-10 / sqrt(max p_i), far below the rounding the factor then takes;
 * *qr_defect = that estimate (NaN when it was not measured: FP64 plans, k = 1
 * plans updated in two passes, or APC_QR_PASSES=2 in the environment).  Any
 * pointer may be NULL. */
apc_status apc_get_setup(apc_plan p, int32_t* qr_passes, double* qr_defect);

/* Launch shape the k-RHS path chose for one of its contractions (which: 0 =
 * pass A, 1 = pass B, 2 = the start x_bar(0) = (1/m) C^T c (FP64; FP32 with
 * APC_BF16_IR), 3 = the FP64
 * residual): rows of the streamed operand per workgroup, split-K factor, and
 * the measured time per launch when it was chosen by timing (0 when fixed by
 * APC_TN_TUNE=0 / APC_TN_RT / APC_TN_SPLIT).  Shapes are timed once per
 * problem shape and process.  which = 4: the single-pass k = 1 update, rows
 * per workgroup and rows per register group (in *splits), *tuned_us = 0.
 * which = 5: the single-launch k = 1 update of apc_iterate, the block rows and
 * columns one workgroup holds (in *splits), *tuned_us = 0.
 * Host pointers, any may be NULL.  APC_EUNSUPPORTED for which 0..3 on a k = 1
 * FP64/FP32 plan, for which = 4 on a plan that updates in two passes and for
 * which = 5 on a plan without the single-launch update. */
apc_status apc_get_launch(apc_plan p, int32_t which, int32_t* rows_per_wg, int32_t* splits,
                          float* tuned_us);

/* Anchor spacing of the FP32 / bf16 k-RHS iteration (plans whose updates use
 * the (y, x_bar) form with APC_F32 or APC_BF16_IR).  With every > 0, the first
 * update after setup (and after each refinement restart) and then every
 * every-th update form X y in FP64 on the FP64 factor and keep it as the anchor
 * (y_ref, u_ref = X y_ref); the updates in between multiply only y - y_ref
 * in low precision and add u_ref, so the error of the stored factor and of the
 * low-precision products acts on a vector that shrinks as the iteration
 * converges instead of on y itself.  every = 0 runs every update in the plan's
 * precision (the plain FP32 / bf16 iteration, whose accuracy levels off near
 * eps_FP32 / mu_min).  Default: 16 for APC_F32, 0 for APC_BF16_IR (there the
 * outer refinement corrects the inner solver).  Call after apc_setup and before
 * the first update.  Host-only.  APC_EUNSUPPORTED for other plans, APC_EINVAL
 * for every < 0 or after an update. */
apc_status apc_set_anchor(apc_plan p, int32_t every);

/* Replace the iteration parameters of eq. (2) (e.g. to probe the derivative in
 * gamma or eta).  Takes effect at the next update; host-only; mu_min, mu_max
 * and rho keep describing the setup's estimate.  APC_EINVAL for non-finite. */
apc_status apc_set_params(apc_plan p, double gamma, double eta);

/* Start Alg. 1 again without refactoring A: with B != NULL, new right-hand
 * sides (device, N x k FP64, entry (r, c) at B[r*ldb + c]; kept by pointer
 * like apc_setup's B); c_i = R_i^{-T} b_i, x_i(0) = Q_i c_i, x_bar(0) = mean
 * (Alg. 1 initialisation, via the stored inverse CholeskyQR factors).  With
 * B == NULL, restarts from the current right-hand sides.  The update count and
 * refinement count return to 0.  Synchronises when B is given (||B||). */
apc_status apc_restart(apc_plan p, const double* B, int64_t ldb);

/* Bytes of device workspace apc_backward needs for T updates with a checkpoint
 * every ckpt_every updates: ceil(T/ckpt_every)+1 saved (y, x_bar) pairs, one
 * recomputed segment of ckpt_every+1 pairs, the adjoint vectors.  0 for a plan
 * without the (y, x_bar) form or invalid arguments. */
size_t apc_backward_workspace_bytes(apc_plan p, int32_t T, int32_t ckpt_every);

/* Reverse-mode derivative of the unrolled iteration (Alg. 1 from its start,
 * T updates of eq. (2a)-(2b), with the plan's gamma and eta) for a scalar L
 * given dL/dx_bar(T) = dXbar (device, n x k FP64, entry (j, c) at
 * dXbar[j*ldd + c]).  Writes dL/dB to dB (device, N x k, entry (r, c) at
 * dB[r*lddb + c]) and dL/dgamma, dL/deta to *dgamma, *deta (host).
 *
 * The forward is run again from the start, keeping (y, x_bar) every
 * ckpt_every updates (~sqrt(T) balances memory and recomputation); the
 * reverse pass recomputes one segment at a time and applies the transpose of
 * each update.  X is symmetric, so the transposed update is the same two
 * contractions as a forward update (W = C v, Z = C^T W) plus an elementwise
 * step; the start x_bar(0) = (1/m) C^T c, c_i = R_i^{-T} b_i, is transposed
 * by one FP64 product and the two inverse CholeskyQR factors.  With L linear
 * in x_bar(T), dL/dB is exact in exact arithmetic; in FP32 plans the
 * products run in FP32 as in the forward.  Needs an APC_F64 / APC_F32 plan in
 * the (y, x_bar) form (k > 1 or APC_REDUCED_FORM; else APC_EUNSUPPORTED).
 * bwd_ws: device, 256-byte aligned, >= apc_backward_workspace_bytes.  The plan
 * is left at x_bar(T) of the forward run (apc_iterations = T).
 * Synchronises. */
apc_status apc_backward(apc_plan p, const double* dXbar, int64_t ldd, int32_t T,
                        int32_t ckpt_every, double* dB, int64_t lddb, double* dgamma,
                        double* deta, void* bwd_ws, size_t bwd_bytes);

/* apc_backward without a workspace argument, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid allocation).  It allocates nothing: its checkpoint scratch is a
 * fixed array of 64 MiB per GPU inside the library, held from the first
 * apc_setup on that GPU until the process ends.  Arguments, outputs, results
 * and synchronisation are those of apc_backward; the caller still provides
 * dXbar, dB and the host scalars.
 * Errors: those of apc_backward, and APC_EINVAL when
 * apc_backward_workspace_bytes(p, T, ckpt_every) exceeds 64 MiB (nothing is
 * enqueued then; use apc_backward with a workspace).
 * Every call on one GPU shares that GPU's array: calls that overlap in time on
 * one GPU (other host threads, or plans on other streams) race and give wrong
 * results.  Each call clears what it needs zeroed itself. */
apc_status apc_backward_noalloc(apc_plan p, const double* dXbar, int64_t ldd, int32_t T,
                                int32_t ckpt_every, double* dB, int64_t lddb, double* dgamma,
                                double* deta);

/* ---- Many independent systems (one persistent launch per pass) ----------
 *
 * A batch runs eq. (2a)-(2b) for many independent systems at once (Sec. 2's
 * machines, Alg. 1, for many problems): every system is a plan from
 * apc_setup, all plans on one stream, each keeping its own factor and state in
 * its own workspace.  Two kinds of plans can be batched:
 *   - k = 1, APC_F32, per-block form;
 *   - the k-RHS (y, x_bar) form with FP32 products (k > 1 or APC_REDUCED_FORM,
 *     k <= 128), with or without FP64 anchor updates.
 * Every launch is a persistent grid of a fixed number of workgroups looping
 * over a work list that covers all systems; items of inactive systems are
 * skipped.  Per update:
 *   - k = 1 plans only, single pass (every row at most 1024 wide): one launch
 *     of (system, row tile) items that form each tile's partial row of
 *     Q_i w_i, one of (system, column chunk) items for the x_i update, the
 *     average and the next differences; otherwise three launches (pass A over
 *     16-row tiles, pass B over (block, column slab) items, the average);
 *   - with k-RHS plans: four launches -- pass-A contraction tiles (W = C y),
 *     split sums of W, pass-B tiles (Z = C^T W), (y, x_bar) update chunks,
 *     preceded on anchor updates by one launch of y_ref chunks -- and the
 *     k = 1 plans' single-pass tiles and combine items ride in launches 1-2
 *     or 3-4 (split between the two by factor size).  All k-RHS plans of one
 *     batch must share k (padded), the anchor spacing and their count of
 *     updates since the start; the batch follows one anchor cycle for them.
 * The grid is chosen at creation by timing the first launch of an update
 * (APC_BATCH_GRID fixes it).  Each system's gamma, eta and ||b|| are captured
 * at creation.  The plans must outlive the batch; apc_get_xbar etc. on a plan
 * see the batch's updates. */
typedef struct apc_batch_s* apc_batch;

/* Bytes of device workspace (descriptors and work lists) for a batch of these
 * plans; 0 when they cannot form a batch. */
size_t apc_batch_workspace_bytes(const apc_plan* plans, int32_t count);

/* Build the batch (host array of count plans; workspace device, 256-byte
 * aligned, caller-owned).  Synchronises.  APC_EUNSUPPORTED for plans of other
 * kinds (FP64, bf16, k-RHS with k > 128) or k-RHS plans that differ in k,
 * anchor spacing or update count, or k = 1 plans that do not update in one
 * pass next to k-RHS plans; APC_EINVAL for mixed streams or a small workspace. */
apc_status apc_batch_create(apc_batch* out, const apc_plan* plans, int32_t count, void* workspace,
                            size_t ws_bytes);

/* T updates of every active system (asynchronous). */
apc_status apc_batch_iterate(apc_batch b, int32_t T);

/* The same T updates through a hipGraph: captured on the batch's stream at the
 * first call for this T (and position in the k-RHS plans' anchor cycle; the
 * stream must not be the default stream), replayed after.  Results are
 * identical to apc_batch_iterate. */
apc_status apc_batch_iterate_graph(apc_batch b, int32_t T);

/* FP64 relative residual ||B_s - A_s X_bar_s||_F / ||B_s||_F of every active system
 * into relres (host, count; inactive systems keep their last value), and
 * deactivate each system whose residual is <= rtol or not finite (rtol < 0:
 * none).  active (host, count, may be NULL) receives the flags.  Synchronises. */
apc_status apc_batch_residuals(apc_batch b, double rtol, double* relres, int32_t* active);

/* Mark every system active again. */
apc_status apc_batch_activate(apc_batch b);

/* Per-system stopping: every system is checked afresh at entry, then
 * residuals every check_every updates; each system stops once its residual is
 * <= rtol (or not finite), until none is left or max_iters updates were
 * applied.  use_graph != 0 runs the updates through apc_batch_iterate_graph.
 * iters_out, relres_out: host arrays of count (may be NULL).  APC_EDIVERGED if
 * some system's residual became non-finite, else APC_ENOCONV if some system
 * did not reach rtol.  Synchronises. */
apc_status apc_batch_solve(apc_batch b, double rtol, int32_t max_iters, int32_t check_every,
                           int32_t use_graph, int32_t* iters_out, double* relres_out);

/* Launch shape: workgroups per persistent launch, work items per pass, and the
 * measured time of the pass over the factors when the grid was chosen by
 * timing.  A batch whose plans all update in one pass over their factor (rows
 * up to 1024 wide) does too: *items_a then counts its row tiles, *items_b is
 * 0 and *items_avg counts the 32-column items of the update + average launch.
 * With k-RHS plans: the items of an ordinary update's first (pass A),
 * third (pass B) and second (split sums) launches.  Host pointers. */
apc_status apc_batch_get_launch(apc_batch b, int32_t* grid, int32_t* items_a, int32_t* items_b,
                                int32_t* items_avg, float* tuned_us);

/* Release the batch (and its captured graphs) after its stream has finished. */
void apc_batch_destroy(apc_batch b);

/* ---- Comparison methods on the same passes (Sec. 4.3, Sec. 6) -----------
 *
 * The distributed heavy-ball method (D-HBM, Sec. 4.3) on plan p's row blocks:
 *     z <- beta z + sum_i C_i^T (C_i x - d_i),     x <- x - alpha z,
 * with [C_i, d_i] = [A_i, b_i] (APC_HBM_PLAIN), or Sec. 6's preconditioned
 * blocks [(A_i A_i^T)^{-1/2} A_i, (A_i A_i^T)^{-1/2} b_i]
 * (APC_HBM_PRECONDITIONED).  The preconditioned blocks are realised as
 * [Q_i^T, c_i] with the plan's factor and c_i = R_i^{-T} b_i: they differ from
 * Sec. 6's by an orthogonal p_i x p_i factor per block, so the gradient
 * C_i^T (C_i x - d_i) = Q_i (Q_i^T x - c_i) is the same.  One update is a row
 * pass (w_r = C_r . x - d_r, FP64 accumulation), a block pass
 * (sum over the block's rows of w_r C_r, per block) and an elementwise step that
 * adds the blocks in a fixed order; the factor or the copy of A is streamed in
 * the plan's precision (APC_F32: FP32), vectors and arithmetic are FP64.
 * Start (not fixed by the paper): x(0) = the plan's x_bar(0) (Alg. 1
 * initialisation), z(0) = 0, so both methods start where APC starts.  Needs a
 * k = 1 APC_F64 / APC_F32 plan in the per-block form (else APC_EUNSUPPORTED).
 * The plan must outlive the object; its own state is not changed. */
typedef struct apc_hbm_s* apc_hbm;

typedef enum {
  APC_HBM_PLAIN = 0,          /* blocks [A_i, b_i] (Sec. 4.3)                  */
  APC_HBM_PRECONDITIONED = 1  /* blocks (A_i A_i^T)^{-1/2} [A_i, b_i] (Sec. 6) */
} apc_hbm_kind;

/* Bytes of device workspace for a heavy-ball run of this kind on plan p:
 * x, z, per-block partial sums, row-pass partials, and for APC_HBM_PLAIN a
 * copy of A in the plan's precision padded like the factor plus a copy of b.
 * 0 for an unsupported plan or kind. */
size_t apc_hbm_workspace_bytes(apc_plan p, int32_t kind);

/* Create the run.  alpha, beta: the step and momentum; if either is NaN both
 * are set to the heavy-ball optimum alpha = 4/(sqrt(L)+sqrt(l))^2,
 * beta = ((sqrt(L)-sqrt(l))/(sqrt(L)+sqrt(l)))^2 for the spectrum [l, L] of
 * sum_i C_i^T C_i: m times the plan's enclosure of X's spectrum for the
 * preconditioned kind (sum_i Q_i Q_i^T = m X), and for the plain kind the
 * enclosure of A^T A's spectrum from the same GPU Lanczos procedure as the
 * plan's (run on the streamed copy of A).  workspace: device, 256-byte
 * aligned, >= apc_hbm_workspace_bytes, caller-owned.  Synchronises.
 * APC_EINVAL for a bad kind or small workspace, APC_ESINGULAR when A^T A is
 * numerically singular. */
apc_status apc_hbm_create(apc_hbm* out, apc_plan p, int32_t kind, double alpha, double beta,
                          void* workspace, size_t ws_bytes);

/* T updates (asynchronous, on the plan's stream). */
apc_status apc_hbm_iterate(apc_hbm h, int32_t T);

/* Back to x(0), z = 0 (asynchronous). */
apc_status apc_hbm_restart(apc_hbm h);

/* Copy x (n doubles) to device memory with entry stride ldx >= 1.
 * Asynchronous. */
apc_status apc_hbm_get_x(apc_hbm h, double* x, int64_t ldx);

/* ||b - A x|| / ||b|| in FP64 (host result).  Synchronises. */
apc_status apc_hbm_residual(apc_hbm h, double* relres);

/* The run's parameters (host pointers, each may be NULL): alpha, beta, the
 * spectrum enclosure [lam_min, lam_max] they came from (NaN when the caller
 * gave alpha and beta), the predicted rate sqrt(beta) at the optimum, the
 * Lanczos steps spent (0 when none ran), and the updates applied. */
apc_status apc_hbm_get_params(apc_hbm h, double* alpha, double* beta, double* lam_min,
                              double* lam_max, double* rho, int32_t* lanczos_steps,
                              int64_t* iters);

/* Release the host-side object. */
void apc_hbm_destroy(apc_hbm h);

/* Number of updates applied since setup (host). */
int64_t apc_iterations(apc_plan p);

/* Release the host-side plan.  Does not touch the caller's device memory. */
void apc_destroy(apc_plan p);

/* Message describing the last non-OK status returned on this thread. */
const char* apc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* APC_H */
