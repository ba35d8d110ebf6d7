/*
 * igs.h -- C ABI of the MI355X (gfx950) iterated Gauss-Seidel GMRES solver.
 *
 * Solves A x = b, A real n x n (Section 1 of the paper), with restarted
 * GMRES(m) whose Arnoldi-QR step needs ONE global reduction per iteration:
 *
 *   gs_iters = 2 : the one-reduce hybrid MGS-CGS step (Algorithm 4.2): the
 *                  reduction [V, u]^T [u, A u], a lagged normalisation
 *                  gamma^2 = u^T u - p^T p, the second Gauss-Seidel sweep
 *                  t = (I + L)^{-1} V^T u lagged by one iteration, the first
 *                  sweep of the next vector through Stephen's trick, and the
 *                  Hessenberg column finished from eq:Aw.
 *   gs_iters = 1 : the two-reduce step (Algorithm 4.1) stopped after its first
 *                  Gauss-Seidel sweep (steps 4-13), which also needs a single
 *                  reduction: [V, w]^T [w, A w].
 *
 * The least-squares problem (eq:llse) is reduced with Givens rotations on the
 * device; x = x0 + V y closes each restart cycle.  Restarts begin from the
 * explicit residual b - A x; the solve is converged when
 * ||b - A x|| <= tol ||b|| at the start of a cycle, and a cycle ends early
 * when its Arnoldi residual |g_J| <= tol ||b||.
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - Return value: IGS_OK (0), IGS_ENOCONV (1, x holds the last iterate), or a
 *    negative error code.  No C++ exception crosses this boundary.
 *    igs_last_error() gives a message for the last failing call on a context.
 *  - "device pointer" means memory the caller allocated on the GPU the
 *    context was created on (e.g. a torch tensor's data_ptr()); the library
 *    never frees caller memory and keeps no reference to it after the call.
 *  - All GPU work runs on the HIP stream passed to igs_create*; the calls are
 *    synchronous: they return after that stream has finished the work.
 *  - A context is not thread-safe; use one context per host thread.
 *  - After IGS_EDEVICE the context must only be destroyed.
 */
#ifndef IGS_H
#define IGS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct igs_ctx igs_ctx;

enum {
  IGS_OK = 0,
  IGS_ENOCONV = 1,    /* iteration budget used up; x holds the last iterate   */
  IGS_EINVAL = -1,    /* invalid argument or input data (nothing was changed) */
  IGS_ENOMEM = -2,    /* device or host allocation failed                      */
  IGS_EDEVICE = -3,   /* a HIP runtime call failed                             */
  IGS_ENOTIMPL = -4,  /* option combination not implemented                   */
  IGS_ENUMERIC = -5   /* a non-finite value appeared during the solve          */
};

/* Why the last restart cycle ended (igs_info.last_cycle_status). */
enum {
  IGS_CYCLE_RUNNING = 0,
  IGS_CYCLE_CONVERGED_AT_START = 1, /* ||r0|| <= tol ||b||: solve converged   */
  IGS_CYCLE_ARNOLDI_CONVERGED = 2,  /* |g_J| <= tol ||b||                     */
  IGS_CYCLE_FULL = 3,               /* m columns finished                     */
  IGS_CYCLE_BREAKDOWN = 4,          /* gamma_j <= n eps ||H[0:j, j-1]||       */
  IGS_CYCLE_LAGNORM = 5,            /* lagged norm cancelled; explicit norm   */
  IGS_CYCLE_MAXIT = 6,              /* iteration budget reached               */
  IGS_CYCLE_NONFINITE = 7           /* NaN or Inf in a reduction              */
};

/* Optional solver settings (igs_solve_opts).  Zero-initialise, then set. */
typedef struct igs_opts {
  int64_t maxit;        /* iteration budget; <= 0 means 20 n                    */
  double lagnorm_tau;   /* gs_iters=2: if u^T u - p^T p < tau u^T u the norm is
                           recomputed explicitly as ||u - V t|| (one extra
                           reduction) and the cycle ends; <= 0 means 1e-4      */
  int final_basis_vector; /* 1: also normalise v_J when a cycle ends, so the
                             debug copy of V holds J+1 valid columns           */
  int profile;          /* 1: time every launch of the step kernels with HIP
                           events (igs_profile_get)                            */
  int max_cycles;       /* > 0: stop after this many restart cycles            */
  int keep_first_basis; /* 1: keep a device copy of the first cycle's V for
                           igs_debug_copy_V (costs one copy of the basis)      */
  int profile_kernels;  /* with profile = 1: bit (1 << IGS_K_*) selects the
                           kernels to time; 0 means all                        */
  int inner_fp32;       /* 1: mixed precision (the paper's Conclusions name it
                           as future work).  Each restart cycle runs in FP32
                           (operator apply with FP32 values, the fused
                           reduction with FP64 sums, the basis update with FP64
                           coefficients), while the residual b - A x, the
                           small solve, the Givens least squares and
                           x = x0 + V y stay in FP64: iterative refinement with
                           one FP32 Arnoldi cycle per correction.  CSR
                           operators only (IGS_ENOTIMPL otherwise).            */
  int two_reduce;       /* 1 with gs_iters = 2: the two-reduce Algorithm 4.1
                           (Section 4): after the first sweep a second
                           reduction r2 = V^T u, r3 = (I + L)^{-1} r2,
                           w = u - V r3 and the column r1 + r3; two global
                           reductions per iteration (a comparator for the
                           one-reduce default)                                 */
  int separate_apply;   /* 1: the operator apply as a kernel of its own before
                           the reduction.  By default, with an ELL form (rows
                           of at most 8 entries) and n a multiple of 4, each
                           block of the reduction forms its own rows of A u
                           first (one launch and one read of u and of A u
                           less per iteration, the ELL columns read as 16-bit
                           offsets where they fit); the results are
                           bit-identical either way.                        */
  double inner_rtol;    /* inner_fp32: a cycle also ends once its Arnoldi
                           residual is <= inner_rtol * ||r0|| of the cycle;
                           <= 0 means 1e-5                                     */
  int batch_reduce_rows;  /* batches (igs_solve_batch, igs_serve_batched): at
                             least this many rows per block of the fused
                             reduction (fewer, larger blocks when many
                             instances share a launch).  1: the grid a lone
                             solve launches (then every member is
                             bit-identical to igs_solve_opts, except the
                             explicit norm of a lagged-norm fallback, whose
                             per-thread partial sums follow the update's
                             tiles); <= 0: 2048                              */
  int batch_update_tiles; /* batches: at least this many tiles (2,048 rows of
                             FP64, 4,096 of FP32) per block of the update.
                             1 (the default; <= 0 means 1): one tile per
                             block                                           */
  int cycle_graph;      /* 1: record the launches of a restart cycle in a HIP
                           graph once and replay it for every cycle (one
                           launch instead of about 2(m+1)+4); the graph is kept in
                           the context and reused while b, x and the settings
                           stay the same.  Not with profile or two_reduce
                           (ignored there).  Results are bit-identical.      */
  int mgs;              /* 1: the comparator the paper measures against:
                           restarted GMRES on modified Gram-Schmidt Arnoldi
                           (Section 1), FP64, c + 2 grid-wide reductions for
                           column c (one kernel each) where IGS-GMRES has one.
                           gs_iters, lagnorm_tau and final_basis_vector do
                           not apply; not with inner_fp32 or two_reduce
                           (IGS_ENOTIMPL); profile and cycle_graph are
                           ignored.                                           */
  int products_in_update; /* 1: every block of the update kernel forms the
                             small products with T and H itself also when
                             they no longer fit its shared memory (large
                             restart lengths).  By default a kernel of their
                             own forms them first, one wave per output over
                             many CUs (Section 4's operation counts: the
                             triangular work grows as j^2); the results are
                             bit-identical either way.                     */
} igs_opts;

/* Result summary of a solve.  Any pointer argument of this type may be NULL. */
typedef struct igs_info {
  int64_t iters;            /* Arnoldi iterations = sum of finished columns     */
  int64_t cycles;           /* restart cycles run, incl. check cycles (the
                               explicit residual and iteration 0 only: after
                               the iteration budget, and after a cycle that
                               met the tolerance by its Arnoldi residual)     */
  double relres_true;       /* ||b - A x|| / ||b|| at the last explicit residual */
  double arnoldi_relres;    /* |g_J| / ||b|| at the end of the last full cycle  */
  double bnorm;             /* ||b||                                            */
  int converged;            /* 1 when relres_true <= tol                        */
  int breakdowns;           /* cycles ended by (happy) breakdown                */
  int lagnorm_fallbacks;    /* explicit-norm recomputations (gs_iters=2)        */
  int last_cycle_status;    /* IGS_CYCLE_* of the last cycle                     */
  int first_cycle_J;        /* columns finished in the first cycle              */
  int stagnant_cycles;      /* restart cycles after which the true residual
                               ||b - A x|| was above (1 - 1e-3) times its value
                               at the cycle's start (a restarted solve that
                               stalls shows a growing count)                  */
  double seconds;           /* wall time of the call                            */
} igs_info;

/*
 * Create a solver context for a CSR operator (Section 1: a real n x n A).
 *   row_ptr: int32[n+1], non-decreasing, row_ptr[0] = 0, row_ptr[n] = nnz.
 *   col_idx: int32[nnz], each in [0, n).  vals: float64[nnz], finite.
 *   ptrs_on_device: 0 = the three arrays are host memory, 1 = device memory.
 *   hip_stream: hipStream_t for all work of this context (NULL: null stream).
 * The arrays are validated and copied; the caller keeps ownership.  When
 * every row has at most 8 entries (and the mean row length is above 4), the
 * context also keeps a column-major ELL copy (K x n values and int32
 * columns, K the longest row) and, when every entry lies within 32,767
 * columns of its row, the ELL columns as int16 offsets from the row: 12
 * bytes per ELL slot, 2 more for the offsets (and 4 for FP32 values once a
 * solve runs FP32 cycles), beside the CSR arrays.
 * Errors: IGS_EINVAL (n < 1, nnz < 0, malformed CSR, non-finite values),
 *         IGS_ENOMEM, IGS_EDEVICE.  On error *out is set to NULL.
 */
int igs_create(igs_ctx **out, int64_t n, int64_t nnz, const int32_t *row_ptr,
               const int32_t *col_idx, const double *vals, int ptrs_on_device,
               void *hip_stream);

/*
 * Create a solver context for a dense operator (Section 1: a real n x n A;
 * the dense non-normal test matrices of Section 5 are of this kind).
 *   A: float64, row-major, n rows of leading dimension lda >= n, finite.
 *   ptr_on_device: 0 = host memory, 1 = device memory.
 * The matrix is copied into device memory the context owns.
 * Errors as igs_create.
 */
int igs_create_dense(igs_ctx **out, int64_t n, const double *A, int64_t lda,
                     int ptr_on_device, void *hip_stream);

/*
 * Solve A x = b.
 *   b: device pointer, float64[n], 16-byte aligned.
 *   x: device pointer, float64[n], 16-byte aligned; in: x0, out: the solution.
 *   restart: m >= 1 (clamped to n and to IGS_MAX_RESTART).
 *   tol: relative residual tolerance >= 0.
 *   gs_iters: 1 or 2 (see the top of this file).
 *   info: optional result summary.
 * Workspace (the n x (m+1) basis and the small matrices) is allocated on the
 * first call and reused while restart does not grow.
 * Returns IGS_OK when converged, IGS_ENOCONV when the budget ran out (x holds
 * the last iterate), IGS_EINVAL (bad argument, non-finite b or x0; x is
 * unchanged), IGS_ENUMERIC, IGS_ENOMEM or IGS_EDEVICE.
 */
int igs_solve(igs_ctx *ctx, const double *b, double *x, int restart, double tol,
              int gs_iters, igs_info *info);

/* igs_solve with optional settings (opts may be NULL = defaults). */
int igs_solve_opts(igs_ctx *ctx, const double *b, double *x, int restart, double tol,
                   int gs_iters, const igs_opts *opts, igs_info *info);

/* Release the context and everything it allocated.  NULL is accepted. */
int igs_destroy(igs_ctx *ctx);

/* Message of the last failing call on ctx ("" if none); valid until the next
 * call on ctx.  With ctx == NULL: the last failure of igs_create*. */
const char *igs_last_error(const igs_ctx *ctx);

/* Largest supported restart length. */
#define IGS_MAX_RESTART 512

/* ---- Serving: continuous batching of independent solves ------------------ */

/* One request of a serving trace: a CSR system A x = b (host arrays, the same
 * format and checks as igs_create) that arrives `arrival` seconds after the
 * start of igs_serve.  The caller owns every array; x receives the solution
 * (from x0 = 0).  Outputs: t_admit and t_done (seconds after the start; -1
 * when the request never ran), iters, rc (the igs_solve_opts return value)
 * and status (IGS_CYCLE_* of its last cycle). */
typedef struct igs_request {
  int64_t n, nnz;
  const int32_t *row_ptr, *col_idx;
  const double *vals, *b;
  double *x;
  double arrival;
  double t_admit, t_done;  /* out */
  int64_t iters;           /* out */
  int rc;                  /* out */
  int status;              /* out */
} igs_request;

/*
 * Serve a trace of independent GMRES(restart) solves on the current device
 * with continuous batching: a request joins a FIFO queue at its arrival time
 * and is admitted as soon as one of `slots` solver slots is free and the
 * device memory it holds (its operator, b, x, the Krylov basis V and the
 * Hessenberg and triangular matrices, kept resident while it runs) fits
 * within mem_cap bytes together with the requests already running.  Each slot
 * owns a stream and a context sized for the largest request, so admitted
 * solves overlap on the device and the loop allocates nothing per request.
 * A request's result does not depend on what runs beside it (every kernel
 * reduces in a fixed order): x is bit-identical to a lone igs_solve_opts of
 * the same system with the same arguments.
 *   tol, gs_iters, opts: as igs_solve_opts (opts may be NULL; profile and
 *     keep_first_basis are ignored).  *wall_seconds: time from the start to
 *     the last completion (may be NULL).
 * The memory a request holds is 12 nnz + 4 (n+1) + 8 n (m'+5) + 32 (m'+2)^2
 * bytes with m' = min(restart, n), plus 4 nnz + 4 n (m'+2) with inner_fp32
 * (the FP32 basis and values).  Each slot holds the footprint of the
 * largest request of the trace (n and nnz taken at their maxima), allocated
 * once at the start; the loop runs min(slots, mem_cap / that footprint)
 * slots, at least one, so that the slots' device memory stays within
 * mem_cap whenever one slot fits it.
 * Returns IGS_OK when the trace was served: each request's rc tells its own
 * outcome (IGS_EINVAL for a malformed CSR, IGS_ENOCONV, ...), and the other
 * requests run regardless.  IGS_EINVAL for bad arguments or a request larger
 * than mem_cap, IGS_ENOMEM/IGS_EDEVICE when the slots cannot be set up
 * (nothing ran in these cases; message in igs_last_error(NULL)), IGS_EDEVICE
 * when a request hit a device error.
 */
int igs_serve(igs_request *reqs, int nreq, int slots, int64_t mem_cap, int restart,
              double tol, int gs_iters, const igs_opts *opts, double *wall_seconds);

/* ---- Batches: many independent solves advanced by each launch ------------ */

/* Most solves one batch advances together. */
#define IGS_MAX_BATCH 32

/*
 * Solve count independent systems A_k x_k = b_k (Section 4, Algorithm 4.2,
 * as igs_solve_opts) together: every step of the restart cycle (operator
 * apply, fused reduction, small solve and update, least squares, x update)
 * is one kernel launch for all members, each member on a contiguous range of
 * the grid equal to the grid its lone solve launches.  Members may differ in
 * n and in their operators; a member whose cycle ended waits, at no cost
 * beyond the launches, until the others end theirs.  Each x_k is
 * bit-identical to igs_solve_opts(ctxs[k], b[k], x[k], ...) alone.
 *   ctxs[k]: distinct CSR contexts on one device; the batch runs on the
 *            stream of ctxs[0] after each member's stream is synchronised.
 *   b[k], x[k]: device float64[n_k], 16-byte aligned; x[k] holds x0 on entry
 *            and the solution on return.
 *   count: 1..IGS_MAX_BATCH.  restart, tol, gs_iters, opts: as
 *            igs_solve_opts (opts may be NULL).  two_reduce and
 *            keep_first_basis are not supported here (IGS_ENOTIMPL).
 *   infos[k] (may be NULL): as igs_solve_opts reports for member k.
 *   rcs[k] (may be NULL): member k's return code as igs_solve_opts gives it.
 * Returns IGS_OK when every member converged, IGS_ENOCONV when some did not,
 * a negative code when a member failed (see rcs) or the call is invalid
 * (message in igs_last_error(ctxs[0]), or igs_last_error(NULL) when ctxs or
 * count is invalid).
 */
int igs_solve_batch(igs_ctx *const *ctxs, const double *const *b, double *const *x, int count,
                    int restart, double tol, int gs_iters, const igs_opts *opts,
                    igs_info *infos, int *rcs);

/*
 * igs_serve with batched kernels: one stream and up to `batch`
 * (1..IGS_MAX_BATCH) requests advanced by each launch, as igs_solve_batch.
 * Admission happens between restart cycles: after every cycle the finished
 * requests leave (x copied back) and the oldest arrived requests join while a
 * member is free and the memory cap allows.  Requests, memory accounting,
 * outputs and return codes are those of igs_serve; each x is bit-identical to
 * a lone solve.  The batch is limited to the members the cap holds at the
 * largest footprint, as igs_serve limits its slots.  two_reduce is not
 * supported (IGS_ENOTIMPL).
 */
int igs_serve_batched(igs_request *reqs, int nreq, int batch, int64_t mem_cap, int restart,
                      double tol, int gs_iters, const igs_opts *opts, double *wall_seconds);

/* ---- Autotuning of launch shapes ---------------------------------------- */

typedef struct igs_tune_report {
  double cycle_ms_before;  /* one full restart cycle with the default shapes  */
  double cycle_ms_after;   /* the same with the chosen shapes                  */
  int spmv_rpg;            /* rows per lane group of the operator apply (0:
                              the default kept)                               */
  int reduce_halved;       /* iterations j whose fused reduction runs with
                              half the blocks (twice the rows per block)      */
  int update_halved;       /* the same for the basis update                  */
  int reserved;
} igs_tune_report;

/*
 * Choose launch shapes for this context by timing them on the device: two
 * full restart cycles of GMRES(restart) with gs_iters sweeps (tol 0, a fixed
 * right-hand side, HIP events around every launch) per candidate.  The
 * candidates are, per iteration j, the fused reduction and the update with
 * half their default blocks (kept where they save more than 3%), and for a
 * CSR operator the rows per lane group of the operator apply.  The choice
 * stays in the context and applies to every later igs_solve_opts on it; the
 * results change by summation order only (the grid of the reductions
 * changes), and stay deterministic.  Takes a few cycles of device time;
 * allocates and frees two vectors of n doubles.  The profile counters are
 * reset.  report may be NULL.  Errors: IGS_EINVAL, IGS_ENOMEM, IGS_EDEVICE.
 */
int igs_tune(igs_ctx *ctx, int restart, int gs_iters, igs_tune_report *report);

/* Back to the default launch shapes. */
int igs_tune_reset(igs_ctx *ctx);

/* ---- Inspection of the FIRST restart cycle of the last solve (tests) ----- */

/* Copy the Hessenberg matrix H (before Givens rotation) of the first cycle to
 * host memory, column-major with leading dimension ldh >= J+1; *ncols = J.
 * H_host must hold ldh * J doubles.  H is the (J+1) x J matrix of the Arnoldi
 * relation A V_J = V_{J+1} H (Section 1; with two sweeps each column is
 * finished from eq:Aw, Section 4). */
int igs_debug_copy_H(igs_ctx *ctx, double *H_host, int ldh, int *ncols);

/* Copy the basis V of the first cycle (J+1 columns, of which column J is
 * valid only with final_basis_vector) to a device buffer, column-major with
 * leading dimension ldv >= n; *ncols = J + 1.  V_dev must hold ldv*(J+1).
 * Needs opts.keep_first_basis = 1 in the last solve, else IGS_EINVAL.  V is
 * the orthonormal Krylov basis of the Arnoldi relation (Section 1), whose
 * loss of orthogonality ||I - V^T V|| Section 4 bounds. */
int igs_debug_copy_V(igs_ctx *ctx, double *V_dev, int64_t ldv, int *ncols);

/* Estimate of ||A||_2 from the last solve (the backward error's
 * denominator, eq:nrbe): the largest singular value of the first cycle's
 * (J+1) x J Hessenberg matrix, computed on the host from the copy the solve
 * keeps (Lanczos on H^T H, exact for J <= 100).  With the orthonormal basis,
 * A V_J = V_{J+1} H (Section 1, the Arnoldi relation), so it equals
 * ||A V_J||_2, a lower bound of ||A||_2; a backward error formed with it is
 * an upper bound.  Not part of the solve's time.  Errors: IGS_EINVAL when the
 * first cycle finished no column. */
int igs_anorm_estimate(igs_ctx *ctx, double *anorm_out);

/* Kernel of the dense operator apply z = A u (Section 1's real n x n A):
 *   IGS_DENSE_VALU: one wavefront per row, 16-byte loads, a wave sum;
 *   IGS_DENSE_MFMA: the matrix cores (v_mfma_f64_16x16x4f64), a block per 16
 *                   rows, the vector as the A operand of each product;
 *   IGS_DENSE_LDS:  the vector staged in shared memory once per block of 16
 *                   rows (n <= 8192).
 * All are bound by the matrix's bytes; a context starts with the fastest on
 * MI355X.  Errors: IGS_EINVAL (not a dense context, an unknown variant, or
 * IGS_DENSE_LDS with n > 8192). */
enum { IGS_DENSE_VALU = 0, IGS_DENSE_MFMA = 1, IGS_DENSE_LDS = 2 };
int igs_dense_variant(igs_ctx *ctx, int variant);

/* ---- Step kernels on caller buffers (unit tests of each hot-path step) --- */

/* z = A u with the context's operator kernel.  u, z: device float64[n]. */
int igs_kernel_spmv(igs_ctx *ctx, const double *u, double *z);

/* The fused reduction of one iteration: with u = V[:, j],
 *   P[c] = V[:, c]^T u and Q[c] = V[:, c]^T z for c = 0..j.
 * V: device, column-major, ldv >= n, j+1 columns; z: device float64[n] or
 * NULL (then Q is not formed).  P_host, Q_host: host float64[j+1] (Q_host may
 * be NULL).  0 <= j < IGS_MAX_RESTART. */
int igs_kernel_reduce(igs_ctx *ctx, const double *V, int64_t ldv, int j,
                      const double *z, double *P_host, double *Q_host);

/* The basis update of one iteration, in place on V:
 *   v = (V[:, j] - V[:, 0:j] t) * inv_gamma            -> V[:, j]
 *   u = z * inv_gamma - V[:, 0:j] r1[0:j] - v r1[j]    -> V[:, j+1]
 * V: device, column-major, ldv >= n, j+2 columns; z: device float64[n];
 * t_host: host float64[j] (NULL = zeros); r1_host: host float64[j+1]. */
int igs_kernel_update(igs_ctx *ctx, double *V, int64_t ldv, int j, const double *z,
                      const double *t_host, const double *r1_host, double inv_gamma);

/* ---- Without allocation ---------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * igs_kernel_reduce without a context: the same kernel and launch shape, so
 * the same sums bit for bit, with its per-block partial sums, group totals
 * and arrival counters in a static device array of the library
 * (IGS_NOALLOC_BYTES on each GPU it runs on, held until the process ends)
 * instead of a workspace:
 *   PQ[c]         = V[:, c]^T u   (u = V[:, j]),
 *   PQ[j + 1 + c] = V[:, c]^T z   (0 when z is NULL),   c = 0..j.
 * V: device, column-major, ldv >= n >= 1, j + 1 columns; z: device float64[n]
 * or NULL; PQ: device float64[2 (j + 1)], written by the call.
 * 0 <= j < IGS_NOALLOC_MAX_COLS.  hip_stream: a stream of the current
 * device (NULL: its null stream).
 * Asynchronous: returns once the work is queued (no synchronisation, no
 * memset: a counter-clearing kernel and the reduction), so a caller may
 * record it into a graph.  The first call on a device also looks up the
 * array's device address and the occupancy of every reduction shape; make
 * that first call outside a capture.
 * Every call on one GPU shares that GPU's array and leaves it holding its own
 * sums: calls that overlap on one GPU (other streams, other host threads)
 * race and must be serialised by the caller.
 * Errors: IGS_EINVAL (NULL V or PQ, n < 1, ldv < n, j out of range; checked
 * before any device call), IGS_EDEVICE (a launch failed).  The message is
 * igs_last_error(NULL). */
#define IGS_NOALLOC_MAX_COLS 256
#define IGS_NOALLOC_BYTES ((2048 + 64) * 2 * IGS_NOALLOC_MAX_COLS * 8 + 512)
int igs_kernel_reduce_noalloc(const double *V, int64_t ldv, int64_t n, int j,
                              const double *z, double *PQ, void *hip_stream);

/* ---- Per-kernel timing (opts.profile = 1) --------------------------------- */

enum { IGS_K_SPMV = 0, IGS_K_REDUCE = 1, IGS_K_UPDATE = 2, IGS_K_XUPDATE = 3,
       IGS_K_RESIDUAL = 4,
       IGS_K_OPREDUCE = 5,   /* the operator apply fused into the reduction */
       IGS_K_COUNT = 6 };

/* Totals over the timed launches of kernel `which` since the last reset:
 * launches, summed HIP-event milliseconds, and summed algorithmic bytes
 * (the minimum HBM traffic of each launch, computed from its shape). */
int igs_profile_get(igs_ctx *ctx, int which, int64_t *launches, double *total_ms,
                    double *total_bytes);
int igs_profile_reset(igs_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* IGS_H */
