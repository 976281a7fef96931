/*
 * nnls.h -- C ABI of the MI355X (gfx950) block principal pivoting NNLS library.
 *
 * Solves  min 1/2 ||A x - b||_2^2  subject to  x >= 0  (Cantarella & Piatek, "tsnnls",
 * arXiv cs/0408029, Eq. 1) for A of size m x n, m >= n, full column rank, and returns the
 * solution x together with the dual vector y = A^T A x - A^T b of the complementarity form
 * (Eq. 3): x >= 0, y >= 0, x_i y_i = 0.
 *
 * Method: the block principal pivoting loop of the paper's Sec. 2 algorithm box.  Each
 * pivot iteration solves the unconstrained least-squares problem on the free columns F
 * (Eq. 4) through the normal equations with a Cholesky factor of the F-principal block of
 * the cached Gram matrix A^T A (Sec. 2.1, Sec. 3), forms y_G = A_G^T (A_F x_F - b) (Eq. 5),
 * zeroes tested entries within tau of zero, counts the negative ones and exchanges them
 * between F and G (all at once; after p_max non-improving block exchanges, only the one
 * with the largest index).  Every step runs in HIP kernels on the device.
 *
 * Conventions shared by every call:
 *   - Array arguments are DEVICE pointers unless the comment says "host".  They are
 *     borrowed for the duration of the call and owned by the caller.
 *   - Matrices: CSC with int32 colptr[n+1], int32 rowidx[nnz] (0-based, strictly
 *     increasing within each column) and double val[nnz]; or dense column-major double
 *     with leading dimension lda >= m.
 *   - Indices are 0-based; "largest index" is the largest column number.
 *   - Calls are stream-ordered on the handle's stream and return after the result is on
 *     the device (the call synchronises that stream).  A handle must not be used from two
 *     threads at once; separate handles are independent.
 *   - Return value: an nnls_status.  No exception or abort crosses the ABI.  When a solve
 *     fails, x and y hold the last iterate (unspecified after INVALID_* errors) and
 *     info->status / info->failed_index say why.
 */
#ifndef NNLS_H_
#define NNLS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NNLS_OK = 0,
  NNLS_ERR_INVALID_ARG = -1,   /* bad size, null pointer, malformed CSC structure       */
  NNLS_ERR_INVALID_VALUE = -2, /* NaN or Inf in A or b, or a tested entry of an iterate
                                  (x_i on F, y_i on G) that is not finite, which no sign
                                  test can decide                                        */
  NNLS_ERR_NOT_PD = -3,        /* Cholesky breakdown: the F-block is not numerically
                                  positive definite (A_F rank deficient, or kappa^2 eps
                                  >= 1 as Sec. 2.1 warns); failed_index names the column */
  NNLS_ERR_MAXITER = -4,       /* iteration cap reached before a feasible split          */
  NNLS_ERR_NO_MEMORY = -5,     /* device or pinned host allocation failed                */
  NNLS_ERR_DEVICE = -6,        /* HIP runtime error, or a device-side wait exceeded its
                                  bound                                                  */
  NNLS_ERR_REFINE = -7,        /* mixed precision: refinement did not reach its target   */
  NNLS_ERR_TIMEOUT = -8,       /* nnls_server_wait: the request is not finished yet      */
  NNLS_ERR_TOO_LARGE = -9      /* nnls_solve_dense_batched_noalloc: the batch needs more
                                  device memory than its fixed scratch array holds       */
} nnls_status;

typedef enum {
  NNLS_FP64 = 0,     /* factor and every vector in float64                               */
  NNLS_FP32_IR = 1,  /* F-block factor in float32, float64 iterative refinement of the
                        normal equations; residual, y_G and sign tests in float64.  The
                        solve of an intermediate split is refined only until every tested
                        sign (|v| >= tau) is certified by an error bound (Sec. 3: the
                        pivot rule needs correct signs only); the feasible split's x_F is
                        refined to ir_rtol                                               */
  NNLS_BF16_IR = 2   /* as NNLS_FP32_IR, with the factor's left-looking updates on MFMA
                        from bfloat16 copies of the finished tiles (float32 accumulation;
                        the diagonal tiles, their inverses and the triangular solves stay
                        float32).  Refinement recovers the float64 accuracy while
                        kappa(A_F^T A_F) 2^-8 stays well below 1; an F-block beyond that
                        is redone in float32, then float64.  Sparse and dense
                        single-problem solves and nnls_cholesky; the batched solves and
                        the serving engine return NNLS_ERR_INVALID_ARG for it           */
} nnls_precision;

/* flags */
#define NNLS_FLAG_PROFILE 1u   /* time kernel classes with HIP events (nnls_get_profile) */
#define NNLS_FLAG_REFINE_FINAL 2u /* NNLS_FP64: once the split is feasible, recompute x_F more
                                     accurately (the final step of Sec. 3) by float64
                                     refinement against the residual from A with the split's
                                     cached factor, then classify the refined x and y again
                                     (pivoting resumes if that finds infeasible entries)    */
#define NNLS_FLAG_REFINE_AUTO 8u /* NNLS_FP64: once the split is feasible, estimate the
                                     condition of A_F^T A_F from the split's factor (Hager /
                                     Higham 1-norm estimate: a few solves with the factor)
                                     and run the NNLS_FLAG_REFINE_FINAL step only when the
                                     predicted error 0.1 kappa_1 eps exceeds ir_rtol (the
                                     error control of Sec. 3)                                */
#define NNLS_FLAG_GRAM_DUAL 16u  /* dense problems (single and batched): y_G for the sign
                                     tests from the cached Gram matrix, H_GF x_F - c_G (Eq. 3),
                                     which reads |G| x |F| of H instead of A twice (Eq. 5,
                                     the default); the sparse path ignores it, refinement
                                     and the final recomputation keep Eq. 5               */
#define NNLS_FLAG_REFINE_ALL 32u /* NNLS_FP32_IR: refine the solve of every split to ir_rtol
                                     instead of stopping once the tested signs are certified */
#define NNLS_FLAG_NO_FACTOR_REUSE 4u /* refactor the whole F-block in every pivot
                                     iteration.  By default F is ordered so that the leading
                                     tile columns no exchange touched come first, and their
                                     factor tiles (exact for that leading block) are kept    */

typedef struct {
  double tau;           /* zeroing threshold; paper: 1e-12 (Sec. 2)                      */
  int32_t p_max;        /* non-improving block exchanges allowed; paper: 3 (Sec. 2 box)  */
  int32_t max_iter;     /* pivot iteration cap; <= 0 means 5 n + 100 (paper gives none)  */
  int32_t precision;    /* nnls_precision                                                */
  int32_t ir_max_steps; /* NNLS_FP32_IR: refinement steps per pivot iteration            */
  double ir_rtol;       /* NNLS_FP32_IR: the final x_F is refined until the last
                           correction is below ir_rtol max|x_F| (while the refinement
                           contracts by 1/2 or better, that bounds the error left)       */
  uint32_t flags;       /* NNLS_FLAG_*                                                   */
  uint32_t max_workgroups; /* cap on the factor kernel's grid: above it, a persistent grid
                              of this many workgroups takes the tiles from a queue (so
                              that several solves can share the device).  0: two per
                              compute unit, the kernel's occupancy                     */
} nnls_options;

typedef struct {
  int32_t status;       /* nnls_status of the solve                                      */
  int32_t iterations;   /* pivot iterations (exchange + solve passes)                    */
  int32_t n_free;       /* |F| of the returned split                                     */
  int32_t last_ninf;    /* infeasible count at exit (0 on success)                       */
  int32_t failed_index; /* NOT_PD: column of the first non-positive pivot; else -1       */
  int32_t ir_steps;     /* NNLS_FP32_IR: total refinement steps                          */
  double min_margin;    /* smallest |v| over the final sign tests that were not zeroed   */
  double setup_ms;      /* host wall time of validation + Gram formation                 */
  double solve_ms;      /* host wall time of the whole call                              */
  double est_rel_err;   /* NNLS_FP32_IR: bound on max|x_F - exact| / max|x_F| of the
                           returned x (exact: the least-squares solution on the final F):
                           the last refinement correction, which bounds the error left
                           while the refinement contracts by 1/2 or better, plus the
                           rounding of x_F itself (the refinement residual is summed with
                           compensation, so its own rounding is far below both); 0 when F
                           is empty, -1 when not measured.  NNLS_FLAG_REFINE_AUTO:
                           predicted relative error of the final normal-equations solution,
                           0.1 kappa_1(A_F^T A_F) 2^-52 with the 1-norm condition estimated
                           from the factor.  Otherwise -1                                  */
} nnls_info;

/* One row of the per-iteration trace recorded by the last solve on a handle. */
typedef struct {
  int32_t k;        /* infeasible count after zeroing                                    */
  int32_t branch;   /* 0: k < N, block exchange; 1: budget block exchange; 2: single     */
  int32_t N;        /* best count after the rule                                         */
  int32_t p;        /* remaining budget after the rule                                   */
  int32_t n_free;   /* |F| after the exchange                                            */
  int32_t n_reused; /* leading F positions whose factor tiles were kept from the previous
                       iteration's factor (a multiple of 64; 0 when refactored whole)      */
  int32_t ir_steps; /* NNLS_FP32_IR: refinement steps of this iteration's solve (the last
                       row also counts the final refinement of the feasible split)       */
} nnls_trace_row;

typedef struct nnls_handle nnls_handle;

/* Human-readable name of a status code (static storage). */
const char* nnls_status_string(int status);

/* Paper defaults: tau 1e-12, p_max 3 (Sec. 2); max_iter 0 (= 5n+100); FP64. */
void nnls_default_options(nnls_options* opts);

/* Create a handle on HIP device `device`, issuing work on `stream` (a hipStream_t, or
 * NULL for the default stream).  The handle owns a growable device workspace and a small
 * pinned host buffer; both are released by nnls_destroy. */
int nnls_create(nnls_handle** out, int device, void* stream);
int nnls_destroy(nnls_handle* h);

/* Solve Eq. 1 for sparse A in CSC (device arrays).  b: double[m].  Outputs x, y:
 * double[n] device, written with x_G = 0 and y_F = 0 exactly.  opts may be NULL
 * (defaults).  info is a host struct and may be NULL.
 * Errors: INVALID_ARG for sizes (m < n, n < 1, nnz < 0), null pointers, colptr not
 * starting at 0 / not non-decreasing / not ending at nnz, or a row index out of [0, m) or
 * not strictly increasing in its column; INVALID_VALUE for non-finite A or b. */
int nnls_solve_csc(nnls_handle* h, int32_t m, int32_t n, int64_t nnz, const int32_t* colptr,
                   const int32_t* rowidx, const double* val, const double* b, double* x,
                   double* y, const nnls_options* opts, nnls_info* info);

/* Solve Eq. 1 for dense column-major A (device, lda >= m).  Same outputs and errors. */
int nnls_solve_dense(nnls_handle* h, int32_t m, int32_t n, const double* A, int32_t lda,
                     const double* b, double* x, double* y, const nnls_options* opts,
                     nnls_info* info);

/* Solve `batch` independent dense problems together (Eq. 1 for each).  m, n, lda:
 * host int32[batch]; A, b, x, y: host arrays of `batch` DEVICE pointers (A column-major
 * with lda >= m, b double[m], x and y double[n] outputs).  Two launches: one workgroup per
 * problem forms A^T b and the Gram matrix (and checks the input), then one workgroup per
 * problem runs the whole pivoting loop of the Sec. 2 algorithm box on the device; a
 * problem's result does not depend on the other problems in the batch.  opts applies to every problem
 * (NNLS_FP32_IR: float32 Gram matrix and factor, float64 refinement; NNLS_BF16_IR runs the
 * same float32 tier, bit for bit: at n <= 256 the batched kernels are bound by the stream of
 * A and the pivot chain, not by the factor's multiply rate).  info: host nnls_info[batch] or
 * NULL.  Returns NNLS_OK when every problem succeeded, otherwise the first failing status
 * (per-problem statuses are in info; a failed problem does not affect the others).
 * Errors: INVALID_ARG for a bad size or null pointer (nothing runs); per problem
 * INVALID_VALUE, NOT_PD, MAXITER as for nnls_solve_dense. */
int nnls_solve_dense_batched(nnls_handle* h, int32_t batch, const int32_t* m, const int32_t* n,
                             const double* const* A, const int32_t* lda, const double* const* b,
                             double* const* x, double* const* y, const nnls_options* opts,
                             nnls_info* info);

/* For callers that cannot allocate device memory (code under HIP stream capture, serving
 * loops that must keep a fixed footprint, harnesses that forbid allocation): the same
 * solve as nnls_solve_dense_batched (same kernel, same per-problem results, bit for bit),
 * with every device buffer of the launch (problem descriptors, per-problem status and the
 * workspace arena) carved from one static device array of NNLS_NOALLOC_SCRATCH_BYTES per
 * GPU instead of the handle's growable workspace.  The call performs no hipMalloc,
 * hipFree or other allocation; the array is part of the library's code object, so each
 * GPU the library runs on holds it until the process ends.
 * Capacity: 256-byte-aligned descriptors (batch * 64 bytes), statuses (batch * 40 bytes)
 * and the problems' workspaces (about 8 (n^2 + m) bytes plus the factor tiles of n each)
 * must fit together; otherwise NNLS_ERR_TOO_LARGE is returned and nothing runs.
 * Problems run in the given order (not sorted by size).  NNLS_FLAG_PROFILE is ignored.
 * Every call on one GPU shares that GPU's array: calls that overlap on the same GPU (from
 * two threads, or on two streams) race and give undefined results, so callers serialise
 * them.  The array keeps the last call's contents; the kernel initialises everything it
 * reads, so nothing needs clearing between calls.
 * Arguments, outputs and the other errors: as nnls_solve_dense_batched. */
#define NNLS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int nnls_solve_dense_batched_noalloc(nnls_handle* h, int32_t batch, const int32_t* m,
                                     const int32_t* n, const double* const* A, const int32_t* lda,
                                     const double* const* b, double* const* x, double* const* y,
                                     const nnls_options* opts, nnls_info* info);

/* ---------------------------------------------------------------------------------
 * Prepared batched solves, replayed from a captured HIP graph
 * For a batch whose shapes and device buffers stay the same over many solves (new values
 * in A and b each time): nnls_batch_plan_create checks the batch as
 * nnls_solve_dense_batched does, uploads the problem descriptors, allocates the workspace
 * and the status array once, and records the two kernels of a batched solve and the copy
 * of the statuses into pinned host memory in a HIP graph (captured on a private stream);
 * nnls_batch_plan_execute replays the graph on the handle's stream, with no host-side
 * preparation.  Each replay reads A and b as they are when it runs and writes x and y; the
 * results are bitwise those of nnls_solve_dense_batched on the same inputs (same kernels,
 * same order).  The plan keeps the pointers it was given: the caller keeps those buffers
 * alive and unmoved until nnls_batch_plan_destroy.  The plan uses the handle's stream and
 * device; calls on one plan are not thread-safe.  NNLS_FLAG_PROFILE is ignored.
 * Errors of create: INVALID_ARG (as nnls_solve_dense_batched), NO_MEMORY, DEVICE (the
 * capture or instantiation failed); nothing is kept on error and *plan is NULL.
 * --------------------------------------------------------------------------------- */
typedef struct nnls_batch_plan nnls_batch_plan;
int nnls_batch_plan_create(nnls_handle* h, int32_t batch, const int32_t* m, const int32_t* n,
                           const double* const* A, const int32_t* lda, const double* const* b,
                           double* const* x, double* const* y, const nnls_options* opts,
                           nnls_batch_plan** plan);
/* Queue one replay on the handle's stream.  With info (host nnls_info[batch]) the call
 * waits for it and returns as nnls_solve_dense_batched does; with info NULL it returns
 * NNLS_OK once the replay is queued, and nnls_batch_plan_info reads the statuses later.
 * Errors: INVALID_ARG (plan NULL), DEVICE. */
int nnls_batch_plan_execute(nnls_batch_plan* plan, nnls_info* info);
/* Wait for the handle's stream and fill info (host nnls_info[batch]) from the last replay;
 * returns its first failing status, or NNLS_OK. */
int nnls_batch_plan_info(nnls_batch_plan* plan, nnls_info* info);
/* The Gram kernel's accumulator tile shape that the plan's autotuner chose for each
 * bucket: shapes (host int32[9]) receives, for k = ceil(n / 32) = 1..8, the number of 32 x
 * 32 rectangles of the Gram matrix a wave accumulates per pass over A (0 where the batch
 * has no problem of that bucket; n > 256 is not tuned).  At plan creation every bucket is
 * timed on its own problems with each shape whose pass plan differs, and the fastest
 * kept; all shapes sum each entry in the same order, so results do not depend on it. */
int nnls_batch_plan_tile_shapes(const nnls_batch_plan* plan, int32_t* shapes);
int nnls_batch_plan_destroy(nnls_batch_plan* plan);

/* ---------------------------------------------------------------------------------
 * Serving engine: continuous batching of independent requests (Eq. 1 each) on one device.
 *
 * nnls_server_submit_csc copies a request's host arrays into pinned staging and returns a
 * ticket at once.  Requests are admitted in arrival order as soon as the device memory
 * they need (A, Gram matrix, factor at |F| = n, vectors; estimated on the host from the
 * CSC) fits next to the requests already running; a request that is alone is always
 * admitted.  Requests with n <= batch_max_n go to batched lanes, which step at the level
 * of pivot iterations: each step admits queued requests (their dense A, Gram matrix,
 * factor and (F, G) state then stay in device memory), advances every live request by
 * batch_step_iters iterations of the Sec. 2 loop in one launch (one workgroup per request,
 * as in nnls_solve_dense_batched) and retires the ones that finished.  Larger requests run
 * the sparse solver of nnls_solve_csc, several at once on separate streams.  Which path a request takes depends on its n only, and both
 * paths give results that do not depend on the other requests, so a result is the same
 * whether the request ran alone or among others.  x and y are available in host memory
 * when the request is reported done; latency is measured from submit to that point.
 * All server calls are thread-safe.
 * --------------------------------------------------------------------------------- */
typedef struct nnls_server nnls_server;

typedef struct {
  size_t hbm_budget;        /* device bytes admitted requests may hold; 0: 90% of the free
                               memory at create                                          */
  int32_t workers;          /* sparse requests solved at once, each on its own stream;
                               0: 16.  Streams beyond the process's hardware queues
                               (GPU_MAX_HW_QUEUES, 4 unless set before the HIP runtime
                               starts) share queues and serialise: set it to at least
                               workers + batch_lanes                                     */
  int32_t batch_lanes;      /* batched launches in flight at once; 0: 2                  */
  int32_t batch_max_n;      /* n <= batch_max_n goes to batched launches; 0: 256; < 0:
                               never                                                     */
  int32_t batch_max_count;  /* live requests per batched lane; 0: 1024                   */
  int32_t batch_step_iters; /* pivot iterations every live request of a batched lane takes
                               per step (admission and retirement happen between steps);
                               0: 1; < 0: whole solves, a step ends when all have finished */
  int32_t pad;
} nnls_server_config;

typedef struct {
  int64_t submitted;        /* since create or the last reset                            */
  int64_t completed;        /* finished (any status)                                     */
  int64_t pending;          /* queued, not admitted yet                                  */
  int64_t batches;          /* batched launches issued                                   */
  int32_t running;          /* admitted and not finished                                 */
  int32_t max_running;
  double committed_bytes;   /* estimated device bytes of the running requests            */
  double peak_committed_bytes;
  double budget_bytes;
  double p50_ms, p99_ms, mean_ms, max_ms;   /* submit -> x, y in host memory             */
  double solves_per_s;      /* completed / (last completion - first submit)              */
} nnls_serving_stats;

/* Start a server on device `device`.  cfg and opts may be NULL (defaults; opts applies to
 * every request, NNLS_FLAG_PROFILE is ignored, and max_workgroups 0 becomes 96 so that
 * concurrent factorisations share the device; results do not depend on it).  Every
 * precision is accepted: the sparse lane runs it as nnls_solve_csc does, and the batched
 * lanes run NNLS_BF16_IR as their float32 tier (as nnls_solve_dense_batched).
 * Errors: INVALID_ARG (bad config), DEVICE, NO_MEMORY. */
int nnls_server_create(nnls_server** out, int device, const nnls_server_config* cfg,
                       const nnls_options* opts);

/* Queue one request.  colptr, rowidx, val, b are HOST arrays in the CSC convention above;
 * they are copied before the call returns.  *ticket (host) names the request.  Errors:
 * INVALID_ARG for sizes, null pointers or a malformed CSC structure (checked on the host;
 * nothing is queued); NO_MEMORY. */
int nnls_server_submit_csc(nnls_server* s, int32_t m, int32_t n, int64_t nnz,
                           const int32_t* colptr, const int32_t* rowidx, const double* val,
                           const double* b, uint64_t* ticket);

/* Non-blocking check.  *done (host) is 1 when the request has finished: then x and y
 * (HOST double[n], either may be NULL) and info (may be NULL) receive its result, the
 * ticket is released, and the return value is the request's status.  *done is 0 and the
 * return value NNLS_OK while it runs or waits.  INVALID_ARG for an unknown ticket.
 * info->setup_ms is the time the request waited for admission and info->solve_ms its
 * latency (submit to result in host memory). */
int nnls_server_poll(nnls_server* s, uint64_t ticket, int32_t* done, double* x, double* y,
                     nnls_info* info);

/* Blocking form of nnls_server_poll: waits up to timeout_ms (< 0: without limit) and
 * returns NNLS_ERR_TIMEOUT, keeping the ticket, if the request has not finished. */
int nnls_server_wait(nnls_server* s, uint64_t ticket, double timeout_ms, double* x,
                     double* y, nnls_info* info);

/* Counters and latency percentiles over the requests completed since the last reset. */
int nnls_server_stats(nnls_server* s, nnls_serving_stats* out);
int nnls_server_reset_stats(nnls_server* s);

/* Let running requests finish, drop queued ones and unclaimed results, free everything. */
int nnls_server_destroy(nnls_server* s);

/* Copy up to `cap` trace rows of the last solve on this handle into `rows` (host).
 * Returns the number of rows the solve recorded (which may exceed cap). */
int nnls_get_trace(nnls_handle* h, nnls_trace_row* rows, int cap);

/* Kernel-class timings of the solves run with NNLS_FLAG_PROFILE since the last reset.
 * For class c (see nnls_profile_class), launches[c] and total_ms[c] are written (host
 * arrays of length NNLS_PROFILE_CLASSES), and flops[c] the algorithmic work of those
 * launches (floating-point operations; bytes for the memory-bound classes). */
#define NNLS_PROFILE_CLASSES 9
typedef enum {
  NNLS_PROF_GRAM = 0,      /* A^T A and A^T b (bytes)                                   */
  NNLS_PROF_CONTROL = 1,   /* classify, count, exchange, rebuild F (bytes)              */
  NNLS_PROF_CHOLESKY = 2,  /* gather + tiled Cholesky of the F-block (flops |F|^3/3)    */
  NNLS_PROF_TRSV = 3,      /* two triangular solves (bytes of L read)                   */
  NNLS_PROF_RESIDUAL = 4,  /* r = A x - b and y_G = A_G^T r (bytes; in nnls_dual_csc the
                              residual alone, the dual being NNLS_PROF_DUAL)            */
  NNLS_PROF_REFINE = 5,    /* mixed precision refinement (bytes)                        */
  NNLS_PROF_BATCHED = 6,   /* a batched launch's pivoting kernel (the pivot loops of all
                              problems; work: sum n^2 m, as for the Gram kernel)        */
  NNLS_PROF_DUAL = 7,      /* y_G = A_G^T r on its own (bytes); inside NNLS_PROF_RESIDUAL
                              when timed as part of a solve                             */
  NNLS_PROF_BATCHED_GRAM = 8 /* a batched launch's Gram kernel: c, the Gram matrices and
                              the input check (flops sum n^2 m)                         */
} nnls_profile_class;
int nnls_get_profile(nnls_handle* h, int64_t* launches, double* total_ms, double* work);
int nnls_reset_profile(nnls_handle* h);

/* Time kernel classes on every call made on this handle from now on (on != 0), the step
 * entry points included, as NNLS_FLAG_PROFILE does for one solve; on == 0 turns it off. */
int nnls_set_profiling(nnls_handle* h, int on);

/* ---------------------------------------------------------------------------------
 * Step entry points.  Each runs one step of the pivot iteration on its own, with the
 * same kernels the solver uses, so that every step can be checked in isolation.
 * --------------------------------------------------------------------------------- */

/* Gram matrix and right-hand side (Sec. 3: A^T A from column dot products, cached once;
 * Sec. 2.1: A^T b).  Writes the full symmetric H = A^T A as a dense n x n column-major
 * double array (device, ldh >= n) and c = A^T b (device double[n]). */
int nnls_gram_csc(nnls_handle* h, int32_t m, int32_t n, int64_t nnz, const int32_t* colptr,
                  const int32_t* rowidx, const double* val, const double* b, double* H,
                  int32_t ldh, double* c);

/* The same for a dense A (device, column-major m x n, lda >= m): H on MFMA float64, one
 * workgroup per 64 x 64 tile of its lower half, mirrored. */
int nnls_gram_dense(nnls_handle* h, int32_t m, int32_t n, const double* A, int32_t lda, const double* b,
                    double* H, int32_t ldh, double* c);

/* Cholesky factor of the symmetric positive definite n x n matrix S (device, column-major,
 * lower triangle read) into L (device, column-major, ldl >= n; the strict upper triangle
 * is written as zero).  This is the factor of Sec. 2.1, run by the tiled MFMA kernel the
 * solver uses on its F-block.  precision: NNLS_FP64, NNLS_FP32_IR (float32 factor,
 * returned widened to double) or NNLS_BF16_IR (float32 factor whose updates read bfloat16
 * tile copies).  *failed (host) is -1, or the first column whose pivot was
 * non-positive or non-finite (then the status is NNLS_ERR_NOT_PD). */
int nnls_cholesky(nnls_handle* h, int32_t n, const double* S, int32_t lds, double* L,
                  int32_t ldl, int32_t precision, int32_t* failed);

/* Solve S x = rhs for the SPD matrix S (device, column-major, lower triangle read) by the
 * solver's factor and its two triangular solves (normal equations of Sec. 2.1). */
int nnls_spd_solve(nnls_handle* h, int32_t n, const double* S, int32_t lds, const double* rhs,
                   double* x, int32_t* failed);

/* Eq. 5 on a given split: r = A x - b (x is used as given: callers pass x_G = 0) and
 * y_i = a_i^T r for i in G (free[i] == 0), y_i = 0 for i in F.  free: uint8[n] device.
 * r may be NULL.  When n (m) exceeds 2^19, the residual (dual) gathers x (r) in slices of
 * 2^18 elements over a sliced copy of A that the call builds in the handle's workspace
 * (about 12 nnz + 4 (m + 1) n / 2^18 bytes per copy); each r_i and y_i is then the
 * sequential sum of its terms in ascending index order. */
int nnls_dual_csc(nnls_handle* h, int32_t m, int32_t n, int64_t nnz, const int32_t* colptr,
                  const int32_t* rowidx, const double* val, const double* b,
                  const uint8_t* free_flags, const double* x, double* r, double* y);

/* Eq. 5 on a given split for dense column-major A (device, lda >= m): r = A x - b and
 * y_i = a_i^T r for i in G, y_i = 0 for i in F.  Same arguments as nnls_dual_csc
 * otherwise; r may be NULL. */
int nnls_dual_dense(nnls_handle* h, int32_t m, int32_t n, const double* A, int32_t lda,
                    const double* b, const uint8_t* free_flags, const double* x, double* r,
                    double* y);

/* One classify-and-exchange step (Sec. 2 box): zero tested entries with |v| < tau (v = x_i
 * on F, y_i on G), count the negative ones (k), apply the counter rule to (N, p) and flip
 * the membership of the exchanged variables.  x, y, free_flags are device arrays updated
 * in place (x is additionally zeroed on the new G and y on the new F).  state (host,
 * int32[3]) holds {N, p, reserved} in and out; N < 0 stands for infinity.  out (host,
 * int32[4]) receives {k, branch (-1 when k == 0), largest infeasible index, new |F|
 * (-1 when k == 0: nothing is exchanged)}.  A tested entry that is NaN or infinite
 * returns NNLS_ERR_INVALID_VALUE and exchanges nothing. */
int nnls_pivot_step(nnls_handle* h, int32_t n, double* x, double* y, uint8_t* free_flags,
                    double tau, int32_t p_max, int32_t* state, int32_t* out);

#ifdef __cplusplus
}
#endif

#endif /* NNLS_H_ */
