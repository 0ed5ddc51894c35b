/* hmlik.h -- H-matrix Gaussian log-likelihood on AMD MI355X (gfx950).
 *
 * C ABI of the library libhmlik.so.  The method is that of Litvinenko, Sun,
 * Genton, Keyes, "Likelihood Approximation With Hierarchical Matrices For
 * Large Spatial Datasets" (arXiv:1709.04419):
 *
 *   L~(theta) = -n/2 log(2 pi) - sum_i log L~_ii - 1/2 v^T v,   L~ v = Z     (eq. 4, Sect. 3.1)
 *
 * where L~ is the H-Cholesky factor (Sect. 3.2) of the H-matrix approximation
 * (Sect. 2.1, Def. 2.1, Remark 2.4) of the Matern covariance (eq. 2,
 * Sect. 2.2) plus a nugget tau^2 I (remark in Sect. 2.4), built over a
 * geometric cluster tree with standard admissibility (App. B, Defs. B.1-B.3).
 *
 * Conventions
 *   - Every function returns hm_status; nothing throws or aborts across the ABI.
 *   - Arrays passed in are owned by the caller and are copied before the call
 *     returns (host pointers) or used only in the call's stream order
 *     (device pointers).  Handles are owned by the library.
 *   - Matrices are column-major; coordinates are n x 2 row-major (x0 y0 x1 y1 ...).
 *   - Arithmetic is FP64 (prec = HM_FP64), or FP64 with FP32-valued low-rank
 *     factors and FP32 low-rank products (prec = HM_MIXED, see hm_approx).
 *     Results are deterministic: the same inputs give bitwise-equal outputs
 *     (a level schedule only reorders tasks that do not depend on each other).
 *   - Calls on one dataset must not overlap; different datasets may be used
 *     from different threads only with different contexts.  While a request
 *     server (hm_server_*) exists on a context, it alone issues that context's
 *     device work: the evaluation, set-up and readback calls on the context
 *     and its datasets return HM_ERR_BUSY (the introspection calls
 *     hm_dataset_info, _export_tree, _export_blocks and _footprint still work).
 */
#ifndef HMLIK_H
#define HMLIK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HM_OK = 0,
  HM_ERR_ARG = 1,       /* invalid argument (null pointer, size, non-finite value, theta <= 0) */
  HM_ERR_NOT_SPD = 2,   /* a pivot of the H-Cholesky was <= 0 (the paper's breakdown at coarse
                           accuracy, Tables 6 and 7); outputs are NaN, fail_block/fail_pivot set */
  HM_ERR_OOM = 3,       /* device allocation failed, or (hm_dataset_create) the task graph exceeds the
                           schedule's 32-bit offsets (about 1.8e9 dependencies at n = 2,000,000) */
  HM_ERR_DEVICE = 4,    /* a HIP runtime call failed */
  HM_ERR_INTERNAL = 5,  /* an internal invariant failed (planner error on unusual input) */
  HM_ERR_CANCELLED = 6, /* the request was cancelled before it finished */
  HM_ERR_BUSY = 7       /* a request server owns the context (see Conventions) */
} hm_status;

typedef struct hm_ctx hm_ctx;
typedef struct hm_dataset hm_dataset;
typedef struct hm_server hm_server;

/* theta = (sigma^2, ell, nu) of eq. (2) and the nugget tau^2. */
typedef struct {
  double sigma2; /* > 0 */
  double ell;    /* > 0, the argument of K_nu is h / ell (eq. 2 as printed) */
  double nu;     /* > 0 */
  double nugget; /* >= 0, added on the diagonal only */
} hm_theta;

/* Cluster tree options (App. B): leaf size n_min (1..64) and admissibility eta >= 0. */
typedef struct {
  int32_t leaf_size;
  double eta;
} hm_tree_opts;

/* Arithmetic of an evaluation.  HM_FP64: every step in FP64.  HM_MIXED: the
 * low-rank factors U, V of C~ and L~ and the products of the H-Cholesky
 * updates in FP32, the dense leaves, log-determinant and recompressions in
 * FP64, and C~^{-1} Z improved by iterative refinement (see hm_result). */
typedef enum { HM_FP64 = 0, HM_MIXED = 1 } hm_precision;

/* Accuracy (Remark 2.4 / Def. 2.1): exactly one of
 *   fixed_rank > 0 (ranks <= fixed_rank, eps ignored), or
 *   fixed_rank == 0 and eps > 0 (relative spectral accuracy per block).
 * prec selects the arithmetic (hm_precision).  refine_max_iter >= 0 and
 * refine_tol >= 0 bound the iterative refinement of x = C~^{-1} Z in the
 * HM_MIXED form (stop after that many steps or once the relative residual
 * ||Z - C~ x|| / ||Z|| is at most refine_tol); they must be 0 in HM_FP64. */
typedef struct {
  int32_t fixed_rank;
  double eps;
  int32_t prec;            /* hm_precision */
  int32_t refine_max_iter;
  double refine_tol;
} hm_approx;

/* One evaluation: one entry per right-hand side (column of Z). */
typedef struct {
  double loglik;      /* eq. (4) */
  double logdet;      /* log|C~| = 2 sum log L~_ii */
  double quadform;    /* v^T v = Z^T (L~ L~^T)^{-1} Z, L~ v = Z (eq. 4) */
  int64_t n;          /* number of locations */
  int32_t max_rank;   /* largest rank of a low-rank block of the factor */
  int32_t rank_capped; /* ACA runs and truncations (assembly and factorisation) in which the rank
                           cap of 64 bound in the accuracy mode, so that the block misses eps; 0 = none */
  int64_t bytes_C;    /* storage of C~ at its actual ranks: 8 (dense entries + sum (m + n) k) */
  int64_t bytes_L;    /* the same for L~ (0 after a breakdown) */
  int32_t status;     /* hm_status of the evaluation */
  int32_t fail_pivot; /* row of the failed pivot inside fail_block, else -1 */
  int64_t fail_block; /* block id of the failed pivot (HM_ERR_NOT_SPD), else -1 */
  double refine_quad; /* Z^T x with x the refined C~^{-1} Z (HM_MIXED); equals quadform in HM_FP64 */
  double refine_resid; /* ||Z - C~ x|| / ||Z|| of that x (HM_MIXED); 0 in HM_FP64 */
  int32_t refine_iters; /* refinement steps taken (0 in HM_FP64) */
  int32_t reserved;
  double t_assemble, t_factor, t_solve; /* seconds (device events) */
} hm_result;

/* Create a context on HIP device `device`.  `stream` is a hipStream_t (NULL =
 * the default stream) on which all work of this context is ordered.  The
 * context owns the work-group workspace its datasets share (grown, with a
 * synchronisation, when a dataset that needs more is created). */
hm_status hm_ctx_create(int device, void *stream, hm_ctx **out);
/* Destroy every dataset of a context before the context itself.  A server
 * still running on the context is destroyed first (hm_server_destroy). */
void hm_ctx_destroy(hm_ctx *ctx);

/* Build the cluster tree and block cluster tree for n locations s_i (Sect. 2.2,
 * App. B, Defs. B.1-B.3) and the theta-independent H-Cholesky schedule, and
 * upload them.  coords: n x d row-major, finite; d must be 2 (the paper's
 * spatial setting; other d return HM_ERR_ARG).  coords_on_device != 0: coords is
 * a device pointer on the context's device, read (copied) during the call. */
hm_status hm_dataset_create(hm_ctx *ctx, const double *coords, int64_t n, int32_t d, const hm_tree_opts *opts,
                            int32_t coords_on_device, hm_dataset **out);
/* Frees all of the dataset's device memory.  If a server runs on its context,
 * the server's queued requests on ds are cancelled and the call waits until
 * none of them is on the device. */
void hm_dataset_destroy(hm_dataset *ds);

/* Device memory of a dataset.  resident_bytes: trees, schedule, Z and the
 * small per-evaluation arrays, held from creation to destruction.
 * factor_bytes: the factor storage (dense leaves, low-rank factors U, V at
 * rank cap 64, update-term buffers) that the evaluations assemble C~ into and
 * factorise in place; *attached says whether it is currently allocated.  Any
 * pointer may be NULL. */
hm_status hm_dataset_footprint(const hm_dataset *ds, int64_t *resident_bytes, int64_t *factor_bytes,
                               int32_t *attached);

/* Frees the factor storage (the last matrix and factor are lost; hm_get_block
 * then returns HM_ERR_ARG).  The next evaluation allocates it again
 * (HM_ERR_OOM if that fails).  Lets many datasets stay resident with only the
 * factor storage of those being evaluated allocated. */
hm_status hm_dataset_release(hm_dataset *ds);

/* Data Z: n x r column-major in input (not permuted) order, 1 <= r <= 64.
 * on_device != 0: Z is a device pointer (on the context's device, n * r
 * doubles) read in stream order during this call.  A host Z must be finite.
 * On any error the dataset keeps its previous Z. */
hm_status hm_dataset_set_z(hm_dataset *ds, const double *Z, int32_t r, int32_t on_device);

/* Assemble C~(theta): Matern entries of the dense leaves, ACA + truncation of
 * the admissible blocks (Sect. 2.1, Remark 2.4). */
hm_status hm_assemble(hm_dataset *ds, const hm_theta *theta, const hm_approx *approx);

/* H-Cholesky of the assembled matrix, in place (Sect. 3.2).  Returns
 * HM_ERR_NOT_SPD on a non-positive pivot (the factor then holds NaNs).  On a
 * dataset with a stream program (hm_tune_schedule) the program also runs the
 * forward solve L~ v = Z of the current Z beside the factorisation. */
hm_status hm_factor(hm_dataset *ds);

/* Forward solve L~ v = Z, log-determinant and eq. (4) for every column of Z;
 * out has r entries.  If the last hm_factor already solved for the current Z
 * (and no hm_dataset_set_z, hm_assemble or earlier hm_solve came between),
 * only the sums remain; the results are bitwise the same either way. */
hm_status hm_solve(hm_dataset *ds, hm_result *out);

/* hm_assemble + hm_factor + hm_solve. out has r entries. */
hm_status hm_loglik(hm_dataset *ds, const hm_theta *theta, const hm_approx *approx, hm_result *out);

/* Schedule tuning (Z must be set): runs one evaluation at theta (assembly and
 * factorisation, with per-task timing), then rebuilds the factorisation's
 * levels from the timed durations: each level is led by the ready task with the
 * longest timed chain to the end, takes every ready task that would lengthen
 * the schedule if deferred, and every other ready task no longer than the
 * level already is; longer tasks run first within a level.  From the same
 * durations it builds a stream program that later factorisations run instead:
 * the big blocks' flush steps, the long low-rank flushes and the other tasks
 * (with the data's forward solve) on streams of their own, ordered by events.
 * Eight streams if the HIP runtime has at least 9 hardware queues, six from 7,
 * else four (GPU_MAX_HW_QUEUES, read when HIP initialises: streams sharing a
 * queue run one after the other); the environment variable HMLIK_STREAMS = 1,
 * 4, 6 or 8 overrides (1: the levels on the context's stream only).  Later
 * factorisations of the dataset, at any theta, use the new schedule; they run
 * the same tasks on the same inputs, so results are bitwise unchanged.
 * Returns the evaluation's status (on HM_ERR_NOT_SPD the schedule is left as
 * it was).  Allocates the timing records on first use. */
hm_status hm_tune_schedule(hm_dataset *ds, const hm_theta *theta, const hm_approx *approx);

/* Batched evaluation of eq. (4) (Monte-Carlo replicates, several theta on
 * copies of one dataset, or unrelated datasets): dataset ds[i] is evaluated at
 * theta[i] and approx[i], i < m.  Runs a request server (below) on ctx for
 * the duration of the call, with one batch slot per dataset (at most 16 at
 * once): each evaluation runs on a stream of its own with its share of the
 * workspace, so that the datasets fill work-groups one alone leaves idle.
 * Every dataset gets bitwise the results of hm_loglik alone.  out receives
 * sum_i r_i results, dataset by dataset (r_i = columns of its Z).  The
 * datasets must be distinct, belong to ctx and have Z set (else HM_ERR_ARG);
 * HM_ERR_BUSY if ctx already has a server.  Returns HM_ERR_NOT_SPD if any
 * factorisation broke down (the per-result status says which); the t_*
 * fields are each evaluation's own (overlapping) device times. */
hm_status hm_loglik_batch(hm_ctx *ctx, int32_t m, hm_dataset *const *ds, const hm_theta *theta,
                          const hm_approx *approx, hm_result *out);

/* Introspection: sizes of the trees and of the factorisation's task graph.
 * nlevels is the number of executor kernel launches per factorisation of the
 * schedule in use: the dependency levels of the graph (longest path, or as
 * rebuilt by hm_tune_schedule), or the launches of the stream program that
 * hm_tune_schedule builds (those overlap in time).  Any pointer may be
 * NULL (that value is not written). */
hm_status hm_dataset_info(const hm_dataset *ds, int64_t *n, int64_t *nclusters, int64_t *nblocks,
                          int64_t *ntasks, int64_t *nlevels);

/* Permutation (perm[i] = input index at permuted position i, n entries),
 * cluster ranges (2 per cluster: begin, end), boxes (4 per cluster: lo_x,
 * lo_y, hi_x, hi_y), in pre-order.  Any pointer may be NULL. */
hm_status hm_dataset_export_tree(const hm_dataset *ds, int64_t *perm, int64_t *ranges, double *boxes);

/* Blocks in pre-order: rc (4 per block: row begin, col begin, rows, cols) and
 * kind (0 internal, 1 dense leaf, 2 low-rank leaf).  Either pointer may be NULL. */
hm_status hm_dataset_export_blocks(const hm_dataset *ds, int64_t *rc, int8_t *kind);

/* Copy one leaf block of the current matrix / factor to host memory.
 * Dense leaf: data receives rows*cols doubles (column-major), *rank = -1.
 * Low-rank leaf: data receives U (rows x k) followed by V (cols x k), *rank = k;
 * data must hold (rows + cols) * 64 doubles. */
hm_status hm_get_block(hm_dataset *ds, int64_t block, double *data, int32_t *rank);

/* Algorithmic floating-point operations of the last hm_factor (dense leaf
 * Cholesky / triangular solves / update products, low-rank products, QR and
 * SVD recompressions, forward substitutions), counted by the device from the
 * actual sizes and ranks.  Used for roofline fractions. */
hm_status hm_factor_flops(hm_dataset *ds, double *flops);

/* Test hook: the update term `term` of the H-Cholesky schedule (in the order
 * the recursion records them): kind (0: X = U_A, Y = L_B V_A; 1: X = L_A V_B,
 * Y = U_B; 2: X = D_A, Y = D_B), the factor blocks A and B, and for kinds 0/1
 * the computed factor (rows x k, column-major) copied into data (may be NULL;
 * must hold rows * 64 doubles). */
hm_status hm_get_term(hm_dataset *ds, int64_t term, double *data, int32_t *kind, int64_t *A, int64_t *B,
                      int64_t *rows, int32_t *k);

/* Test hook for the truncation step (Remark 2.4): one work-group computes the
 * best approximation of X Y^T (X: m x r, Y: n x r, host, column-major,
 * 1 <= r <= 128) at relative accuracy eps (fixed_rank == 0) or rank
 * fixed_rank, through the same device routine the H-Cholesky uses.  U (m x 64)
 * and V (n x 64) receive the k = *k factors; seconds (4 entries, may be NULL)
 * the kernel time and its QR, SVD and back-transformation phases.  With
 * Y == NULL and r == 0, X is instead an explicit m x n matrix (n <= 256)
 * truncated by the routine of the explicit flush of small low-rank blocks
 * (pivoted QR, then one-sided Jacobi on R^T); the phases are then the pivoted
 * QR, the Jacobi iteration and the formation of U and V.  Uses the dataset's
 * workspace (HM_ERR_ARG if the matrices do not fit in one slot of it). */
hm_status hm_test_truncate(hm_dataset *ds, const double *X, int64_t m, const double *Y, int64_t n, int32_t r,
                           double eps, int32_t fixed_rank, double *U, double *V, int32_t *k, double *seconds);

/* ---------------------------------------------------------------- operators
 *
 * Products and solves with the last evaluation's factor L~ and matrix C~, for
 * simulating data (Sect. 4: Z = L~ W with W standard normal), the accuracy
 * diagnostics of Sect. 2.4 and the refinement of C~^{-1} Z (Sect. 3.1).
 * W and Y are n x r column-major (1 <= r <= 64) in input (not permuted)
 * order; the library applies the tree permutation P itself, so the operators
 * are those of the input ordering: with M the matrix in tree order, Y =
 * P^T M P W.  on_device != 0: W and Y are device pointers on the dataset's
 * device, else host pointers (a host W must be finite).  Each call waits for
 * its result.  Uses three n x 64 device buffers of the dataset, allocated on
 * the first call. */
typedef enum {
  HM_OP_L = 0,        /* Y = L~ W (requires a successful factorisation) */
  HM_OP_LT = 1,       /* Y = L~^T W */
  HM_OP_C = 2,        /* Y = C~ W with the assembled H-matrix (requires hm_dataset_keep_matrix
                         before the last assembly) */
  HM_OP_SOLVE = 3,    /* Y = (L~ L~^T)^{-1} W: forward, then backward substitution */
  HM_OP_C_EXACT = 4   /* Y = C(theta) W with the exact covariance of eq. (2) plus the nugget on
                         the diagonal, theta of the last assembly; n^2 entries formed on the fly */
} hm_operator;

/* keep != 0: every later assembly also copies C~ (its dense leaves, low-rank
 * factors and ranks, one device allocation of the size of the matrix
 * storage) for HM_OP_C; keep == 0 frees the copy. */
hm_status hm_dataset_keep_matrix(hm_dataset *ds, int32_t keep);

/* Y = op W (hm_operator).  HM_ERR_ARG when the operator's matrix is not
 * available (no successful factorisation, no kept copy, no assembly). */
hm_status hm_apply(hm_dataset *ds, int32_t op, const double *W, double *Y, int32_t r, int32_t on_device);

/* Simulated data (Sect. 4): assembles and factorises C~(theta) at accuracy
 * approx, then Z = L~ W for the caller's standard-normal W (n x r, input
 * order), so that Cov(Z) = C~(theta).  HM_ERR_NOT_SPD on a breakdown. */
hm_status hm_simulate(hm_dataset *ds, const hm_theta *theta, const hm_approx *approx, const double *W, double *Z,
                      int32_t r, int32_t on_device);

/* Accuracy of the factorisation (Sect. 2.4, Theorem 1's eps): *norm ~
 * ||I - (L~ L~^T)^{-1} C||_2 with C the exact covariance at the last theta, by
 * `iters` steps of the power iteration on A^T A, A = I - (L~ L~^T)^{-1} C,
 * from the start vector x0 (n entries, host, input order, not zero).  Each
 * step applies C twice (n^2 entries each) and solves with L~ L~^T twice. */
hm_status hm_inverse_accuracy(hm_dataset *ds, const double *x0, int32_t iters, double *norm);

/* Entries of the exact covariance C(theta) of eq. (2) plus the nugget on the
 * diagonal (Sect. 2.2, 2.4), at the theta of the last assembly, in input
 * order: out[a + b ldo] = C(i0 + a, j0 + b) for a < ni, b < nj (column-major,
 * ldo >= ni).  The reference side of the accuracy diagnostics of Sect. 2.4
 * (KLD and the error of log|C~| need C itself).  out is a host array, or a
 * device array on the context's GPU with on_device = 1 (checked).
 * HM_ERR_ARG for a range outside 0 .. n-1, ldo < ni, no assembly yet, or a
 * pointer of the wrong kind; HM_ERR_OOM if the index map or the host staging
 * buffer (ni nj doubles) cannot be allocated.  Allocates the index map (n
 * int64) on first use. */
hm_status hm_exact_block(hm_dataset *ds, int64_t i0, int64_t ni, int64_t j0, int64_t nj, double *out, int64_t ldo,
                         int32_t on_device);

/* Allocation-free truncation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the computation of hm_test_truncate -- the best approximation
 * of X Y^T (X: m x r, Y: n x r, 1 <= r <= 128), or of the explicit m x n
 * matrix X when Y == NULL and r == 0 (n <= 256), at relative accuracy eps
 * (fixed_rank == 0) or rank fixed_rank -- with every pointer a device
 * pointer on ctx's device: X, Y are read, U (m x 64) and V (n x 64) receive
 * the k factors (column-major, leading dimensions m and n) and *k (a device
 * int32) the rank.  The work is enqueued on ctx's stream and the call returns
 * without waiting; nothing is allocated or freed.  The workspace is one fixed
 * array per GPU of 4 Mi doubles (32 MiB, held until the process ends): a call
 * whose workspace (m + n) r + 2 (r + 1) r + 64 doubles, or m n + (n | 1)
 * min(m, n) + 64 in the explicit form, exceeds 4 Mi - 64 is refused with
 * HM_ERR_ARG before anything is enqueued.  Every
 * call on a GPU shares that array, so calls that overlap on one GPU (other
 * streams, other contexts, other threads) race and must be ordered by the
 * caller. */
hm_status hm_truncate_noalloc(hm_ctx *ctx, const double *X, int64_t m, const double *Y, int64_t n, int32_t r,
                              double eps, int32_t fixed_rank, double *U, double *V, int32_t *k);

/* ------------------------------------------------------------------ serving
 *
 * A request server evaluates eq. (4) (Sect. 3.1) for a stream of requests
 * (dataset, theta, accuracy), the calls a likelihood maximiser issues, on
 * resident datasets of one context, with continuous batching: every batch slot
 * has a HIP stream of its own (default priority) and its own share of the
 * context's work-group workspace, and an admitted request's assembly,
 * H-Cholesky levels and forward solve run on its slot's stream, so admitted
 * requests advance independently and their kernels overlap on the device.  A
 * worker thread feeds the streams (levels in chunks), retires finished
 * requests and admits queued ones as slots and memory free up; a request that
 * arrives while others run starts at once if a slot is free.  Each request
 * gets bitwise the result of hm_loglik alone.
 *
 * Admission, in arrival order, takes a request when a batch slot is free, no
 * other admitted request uses its dataset (requests on one dataset run in
 * arrival order), and its dataset's factor storage fits the HBM budget: the
 * factor storage attached over all datasets of the context, plus what the
 * request needs if its dataset has none attached, must stay within
 * hbm_budget bytes.  To make room, the server releases the factor storage of
 * datasets that no admitted request uses, least recently used first.  A
 * request that cannot get room waits, and so do the requests after it (no
 * later request overtakes a request held back for memory).
 *
 * Overlap needs one hardware queue per stream: the HIP runtime maps streams to
 * GPU_MAX_HW_QUEUES hardware queues (4 by default) and streams that share a
 * queue run one after the other.  With the context's stream counted, set
 * GPU_MAX_HW_QUEUES >= max_active + 1 in the environment before the process
 * first uses HIP (measured at n = 256k: four requests at once took 72-77 s each
 * with 8 queues, while two of them took 145 s with 4).
 */
typedef struct {
  int32_t max_active; /* batch slots (requests on the device at once), 1..16; each slot's
                         kernels use 512 / max_active work-groups at most */
  int64_t hbm_budget; /* bytes of attached factor storage over the context's datasets; 0 = no limit */
} hm_server_opts;

/* Per-request timing and batching record. */
typedef struct {
  double t_queue;      /* seconds from submission to admission (host clock) */
  double t_latency;    /* seconds from submission to the result being ready (host clock) */
  int32_t steps;       /* chunks of levels enqueued for the request's factorisation */
  int32_t peak_batch;  /* largest number of requests admitted at once while it was admitted */
} hm_request_stats;

/* Starts a server (worker thread, one stream per batch slot) on ctx.  The
 * context's datasets must already exist: dataset creation is refused while
 * the server runs.  HM_ERR_ARG if ctx has no dataset or the options are out of
 * range; HM_ERR_BUSY if ctx already has a server.  Allocates the slots' pinned
 * host records (ranks, breakdown record, solve output). */
hm_status hm_server_create(hm_ctx *ctx, const hm_server_opts *opts, hm_server **out);

/* Queues the evaluation of ds (with its current Z) at theta and approx;
 * *ticket identifies it.  HM_ERR_ARG for invalid theta/approx, a dataset of
 * another context or one without Z; HM_ERR_OOM if the dataset's factor storage
 * alone exceeds the budget; HM_ERR_DEVICE after a device failure of the
 * server.  Thread-safe. */
hm_status hm_server_submit(hm_server *sv, hm_dataset *ds, const hm_theta *theta, const hm_approx *approx,
                           uint64_t *ticket);

/* Result of a request.  wait != 0 blocks until it is ready.  When ready,
 * *done = 1, out receives r results (r = columns of the dataset's Z at
 * submission), stats (may be NULL) its record, the ticket is retired, and the
 * request's status is returned (HM_OK, HM_ERR_NOT_SPD, HM_ERR_CANCELLED,
 * HM_ERR_DEVICE, ...).  When not ready (wait == 0), *done = 0 and HM_OK.
 * HM_ERR_ARG for an unknown or retired ticket.  Thread-safe. */
hm_status hm_server_poll(hm_server *sv, uint64_t ticket, int32_t wait, hm_result *out, hm_request_stats *stats,
                         int32_t *done);

/* Cancels a request: a queued one at once, an admitted one at the end of its
 * chunk of levels in flight (one whose forward solve has started completes
 * normally).  Its poll then returns HM_ERR_CANCELLED.  HM_ERR_ARG for an unknown ticket, HM_OK (no
 * effect) if it already finished.  Thread-safe. */
hm_status hm_server_cancel(hm_server *sv, uint64_t ticket);

/* Cancels queued requests, lets admitted ones finish, joins the worker and
 * frees the server; the context's direct entry points work again.  Must not
 * overlap any other call on sv (unretired tickets become invalid). */
void hm_server_destroy(hm_server *sv);

const char *hm_status_string(hm_status s);

#ifdef __cplusplus
}
#endif
#endif /* HMLIK_H */
