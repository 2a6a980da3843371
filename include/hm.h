/* hm.h — C-ABI of the MI355X H-matrix LU library (libhm.so).
 *
 * Method: Boerm, Christophersen, Kriemann, "Semi-Automatic Task Graph
 * Construction for H-Matrix Arithmetic" (arXiv 1911.07531).
 *   build_htree  cluster tree (Def. 2.1) by geometric bisection and block tree
 *                (Def. 2.2) with standard admissibility (Sec. 5.1)
 *   h_assemble   H-matrix of Def. 2.3: dense inadmissible leaves, low-rank
 *                U V^T admissible leaves compressed to precision eps
 *   h_lu         H-LU of Algorithm 2 (with Algorithms 1 and 3 and the
 *                truncated low-rank addition of Sec. 2.3); the recursion is
 *                traced on the host into a task DAG (Sec. 3, Def. 3.1/3.2)
 *                and replayed on the GPU
 *   h_solve      forward/backward substitution through the factors, with
 *                optional iterative refinement against h_matvec (not in the
 *                paper: textbook block substitution)
 *   h_matvec     y = alpha A_H x + beta y over all leaves (not in the paper)
 *
 * Conventions
 *   - Every call returns hm_status: 0 on success, a negative code otherwise;
 *     hm_last_error() returns a thread-local message for the last failure.
 *   - Handles are opaque and owned by the library; release them with the
 *     matching *_free.  A tree must outlive every matrix and factor built on
 *     it; a matrix must outlive refinement calls that name it.
 *   - Vectors cross the boundary in the caller's original point ordering,
 *     FP64, column-major with a leading dimension.  Vector arguments are
 *     device pointers owned by the caller, and must stay valid until the
 *     work on `stream` has completed.
 *   - `stream` is a hipStream_t (NULL = default stream).  h_assemble, h_lu
 *     and h_solve synchronise the stream before returning (they report pivot,
 *     rank and executor status); h_matvec and h_solve_async are stream-ordered
 *     and asynchronous.
 *   - Device memory of handles comes from the allocator installed with
 *     hm_set_allocator, else hipMalloc/hipFree.
 *   - Nothing here falls back to the CPU: the compute entry points return
 *     HM_EDEVICE when no gfx950 device is usable.
 */
#ifndef HM_H_
#define HM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HM_OK = 0,
  HM_EINVAL = -1,     /* bad argument: n < 1, leaf < 1, eta <= 0, eps < 1e-8, null pointer, ... */
  HM_ENOMEM = -2,     /* host or device allocation failed */
  HM_ESINGULAR = -3,  /* exact zero pivot in a diagonal leaf; *info = permuted global row */
  HM_ENOCONV = -4,    /* refinement did not reach rtol within max_iter */
  HM_EDEVICE = -5,    /* HIP error, no usable device, or executor timeout */
  HM_ERANK = -6       /* with max_rank = 0: a truncation wanted more than the stored
                         rank capacity (64); the result is kept at rank 64 */
} hm_status;

typedef enum {
  HM_FP64 = 0,  /* every block FP64 */
  HM_MIXED = 1  /* FP32 off-diagonal blocks and products; FP64 diagonal leaves,
                   pivots, Gram/core SVD of truncations, residuals */
} hm_precision;

typedef enum {
  HM_LAPLACE3D = 0, /* a_ij = 1 / (4 pi |x_i - x_j|) */
  HM_LOG2D = 1      /* a_ij = -log |x_i - x_j| / (2 pi); with points on a line the
                       kernel of the one-dimensional model problem (Sec. 5.1)
                       up to the factor -1/(2 pi) */
} hm_kernel;

typedef enum {
  HM_EXEC_DATAFLOW = 0, /* one persistent launch; workgroups take ready tasks */
  HM_EXEC_LEVEL = 1     /* one launch per DAG level */
} hm_exec;

typedef struct {
  int leaf;         /* cluster leaf size (Def. 2.1 stop criterion |t| <= leaf) */
  double eta;       /* admissibility parameter, min diam <= eta * dist */
  double eps;       /* relative truncation accuracy (keep sigma_i > eps sigma_1,
                       Sec. 2.1 / 2.3); at least 1e-8: the truncation's FP64
                       Gram-matrix route resolves directions down to about
                       sqrt(u) of the largest, so smaller eps (and the exact
                       case eps = 0) is rejected with HM_EINVAL */
  int max_rank;     /* rank cap, 0 = none (then the capacity 64 bounds it) */
  int prec;         /* hm_precision */
  int exec;         /* hm_exec of the factorization; the substitution DAGs of
                       h_solve, a few tasks per level, always run on the
                       persistent executor with 64 workgroups */
  int lazy;         /* 0: truncate every update of a low-rank leaf when it is
                       produced, in the sequential order of Algorithm 1;
                       1: collect the updates of a low-rank leaf and add them
                       with a balanced tree of truncations when the leaf is
                       next read (the accumulator arithmetic of Sec. 2.3,
                       applied per leaf);
                       2: the accumulated H-LU of Algorithms 4-8: every block
                       carries an accumulator and pending products, shifted
                       to its sons at each recursion (shift_upd) and applied
                       before a leaf is factored, solved with or read
                       (apply_upd).  Other values: HM_EINVAL */
  int coarsen;      /* stop refining the substitution at diagonal blocks of at
                       most this many rows (the remark after Algorithm 11 on
                       stopping task refinement at a block size): each such
                       block's forward or backward substitution runs as one
                       task with the block's panel rows on chip, and the
                       product from the neighbouring block joins it; 0 = off
                       (leaf-level tasks), at most 1024, else HM_EINVAL.  The
                       H-LU's DAG is not coarsened. */
} hm_opts;

typedef struct hm_tree_s* hm_tree;
typedef struct hm_matrix_s* hm_matrix;
typedef struct hm_lu_s* hm_lu;

typedef struct {
  int64_t ntasks, nedges, nlevels;
  int64_t tasks_by_op[16]; /* tasks per task kind (index = task kind) */
  int64_t bytes_alg;   /* algorithmic bytes of the executed tasks (run-time ranks) */
  int64_t flops_alg;
  double exec_ms;      /* device time of the executor launch(es), HIP events */
  int64_t temp_bytes;  /* temporaries of the traced DAG */
  int64_t rank_overflows; /* truncations whose rank the cap (max_rank, else the
                             capacity 64) or min(m, n) bounded */
  double op_busy_ms[16];  /* summed workgroup-busy time per task kind (index = task kind) */
  double trunc_phase_ms[12]; /* truncation phases Gram, Cholesky, core, SVD, solve, rebuild:
                                [0..5] stacked rank <= 32, [6..11] larger */
  double trunc_mean_k, trunc_mean_mn; /* mean stacked rank K and mean m + n of truncations */
} hm_lu_stats;

/* Launch choices of the executors, set by the autotuner of the Python package
 * (paper_1911_07531_amd/autotune.py) from timed candidates, process-wide.
 *   exec_wg_per_cu  workgroups per compute unit of the H-LU executors (1 or
 *                   2; 0 = as many as fit, which is 2)
 *   solve_wg        workgroups of the persistent substitution executor
 *                   (default 64, or HM_SOLVE_NWG)
 *   batch_order     h_lu_batched queue order of the instances' first tasks:
 *                   0 as given, 1 the instances with the most tasks first */
typedef struct {
  int exec_wg_per_cu;
  int solve_wg;
  int batch_order;
  int reserved[5];
} hm_tuning;
hm_status hm_get_tuning(hm_tuning* out);
hm_status hm_set_tuning(const hm_tuning* t); /* HM_EINVAL when a field is out of range */

/* Device allocator hook; ctx is passed back.  Both may be NULL to restore
 * hipMalloc/hipFree. */
hm_status hm_set_allocator(void* (*alloc)(size_t bytes, void* stream, void* ctx),
                           void (*dealloc)(void* ptr, size_t bytes, void* stream, void* ctx), void* ctx);

/* Cluster tree + block tree (host only, no device needed).
 * pts_host: n x dim, row-major, FP64, caller-owned (copied).  dim in {1, 2, 3};
 * points are embedded in R^3 with zero trailing coordinates (the kernels of
 * h_assemble see the 3D distance).  Uses opts->leaf and opts->eta. */
hm_status build_htree(const double* pts_host, int64_t n, int dim, const hm_opts* opts, hm_tree* out);

/* Tree tables (host): sizes, then copies.  Any output pointer may be NULL.
 * clusters: ncl x 5 int64 (begin, end, son0, son1, level), boxes ncl x 6
 * (lo[3], hi[3]); blocks: nbl x 7 int32 (tau, sigma, kind 0 struct / 1 dense
 * / 2 low-rank, son00, son01, son10, son11); perm: n int64, perm[k] =
 * original index of permuted index k.  Both tables are depth-first pre-order. */
hm_status hm_tree_sizes(hm_tree t, int64_t* n, int64_t* nclusters, int64_t* nblocks);
hm_status hm_tree_export(hm_tree t, int64_t* perm, int64_t* clusters, double* boxes, int32_t* blocks);

/* Assemble the H-matrix of Def. 2.3 on the device: dense leaves hold the
 * kernel entries (a_ii = diag), admissible leaves the adaptive cross
 * approximation recompressed to eps (opts->eps, opts->max_rank).  The matrix
 * is stored in FP64.  Synchronises `stream`. */
hm_status h_assemble(hm_tree t, int kernel, double diag, const hm_opts* opts, void* stream, hm_matrix* out);

/* H-LU (Algorithm 2) of A into new factors; A is not modified.  Uses
 * opts->eps, max_rank, prec, exec.  On HM_ESINGULAR, *info (may be NULL) is the
 * permuted global row of the first exact zero pivot; the factors are invalid.
 * Synchronises `stream`. */
hm_status h_lu(hm_matrix A, const hm_opts* opts, void* stream, hm_lu* out, int64_t* info);

/* H-LU and substitution as one task DAG (the fusion of composed operations
 * that the semi-automatic construction allows, Sec. 6; cf. the merged DAGs of
 * Sec. 4.3): the H-LU of A (Algorithm 2) and the forward/backward substitution of the first
 * min(nrhs, 64) columns of B are traced into one DAG and run by one persistent
 * launch, so that a block row's substitution starts as soon as its factors
 * are final; further columns are solved after it as by h_solve without
 * refinement.  B: device, n x nrhs, column-major, ldb >= n, overwritten by
 * the solution.  The factors equal those of h_lu (task for task the same
 * H-LU); *out and *info as for h_lu (on failure B is unspecified).  opts->exec
 * is ignored (always the persistent executor).  Synchronises `stream`. */
hm_status h_lu_solve(hm_matrix A, const hm_opts* opts, double* B, int64_t ldb, int64_t nrhs, void* stream, hm_lu* out,
                     int64_t* info);

/* H-LU (Algorithm 2) of `count` independent H-matrices (each on its own tree,
 * of any size, geometry and leaf size) as one task DAG on one launch: each
 * matrix's traced DAG (Sec. 3) is relocated into one factor arena and the
 * union runs on the persistent executor (opts->exec = HM_EXEC_DATAFLOW) or
 * one launch per DAG level across all matrices (HM_EXEC_LEVEL), so that
 * small and large factorizations fill the GPU together.  opts (eps, max_rank,
 * prec, lazy) apply to every matrix; each A_i must have been assembled with
 * opts->max_rank.  outs: count handles, each as from h_lu (their factors
 * share one device allocation, released with the last of them; the same
 * factors as h_lu of that matrix alone).  infos (may be NULL): count int64,
 * all 0; on HM_ESINGULAR the permuted row of the first exact zero pivot at
 * the instance that has it and -1 at every other (all outs NULL then).  The temporaries of the batch
 * span HM_BATCH_TEMP_GB GiB (default 16) shared in proportion to n.
 * hm_lu_stats of every handle describe the whole batch launch.
 * Synchronises `stream`. */
hm_status h_lu_batched(const hm_matrix* As, int count, const hm_opts* opts, void* stream, hm_lu* outs,
                       int64_t* infos);

/* The combined DAG of h_lu_batched over `count` trees (host only, for
 * inspection and tests; the plans are traced as h_lu_batched traces them).
 * sizes (7 int64): ntasks, nedges, nlevels, FP64 / FP32 / pivot arena
 * elements, rank slots.  Any other output may be NULL: tasks (ntasks
 * records), succ_ptr (ntasks + 1), succ_idx (nedges), order (ntasks, level
 * order), level_ptr (nlevels + 1), lr (rank slots x 6 int64: u_off, v_off,
 * m, n, cap, type; zeros at the slots of a solve's column count), bases
 * (count x 8 int64: FP64, FP32 and pivot arena bases, first rank slot,
 * first row, first task, first edge, tasks of the instance). */
hm_status hm_batch_dag_export(const hm_tree* trees, int count, const hm_opts* opts, int64_t* sizes, void* tasks,
                              int32_t* succ_ptr, int32_t* succ_idx, int32_t* order, int32_t* level_ptr, int64_t* lr,
                              int64_t* bases);

/* Solve A X = B in place through the factors: forward and backward block
 * substitution (not in the paper; the textbook substitution through L and U
 * of Sec. 2.2's A = LU, with the leaf pivots applied per diagonal leaf).
 * A diagonal leaf's triangles are applied through their inverses, computed
 * once per factorization right after the leaf's getrf; with opts->coarsen
 * of the factorization, each diagonal block of at most that many rows is
 * substituted by one task (the remark after Algorithm 11).
 * B: device, n x nrhs, column-major, leading dimension ldb >= n, caller-owned.
 * With A_or_null != NULL the solution is refined with r = b - A_H x (FP64
 * h_matvec) until every column has ||r|| / ||b|| <= rtol or max_iter
 * corrections were applied (then HM_ENOCONV, X still the last iterate).
 * iters_host (ceil(nrhs / 64) ints: corrections per group of 64 columns) and
 * relres_host (nrhs doubles: final relative residuals, NaN where no
 * refinement ran) may be NULL.  A column's result does not depend on the
 * other columns of the call beyond rounding: the substitution's FP64
 * reductions are grouped by the number of columns, so a column solved alone
 * and in a wider call agree to about 1e-15 relative, not always bit for bit.  Synchronises `stream`; HM_EDEVICE if the
 * substitution executor gave up (X is then unspecified).  Allocates the
 * refinement vectors on the first refined call and keeps them with F. */
hm_status h_solve(hm_lu F, hm_matrix A_or_null, double* B, int64_t ldb, int64_t nrhs, double rtol, int max_iter,
                  void* stream, int* iters_host, double* relres_host);

/* The substitution of h_solve without refinement, stream-ordered and
 * asynchronous (for a serving loop that keeps factors resident and overlaps
 * requests): returns once the work is queued on `stream`; when it completes,
 * *status_dev (a device-accessible int32 owned by the caller) holds HM_OK or
 * HM_EDEVICE (the executor gave up; B unspecified).  Argument errors are
 * returned directly.  Calls on one F share its substitution workspace and
 * must be ordered (one stream per F); calls on different factors may overlap. */
hm_status h_solve_async(hm_lu F, double* B, int64_t ldb, int64_t nrhs, void* stream, int32_t* status_dev);

/* h_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments and results, but the refinement vectors live in a fixed
 * 32 MiB device array of the library (one per GPU, held until the process
 * ends) instead of memory allocated on the first call, and nothing is
 * allocated.  Refinement runs on chunks of cw columns, the largest cw <= 64
 * with (2 n cw + 4 cw) doubles <= 32 MiB; HM_EINVAL when even one column does
 * not fit (n > ~2.1 million).  iters_host (may be NULL) receives one int: the
 * largest number of corrections of any chunk.  Every call on a GPU shares that
 * GPU's array: calls that overlap on one GPU (other streams, other threads)
 * race and must be serialised by the caller.  Synchronises `stream`. */
hm_status h_solve_noalloc(hm_lu F, hm_matrix A_or_null, double* B, int64_t ldb, int64_t nrhs, double rtol,
                          int max_iter, void* stream, int* iters_host, double* relres_host);

/* Y = alpha A_H X + beta Y; X, Y device, n x nrhs column-major. */
hm_status h_matvec(hm_matrix A, double alpha, const double* X, int64_t ldx, double beta, double* Y, int64_t ldy,
                   int64_t nrhs, void* stream);

/* Device bytes held by a handle: kind 0 matrix, 1 factors, 2 factor workspace
 * (temporaries, scratch and DAG). */
hm_status hm_footprint(const void* handle, int kind, size_t* bytes);

/* An H-matrix from host leaf data on the block structure of t (parity hook,
 * the inverse of hm_export_leaf kind 0): the matrix any outside assembly (for
 * example an FP64 reference's truncated SVDs) produced, factored and applied
 * by the device path as one assembled by h_assemble.  ranks: one int32 per
 * block of hm_tree_export's table (read at low-rank leaves: their rank k;
 * ignored elsewhere).  data (FP64, host, caller-owned, copied): the leaves in
 * block-table order, a dense leaf as its m x n entries, a low-rank leaf as U
 * (m x k) then V (n x k), all column-major; ndata = the total count.  Uses
 * opts->max_rank (rank capacity; a larger k gives HM_ERANK) and eps (kept
 * with the matrix).  HM_EINVAL when ndata does not match.  Synchronises
 * `stream`. */
hm_status hm_import(hm_tree t, const hm_opts* opts, const int32_t* ranks, const double* data, int64_t ndata,
                    void* stream, hm_matrix* out);

/* Copy one leaf block to the host in FP64 (parity hook).  kind 0: matrix,
 * 1: factors.  Dense leaf: data (m x n column-major), *rank = -1.  Low-rank
 * leaf: data = U (m x rank) then V (n x rank), column-major, *rank = rank
 * (call with data = NULL first to learn the rank).  Diagonal leaves of
 * factors also fill piv (m int32, LAPACK interchanges, 0-based) if non-NULL. */
hm_status hm_export_leaf(const void* handle, int kind, int64_t block, double* data, int32_t* rank, int32_t* piv);

/* Per-task timeline of the last h_lu on F, recorded only when the
 * environment variable HM_DEBUG_TRACE=1 was set before h_lu: out (may be
 * NULL to query sizes) receives ntasks x 8 uint64 (start tick, end tick,
 * info, info2, three words of truncation-phase ticks, the tick at which the
 * dataflow executor queued the task (0 for the first tasks)) in trace order;
 * ticks count at clock_khz kHz.  info bits 0-15
 * hold the workgroup; for truncations bits 16-31 the width of the added
 * terms and bits 32-47 / 48-63 the rows m / columns n of the low-rank leaf,
 * and info2 the route (bits 0-7: 1 small-rank, 2 / 3 dense / Gram with a
 * QR-reduced core SVD, 4 / 5 dense / Gram with a full core SVD), the SVD
 * operand's rows p and columns q (bits 8-19, 20-31), the Jacobi sweeps
 * (32-39) and the new rank (40-47).  Words 4-6 hold the ticks of the six
 * truncation phases (Gram, factor, core, SVD, solve, rebuild), two 32-bit
 * counts per word, low half first. */
hm_status hm_lu_trace(hm_lu F, uint64_t* out, int64_t* ntasks, int64_t* clock_khz);

/* The timeline of the last substitution pass of h_solve on F (recorded when
 * HM_DEBUG_TRACE=1 was set before h_lu), one record of 8 words per task of
 * the substitution DAG, laid out as in hm_lu_trace.  For a coarsened block
 * (task kind 12) info's bits 48-63 hold its micro-operation count and words
 * 4-6 the ticks of its triangular solves and dense products, of its low-rank
 * products and panel copies, and the counts of its triangular solves and
 * products (two 32-bit counts per word, low half first). */
hm_status hm_solve_trace(hm_lu F, uint64_t* out, int64_t* ntasks, int64_t* clock_khz);

/* Statistics of the last h_lu on F. */
hm_status hm_lu_stats_get(hm_lu F, hm_lu_stats* out);

/* The traced DAG without a device (host only), for inspection and tests.
 * which: 0 = H-LU, 1 = solve, 2 = H-LU + solve (the DAG of h_lu_solve).  sizes: ntasks, nedges, nlevels, task_bytes
 * (sizeof one task record), n_f64, n_f32, n_piv (arena sizes in elements),
 * nlr (low-rank leaves), nranks.  hm_dag_export copies (any pointer may be
 * NULL): tasks (ntasks records), succ_ptr (ntasks + 1), succ_idx (nedges),
 * level (ntasks), block_off (nblocks x 4 int64: data offset, data type,
 * low-rank index, pivot offset; -1 where absent), lr (nlr x 6 int64: u_off,
 * v_off, m, n, cap, type). */
hm_status hm_dag_sizes(hm_tree t, const hm_opts* opts, int which, int64_t* sizes);
hm_status hm_dag_export(hm_tree t, const hm_opts* opts, int which, void* tasks, int32_t* succ_ptr, int32_t* succ_idx,
                        int32_t* level, int64_t* block_off, int64_t* lr);

/* The micro-operations of the coarsened substitution blocks of a traced DAG
 * (host only; opts->coarsen > 0, which = 1): *nseq records of task_bytes each,
 * copied to seq when it is not NULL.  An OP_SEQ task runs records
 * [piv, piv + lr) in order; views flagged block-local address the block's
 * rows of the panel relative to its first row. */
hm_status hm_dag_seq_export(hm_tree t, const hm_opts* opts, int which, int64_t* nseq, void* seq);

/* The paper-level leaf call of every traced task (host only): ncalls calls of
 * 4 int32 each (kind 0 hlu, 1 htrsl, 2 htrsu, 3 hmul; then the blocks: hlu
 * (d, d, d), htrsl (L, M, M), htrsu (U, M, M), hmul (A, B, C), block indices
 * of hm_tree_export), and task_call (ntasks int32, the call of each task, -1
 * outside any call).  which as for hm_dag_sizes.  Any output may be NULL. */
hm_status hm_dag_calls(hm_tree t, const hm_opts* opts, int which, int64_t* ncalls, int32_t* calls, int32_t* task_call);

/* The H-LU task graph by the paper's semi-automatic construction (host only):
 * task refinement from the single task hlu(A, L, U) with inherited and refined
 * dependencies of Definition 3.2 (Sec. 3, Algorithms 9-11), and with
 * sparsify != 0 the removal of redundant edges after every refinement step
 * (Sec. 4.1, Algorithm 12, paths of at most max_path edges, 0 = unbounded).
 * tasks: ntasks x 4 int32 as in hm_dag_calls; edges: nedges x 2 int32 (task
 * indices, predecessor first).  Call with NULL arrays to learn the sizes
 * (each call recomputes the graph). */
hm_status hm_semiauto_dag(hm_tree t, int sparsify, int max_path, int64_t* ntasks, int64_t* nedges, int32_t* tasks,
                          int32_t* edges);

void hm_tree_free(hm_tree t);
void hm_matrix_free(hm_matrix A);
void hm_lu_free(hm_lu F);
const char* hm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HM_H_ */
