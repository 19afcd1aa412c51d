/* C ABI of the MI355X adaptive H2-matrix product.
 *
 * Problem (Section 3 of the paper): given H2-matrices X (row tree T_I, column
 * tree T_J) and Y (row tree T_J, column tree T_K) sharing the middle cluster
 * tree, approximate Z = X Y by an H2-matrix on the block tree T_{IxK} built by
 * the admissibility condition, with isometric nested row and column bases
 * (Section 5.2) chosen adaptively so that every admissible block b satisfies
 * ||(XY)|_b - C|_b||_2 <= eps ||(XY)|_b||_2 (Section 5.3, block-relative error
 * control).  Inadmissible blocks are the exact product up to FP64 rounding
 * (with the FP32 bulk: up to the FP32 rounding of the exact product).
 *
 * Conventions
 *  - Every call returns h2_status; no exception crosses the ABI.  On failure
 *    output handles are set to NULL, nothing partial is returned, and
 *    h2_last_error() gives a message for the calling thread.
 *  - Host arrays passed in are copied during the call; the caller keeps them.
 *    Handles are created by the library and released by the caller with the
 *    matching *_destroy call.  Output buffers are caller-allocated.
 *  - Matrices are row-major.  Index sets of dense outputs are in the ORIGINAL
 *    point order (not the tree's permuted order).
 *  - Device memory and the HIP stream belong to the context; all device work
 *    of a call is ordered on that stream and completed before the call
 *    returns.
 */
#ifndef H2_H
#define H2_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  H2_OK = 0,
  H2_ERR_INVALID_ARG = 1,   /* null/invalid pointer, size, eps not in (0,1), non-finite input */
  H2_ERR_OUT_OF_MEMORY = 2, /* device or host allocation failed */
  H2_ERR_DEVICE = 3,        /* HIP error (message holds the HIP string) */
  H2_ERR_INCOMPATIBLE = 4,  /* X's column tree is not Y's row tree */
  H2_ERR_TOO_LARGE = 5,     /* size above a documented limit (rank cap, dense size) */
  H2_ERR_NOT_CONVERGED = 6  /* a Jacobi SVD of a truncation still rotated after its sweep cap */
} h2_status;

typedef struct h2_context_s* h2_context;
typedef struct h2_tree_s* h2_tree;
typedef struct h2_matrix_s* h2_matrix;
typedef struct h2_job_s* h2_job;

/* Context on HIP device `device` with its own stream. */
h2_status h2_context_create(int device, h2_context* out);
void h2_context_destroy(h2_context ctx);
/* Message of the calling thread's last failure ("" if none).  Valid until the
 * thread's next library call. */
const char* h2_last_error(void);

/* Cluster tree (Definition 1) of n points (row-major n x dim, dim 1..3) by
 * geometric bisection: a cluster with more than leaf_size points is split
 * along the longest edge of its bounding box at the midpoint (first axis on
 * ties; points below the midpoint go to the first child; if one side would be
 * empty, the cluster is halved by a stable sort along that axis).
 * Errors: INVALID_ARG for n < 1, dim outside 1..3, leaf_size < 1, non-finite
 * coordinates. */
h2_status h2_build_cluster_tree(h2_context ctx, const double* points, int64_t n, int dim, int leaf_size,
                                h2_tree* out);
/* perm[k] = original index of the k-th point in tree order (n entries). */
h2_status h2_tree_permutation(h2_tree tree, int64_t* perm);
/* Sizes: n, number of clusters, depth (levels), number of leaves. */
h2_status h2_tree_info(h2_tree tree, int64_t* n, int* nclusters, int* depth, int* nleaves);
/* Cluster arrays (nclusters entries each, any may be NULL): first/one-past-last
 * position in tree order, parent (-1 at the root), level. */
h2_status h2_tree_clusters(h2_tree tree, int64_t* begin, int64_t* end, int* parent, int* level);
void h2_tree_destroy(h2_tree tree);

typedef enum {
  H2_KERNEL_NEG_LOG = 0,   /* -log|x-y|                                  */
  H2_KERNEL_LAPLACE_SLP = 1, /* 1/(4 pi |x-y|)                           */
  H2_KERNEL_LAPLACE_DLP = 2  /* (x-y).n_y / (4 pi |x-y|^3), normals given */
} h2_kernel;

typedef enum {
  H2_DIAG_ZERO = 0,              /* g(x,x) = 0                                       */
  H2_DIAG_ROW_NEARFIELD_MEAN = 1 /* mean of the row's other nearfield kernel values  */
} h2_diag_rule;

/* H2-matrix of the point-collocation kernel matrix g(x_i, y_j) by tensor
 * Chebyshev interpolation of order `order` per axis (rank k = order^dim) on the
 * clusters' bounding boxes (eq. interpolation/vsw, transfers eq. transfer).
 * Block tree by the admissibility condition max(diam) <= 2 eta dist.
 * Double layer: normals (host, n x 3, unit) for the column points; the column
 * basis holds normal derivatives of the Lagrange polynomials.
 * Errors: INVALID_ARG (order < 1, order^dim > 64, eta <= 0, DLP without normals
 * or dim != 3, non-finite normals), OUT_OF_MEMORY, DEVICE. */
h2_status h2_build_interpolated(h2_context ctx, h2_tree rows, h2_tree cols, int kernel, const double* normals,
                                int order, double eta, int diag, h2_matrix* out);

typedef enum { H2_PREC_FP64 = 0, H2_PREC_FP32_BULK = 1 } h2_precision;

typedef struct {
  int precision;       /* h2_precision; FP32 bulk is used only for eps >= 1e-5, tighter
                          eps runs the bulk in FP64.  A product whose FP32 bulk exceeds
                          a rank cap (rounding noise kept as rank where the product
                          cancels) is recomputed in FP64, and later products of the
                          same pair at that eps or tighter use FP64 directly.
                          stats.prec_used tells which ran.                              */
  double theta;        /* weight base, 0 => 1/(2*sigma), sigma = max children (= 2)   */
  double budget_coarse;/* fractions of eps for coarsening, rows, columns; 0 => 1/4 */
  double budget_row;
  double budget_col;
  int max_rank;        /* rank cap of the result bases (<= 64; 0 => default)          */
  int coarse_rank;     /* rank cap of a coarsened block (<= 64; 0 => default 64)       */
  int timing;          /* 1: per-phase device times; 2: also device times of every kernel
                          launch (events around each); 3: as 2, plus the algorithmic work of
                          every kernel from the sizes the kernels report (one extra
                          device-to-host copy after the product)                         */
  int graph;           /* 1: run the product's launches as a HIP graph, captured at the
                          first such call for the plan and replayed afterwards (fewer
                          launch gaps for small products); needs timing = 0. 0: launch
                          every kernel from the host.                                    */
  int jacobi_sweeps;   /* sweep cap of the one-sided Jacobi SVDs (0 => 40).  A truncation
                          whose Jacobi still rotates after the cap makes the product fail
                          with H2_ERR_NOT_CONVERGED instead of returning vectors that are
                          not singular vectors.                                          */
  int chunks;          /* 0: automatic.  The exact product and the coarsening run in this
                          many chunks of result-block subtrees, one after the other, so
                          that a chunk's workspace is reused by the next (same arithmetic,
                          more launches).  Automatic: one chunk while the plan's
                          workspace fits the device, else 4, 16, ... chunks.            */
} h2_mul_options;

/* Number of kernels in the per-kernel statistics; h2_kernel_name(i) names kernel i. */
#define H2_NKERNEL 13

typedef struct {
  double t_phase[8];   /* device ms: 0 operand prep, 1 exact product, 2 leaf assembly,
                          3 coarsening, 4 row and column bases (built together, level by
                          level), 5 reserved (0), 6 couplings, 7 total                   */
  double t_plan_ms;    /* host planning time of this call (0 when the plan was cached)   */
  double bytes_alg;    /* algorithmic bytes of the product from the planned sizes          */
  double flops_alg;    /* algorithmic flops of the product from the planned sizes          */
  int prec_used;       /* h2_precision actually used for the bulk                        */
  int rank_max_row, rank_max_col, coarse_rank_max;
  int64_t n_adm, n_inadm;
  int64_t launches;    /* kernel launches of the product                                  */
  /* per kernel i < H2_NKERNEL:
     t_kernel        device ms summed over the kernel's launches (timing >= 2)
     launches_kernel launches of the kernel
     units_kernel    matrices (tasks) the kernel processed (timing == 3)
     flops_kernel    algorithmic flops: QR 2mw^2 - 2w^3/3 of each factored m x w
                     matrix (2wm^2 - 2m^3/3 when m < w), SVD the pivoted QR steps and
                     Jacobi rotations it ran, GEMM 2mnk with the m, n and summed inner
                     dimension k that each task reports from the device (timing == 3)
     bytes_kernel    algorithmic bytes: each input read once, each output written
                     once, with the same device-side sizes (timing == 3)               */
  double t_kernel[H2_NKERNEL];
  int64_t launches_kernel[H2_NKERNEL];
  double units_kernel[H2_NKERNEL];
  double flops_kernel[H2_NKERNEL];
  double bytes_kernel[H2_NKERNEL];
} h2_mul_stats;

/* Default options (all fields as documented above).  h2_mul and h2_mul_submit
 * reject (INVALID_ARG) a budget that is negative or not finite, resolved
 * budgets (0 => 1/4) summing above 1, theta outside [0, 1/sigma), a negative
 * jacobi_sweeps. */
void h2_mul_default_options(h2_mul_options* opt);

/* Name of kernel i of the per-kernel statistics (the kernel's template
 * instantiation as a profiler lists it); "" for i out of range.  The string
 * is static. */
const char* h2_kernel_name(int i);

/* C = X Y with the block-relative bound eps (0 < eps < 1), see the header
 * comment.  X and Y are read-only and stay resident.  The product plan
 * (integer work lists) is cached on the pair (X, Y) and reused.
 * Errors: INVALID_ARG, INCOMPATIBLE (X's column tree differs from Y's row
 * tree), TOO_LARGE (a rank cap was exceeded: raise max_rank / coarse_rank, or
 * an operand rank above 64), OUT_OF_MEMORY, DEVICE. */
h2_status h2_mul(h2_context ctx, h2_matrix X, h2_matrix Y, double eps, const h2_mul_options* opt,
                 h2_matrix* C, h2_mul_stats* stats);

/* Dense matrix (rows x cols, row-major, leading dimension ld >= cols, original
 * index order) of an H2-matrix as Definition 4 defines it: V_t S_b W_s^* on
 * every admissible leaf b = (t,s) (V_t, W_s expanded from the leaf bases and
 * transfer matrices) and the stored nearfield block on every inadmissible
 * leaf.  For small cases only: rows*cols <= 2^26, else TOO_LARGE. */
h2_status h2_to_dense(h2_matrix M, double* out, int64_t ld);

/* One leaf block of M as dense: block index b in [0, n_adm + n_inadm) (first
 * the admissible leaves, then the inadmissible ones, in the order of
 * h2_matrix_blocks).  out: |t| x |s| row-major in tree order. */
h2_status h2_block_dense(h2_matrix M, int64_t b, double* out);

/* Asynchronous products (batched and served products: many independent
 * h2_mul calls whose device work overlaps). A context has `nlanes` lanes
 * (1..8, default 4 at the first submit); a lane is a stream of its own plus
 * two for the size classes of its QR/SVD steps. h2_mul_submit plans the
 * product if its plan is not cached (host, synchronous), enqueues it and the
 * copies of its result on a lane and returns: on the plan's lane while
 * earlier jobs of that plan (same operand pair and precision) are in flight,
 * since a plan's workspace admits one product at a time, else on the least
 * loaded lane. At most 64 jobs may be in flight per lane (TOO_LARGE).
 * X and Y must stay alive until the job is waited for or destroyed.
 * h2_job_poll sets *done = 1 once the job's device work has finished.
 * h2_job_wait blocks until then and returns the result and stats, as h2_mul
 * would (per-kernel timing is not recorded on this path); a rank-cap overflow
 * is resolved by the synchronous h2_mul path. Waiting twice is INVALID_ARG.
 * h2_job_destroy releases a job (waiting for its device work first). The
 * result of a job is the same, bit for bit, as that of h2_mul with the same
 * arguments. Not thread-safe: one host thread per context. */
h2_status h2_context_set_lanes(h2_context ctx, int nlanes);
/* Device memory admission (h2_mul and h2_mul_submit).  Before a product
 * allocates anything, the library adds up what it still needs (a larger
 * workspace arena for its lane, its launch descriptors if not uploaded yet,
 * its result arrays) and compares it with what can be given: free device
 * memory, the arena it replaces and the arenas of idle lanes.  If that is
 * not enough, cached product plans without jobs are dropped, least recently
 * used first (their descriptors are freed; such a plan is built again when
 * its operands are multiplied again), but only when dropping them all would
 * make room; otherwise the product fails with H2_ERR_OUT_OF_MEMORY and
 * nothing is allocated or dropped.  h2_context_set_memory_limit(ctx, bytes)
 * makes the admission treat the device as holding at most `bytes` (memory in
 * use by anyone counts against it; 0 = the whole device), e.g. to leave room
 * for other work on the GPU; it also bounds the workspace budget of new
 * plans (chunking).  It does not restrict allocations outside products. */
h2_status h2_context_set_memory_limit(h2_context ctx, uint64_t bytes);
h2_status h2_mul_submit(h2_context ctx, h2_matrix X, h2_matrix Y, double eps, const h2_mul_options* opts,
                        h2_job* job);
h2_status h2_job_poll(h2_job job, int* done);
h2_status h2_job_wait(h2_job job, h2_matrix* C, h2_mul_stats* stats);
void h2_job_destroy(h2_job job);

/* Leaves of the block tree of (rows, cols) with admissibility parameter eta
 * (the condition max(diam) <= 2 eta dist of Section 2, the tree of every
 * matrix built here): *n_adm admissible and *n_inadm inadmissible leaves.
 * If pairs is not NULL it receives 2 (n_adm + n_inadm) ints, the cluster
 * pairs (t, s), admissible leaves first: the order h2_recompress expects.
 * Call with pairs = NULL to learn the sizes. */
h2_status h2_block_tree_leaves(h2_tree rows, h2_tree cols, double eta, int64_t* n_adm, int64_t* n_inadm,
                               int* pairs);

/* H -> H2 recompression with block-relative error (the second half of the
 * method, Section 5, on its own): an H-matrix G on the block tree of (rows,
 * cols, eta) becomes an H2-matrix C with adaptively chosen row and column
 * bases and ||G|_b - C|_b||_2 <= eps ||G|_b||_2 on every admissible leaf b
 * (the same error split as h2_mul: truncation of each block, row basis,
 * column basis); the nearfield is copied.
 *   ranks[i], U, Z: admissible leaf i (order of h2_block_tree_leaves) is
 *     G_i = U_i Z_i^T with U_i |t| x k_i and Z_i |s| x k_i, k_i = ranks[i] in
 *     [1, 128] (a zero block: rank 1, zero factors); the U_i are packed one
 *     after the other in leaf order, row-major, rows in tree order (cluster
 *     t covers positions begin(t) .. end(t)-1 of h2_tree_permutation), and
 *     the Z_i likewise.
 *   near: the inadmissible leaves' dense |t| x |s| blocks, row-major, packed
 *     in leaf order.
 * Host arrays, read during the call. opts: max_rank, coarse_rank (truncated
 * block rank cap), theta, budgets and timing as for h2_mul; precision is
 * FP64. Errors: INVALID_ARG (ranks, eps, non-finite input), TOO_LARGE (a
 * rank cap), OUT_OF_MEMORY. Synchronous. */
h2_status h2_recompress(h2_context ctx, h2_tree rows, h2_tree cols, double eta, const int* ranks, const double* U,
                        const double* Z, const double* near, double eps, const h2_mul_options* opts, h2_matrix* C,
                        h2_mul_stats* stats);

/* Matrix-vector product with an H2-matrix (Section 2: O(nk) operations with
 * the nested bases): y = M x (trans = 0) or y = M^T x (trans = 1) for nrhs
 * vectors at once.  x holds cols(M) x nrhs (rows(M) x nrhs when trans) and y
 * the other side, host memory, row-major (vector j is column j), original
 * point order.  Runs on the device with a cached plan per (M, trans, nrhs);
 * synchronous.  nrhs >= 1, else INVALID_ARG. */
h2_status h2_matvec(h2_matrix M, int trans, int64_t nrhs, const double* x, double* y);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): h2_matvec
 * with no device allocation at all.  Same arguments, errors and result as
 * h2_matvec (bit for bit: the same kernels on the same launch descriptors).
 * Every device buffer of the call (input and output vectors in tree order,
 * the coefficient vectors of the nested bases, the launch descriptors) lives
 * in one library-owned device array of H2_MATVEC_SCRATCH_BYTES per GPU,
 * created when the library is loaded on that GPU and held until the process
 * ends; its address is looked up by h2_context_create.  A call that needs
 * more (8 (n_rows + n_cols) nrhs + 8 (ncl_rows + ncl_cols) kc nrhs bytes plus
 * the descriptors, which grow with the number of blocks) fails with
 * H2_ERR_TOO_LARGE before any device work.  The array keeps the last call's
 * contents; nothing in it needs to start at zero.  All calls on one GPU share
 * it (every context, every host thread): calls that overlap on one GPU race,
 * so the caller serialises them.  Synchronous. */
#define H2_MATVEC_SCRATCH_BYTES (32u * 1024u * 1024u)
h2_status h2_matvec_noalloc(h2_matrix M, int trans, int64_t nrhs, const double* x, double* y);

/* Global error of a product as the experiments of Section 6 report it: the
 * relative spectral error ||XY - C||_2 / ||XY||_2, both norms estimated by
 * `iters` steps of the power iteration (the paper uses ten).  Each step on
 * E^T E (E = XY - C, resp. XY) takes z of unit norm, sets sigma = ||E z|| and
 * z = E^T E z / ||E^T E z||; the estimate is the last sigma (a lower bound of
 * ||E||_2).  z0: cols(Y) entries, host, original order, not all zero (the
 * caller supplies it, e.g. seeded random).  C may be NULL (then *err_norm =
 * 0).  X's column tree must be Y's row tree and C must have X's row tree and
 * Y's column tree, else INCOMPATIBLE.  Device matrix-vector products only;
 * synchronous. */
h2_status h2_product_error(h2_matrix X, h2_matrix Y, h2_matrix C, int iters, const double* z0, double* err_norm,
                           double* xy_norm);

/* Sizes of M: numbers of admissible / inadmissible leaves, rank cap, maximal
 * row and column ranks. */
h2_status h2_matrix_info(h2_matrix M, int64_t* n_adm, int64_t* n_inadm, int* kcap, int* rank_max_row,
                         int* rank_max_col);
/* Leaf blocks as (row cluster, column cluster) pairs: first the admissible
 * ones, then the inadmissible ones (2*(n_adm+n_inadm) ints). */
h2_status h2_matrix_blocks(h2_matrix M, int* pairs);
/* Ranks of the row and column cluster bases (nclusters entries each). */
h2_status h2_matrix_ranks(h2_matrix M, int* row_ranks, int* col_ranks);
/* Packed arrays of an H2-matrix (Definition 4: leaf bases, transfer matrices,
 * coupling matrices of the admissible leaves, dense nearfield of the
 * inadmissible leaves), copied to host memory, e.g. to check that the row and
 * column bases of a product are isometric and nested (Section 5.2).
 * All arrays are row-major, rows in tree order (cluster t covers positions
 * begin(t) .. end(t)-1, see h2_tree_clusters), coefficients padded to kc:
 *   v_leaf      n_rows x kc.  For a leaf cluster t, rows begin(t)..end(t)-1
 *               hold V_t; columns k_t .. kc-1 are zero (k_t = rank_row[t]).
 *   v_transfer  ncl_rows x kc x kc.  Entry t holds E_t (k_t x k_parent in its
 *               top left corner, zero elsewhere): V_parent restricted to t's
 *               rows equals V_t E_t.  The root's entry is zero.
 *   w_leaf, w_transfer   the same for the column basis (W, F; rank_col).
 *   couplings   n_adm x kc x kc: S_b (k_t x k_s in its top left corner) of
 *               admissible leaf b in the order of h2_matrix_blocks.
 *   near        near_size doubles: inadmissible leaf i's |t| x |s| block at
 *               offset near_offset[i] (n_inadm + 1 offsets, the last one is
 *               near_size).
 *   rank_row, rank_col   ncl_rows / ncl_cols ranks.
 * The call always fills the size fields; it copies every array whose pointer
 * is not NULL (caller-allocated with the sizes above), so a first call with
 * all pointers NULL learns the sizes.  Synchronous (waits for the context's
 * device work).  Errors: INVALID_ARG (null M or view), DEVICE. */
typedef struct {
  int64_t n_rows, n_cols;  /* filled: points of the row and column trees */
  int ncl_rows, ncl_cols;  /* filled: clusters of the row and column trees */
  int kc;                  /* filled: padded rank of every coefficient array */
  int64_t n_adm, n_inadm;  /* filled: admissible and inadmissible leaves */
  int64_t near_size;       /* filled: doubles of the packed nearfield */
  double* v_leaf;
  double* v_transfer;
  double* w_leaf;
  double* w_transfer;
  double* couplings;
  double* near;
  int64_t* near_offset;
  int* rank_row;
  int* rank_col;
} h2_host_view;
h2_status h2_export_host(h2_matrix M, h2_host_view* view);

/* Storage of M in bytes (bases, transfers, couplings, nearfield). */
h2_status h2_matrix_storage(h2_matrix M, int64_t* bytes);
void h2_matrix_destroy(h2_matrix M);

/* Diagnostic: runs every device kernel (batched GEMM in FP64 and FP32 with all
 * transpose combinations, streaming QR, Jacobi SVD, Cholesky
 * orthonormalisation) on seeded data and writes each kernel's error against a
 * host evaluation of its definition into errors[0..min(nerrors,*ntests)-1];
 * *ntests receives the number of tests.  Synchronous; allocates its own
 * device memory.  Not used by h2_mul. */
h2_status h2_selftest(h2_context ctx, double* errors, int nerrors, int* ntests);

#ifdef __cplusplus
}
#endif

#endif /* H2_H */
