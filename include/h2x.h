/*
 * h2x -- H^2-matrix x block-of-vectors products and block CG on AMD MI355X (gfx950).
 *
 * C ABI of the library paper_2509_17257_amd/libh2x.so.  The operations follow
 * "On efficient block Krylov solvers for H^2-matrices" (arXiv 2509.17257):
 *
 *   - the cluster tree, block tree and admissibility condition of section 2
 *     (Definitions "Cluster tree", "Block tree", the standard admissibility
 *     condition max(diam) <= eta * dist) and the per-row-cluster block lists of
 *     Algorithm "prepare_addeval" (section 3);
 *   - the H^2 representation of section 2 (nested cluster basis with transfer
 *     matrices, coupling matrices S_b for admissible leaves, dense near-field
 *     blocks), built by tensor Chebyshev interpolation of the kernel
 *     g(x, y) = exp(-|x - y| / ell), plus shift * delta_ij on the diagonal;
 *   - the product Y <- beta Y + alpha A X of Algorithm "H2_mvm" in its matrix
 *     form (section 4): forward transformation, multiplication phase over the
 *     lists C_t of every cluster, backward transformation;
 *   - block CG (section 5.1): m independent CG iterations sharing one H^2 x P
 *     product per iteration, stopping when every column has converged.
 *
 * Conventions
 *   - Every call returns h2x_status and never throws.  On a non-OK status,
 *     h2x_last_error() returns a thread-local message.
 *   - Arguments are validated before anything is launched (H2X_EINVAL,
 *     H2X_ENOMEM for a workspace that is too small).  A failing HIP call gives
 *     H2X_EHIP.
 *   - Device memory is owned by the caller: the library never allocates device
 *     memory.  Every entry point that needs device storage takes a workspace
 *     pointer and its size, obtained from the matching *_workspace_bytes call.
 *     Workspaces must be 256-byte aligned.
 *   - Streams are the caller's (a hipStream_t passed as void*; NULL is the null
 *     stream).  Calls marked "async" only enqueue work on that stream.
 *   - Dense blocks of vectors (X, Y, B) are row-major n x m with leading
 *     dimension ld >= m, in the caller's original point order, FP64.
 *   - Handles are not thread-safe; use one handle per thread or lock.
 */
#ifndef H2X_H
#define H2X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    H2X_OK = 0,
    H2X_EINVAL = 1,       /* invalid argument */
    H2X_ENOMEM = 2,       /* workspace too small */
    H2X_EHIP = 3,         /* a HIP runtime call failed */
    H2X_EBREAKDOWN = 4,   /* CG breakdown (p^T A p <= 0 or non-finite) in >= 1 column */
    H2X_ENOCONV = 5,      /* CG reached max_iter with >= 1 unconverged column */
    H2X_EUNSUPPORTED = 6  /* option not supported by this library version */
} h2x_status;

/* Storage / compute precision of the H^2 operator (V, E, S; near field see h2x_mat_create). */
typedef enum { H2X_F64 = 0, H2X_F32 = 1, H2X_BF16 = 2 } h2x_prec;

typedef enum {
    H2X_KERNEL_EXP = 0,   /* g = exp(-|x - y| / ell) + shift * delta_ij                */
    H2X_KERNEL_POLY = 1,  /* g = (1 + x.y)^2 + shift * delta_ij; reproduced exactly by
                             interpolation order >= 3 (a test kernel)                    */
    H2X_KERNEL_CONST = 2, /* g = 1 + shift * delta_ij, i.e. A = shift I + 1 1^T (test)  */
    H2X_KERNEL_HELMHOLTZ = 3 /* complex: g = (4 pi / n) exp(i kappa r) / (4 pi r) for
                             x != y (the single-layer kernel of section 5.2's examples
                             with equal quadrature weights, kappa = ell), 0 for coinciding
                             points, + shift * delta_ij.  The operator is complex (FP64
                             storage, k = 64 or k <= 32); products and GMRES take m complex
                             columns as 2m real columns (pairs real, imaginary, i.e. the
                             memory of a row-major complex128 array)                     */
} h2x_kernel;

typedef struct {
    h2x_kernel kernel;
    double ell;         /* length scale of the exponential kernel, > 0            */
    double shift;       /* added to every diagonal entry                           */
    double eta;         /* admissibility parameter, > 0                            */
    int32_t leaf_size;  /* a cluster with <= leaf_size points is a leaf, >= 1      */
    int32_t cheb_order; /* Chebyshev nodes per dimension p, 1..8; rank k = p^3    */
} h2x_params;

typedef struct {
    int64_t n, clusters, leaves, n_adm, n_near, near_entries;
    int32_t depth, k;
    int64_t bytes_operator[3]; /* V + E + S bytes per h2x_prec, near field excluded */
    int64_t bytes_near;        /* near-field bytes at FP64                          */
    int32_t adm_depth;         /* shallowest depth of a cluster in an admissible block */
    int32_t split_depth;       /* depth that splits the coupling rows into a deep part and
                                  the rest (tuning option split), 0 when not split     */
    int64_t deep_blocks;       /* admissible blocks in the rows of the deep part       */
} h2x_stats;

typedef struct h2x_plan h2x_plan; /* host topology: trees, lists, permutation */
typedef struct h2x_mat h2x_mat;   /* a plan plus views into a filled device workspace */

/* ---- planning (host only, no GPU needed) -------------------------------- */

/* Build the cluster tree (binary bisection of the tight bounding box at the
 * midpoint of its widest dimension, points strictly below the midpoint first;
 * a cluster is a leaf when it has <= leaf_size points or all its points
 * coincide), the block tree (admissible when dist > 0 and
 * max(diam_t, diam_s) <= eta * dist of the tight boxes) and the lists C_t.
 * pts: host, n x 3 row-major, read during the call only. */
h2x_status h2x_plan_create(const double *pts, int64_t n, const h2x_params *prm, h2x_plan **out);
void h2x_plan_destroy(h2x_plan *plan);
h2x_status h2x_plan_stats(const h2x_plan *plan, h2x_stats *out);

/* perm[i] = original index of the point at tree position i (host, n entries). */
h2x_status h2x_plan_perm(const h2x_plan *plan, int64_t *perm);

/* Clusters in pre-order (host arrays of `clusters` entries, caller-owned; any
 * pointer may be NULL): first tree position, size, parent (-1 for the root),
 * sons (-1 for leaves), depth. */
h2x_status h2x_plan_clusters(const h2x_plan *plan, int64_t *first, int64_t *size, int64_t *parent,
                             int64_t *son0, int64_t *son1, int64_t *depth);

/* Admissible leaves in the library's storage order (row cluster ascending; in
 * block-tree pre-order within a row): row and column cluster of each of the
 * n_adm coupling matrices.  Near-field leaves likewise (n_near entries). */
h2x_status h2x_plan_blocks(const h2x_plan *plan, int64_t *adm_t, int64_t *adm_s, int64_t *near_t,
                           int64_t *near_s);

/* Block-diagonal union of `count` plans (host, count >= 1): one plan whose
 * operator is diag(A_1, ..., A_count), each system keeping its own cluster tree,
 * blocks, lists and kernel parameters (kernel, ell, shift, leaf size, eta).  All
 * plans must have the same cheb_order.  Rows (original and tree order) are the
 * systems' rows concatenated in order.  Used to run many independent systems
 * with one launch per stage and level.  The inputs stay owned by the caller. */
h2x_status h2x_plan_merge(const h2x_plan *const *plans, int32_t count, h2x_plan **out);

/* Number of systems of a plan (1 unless merged) and, if row_offsets is not
 * NULL, the first row of each system plus the total (count + 1 host entries). */
h2x_status h2x_plan_systems(const h2x_plan *plan, int32_t *count, int64_t *row_offsets);

/* ---- operator ------------------------------------------------------------ */

/* Bytes of device workspace an operator needs (topology + V, E, S in `storage`
 * precision + near field; the near field is FP64 for H2X_F64 and FP32 for the
 * low-precision storages). */
size_t h2x_mat_workspace_bytes(const h2x_plan *plan, h2x_prec storage);

/* Upload the topology and fill V, E, S and the near field on the device.
 * dev_ws must stay valid (and untouched) until h2x_mat_destroy.  The plan must
 * outlive the operator.  Blocking: returns after the fill has completed. */
h2x_status h2x_mat_create(const h2x_plan *plan, h2x_prec storage, void *dev_ws, size_t ws_bytes,
                          void *hip_stream, h2x_mat **out);
void h2x_mat_destroy(h2x_mat *mat);

/* ---- product ------------------------------------------------------------- */

#define H2X_TREE_ORDER 1 /* X and Y are in tree order (rows permuted by perm) */

/* Bytes of device workspace h2x_matmul needs for m columns (x-hat, y-hat). */
size_t h2x_matmul_workspace_bytes(const h2x_mat *A, int64_t m);

/* Y <- beta Y + alpha A X, A the H^2 matrix (async).  X: device, n x m, ldx;
 * Y: device, n x m, ldy; X and Y must not overlap.  beta == 0 ignores Y's
 * contents (NaN-safe).  m >= 1. */
h2x_status h2x_matmul(const h2x_mat *A, int64_t m, double alpha, const double *X, int64_t ldx,
                      double beta, double *Y, int64_t ldy, int32_t flags, void *dev_ws,
                      size_t ws_bytes, void *hip_stream);

/* Same product as h2x_matmul, with HIP events recorded on the stream around
 * each stage.  Blocking: returns after the product has completed, with the
 * stage durations in milliseconds in stage_ms[H2X_NUM_STAGES] (host array):
 * forward leaf (including any reordering of X), forward transfer passes,
 * coupling, backward transfer passes, leaf stage (leaf basis and near field). */
#define H2X_NUM_STAGES 5
h2x_status h2x_matmul_timed(const h2x_mat *A, int64_t m, double alpha, const double *X, int64_t ldx,
                            double beta, double *Y, int64_t ldy, int32_t flags, void *dev_ws,
                            size_t ws_bytes, void *hip_stream, double *stage_ms);

/* Stage timing without synchronization, for products inside a timed loop.  A timer holds
 * `slots` sets of HIP events (library-owned, destroyed with the timer).  h2x_matmul_marked
 * is h2x_matmul that also records the stage boundaries of this product into one slot on
 * hip_stream (the stages then run one after another on that stream, as with
 * h2x_matmul_timed); it returns without waiting.  h2x_timer_read waits for the slot's last
 * event and writes the stage durations of its latest product in milliseconds to
 * stage_ms[H2X_NUM_STAGES] (host).  H2X_EINVAL: slot out of range, NULL arguments. */
typedef struct h2x_timer h2x_timer;
h2x_status h2x_timer_create(int32_t slots, h2x_timer **out);
void h2x_timer_destroy(h2x_timer *timer);
h2x_status h2x_matmul_marked(const h2x_mat *A, int64_t m, double alpha, const double *X, int64_t ldx,
                             double beta, double *Y, int64_t ldy, int32_t flags, void *dev_ws,
                             size_t ws_bytes, void *hip_stream, h2x_timer *timer, int32_t slot);
h2x_status h2x_timer_read(const h2x_timer *timer, int32_t slot, double *stage_ms);

/* ---- block CG ------------------------------------------------------------ */

typedef struct {
    double rtol;              /* stop column i when ||r_i|| <= rtol ||b_i||              */
    int32_t max_iter;         /* iterations of the shared loop                           */
    int32_t freeze_converged; /* 0: converged columns keep iterating (the paper's rule);
                                 1: converged columns stop updating                       */
    int32_t check_every;      /* read the device convergence flag every this many steps */
    int32_t variant;          /* H2X_CG_INDEPENDENT or H2X_CG_SHARED                     */
    int32_t graph;            /* H2X_CG_INDEPENDENT: 1 captures check_every iterations (the
                                 product and the CG kernels) once into a HIP graph on a
                                 private stream and replays it; 0 launches every kernel     */
} h2x_cg_params;

/* H2X_CG_INDEPENDENT: the paper's block CG -- m independent CG iterations that
 *   share only the H^2 x P product (section 5.1).
 * H2X_CG_SHARED: block CG over one shared block Krylov space (O'Leary's block CG,
 *   which the paper cites as the alternative that enriches the Krylov space):
 *   m x m Gram matrices, their Cholesky factorizations and a Cholesky-QR
 *   orthonormalisation of the search block with deflation of directions whose
 *   remaining norm falls below 1e-6 of the largest; m <= 64; freeze_converged
 *   and check_every are ignored (convergence is read every iteration). */
#define H2X_CG_INDEPENDENT 0
#define H2X_CG_SHARED 1

typedef struct {
    int32_t iters;       /* iterations of the shared loop (refined solve: all inner iterations) */
    int32_t status;      /* H2X_OK, H2X_EBREAKDOWN or H2X_ENOCONV                     */
    int32_t outer_iters; /* refinement steps (h2x_block_cg_refine); 0 otherwise        */
    double *col_relres;  /* host, m entries or NULL: final ||r_i|| / ||b_i|| (recursive) */
    int32_t *col_iters;  /* host, m entries or NULL: iteration at which column i first met
                            the tolerance (iters if it never did)                      */
    int32_t *col_status; /* host, m entries or NULL: 0 ok, 1 breakdown, 2 not converged */
    int32_t *sys_iters;  /* host, one entry per system or NULL: iteration at which the
                            system stopped (every column converged or broken down)   */
} h2x_cg_info;

size_t h2x_block_cg_workspace_bytes(const h2x_mat *A, int64_t m);

/* Solve A X = B for m right-hand sides with block CG: one H^2 x P product per
 * iteration, per-column step sizes (the paper's block CG).  For an operator on
 * a merged plan (h2x_plan_merge) every system is solved independently in the
 * same iterations: dot products, step sizes and convergence per system and
 * column, and a system stops updating once all its columns have converged; the
 * per-column info arrays then hold systems x m entries, system-major.  B: device n x m,
 * ldb; X: device n x m, ldx, holds X0 on entry and the iterate on exit.  A
 * column whose p^T A p is <= 0 or non-finite is frozen and reported.
 * Blocking: returns after the solve.  The return value reports argument and
 * HIP errors only; the solver outcome (H2X_OK, H2X_EBREAKDOWN, H2X_ENOCONV)
 * is info->status, with per-column detail.  info may be NULL. */
h2x_status h2x_block_cg(const h2x_mat *A, const h2x_cg_params *prm, int64_t m, const double *B,
                        int64_t ldb, double *X, int64_t ldx, void *dev_ws, size_t ws_bytes,
                        h2x_cg_info *info, void *hip_stream);

/* Mixed precision: FP64 iterative refinement around block CG with a
 * low-precision operator (the paper itself computes in FP64 throughout).
 * A: the FP64 operator (H2X_F64 storage); A_lo: the same plan stored in FP32 or
 * BF16 (its products accumulate in FP32).  Outer step: R = B - A X in FP64; stop
 * when every column has ||R_i|| <= rtol ||B_i||; otherwise solve A_lo D = R with
 * block CG (FP64 vectors, dot products and step sizes) to inner->rtol relative to
 * ||R_i||, and set X += D.  At most max_outer steps; a step that does not halve
 * the worst column's relative residual is a stall, and two stalls end the solve
 * with H2X_ENOCONV (the low-precision operator is too far from A for this
 * system's conditioning).  Every column returns its outer iterate with the
 * smallest FP64 true residual (X0 included), so a refinement that diverges
 * returns its best iterate.  Blocking.  info->iters is the
 * total number of inner iterations, info->outer_iters the number of steps,
 * info->col_relres the FP64 true residuals ||B_i - A X_i|| / ||B_i|| of the
 * returned columns, info->status H2X_ENOCONV if one of them misses rtol.  The
 * workspace holds one n x m block for the best iterate besides the solve's. */
size_t h2x_block_cg_refine_workspace_bytes(const h2x_mat *A, const h2x_mat *A_lo, int64_t m);
h2x_status h2x_block_cg_refine(const h2x_mat *A, const h2x_mat *A_lo, const h2x_cg_params *inner, double rtol,
                               int32_t max_outer, int64_t m, const double *B, int64_t ldb, double *X,
                               int64_t ldx, void *dev_ws, size_t ws_bytes, h2x_cg_info *info,
                               void *hip_stream);

/* Mixed precision in one CG run (residual replacement, van der Vorst and Ye,
 * "Residual replacement strategies for Krylov subspace iterative methods for the
 * convergence of true residuals", 2000): every iteration is block CG
 * (H2X_CG_INDEPENDENT) with the low-precision operator A_lo; after an iteration in
 * which an open column's recursive residual has fallen below delta times its
 * largest value since the last replacement (checked every prm->check_every
 * iterations), and whenever every column looks converged, the residual is
 * recomputed as R = B - A X with the FP64 operator A and the iteration continues
 * from it with the same search directions.  The solve stops when every column
 * meets prm->rtol on the recomputed residual (or has broken down, or max_iter
 * is reached).  Every column returns the iterate with the smallest recomputed
 * true residual (X0 included), so a solve that breaks down or diverges returns
 * its best iterate.  info->outer_iters is the number of replacements,
 * info->col_relres the true residuals of the returned columns, info->status
 * H2X_EBREAKDOWN if a column broke down, else H2X_ENOCONV if a returned column
 * misses rtol.  A and A_lo: one plan with one system; A stored in FP64.
 * 0 < delta < 1 (0.1 is usual).  Blocking. */
size_t h2x_block_cg_mixed_workspace_bytes(const h2x_mat *A, const h2x_mat *A_lo, int64_t m);
h2x_status h2x_block_cg_mixed(const h2x_mat *A, const h2x_mat *A_lo, const h2x_cg_params *prm, double delta,
                              int64_t m, const double *B, int64_t ldb, double *X, int64_t ldx, void *dev_ws,
                              size_t ws_bytes, h2x_cg_info *info, void *hip_stream);

/* ---- block GMRES ------------------------------------------------------------ */
/* Block GMRES(restart) without a preconditioner (section 5.2, the block form of
 * the generalized minimal residual method with M = I): m independent GMRES
 * processes that share one H^2 x Q product per Arnoldi step.  Per column and
 * cycle: r = b - A x, rhat = ||r|| e_0, q_0 = r / ||r||; each step takes the
 * product a = A q_k, classical Gram-Schmidt against q_0..q_k (all projections
 * from the same a), h[k+1][k] = ||a||, q_{k+1} = a / h[k+1][k], and Givens
 * rotations that keep the Hessenberg matrix upper triangular and carry rhat.  A
 * column stops extending its basis once |rhat| <= rtol ||b_i||; at the end of a
 * cycle each column solves its triangular system with its own number of steps
 * and updates x; the next cycle restarts from the improved x.  A column is done
 * when its true residual ||b_i - A x_i|| <= rtol ||b_i|| at the start of a
 * cycle.  Not for merged (batched) plans.
 *
 * restart: Arnoldi steps per cycle (>= 1); the workspace holds restart + 1 basis
 * blocks of n x m doubles.  max_iter: Arnoldi steps over all cycles (>= 0).
 * check_every: the host reads the device's convergence flag every this many
 * steps (>= 1; steps launched after every column has closed do nothing).
 * X holds X0 on entry and the iterate on exit (row-major, leading dimension ldx);
 * B is row-major with leading dimension ldb.  Blocking: returns after the solve.
 * Returns H2X_OK when the solve ran; the outcome is in info->status (H2X_OK, or
 * H2X_ENOCONV when a column did not converge within max_iter, H2X_EBREAKDOWN when
 * a column met a singular projected matrix).  info arrays are host, m entries,
 * nullable: col_iters (steps in which the column was open), col_status (0
 * converged, 1 breakdown, 2 not converged), col_res (|rhat| / ||b_i|| after the
 * column's last cycle, the GMRES estimate of its relative residual).
 * Complex operator (H2X_KERNEL_HELMHOLTZ): the same method over C (inner product
 * u^H v, complex Givens rotations); m counts real columns, two per complex column
 * (real, imaginary part; m even), and the info arrays have m / 2 entries. */
typedef struct {
    double rtol;
    int32_t restart;
    int32_t max_iter;
    int32_t check_every;
    int32_t reserved;
} h2x_gmres_params;

typedef struct {
    int32_t iters;   /* Arnoldi steps run */
    int32_t cycles;  /* restart cycles run */
    int32_t status;
    int32_t reserved;
    double *col_res;
    int32_t *col_iters;
    int32_t *col_status;
} h2x_gmres_info;

size_t h2x_block_gmres_workspace_bytes(const h2x_mat *A, int64_t m, int32_t restart);
h2x_status h2x_block_gmres(const h2x_mat *A, const h2x_gmres_params *prm, int64_t m, const double *B, int64_t ldb,
                           double *X, int64_t ldx, void *dev_ws, size_t ws_bytes, h2x_gmres_info *info,
                           void *hip_stream);

/* ---- right-hand-side chunking --------------------------------------------------- */
/* Section 5 (the remarks on the memory footprint of block CG and block GMRES): the
 * solvers' auxiliary storage grows linearly in the number of right-hand sides -- block
 * CG O(6 n m), block GMRES O(n (restart + 1) m) -- so for a large m the columns are
 * solved in chunks of at most m_chunk; the paper's conclusions name choosing m_chunk
 * adaptively from the available memory and the compute rate as the next step. */
typedef enum { H2X_SOLVER_CG = 0, H2X_SOLVER_GMRES = 1 } h2x_solver;

/* Device workspace of one solve of m right-hand sides (h2x_block_cg_workspace_bytes or
 * h2x_block_gmres_workspace_bytes of an operator built from this plan and storage),
 * computed from the plan alone.  0 on bad arguments. */
size_t h2x_solve_workspace_bytes(const h2x_plan *plan, h2x_prec storage, int32_t solver, int64_t m,
                                 int32_t restart);

/* m_chunk for m right-hand sides under a device-memory budget of mem_bytes for the
 * solver workspace.  Without a throughput curve (cand_ms NULL or ncand 0): the largest
 * chunk <= m whose workspace fits.  With one (cand_m[i] columns take cand_ms[i] ms per
 * product, e.g. from h2x_product_times): among the candidates that fit, the one with the
 * least predicted time ceil(m / c) * cand_ms(c), ties to the larger chunk (candidates
 * larger than m count as m; none fitting falls back to the memory rule).  Host only.
 * H2X_ENOMEM when a single column does not fit; H2X_EINVAL on bad arguments. */
h2x_status h2x_choose_chunk(const h2x_plan *plan, h2x_prec storage, int32_t solver, int32_t restart, int64_t m,
                            size_t mem_bytes, int32_t ncand, const int64_t *cand_m, const double *cand_ms,
                            int64_t *m_chunk);

/* The throughput curve: mean time of one product (h2x_matmul, tuned tile shapes if any)
 * for each candidate column count, reps timed products after an untimed one, HIP events on
 * the given stream.  ms: host, ncand entries.  Blocking. */
size_t h2x_product_times_workspace_bytes(const h2x_mat *A, int32_t ncand, const int64_t *cand_m);
h2x_status h2x_product_times(const h2x_mat *A, int32_t ncand, const int64_t *cand_m, int32_t reps, void *dev_ws,
                             size_t ws_bytes, void *hip_stream, double *ms);

/* Block CG / block GMRES over the columns in chunks of m_chunk (the last may be smaller):
 * each chunk is an independent solve of the column slice (B + c0, ldb) -> (X + c0, ldx),
 * in place, with a workspace for m_chunk columns.  info: per-column arrays (m entries) are
 * filled chunk by chunk; iters / cycles / outer_iters are the maxima over the chunks;
 * status is the first non-OK chunk status. */
h2x_status h2x_block_cg_chunked(const h2x_mat *A, const h2x_cg_params *prm, int64_t m, int64_t m_chunk,
                                const double *B, int64_t ldb, double *X, int64_t ldx, void *dev_ws, size_t ws_bytes,
                                h2x_cg_info *info, void *hip_stream);
h2x_status h2x_block_gmres_chunked(const h2x_mat *A, const h2x_gmres_params *prm, int64_t m, int64_t m_chunk,
                                   const double *B, int64_t ldb, double *X, int64_t ldx, void *dev_ws,
                                   size_t ws_bytes, h2x_gmres_info *info, void *hip_stream);

/* ---- tuning ----------------------------------------------------------------- */
/* Tile shapes of the matrix-core kernels: columns per work-group of the forward
 * leaf and transfer passes (16 * nj_transfer), of the coupling (16 * nj_coupling)
 * and of the leaf stage (32 * np_leaf); 0 means the built-in rule.  On the FP64
 * matrix-core path the near-field term can run on a second stream of the operator
 * while the transfer passes and the coupling run on the caller's stream (the
 * basis term joins it); the product then adds the two terms to Y in two steps. */
typedef struct {
    int32_t nj_transfer, nj_coupling, np_leaf;
    int32_t overlap;   /* near field beside the transfer passes: 0 (built-in rule) and 2
                          off; on a second stream with its grid capped at 256 (1), 128 (3)
                          or 512 (4) work-groups; 5 in shares inside the launches of the
                          transfer levels; 6 in two halves on a second stream, one beside
                          the upward and one beside the downward pass, at most three
                          near work-groups per CU (5 and 6: leaf_kind 3, k = 64)         */
    int32_t fuse_up;   /* forward leaf and upward pass in one launch: 1 on; 0 (built-in
                          rule) and 2 level by level                                   */
    int32_t leaf_kind; /* leaf stage (32 * np_leaf columns per wave): 0 built-in rule
                          (3 where its table of near rows fits in LDS and the operator
                          is real, else 1); 1 a work-group per leaf, each wave a 64-row
                          tile of its share of the terms; 2 a wave per 32-row band of a
                          leaf, every term in turn (FP64 only; 1 for FP32 / BF16); 3 a
                          work-group per leaf, the near blocks and the basis as one
                          contraction in rounds of 16 rows, 16-row tiles of the leaf
                          (FP64, FP32 and BF16 storage)                                 */
    int32_t split;     /* coupling rows in two parts, the deep part (rows whose lists are
                          complete once the upward pass has reached a split depth) on a
                          second stream beside the upper transfer levels, the coupling of
                          the other rows and the upper downward levels: 0 built-in rule,
                          1 on (the deep part leaves room on every CU for a work-group
                          of the transfer passes), 2 off, 3 on without that reserve     */
    double ms_default; /* product time with the built-in rule */
    double ms_tuned;   /* product time with the chosen shapes */
} h2x_tune_info;

/* Autotune the operator for m columns: time the product with each candidate
 * shape per stage (HIP events, a few runs each, on synthetic right-hand sides
 * inside the workspace), keep the fastest per stage if the combination beats
 * the built-in rule, and store the choice in the operator for every column
 * count with the same ceil(m / 16) (counts above 64 share one entry).  Later
 * products and solves on the operator use it.  Blocking.  info may be NULL.
 * Must not run concurrently with other calls on the same operator. */
size_t h2x_mat_autotune_workspace_bytes(const h2x_mat *A, int64_t m);
h2x_status h2x_mat_autotune(h2x_mat *A, int64_t m, void *dev_ws, size_t ws_bytes, void *hip_stream,
                            h2x_tune_info *info);

/* Read / write the shapes stored for m's entry (every column count with the same
 * ceil(m / 16), counts above 64 sharing one): a choice kept from an earlier autotune
 * run, or a fixed shape, without timing.  Set: the shape fields of cfg are used
 * (ms_default / ms_tuned ignored); all zero restores the built-in rule; ranges
 * nj_transfer, nj_coupling 0..4, np_leaf 0..2, overlap 0..6, fuse_up 0..2, leaf_kind
 * 0..3, split 0..3, else H2X_EINVAL.  Get: ms_default = ms_tuned = 0.  Host only; must
 * not run concurrently with products on the same operator. */
h2x_status h2x_mat_set_tune(h2x_mat *A, int64_t m, const h2x_tune_info *cfg);
h2x_status h2x_mat_get_tune(const h2x_mat *A, int64_t m, h2x_tune_info *cfg);

/* ---- batches ---------------------------------------------------------------- */
/* A batch is a list of operators (typically one merged plan per Chebyshev order
 * and storage precision) whose rows are concatenated in order: operator j owns
 * rows [r_j, r_j + n_j) of every n_total x m block passed to the batch calls.
 * The batch only refers to the operators, which must outlive it. */
typedef struct h2x_batch h2x_batch;
h2x_status h2x_batch_create(const h2x_mat *const *mats, int32_t count, h2x_batch **out);
void h2x_batch_destroy(h2x_batch *batch);

/* Y <- beta Y + alpha diag(A_1, ...) X over all operators of the batch (async). */
size_t h2x_batch_matmul_workspace_bytes(const h2x_batch *batch, int64_t m);
h2x_status h2x_batch_matmul(const h2x_batch *batch, int64_t m, double alpha, const double *X, int64_t ldx,
                            double beta, double *Y, int64_t ldy, int32_t flags, void *dev_ws, size_t ws_bytes,
                            void *hip_stream);

/* Block CG (H2X_CG_INDEPENDENT) on every system of the batch at once: each
 * iteration runs the products of all operators and one set of CG kernels over
 * all rows, with per-system dot products and convergence (see h2x_block_cg).
 * info arrays hold (total systems) x m entries.  Columns of B that are zero
 * converge at once, so systems with fewer right-hand sides pad B with zeros. */
size_t h2x_batch_block_cg_workspace_bytes(const h2x_batch *batch, int64_t m);
h2x_status h2x_batch_block_cg(const h2x_batch *batch, const h2x_cg_params *prm, int64_t m, const double *B,
                              int64_t ldb, double *X, int64_t ldx, void *dev_ws, size_t ws_bytes,
                              h2x_cg_info *info, void *hip_stream);

/* ---- differentiation ------------------------------------------------------- */
/* The paper's products use the row lists C_t of section 3 ("prepare_addeval");
 * the adjoint swaps the roles of row and column cluster (lists by column
 * cluster, transposed coupling and near-field blocks), with the same forward
 * and backward transformations, since the row and column bases coincide (W = V,
 * section 2).  The gradients are those of L = <dY, A X> (sum of the entrywise
 * products) with respect to the stored blocks of the representation of section 2
 * and to the kernel length scale ell.  FP64 operators with rank k <= 64 only
 * (H2X_EUNSUPPORTED otherwise). */

/* Bytes of device workspace h2x_matmul_adjoint needs for m columns. */
size_t h2x_matmul_adjoint_workspace_bytes(const h2x_mat *A, int64_t m);

/* Y <- beta Y + alpha A^T X (async): every column cluster s collects
 * S_b^T x-hat_t over the admissible blocks b = (t, s) of its column, and every
 * leaf s collects N_ts^T X|_t over the near-field blocks of its column.  X, Y:
 * device, n x m, original point order; must not overlap; beta == 0 ignores Y. */
h2x_status h2x_matmul_adjoint(const h2x_mat *A, int64_t m, double alpha, const double *X, int64_t ldx,
                              double beta, double *Y, int64_t ldy, void *dev_ws, size_t ws_bytes,
                              void *hip_stream);

/* Bytes of device workspace h2x_grad needs for m columns. */
size_t h2x_grad_workspace_bytes(const h2x_mat *A, int64_t m);

/* Gradients of L = scale * <dY, A X> (async).  X, dY: device n x m (original order).
 * Outputs (device, any may be NULL to skip it):
 *   dS:   n_adm x k x k row-major, in the storage order of h2x_plan_blocks:
 *         dS_b = scale * dyhat_t xhat_s^T, xhat / dyhat the forward transformations;
 *   dN:   near_entries doubles, the blocks in the storage order of
 *         h2x_plan_blocks, each |t| x |s| row-major in tree order of the points:
 *         dN_b = scale * dY|_t X|_s^T;
 *   dell: one double, dL/dell = sum_b <dS_b/dell, dS_b> + sum_b <dN_b/dell, dN_b>
 *         with d g / d ell = (r / ell^2) exp(-r / ell) (0 for the test kernels);
 *         dell_terms selects the terms summed: H2X_DELL_COUPLING (the coupling
 *         matrices), H2X_DELL_NEAR (the near field), or both.  A caller that
 *         supplies its own coupling matrices (which then do not depend on ell)
 *         asks for H2X_DELL_NEAR only.  Reduced in a fixed order (bitwise
 *         reproducible).
 * scale: finite (e.g. -1 for the implicit adjoint of a solve). */
#define H2X_DELL_COUPLING 1
#define H2X_DELL_NEAR 2
h2x_status h2x_grad(const h2x_mat *A, int64_t m, const double *X, int64_t ldx, const double *dY,
                    int64_t lddy, double *dS, double *dN, double *dell, double scale, int32_t dell_terms,
                    void *dev_ws, size_t ws_bytes, void *hip_stream);

/* Refill the coupling matrices and the near field for a new kernel length scale
 * (the cluster tree, block tree, bases and transfers do not depend on ell).
 * Blocking: returns after the refill. */
h2x_status h2x_mat_set_ell(h2x_mat *A, double ell, void *hip_stream);

/* Copy the coupling matrices S_b (FP64 operators) to out (device, n_adm x k x k
 * doubles, row-major S_b[nu][mu] = g(xi_t,nu, xi_s,mu), blocks in the storage
 * order of h2x_plan_blocks), whatever the internal layout (async). */
h2x_status h2x_mat_coupling(const h2x_mat *A, double *out, void *hip_stream);

/* Replace the coupling matrices S_b (FP64 operators) by in (device, same layout
 * as h2x_mat_coupling), e.g. after a gradient step on them (async; in must stay
 * valid until the copy has run).  h2x_mat_set_ell refills them from the kernel. */
h2x_status h2x_mat_set_coupling(h2x_mat *A, const double *in, void *hip_stream);

/* ---- product without a workspace ------------------------------------------- */
/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the product of
 * h2x_matmul, same arguments and semantics, with its scratch memory (x-hat,
 * y-hat, the tree-ordered copy of X) in a static device array of
 * H2X_NOALLOC_MAX_BYTES that the library holds on every GPU it runs on until
 * the process ends.  Nothing is allocated by the call.  The scratch needed is
 * h2x_matmul_workspace_bytes(A, m); a larger need returns H2X_ENOMEM (use
 * h2x_matmul with a workspace).  The array is shared by every call on the same
 * GPU and keeps the last call's contents (the product reads none of it before
 * writing it): calls that overlap on one GPU (several streams or threads) race
 * and must be serialized by the caller.  The calling thread's current device
 * must be the device of A and of hip_stream.  Async. */
#define H2X_NOALLOC_MAX_BYTES ((size_t)128 << 20)
h2x_status h2x_matmul_noalloc(const h2x_mat *A, int64_t m, double alpha, const double *X, int64_t ldx, double beta,
                              double *Y, int64_t ldy, int32_t flags, void *hip_stream);

/* ---- misc ------------------------------------------------------------------ */

const char *h2x_last_error(void);
const char *h2x_version(void);

#ifdef __cplusplus
}
#endif
#endif /* H2X_H */
