/*
 * dwfmm.h -- C ABI of the MI355X dimension weighted FMM library (libdwfmm.so).
 *
 * The library computes y = K~ x, the fast multipole approximation of a kernel
 * matrix K = [K(x_i, x_j)] over N data sites in d dimensions, and solves
 * (K~ + lambda I) alpha = f with conjugate gradients (Harbrecht, Multerer,
 * Quizi, arXiv 2402.09531: Sec 2 eqs. (LGS0)/(LGS) for the systems, Sec 5 for
 * the method).  Everything after setup runs in HIP kernels on a gfx950 GPU.
 *
 * Conventions for every entry point
 *   - Array arguments are DEVICE pointers unless marked "host".
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   - Point and vector arrays are in the caller's original point order;
 *     x, y, f, alpha are N x nrhs row-major FP64.
 *   - Every call returns a dwfmm_status; no exception crosses the ABI and the
 *     library never aborts.  dwfmm_last_error() gives a message for the last
 *     non-OK status of the calling thread.
 *   - Objects are not thread-safe; distinct objects may be used concurrently.
 *   - The library owns all memory of a tree or operator: it is allocated in
 *     dwfmm_build_tree / dwfmm_fmm_create and freed by the destroy calls.
 *     dwfmm_fmm_matvec and dwfmm_fmm_solve allocate nothing.
 */
#ifndef DWFMM_H
#define DWFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DWFMM_OK = 0,
    DWFMM_E_INVALID = 1,        /* argument out of range */
    DWFMM_E_NONFINITE = 2,      /* NaN or Inf in points or weights */
    DWFMM_E_NOMEM = 3,          /* device or host allocation failed */
    DWFMM_E_HIP = 4,            /* a HIP runtime call failed */
    DWFMM_E_NOT_CONVERGED = 5,  /* solve hit max_iter (info still filled) */
    DWFMM_E_BREAKDOWN = 6       /* CG breakdown: |p^T A p| <= 1e-300 or non-finite */
} dwfmm_status;

/* Kernel functions K(x,y) with r = |x - y|_2:
 *   MATERN32     (1 + sqrt(3) r/ell) exp(-sqrt(3) r/ell)
 *   GAUSSIAN     exp(-r^2/ell)
 *   EXPONENTIAL  exp(-r/ell)           (the Sec 6.2 kernel, with the sign read as decaying)
 *   POLY_TEST    1 + sum_{k < (int)ell} x_k y_k + (x_0 y_0)^2  (exactness tests only)  */
typedef enum { DWFMM_MATERN32 = 0, DWFMM_GAUSSIAN = 1, DWFMM_EXPONENTIAL = 2, DWFMM_POLY_TEST = 3 } dwfmm_kernel_kind;

typedef struct {
    int32_t kind;   /* dwfmm_kernel_kind */
    double ell;     /* length scale (> 0) */
} dwfmm_kernel;

/* Dimension weights omega_k of the index set (Sec 4; Thm 4.6; Sec 6.2), computed
 * from the box side lengths b_k given to dwfmm_build_tree:
 *   R1 (default)  omega_k = max(1, log2(b_max / b_k))
 *   R2            omega_k = 1 + log2(b_max / b_k)
 *   R3            Sec 6.2: tau_k = 1/(eta b_k), rho_k = e g(tau_k)/g(tau_1),
 *                 g(t) = 2t + sqrt(1+4t^2), omega_k = log rho_k
 *   EXPLICIT      omega taken from dwfmm_opts.omega (host, length d, > 0)     */
typedef enum { DWFMM_W_R1 = 0, DWFMM_W_R2 = 1, DWFMM_W_R3 = 2, DWFMM_W_EXPLICIT = 3 } dwfmm_weight_rule;

/* Arithmetic of the coupling (M2L) and nearfield (P2P) stages.  Geometry,
 * moments, transfers, CG inner products and residuals are always FP64.
 *   FP32  distances on FP32 MFMA, kernel values and sums in FP32
 *   BF16  FP32 mode, and with several rhs the products on BF16 MFMA with FP32
 *         accumulation: the nearfield K Q with K and Q rounded to BF16, the
 *         coupling S m with S and m each carried as a pair of BF16 numbers
 *         (three products); the nearfield's distances (d >= 5) on FP16 MFMA
 *         from coordinates split into FP16 high and low parts (three
 *         products, about 2^-22 of each term); with one rhs it is FP32 mode  */
typedef enum { DWFMM_FP64 = 0, DWFMM_FP32 = 1, DWFMM_BF16 = 2 } dwfmm_precision;

/* Interpolation nodes on the reference box (Sec 5.4 and the per-axis reading):
 *   CHEB_LEJA  node alpha = (z^(1)_{alpha_1}, ..., z^(d)_{alpha_d}), z^(k) the m_k+1
 *              first-kind Chebyshev points of [0,1] in Leja order (default)
 *   AFP        approximate Fekete points: the n_x pivots of a greedy column-pivoted
 *              QR of the Legendre Vandermonde matrix over Halton candidates (points
 *              1..M over the axes with m_k > 0, in consecutive prime bases; other
 *              coordinates 1/2); a residual norm within relative 1e-12 of the
 *              largest goes to the lowest candidate index                          */
typedef enum { DWFMM_NODES_CHEB_LEJA = 0, DWFMM_NODES_AFP = 1 } dwfmm_node_rule;

/* Index set (Sec 4; Sec 6.1):
 *   WEIGHTED_TOTAL_DEGREE  Lambda = { alpha : sum_k omega_k alpha_k <= q } (default; with
 *                          omega = 1 through DWFMM_W_EXPLICIT it is the total degree set)
 *   TENSOR                 { alpha : max_k alpha_k <= q }, the tensor product set; the
 *                          weights are not used                                      */
typedef enum { DWFMM_INDEX_WEIGHTED_TOTAL_DEGREE = 0, DWFMM_INDEX_TENSOR = 1 } dwfmm_index_rule;

typedef struct {
    int32_t weight_rule;     /* dwfmm_weight_rule, default R1 */
    const double *omega;     /* host, length d, only for DWFMM_W_EXPLICIT */
    int32_t precision;       /* dwfmm_precision of the inner matvec, default FP64 */
    int32_t max_nrhs;        /* largest nrhs a matvec/solve may use (1..32), default 1 */
    int32_t check_every;     /* CG iterations between host convergence checks, default 1 */
    double ir_inner_rtol;    /* reduced precision: inner CG tolerance (0 = 1e-4 FP32, 1e-2 BF16) */
    int32_t ir_max_outer;    /* reduced precision: max refinement steps, default 30 */
    int32_t node_rule;       /* dwfmm_node_rule, default CHEB_LEJA */
    int32_t afp_candidates;  /* AFP: Halton candidates M >= n_x, 0 = max(2000, 50 n_x) */
    /* Optional (NULL = none): called by dwfmm_fmm_solve on the calling thread at each host
     * convergence check (every check_every iterations) with the iteration count, nrhs and
     * the recursive relative residuals |r|/|f| per column (host array, valid during the
     * call).  It must not call into the library for this operator. */
    void (*progress)(void *ctx, int32_t iteration, int32_t nrhs, const double *rel_res);
    void *progress_ctx;
    int32_t index_rule;      /* dwfmm_index_rule, default WEIGHTED_TOTAL_DEGREE */
    int32_t ir_max_inner;    /* reduced precision: max inner CG iterations per refinement step
                                (0 = up to the solve's remaining max_iter) */
    int32_t cache_near;      /* 1: keep the BF16 kernel tiles of the several-rhs nearfield in device
                                memory (2 bytes per nearfield entry, rows padded to 128: ~42 GB at
                                N = 1e6, d = 20); the first BF16 matvec with nrhs > 1 writes them,
                                later ones read them instead of recomputing (same results, bit for
                                bit; not used inside a graph capture).  Needs precision BF16 and
                                max_nrhs > 1 (else E_INVALID); kept only when leaves hold at most 128
                                points and d <= 32.  Default 0. */
} dwfmm_opts;

/* Per right-hand-side result of dwfmm_fmm_solve. */
typedef struct {
    int32_t iters;               /* CG iterations (matvecs) taken, summed over refinement steps */
    int32_t neg_curvature_steps; /* steps with p^T A p < 0 (taken, counted) */
    int32_t refine_steps;        /* outer refinement steps (0 in FP64 mode) */
    int32_t status;              /* DWFMM_OK, DWFMM_E_NOT_CONVERGED or DWFMM_E_BREAKDOWN */
    double rel_res_recursive;    /* |r_k| / |f| from the CG recurrence */
    double rel_res_true;         /* |f - (K~ + lambda I) alpha| / |f|, one extra FP64 matvec */
} dwfmm_solve_info;

typedef struct dwfmm_tree_s *dwfmm_tree;
typedef struct dwfmm_op_s *dwfmm_op;

/* Cluster tree and block partition (Sec 5.1, Def 5.1/5.2; Sec 5.2 eq. (admissibility)).
 *   points       device, N x d row-major FP64, original order (copied; may be freed on return)
 *   n, d         N >= 1, 1 <= d <= 64
 *   dim_weights  host, length d, b_k > 0 (side lengths of the anisotropic box, Sec 2)
 *   leaf_size    >= 1; depth J = min{j : ceil(N/2^j) <= leaf_size}
 *   eta          > 0, admissibility dist(B,B') >= eta max(diam B, diam B')
 * Splits every cluster above depth J along the longest edge of its tight box at
 * the median (left child takes ceil(n/2); ties by original index).  Farfield =
 * admissible blocks whose parent block is not; nearfield = remaining leaf blocks.
 * Synchronises `stream`.  Errors: E_INVALID, E_NONFINITE, E_NOMEM, E_HIP.      */
dwfmm_status dwfmm_build_tree(const double *points, int64_t n, int32_t d, const double *dim_weights,
                              int32_t leaf_size, double eta, void *stream, dwfmm_tree *out);

/* Which box size the admissibility compares against (Sec 5.2 eq. (admissibility) names the
 * diameter; the paper's Sec 6.2 settings are consistent with half of the box diagonal).
 *   FULL_DIAGONAL  dist(B,B') >= eta max(diag B, diag B')          (dwfmm_build_tree)
 *   HALF_DIAGONAL  eta dist(B,B') >= max(diag B, diag B') / 2
 * Both are evaluated squared and inclusive; HALF with eta gives the same partition as FULL
 * with 1/(2 eta) wherever the two products round alike (exactly so for eta = 0.5 and 1).   */
typedef enum {
    DWFMM_ADM_FULL_DIAGONAL = 0,
    DWFMM_ADM_HALF_DIAGONAL = 1
} dwfmm_admissibility;

/* dwfmm_build_tree with the admissibility rule chosen; the rule is kept with the tree and
 * also applies to evaluation at new points (dwfmm_eval_create).  Errors as dwfmm_build_tree,
 * plus E_INVALID for an unknown rule.                                                       */
dwfmm_status dwfmm_build_tree_ex(const double *points, int64_t n, int32_t d, const double *dim_weights,
                                 int32_t leaf_size, double eta, dwfmm_admissibility admissibility,
                                 void *stream, dwfmm_tree *out);

/* FMM operator for a tree (Sec 4 index set; Sec 5.2 interpolation, cluster bases,
 * transfer matrices).  q >= 0 is the weighted total degree.  opts may be NULL.
 * Builds Lambda, the nodes (opts->node_rule), V^-1, the transfer matrices of
 * every cluster and the interpolation nodes of every box, and allocates the
 * workspace for opts->max_nrhs right-hand sides.  The operator keeps a reference
 * on the tree.  Synchronises `stream`.  n_x <= 128 and n_x * d (rounded up to a
 * multiple of 4) <= 3072; above n_x = 64 the coupling runs on the general kernel.
 * Errors: E_INVALID (bad kernel, q, opts, index set too large), E_NOMEM, E_HIP.  */
dwfmm_status dwfmm_fmm_create(dwfmm_tree tree, dwfmm_kernel kernel, double q, const dwfmm_opts *opts,
                              void *stream, dwfmm_op *out);

/* y = K~ x (Sec 5.2 eq. (LowRankBlock) on the farfield, kernel entries on the
 * nearfield), in the operator's precision.  x, y: device N x nrhs, distinct.
 * 1 <= nrhs <= max_nrhs.  Asynchronous on `stream`; allocates nothing.  On the
 * MFMA nearfield paths (one rhs, or up to 32 with leaves of at most 128 points and
 * d <= 32) the farfield (M2M, M2L, L2L) runs on the operator's own side stream
 * beside the nearfield, ordered after the P2M on `stream` and joined back into
 * `stream` before the final combine or L2P, so the result is ordered on `stream`
 * as usual.  The
 * call may be captured into a HIP graph from `stream`; while `stream` is capturing
 * all work stays on `stream` (no library object may be destroyed during a capture:
 * the destroy calls free device memory).  Calls on one operator must not overlap (they share
 * its workspace and side stream).  Errors: E_INVALID, E_HIP.                      */
dwfmm_status dwfmm_fmm_matvec(dwfmm_op op, const double *x, double *y, int32_t nrhs, void *stream);

/* Allocation-free matvec, for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Computes the same
 * y = K~ x as dwfmm_fmm_matvec (same kernels, same bits) but takes the call's workspace --
 * charges in tree order (and their BF16 copy with several rhs), moments and locals, nearfield
 * row and column sums -- from one static
 * device array of DWFMM_STATIC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends, instead of the operator's buffers; it allocates nothing (the first
 * call on a device looks the array's address up once).  1 <= nrhs <= 32, independent of the
 * operator's max_nrhs; the operator's precision applies.  The operator's device must be
 * current.  Every call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (on different streams or host threads) race and must be ordered by the caller; nothing is
 * carried from one call to the next.  Asynchronous on `stream`.
 * The workspace is 8 N nrhs + 16 ncl n_x nrhs bytes, plus 1024 (nleaf + owned blocks) with one
 * rhs or 2 N nrhs with several, each part rounded up to 256 bytes (ncl clusters, nleaf leaves,
 * owned blocks as reported by dwfmm_tree_info / dwfmm_tree_stats).  An operator's stored
 * nearfield tiles (cache_near) are its own memory and are used as by dwfmm_fmm_matvec.
 * Errors: E_INVALID (NULL or equal x/y, nrhs out of range, another device current, or a
 * workspace above DWFMM_STATIC_SCRATCH_BYTES, with the sizes in the message), E_HIP.       */
#define DWFMM_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
dwfmm_status dwfmm_fmm_matvec_static(dwfmm_op op, const double *x, double *y, int32_t nrhs, void *stream);
/* Same as dwfmm_fmm_matvec restricted to parts of the operator (bit 0 nearfield,
 * bit 1 farfield), and with an explicit precision (dwfmm_precision), for
 * stage-by-stage checks.                                                        */
dwfmm_status dwfmm_fmm_matvec_parts(dwfmm_op op, const double *x, double *y, int32_t nrhs, int32_t parts,
                                    int32_t precision, void *stream);

/* Solve (K~ + lambda I) alpha = f by conjugate gradients (eq. (LGS)), one
 * independent iteration per column.  alpha is the start vector on entry and
 * the solution on return.  Stops a column when |r| <= rtol |f| (recursive
 * residual), checked every opts.check_every iterations.  Steps with
 * p^T A p < 0 are taken and counted.  In FP32/BF16 operator precision the
 * solve is iterative refinement: an FP64 residual f - (K~ + lambda I) alpha,
 * an inner CG in reduced precision, alpha += delta; a correction that raises the
 * FP64 residual is taken back and its column stops (NOT_CONVERGED) at the lowest
 * residual it reached.  info: host, nrhs entries.
 * Synchronises `stream`.  Returns the worst per-column status.
 * Errors: E_INVALID, E_HIP, E_NOT_CONVERGED, E_BREAKDOWN.                       */
dwfmm_status dwfmm_fmm_solve(dwfmm_op op, double lambda, const double *f, double *alpha, int32_t nrhs,
                             double rtol, int32_t max_iter, void *stream, dwfmm_solve_info *info);

/* ---- batches of independent problems --------------------------------------
 * A batch runs one matvec (one rhs each) of many operators with one launch per
 * kernel variant and tree level across all of them (work lists of (problem, block)
 * pairs), so that many small problems fill the GPU together.  Operators with a
 * polynomial kernel, leaves above 128 points, d > 32 or n_x > 64 are run one by
 * one inside the same call.  Each problem uses its operator's precision and
 * workspace: do not run an operator alone while its batch runs.  The operators
 * must outlive the batch.
 *   ops    host array of count operators (count >= 1)
 *   flags  DWFMM_BATCH_GRAPH: capture the batched launches as one HIP graph at
 *          creation and replay it on every call
 *          DWFMM_BATCH_TUNE: before any capture, time every compiled tile shape of
 *          each M2L launch (waves per target cluster: 4, 2, or 1 when n_x <= 32;
 *          4 / waves clusters per 256-thread workgroup) on this batch and keep the
 *          fastest.  All shapes split a cluster's farfield list into the same four
 *          classes and add the class sums in the same order, so the choice never
 *          changes a result bit.  Tuning runs M2L on the operators' current moments
 *          (its output is overwritten by the next matvec).
 *          DWFMM_BATCH_M2L_WAVES(w), w in {1, 2, 4}: use w waves per cluster in every
 *          M2L launch where that shape is compiled (else 4); ignored with TUNE.
 *          Default: 4 waves per cluster.
 *          DWFMM_BATCH_M2L_PERSISTENT: every M2L launch is one persistent grid (1024
 *          workgroups, 4 per CU) striding over its whole work list instead of one
 *          workgroup per 4 / waves clusters; with TUNE both layouts of every shape are
 *          timed.  The layout never changes a bit of the result.
 * Synchronises `stream`.  Errors: E_INVALID (also unknown flag bits), E_NOMEM, E_HIP. */
typedef struct dwfmm_batch_s *dwfmm_batch;
#define DWFMM_BATCH_GRAPH 1
#define DWFMM_BATCH_TUNE 2
#define DWFMM_BATCH_M2L_PERSISTENT 4
#define DWFMM_BATCH_M2L_WAVES(w) ((w) << 4)
dwfmm_status dwfmm_batch_create(const dwfmm_op *ops, int32_t count, int32_t flags, void *stream, dwfmm_batch *out);
/* The batch's M2L launches: *count = their number; for i < min(count, cap), wpc[i] = the
 * waves per cluster launch i uses and, if ms is not NULL, ms[3 i + j] = its tuned time in
 * milliseconds with 4, 2 and 1 waves (j = 0, 1, 2; -1 where not timed).  Host arrays.
 * Errors: E_INVALID. */
dwfmm_status dwfmm_batch_m2l_shapes(dwfmm_batch batch, int32_t *wpc, double *ms, int32_t cap, int32_t *count);
/* The layout of the batch's M2L launches: *count = their number; for i < min(count, cap),
 * grid[i] = 0 when launch i uses one workgroup per 4 / waves clusters, else the size of its
 * persistent grid; if ms is not NULL, ms[3 i + j] = the tuned time of the persistent layout
 * with 4, 2 and 1 waves (-1 where not timed).  Host arrays.  Errors: E_INVALID.           */
dwfmm_status dwfmm_batch_m2l_layout(dwfmm_batch batch, int32_t *grid, double *ms, int32_t cap, int32_t *count);
/* y_i = K~_i x_i for every problem i.  xs, ys: host arrays of count device pointers
 * (N_i x 1 each, caller order, x_i != y_i).  Asynchronous on `stream`; allocates nothing. */
dwfmm_status dwfmm_batch_matvec(dwfmm_batch batch, const double *const *xs, double *const *ys, void *stream);
/* Solve (K~_i + lambda I) alpha_i = f_i (eq. (LGS)) for every problem of the batch at once:
 * one CG iteration per problem in lockstep, each iteration one batched matvec (the batch's
 * plan, or a plan over the problems still iterating once they are at most half of it) and
 * one launch per CG vector step for all problems.  Per problem the arithmetic is that of
 * dwfmm_fmm_solve with one rhs on its operator, so each alpha_i, its iteration count and its
 * residuals are bitwise those of solving problem i alone.  All operators must share one
 * precision: FP64 runs CG; FP32/BF16 runs the iterative refinement of dwfmm_fmm_solve with
 * the operators' refinement options (FP64 residuals on an FP64 plan of the same problems,
 * built at the first such call and kept with the batch).  The solve uses each operator's
 * CG workspace (max_nrhs >= 1 suffices).
 *   fs, alphas  host arrays of count device pointers, N_i x 1 each, caller order; alpha_i
 *               is the start vector on entry and the solution on return; alpha_i != f_i
 *   check_every iterations between reads of the problems' states (each read synchronises)
 *   infos       host array of count entries
 * Synchronises `stream`.  Returns the worst per-problem status.
 * Errors: E_INVALID (also mixed precisions), E_NOMEM, E_HIP, E_NOT_CONVERGED, E_BREAKDOWN. */
dwfmm_status dwfmm_batch_solve(dwfmm_batch batch, double lambda, const double *const *fs, double *const *alphas,
                               double rtol, int32_t max_iter, int32_t check_every, void *stream,
                               dwfmm_solve_info *infos);
void dwfmm_batch_destroy(dwfmm_batch batch);

/* ---- evaluation at new points ------------------------------------------------
 * y_i = sum_j K~(t_i, x_j) x_j at targets t_i other than the data sites (the
 * interpolant of a solved alpha at new points).  The targets get a tree of the
 * source tree's depth built by the same rules (Sec 5.1; clusters may be empty);
 * target and source clusters of equal level are paired with the same admissibility
 * (Sec 5.2): farfield blocks are interpolated in both variables with the operator's
 * index set and nodes on the target clusters' own boxes, nearfield leaf pairs are
 * summed directly.  With the data sites as targets it is the operator's matvec.
 *   op       source operator; must outlive the plan; the plan uses the operator's
 *            charge and moment workspace, so the two must not run concurrently
 *   targets  device, m x d row-major, copied at creation (1 <= m <= 2^30)
 * Synchronises `stream`.  Errors: E_INVALID, E_NONFINITE, E_NOMEM, E_HIP.        */
typedef struct dwfmm_eval_s *dwfmm_eval;
dwfmm_status dwfmm_eval_create(dwfmm_op op, const double *targets, int64_t m, void *stream, dwfmm_eval *out);
/* y (device, m x nrhs, target order) = K~(targets, sources) x (device, N x nrhs, caller
 * order), 1 <= nrhs <= the operator's max_nrhs.  Asynchronous on `stream`. */
dwfmm_status dwfmm_eval_apply(dwfmm_eval ev, const double *x, double *y, int32_t nrhs, void *stream);
/* out[0..4] = m, J, clusters, farfield blocks, nearfield blocks. */
dwfmm_status dwfmm_eval_info(dwfmm_eval ev, int64_t *out);
/* Host copies of the target tree and the cross lists: perm[m], begin/end[ncl],
 * lo/hi[ncl*d], Fptr[ncl+1], Fsrc[nF] (source clusters), Nptr[ncl+1], Nsrc[nN]
 * (source clusters); any pointer may be NULL. */
dwfmm_status dwfmm_eval_tree_get(dwfmm_eval ev, int64_t *perm, int64_t *begin, int64_t *end, double *lo, double *hi,
                                 int64_t *Fptr, int64_t *Fsrc, int64_t *Nptr, int64_t *Nsrc);
void dwfmm_eval_destroy(dwfmm_eval ev);

/* ---- solve server (continuous batching) ------------------------------------
 * Requests solve (K~ + lambda I) alpha = f (eq. (LGS)) by FP64 CG from alpha = 0, one
 * rhs each.  Waiting requests are handed, first come first served, to a pool of host
 * threads (each with its own non-blocking stream) while a slot is free and the device
 * bytes they will hold fit the budget (a request is always taken when nothing else holds
 * memory); a thread builds the request's tree, operator and CG start and waits for its
 * own stream.  A tick makes the prepared requests active, runs one batched matvec over
 * every active request on `stream`, one CG update per request (scalars on the device),
 * and every check_every ticks (or when a request used max_iter) synchronises `stream`
 * and retires the requests that converged, broke down or used max_iter: their alpha is
 * copied to the host and their device memory freed.  That check is the only point where
 * a tick waits for the device, except that a tick with nothing active waits for the
 * first prepared request.  A request whose setup fails is finished with that status.
 * Server calls must come from one host thread at a time.                          */
typedef struct dwfmm_server_s *dwfmm_server;
typedef struct {
    int64_t n;                  /* points, >= 1 */
    int32_t d;                  /* 1..64 */
    const double *points;       /* host, n x d row-major (copied at submit) */
    const double *dim_weights;  /* host, d values b_k > 0 */
    const double *f;            /* host, n data values (copied at submit) */
    int32_t leaf_size;          /* 1..1024 */
    double eta;                 /* > 0 */
    dwfmm_kernel kernel;
    double q;                   /* >= 0 */
    double lambda;              /* >= 0 */
    double rtol;                /* > 0 */
    int32_t max_iter;           /* >= 0 */
    int32_t precision;          /* dwfmm_precision of the matvec inside CG (no refinement: a
                                   reduced-precision request converges to its operator's accuracy and
                                   is reported E_NOT_CONVERGED when its FP64 true residual stays above
                                   rtol) */
} dwfmm_request;
dwfmm_status dwfmm_server_create(size_t budget_bytes, int32_t max_active, int32_t check_every, void *stream,
                                 dwfmm_server *out);
/* Queue a request; *id identifies it.  Errors: E_INVALID, E_NOMEM. */
dwfmm_status dwfmm_server_submit(dwfmm_server server, const dwfmm_request *request, int64_t *id);
/* One scheduling step (admission, batched matvec, CG updates, retirement).
 * *n_queued counts requests waiting or being prepared. */
dwfmm_status dwfmm_server_tick(dwfmm_server server, int32_t *n_active, int32_t *n_queued);
/* If request id has finished: *done = 1, alpha (host, n values, may be NULL) and info are
 * filled and the request is forgotten; otherwise *done = 0.  times (host, 4 values, may be
 * NULL): seconds since the server's creation at which the request was submitted, handed to a
 * preparation thread (the end of its wait for a slot and memory), made active (preparation
 * done) and retired (alpha on the host). */
dwfmm_status dwfmm_server_result(dwfmm_server server, int64_t id, double *alpha, dwfmm_solve_info *info,
                                 double *times, int32_t *done);
/* Requests finished and not yet collected by dwfmm_server_result: *count = their number,
 * ids[0 .. min(count, cap)) their ids (host array), in retirement order.  Errors: E_INVALID. */
dwfmm_status dwfmm_server_finished(dwfmm_server server, int64_t *ids, int32_t cap, int32_t *count);
/* Host-side accounting of the ticks so far: out[0..5] = ticks that ran work, batch-plan rebuilds,
 * and the seconds the ticks spent rebuilding plans, launching their work, waiting for the
 * device at checks, and retiring requests (residual, alpha to the host, release).  Host array
 * of 6.  Errors: E_INVALID. */
dwfmm_status dwfmm_server_stats(dwfmm_server server, double *out);
/* Device bytes counted against the budget (requests being prepared or active). */
size_t dwfmm_server_bytes(dwfmm_server server);
void dwfmm_server_destroy(dwfmm_server server);

/* Device bytes a tree plus operator would hold for the given sizes, from the sizes alone: an
 * estimate (the nearfield column sums, 1 KiB per owned leaf pair, are counted at 128 owned
 * pairs per leaf; the true count depends on the geometry).  The solve server reserves this
 * for a request first and re-checks with dwfmm_op_bytes_for once the request's tree is built. */
size_t dwfmm_estimate_bytes(int64_t n, int32_t d, int32_t leaf_size, int32_t n_x, int32_t nrhs);
/* Device bytes held by a tree plus operator. */
size_t dwfmm_op_bytes(dwfmm_op op);
/* Exactly the device bytes dwfmm_op_bytes will report for dwfmm_fmm_create(tree, kernel, q,
 * opts) on this tree (any kernel), computed on the host before anything is allocated; 0 for
 * invalid arguments or an index set that cannot be built.                               */
size_t dwfmm_op_bytes_for(dwfmm_tree tree, double q, const dwfmm_opts *opts);

void dwfmm_op_destroy(dwfmm_op op);
/* Destroying a tree that an operator still references is deferred until that operator is destroyed. */
void dwfmm_tree_destroy(dwfmm_tree tree);

/* Message for the last non-OK status returned on the calling thread. */
const char *dwfmm_last_error(void);

/* ---- introspection (host copies; for tests and statistics) ---------------- */
/* out[0..7] = n, d, J, ncl (clusters), nF (farfield blocks), nN (nearfield blocks), nleaf, leaf_size */
dwfmm_status dwfmm_tree_info(dwfmm_tree tree, int64_t *out);
/* Nearfield list statistics: out[0..2] = the most blocks one leaf owns in the symmetric
 * nearfield (its self block plus the unordered pairs dealt to it), the longest nearfield
 * list of a leaf, and the number of owned blocks.  Host values; E_INVALID on NULL.    */
dwfmm_status dwfmm_tree_stats(dwfmm_tree tree, int64_t *out);
/* The order in which the symmetric nearfield takes the owner leaves (workgroup q runs on XCD
 * q mod 8: 8 contiguous leaf segments of equal nearfield work, segment k on XCD k, costliest leaf
 * first within a segment, -1 padding the shorter segments): *count = its length; order (host, may
 * be NULL) receives min(count, cap) entries; work (host, may be NULL, nleaf entries) the nearfield
 * work of each leaf (owned-block entries plus 128 per point).  Errors: E_INVALID, E_HIP. */
dwfmm_status dwfmm_tree_leaf_order(dwfmm_tree tree, int32_t *order, double *work, int32_t cap, int32_t *count);
/* Tree order and boxes: perm[n] (tree position -> original index), begin/end[ncl],
 * lo/hi[ncl*d]; farfield CSR by target cluster Fptr[ncl+1], Fsrc[nF]; nearfield
 * CSR by target cluster Nptr[ncl+1], Nsrc[nN].  Any pointer may be NULL.      */
dwfmm_status dwfmm_tree_get(dwfmm_tree tree, int64_t *perm, int64_t *begin, int64_t *end, double *lo, double *hi,
                            int64_t *Fptr, int64_t *Fsrc, int64_t *Nptr, int64_t *Nsrc);
/* out[0..6] = n_x, max_nrhs, precision, bytes, then 1 when the FP64 Gaussian nearfield runs
 * split into row, column and cross factors (every nearfield exponent bounded by 600), and 1
 * when the FP32/BF16 one does (bounded by 80), else 0; then the stored nearfield tiles
 * (cache_near): 0 none, 1 allocated and not yet written (the next eager BF16 matvec with
 * nrhs > 1 writes them), 2 written (later ones read them).  out: host, 7 values. */
dwfmm_status dwfmm_op_info(dwfmm_op op, int64_t *out);
/* Index set alpha[n_x*d] (uint8), reference nodes xi[n_x*d], Vinv[n_x*n_x], omega[d]. */
dwfmm_status dwfmm_op_basis(dwfmm_op op, uint8_t *alpha, double *xi, double *Vinv, double *omega);
/* Sampled Lebesgue constant of the operator's nodes (Sec 5.4, the constant
 * max_x sum_a |l_a(x)| over [0,1]^d of the Lagrange basis l = V^-T p): the largest
 * value over the corners x = (0,...,0) and (1,...,1) and the Halton points 1..n_samples
 * (r-th prime base on the r-th axis with m_k > 0, 1/2 on the others; the candidate
 * sequence of the approximate Fekete points).  A lower bound of the constant; host
 * work of n_samples * n_x^2 operations.  out: host, one double.
 * Errors: E_INVALID (NULL op/out, n_samples outside [0, 1e8]).                        */
dwfmm_status dwfmm_op_lebesgue(dwfmm_op op, int64_t n_samples, double *out);
/* Kernel timing for measurement: while enabled, each matvec records HIP events
 * on its stream around the nearfield (P2P) and coupling (M2L) launches.  out
 * (host, 3 doubles, may be NULL) receives the summed P2P ms, summed M2L ms and
 * the number of timed matvecs since the last call; the call then resets the
 * count and sets timing on (enable != 0) or off.  Waits for the recorded events. */
dwfmm_status dwfmm_op_timing(dwfmm_op op, int32_t enable, double *out);
/* Lagrange moments and locals of the last matvec, host [ncl][n_x][nrhs]. */
dwfmm_status dwfmm_op_moments(dwfmm_op op, double *moments, double *locals, int32_t nrhs);

#ifdef __cplusplus
}
#endif
#endif
