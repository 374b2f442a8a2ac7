// Device-side data of a tree and an operator, and the launchers of the HIP
// kernels that make up one matvec and the CG solver.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <utility>
#include <vector>

namespace dwfmm {

// Everything the kernels read about the geometry (device pointers).
struct DevTree {
    int n, d, J, dpad;
    int nleaf, ncl, leaf_first;   // leaf_first = 2^J - 1
    int max_leaf;                 // largest leaf size
    int min_far_level;            // J+1 when there is no farfield
    const double *Xs;             // [dpad][n] coordinates in tree order (rows k >= d are zero)
    const int32_t *perm;          // [n] tree position -> original index
    const int32_t *cbeg, *cend;   // [ncl]
    const int32_t *Fptr, *Fsrc;   // farfield CSR over clusters
    const int32_t *Nptr, *Nsrc;   // nearfield CSR over leaves (leaf-local indices)
    // Symmetric nearfield: every unordered leaf pair {t, s}, t != s, is owned by one of
    // its two leaves (balanced); the owner evaluates the block once and applies it both
    // ways.  own: CSR over owner leaves of partner leaves, block id = CSR position.
    // inc: CSR over partner leaves of the block ids whose column sums they receive.
    int nblk;                     // number of owned blocks of the symmetric nearfield (self blocks included)
    const int32_t *own_ptr, *own_src, *inc_ptr, *inc_blk;
    const double *center;         // [nleaf][dpad] leaf box midpoints (coordinate shift)
    // Order in which the symmetric nearfield launches take the owner leaves: workgroup q runs on
    // XCD q % 8, and XCD k gets the k-th of 8 contiguous leaf segments of equal nearfield work,
    // costliest leaf first; -1 pads the shorter segments.  NULL for trees without a symmetric nearfield.
    const int32_t *leaf_order;
    int n_order;
    // The same for the several-rhs nearfield, which sweeps each target leaf's whole nearfield list:
    // segments of equal list entries, costliest leaf first; near_order_seq has the same segments in
    // leaf order (the launches that read stored BF16 tiles, whose sources then stay in L2).
    const int32_t *near_order;
    const int32_t *near_order_seq;
    int n_near_order;
};

struct DevOp {
    int kind;
    double ell;
    int nx, max_nrhs;
    const double *nodes;          // [ncl][nx][dpad] interpolation nodes of every box
    const double *E;              // [ncl][nx][nx] Lagrange transfer matrices (row a, column b)
    const double *Lb;             // [nx][n] Lagrange basis l_a(a_leaf^-1 x_i), tree order
    double *xt;                   // [n][max_nrhs] x in tree order
    __bf16 *xtb;                  // [n][nrhs] the same charges rounded to BF16 through FP32 (max_nrhs > 1)
    double *M, *L;                // [ncl][nx][max_nrhs] moments and locals
    int nxp;                      // nx rounded up to a multiple of 16
    const double *nodesT;         // [ncl][dk][nxp] nodes, axis-major, zero padded (dk = d rounded up to 4)
    const double *nnorm;          // [ncl][nxp] squared norms of the nodes, zero padded
    double *rowbuf;               // [nleaf][128] owner-side nearfield row sums (one rhs)
    double *colbuf;               // [nblk][128] column sums of owned blocks (one rhs)
    // Gaussian only: every nearfield exponent |x - c|^2 / ell, |y - c|^2 / ell, 2 (x - c).(y - c) / ell
    // (c the owner leaf's midpoint) is at most 600 in magnitude, so the symmetric FP64 nearfield may
    // evaluate exp(-|x-y|^2/ell) = exp(-|x-c|^2/ell) exp(-|y-c|^2/ell) exp(2 (x-c).(y-c)/ell).
    int gauss_split;
    int gauss_split32;            // the same with every exponent within 80 (the FP32 nearfield)
    // Matern only: sqrt(3) max|x - y| / ell log2(e) <= 1000 over the nearfield (from the host's reach
    // bound), so the FP64 nearfield's 2^-s log2(e) needs no underflow clamp
    int matern_in_range;
    // Power of two 2^-e with every centred nearfield coordinate (a point minus its target leaf's
    // midpoint) at most 1 in magnitude after scaling (e from the host's reach bound): the BF16
    // several-rhs nearfield forms its FP16 Gram operands from the scaled coordinates
    float hscale;
    // Tile cache of the BF16 several-rhs nearfield (NULL when off): column tile t of target leaf l
    // (16 stream columns x 8 row tiles of 16 targets, 64 lanes x 4 BF16 each, 4 KiB) sits at
    // near_tiles + (near_tile_off[l] + t) * 512; near_filled points at a host flag set once a
    // launch has written the tiles; near_cache_mode is chosen per launch (0 off, 1 compute and
    // write, 2 read).
    uint2 *near_tiles;
    const int64_t *near_tile_off;
    int *near_filled;
    int near_cache_mode;
};

// Optional HIP events recorded around the nearfield (P2P) and coupling (M2L)
// launches, on the stream they run on.
struct KernelTimer {
    hipEvent_t p2p_start = nullptr, p2p_stop = nullptr, m2l_start = nullptr, m2l_stop = nullptr;
};

// A second stream and two events with which the farfield (M2M, M2L, L2L) of a one-rhs matvec
// runs beside the symmetric nearfield: forked after P2M, joined before the combine.
struct StreamFork {
    hipStream_t side = nullptr;
    hipEvent_t forked = nullptr, joined = nullptr;
};

// One matvec (or parts of it) on `stream` (with `fork`, partly on its side stream; the result
// is ordered on `stream` as without it).  parts: bit0 nearfield, bit1 farfield.
hipError_t launch_matvec(const DevTree &T, const DevOp &O, const double *x, double *y, int nrhs, int parts,
                         int precision, hipStream_t stream, const KernelTimer *timer = nullptr,
                         const StreamFork *fork = nullptr);

// Evaluation at new points: y (targets, caller order) = K~(targets, sources) x (sources, caller
// order).  Tt/Ot: the target tree (cross farfield/nearfield lists naming source clusters and
// leaves) and the target side (box nodes, transfer matrices, basis at the targets, locals);
// Ts/Os: the source tree and operator, whose charge and moment workspace it uses.
hipError_t launch_eval(const DevTree &Tt, const DevOp &Ot, const DevTree &Ts, const DevOp &Os, const double *x,
                       double *y, int nrhs, hipStream_t stream);

// Lagrange basis cache Lb from the boxes and the index set (setup).
hipError_t launch_basis(const DevTree &T, int nx, const double *clo, const double *csc, const double *coff,
                        const int32_t *lidx, int nnz_max, const double *Vinv, int nleg, const int32_t *leg_axis,
                        const int32_t *leg_deg, double *Lb, hipStream_t stream);

// ---- batches of independent problems (one rhs each) ----
struct BatchItem {
    DevTree T;
    DevOp O;
    int far;        // the problem has a farfield
    int precision;  // 0 FP64, 1/2 FP32 nearfield and coupling
};

// One launch of a templated kernel over a slice of the work list.  wpc (M2L only): waves per
// target cluster, 4, 2 or 1; every choice gives bitwise the same locals.
struct BatchLaunch {
    int kind, dk, nxt, prec, off, cnt;
    int wpc = 4;
    int grid = 0;  // M2L: 0 = one workgroup per 4 / wpc list entries; > 0 = a persistent grid of
                   // this many workgroups striding over the list
};
constexpr int kM2lPersistentGrid = 1024;  // 4 workgroups per CU on 256 CUs

// Work list entries are (item, local block); entries with item < 0 are padding.
struct BatchPlan {
    const BatchItem *items = nullptr;
    const double *const *xs = nullptr;
    double *const *ys = nullptr;
    const int2 *work = nullptr;
    int leaf_off = 0, leaf_cnt = 0;
    std::vector<std::pair<int, int>> m2m, l2l;  // (offset, count) per level in launch order
    std::vector<BatchLaunch> m2l, p2p;
};

// With `fork`, the farfield stages run on its side stream beside the nearfield (same bits).
hipError_t launch_batch_matvec(const BatchPlan &P, hipStream_t stream, const StreamFork *fork = nullptr);
// Waves per cluster compiled for an M2L launch with nxt node tiles: 1 only up to two tiles
// (its per-lane accumulators grow with 4 / wpc x nxt).
inline bool m2l_wpc_available(int nxt, int wpc) { return wpc == 4 || wpc == 2 || (wpc == 1 && nxt <= 2); }
// One M2L launch of the plan on its own (the tile-shape tuner times these).
hipError_t launch_batch_m2l(const BatchPlan &P, const BatchLaunch &L, hipStream_t stream);

// ---- CG building blocks (FP64, deterministic fixed-order reductions) ----
// partial[b][c] for b < kDotBlocks (the grid grows with n nrhs up to that); out[c] = sum_b partial[b][c]
// by a fixed-order tree, so a result depends only on n, nrhs and the inputs.
constexpr int kDotBlocks = 1024;
hipError_t launch_dot(const double *a, const double *b, int n, int nrhs, double *partial, double *out,
                      hipStream_t stream);

// ---- FP64 CG for problems with one right-hand side, any number of them per launch ----
// One problem of a CG launch: CG on (K~ + lambda I) x = b, with A p (or A x) already in q when
// a step needs it.  The inner products of a problem are taken over nblk blocks of chunk rows
// (nblk = min(kDotBlocks, ceil(n / 4096)), the grid launch_dot uses for one column) and summed in
// the same fixed order as launch_dot, so a problem's iterates do not depend on what else the
// launch carries.  scal: [0] |r|^2, [1] |b|^2, [2] p.Ap, [3] new |r|^2, [4] step, [5] beta,
// [8] |out|^2 of the residual step; state: [0] 0 active, 1 converged, 2 breakdown, 3 frozen,
// [1] iterations, [2] steps with p.Ap < 0.
struct CgItem {
    double *x, *r, *p, *q;
    const double *b;
    // residual step: out = f - (out + lambda v) with K~ v already in out; add step: acc += x
    const double *f, *v;
    double *out, *acc;
    double *partial;          // [2][kDotBlocks]
    double *scal;
    int32_t *state;
    double lambda, rtol;
    int n, nblk, chunk, blk0;  // blk0: first block of the problem in the launch's block numbering
    int max_it;                // the problem takes no step once state[1] reaches max_it
    int frozen;                // start: the problem starts frozen; residual and add steps skip it
    int zero_x;                // start: x = 0 and q = 0 (= K~ 0) instead of reading them
    double *mirror;            // mirror step: state[0..2], scal[0], scal[1], scal[8], scal[9] (8 doubles)
};
enum CgStep {
    CG_START,      // blocks: q += lambda x, r = b - q, p = r; partial |r|^2 and |b|^2
    CG_START_SUM,  // problems: |r|^2, |b|^2, state (frozen or active), convergence check
    CG_PQ,         // blocks: q += lambda p; partial p.q
    CG_ALPHA,      // problems: p.q, step a = |r|^2 / p.q (breakdown, negative curvature)
    CG_XR,         // blocks: x += a p, r -= a q; partial |r|^2
    CG_BETA,       // problems: new |r|^2, beta, iteration count, convergence check
    CG_P,          // blocks: p = r + beta p
    CG_RES,        // blocks: out = f - (out + lambda v); partial |out|^2
    CG_RES_SUM,    // problems: |out|^2 into scal[8]
    CG_ADD,        // blocks: acc += x
    CG_SUB,        // blocks: acc -= x
    CG_MIRROR      // problems: copy state and scalars to mirror, for one host read of many problems
};
inline int cg_blocks(int n) { return (int)std::max<int64_t>(1, std::min<int64_t>(kDotBlocks, ((int64_t)n + 4095) / 4096)); }
// One step for `nitems` problems (device array `items`, blk0 ascending, nblocks blocks in all),
// or, with items == nullptr, for the single problem `one` passed by value.
hipError_t launch_cg(int step, const CgItem *items, int nitems, int nblocks, const CgItem &one, hipStream_t stream);

}  // namespace dwfmm
