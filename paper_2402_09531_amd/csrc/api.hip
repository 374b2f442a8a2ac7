// C ABI of libdwfmm.so (declared in include/dwfmm.h): object lifetime, uploads,
// argument checks, and the conjugate gradient driver (Sec 2, eq. (LGS)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/dwfmm.h"
#include "device.hpp"
#include "setup.hpp"

using namespace dwfmm;

namespace {

thread_local std::string g_err;

dwfmm_status fail(dwfmm_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

// All device allocations of an object, freed together.
struct Arena {
    std::vector<DevBuf> bufs;
    size_t total = 0;
    hipError_t alloc(void **out, size_t bytes)
    {
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, std::max<size_t>(bytes, 256));
        if (e != hipSuccess) return e;
        bufs.push_back({p, bytes});
        total += bytes;
        *out = p;
        return hipSuccess;
    }
    template <class T>
    hipError_t upload(T **out, const std::vector<T> &v, hipStream_t st)
    {
        hipError_t e = alloc((void **)out, v.size() * sizeof(T));
        if (e != hipSuccess) return e;
        if (!v.empty()) e = hipMemcpyAsync(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st);
        return e;
    }
    void release()
    {
        for (auto &b : bufs) (void)hipFree(b.p);
        bufs.clear();
        total = 0;
    }
};

#define HIP_TRY(expr)                                                                             \
    do {                                                                                          \
        hipError_t _e = (expr);                                                                   \
        if (_e != hipSuccess) {                                                                   \
            return fail(_e == hipErrorOutOfMemory ? DWFMM_E_NOMEM : DWFMM_E_HIP,                  \
                        std::string(#expr) + ": " + hipGetErrorString(_e));                       \
        }                                                                                         \
    } while (0)

// coordinate rows stored per point: a multiple of 4 (the MFMA k-chunk) up to 32, of 8 beyond
int pad_dim(int d) { return d <= 32 ? (d + 3) / 4 * 4 : (d + 7) / 8 * 8; }

}  // namespace

// Host arrays of a tree built but not yet uploaded (the tree's device arrays, in upload order).
struct TreeStage {
    std::vector<double> Xs, clo, csc, coff, center;
    std::vector<int32_t> nsrc_local, nptr_leaf, own_ptr, own_src, inc_ptr, inc_blk, leaf_order, near_order,
        near_order_seq;
    int max_leaf = 0;
};

struct dwfmm_tree_s {
    HostTree H;
    std::unique_ptr<TreeStage> stage;  // between the host build and the upload
    DevTree D{};
    Arena arena;
    double *clo = nullptr, *csc = nullptr, *coff = nullptr;  // [ncl][d] reference-coordinate maps
    // max over nearfield leaf pairs (t, s) of (R_t + |c_s - c_t| + R_s)^2, R the half diagonal and
    // c the midpoint of a leaf box: bounds every squared shifted distance the nearfield forms
    double near_reach2 = 0.0;
    int64_t own_max = 0, own_total = 0, near_max = 0;  // symmetric-nearfield ownership statistics
    std::vector<double> leaf_work;  // nearfield work of each owner leaf (entries of its owned blocks + 128 per point)
    int refs = 1;       // the caller's reference plus one per operator
    bool destroyed = false;
    int device = 0;
};

struct dwfmm_op_s {
    dwfmm_tree tree = nullptr;
    HostBasis B;
    DevOp D{};
    Arena arena;
    int precision = 0, max_nrhs = 1, check_every = 1, ir_max_outer = 30, ir_max_inner = 0;
    double ir_inner_rtol = 0.0;
    void (*progress)(void *, int32_t, int32_t, const double *) = nullptr;
    void *progress_ctx = nullptr;
    // basis tables on the device (Legendre slots, their products, V^-1), kept for evaluation plans
    int32_t *b_lidx = nullptr, *b_la = nullptr, *b_ld = nullptr;
    double *b_Vinv = nullptr;
    int b_nnz = 0, b_nleg = 0;
    // CG workspace
    double *r = nullptr, *p = nullptr, *q = nullptr, *partial = nullptr, *scal = nullptr;
    double *ir_r = nullptr, *ir_d = nullptr;  // refinement: outer residual and correction
    int32_t *state = nullptr;
    // kernel timing: one event pair per timed matvec, summed when read
    bool timing = false;
    std::vector<KernelTimer> timers;
    size_t timers_used = 0;
    StreamFork fork;  // farfield beside the one-rhs nearfield
    int near_filled = 0;  // the BF16 nearfield tile cache holds this operator's tiles
    ~dwfmm_op_s()
    {
        if (fork.forked) (void)hipEventDestroy(fork.forked);
        if (fork.joined) (void)hipEventDestroy(fork.joined);
        if (fork.side) (void)hipStreamDestroy(fork.side);
        for (auto &t : timers) {
            (void)hipEventDestroy(t.p2p_start);
            (void)hipEventDestroy(t.p2p_stop);
            (void)hipEventDestroy(t.m2l_start);
            (void)hipEventDestroy(t.m2l_stop);
        }
    }
};

static void tree_release(dwfmm_tree t)
{
    if (--t->refs == 0) {
        t->arena.release();
        delete t;
    }
}

// ============================================================== build_tree
static dwfmm_status tree_from_host(const std::vector<double> &pts, int64_t n, int32_t d, const double *dim_weights,
                                   int32_t leaf_size, double eta, hipStream_t st, dwfmm_tree *out, int adm_half);

extern "C" dwfmm_status dwfmm_build_tree(const double *points, int64_t n, int32_t d, const double *dim_weights,
                                         int32_t leaf_size, double eta, void *stream, dwfmm_tree *out)
{
    return dwfmm_build_tree_ex(points, n, d, dim_weights, leaf_size, eta, DWFMM_ADM_FULL_DIAGONAL, stream, out);
}

extern "C" dwfmm_status dwfmm_build_tree_ex(const double *points, int64_t n, int32_t d, const double *dim_weights,
                                            int32_t leaf_size, double eta, dwfmm_admissibility admissibility,
                                            void *stream, dwfmm_tree *out)
{
    if (!out) return fail(DWFMM_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!points || !dim_weights) return fail(DWFMM_E_INVALID, "points or dim_weights is NULL");
    if (n < 1 || n > (int64_t)1 << 30) return fail(DWFMM_E_INVALID, "n must be in [1, 2^30]");
    if (d < 1 || d > kMaxDim) return fail(DWFMM_E_INVALID, "d must be in [1, 64]");
    if (leaf_size < 1 || leaf_size > 1024) return fail(DWFMM_E_INVALID, "leaf_size must be in [1, 1024]");
    if (!(eta > 0.0) || !std::isfinite(eta)) return fail(DWFMM_E_INVALID, "eta must be finite and > 0");
    if (admissibility != DWFMM_ADM_FULL_DIAGONAL && admissibility != DWFMM_ADM_HALF_DIAGONAL)
        return fail(DWFMM_E_INVALID, "unknown admissibility rule");
    for (int k = 0; k < d; ++k) {
        if (!std::isfinite(dim_weights[k])) return fail(DWFMM_E_NONFINITE, "dim_weights not finite");
        if (!(dim_weights[k] > 0.0)) return fail(DWFMM_E_INVALID, "dim_weights must be > 0");
    }
    hipStream_t st = (hipStream_t)stream;
    std::vector<double> pts((size_t)n * d);
    HIP_TRY(hipMemcpyAsync(pts.data(), points, pts.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return tree_from_host(pts, n, d, dim_weights, leaf_size, eta, st, out, (int)admissibility);
}

// Launch order of the leaves of a nearfield kernel with per-leaf work w: workgroup q runs on XCD
// q mod 8, so the leaves are cut into 8 contiguous segments of equal work, segment k dealt to XCD
// k (each XCD's L2 then holds the sources of one region of the tree), the costliest leaves first
// within a segment (it ends on short ones) or, with by_cost false, in leaf order (neighbouring
// leaves, which list mostly the same sources, then run at the same time); -1 pads the shorter
// segments.
static std::vector<int32_t> xcd_order(const std::vector<double> &w, bool by_cost = true)
{
    const int64_t nl = (int64_t)w.size();
    double total = 0.0;
    for (double v : w) total += v;
    std::vector<int64_t> cut(9, nl);
    cut[0] = 0;
    double acc = 0.0;
    for (int64_t l = 0, k = 1; l < nl && k < 8; ++l) {
        acc += w[l];
        while (k < 8 && acc >= total * k / 8.0) cut[k++] = l + 1;
    }
    int64_t longest = 0;
    for (int k = 0; k < 8; ++k) longest = std::max(longest, cut[k + 1] - cut[k]);
    std::vector<int32_t> order(8 * longest, -1);
    for (int k = 0; k < 8; ++k) {
        std::vector<int32_t> seg;
        for (int64_t j = cut[k]; j < cut[k + 1]; ++j) seg.push_back((int32_t)j);
        if (by_cost) std::stable_sort(seg.begin(), seg.end(), [&](int32_t a, int32_t b) { return w[a] > w[b]; });
        for (size_t j = 0; j < seg.size(); ++j) order[8 * j + k] = seg[j];
    }
    return order;
}

// Tree from host points (arguments already checked), in two phases: tree_host builds the tree,
// the nearfield ownership and every array the device will hold, on the host only (so the
// device bytes are known before anything is allocated); tree_upload allocates and uploads them.
static dwfmm_status tree_host(const std::vector<double> &pts, int64_t n, int32_t d, const double *dim_weights,
                              int32_t leaf_size, double eta, dwfmm_tree *out, int adm_half)
{
    for (double v : pts)
        if (!std::isfinite(v)) return fail(DWFMM_E_NONFINITE, "points contain NaN or Inf");

    dwfmm_tree t = new (std::nothrow) dwfmm_tree_s();
    if (!t) return fail(DWFMM_E_NOMEM, "host allocation failed");
    std::string err;
    if (!build_tree(pts.data(), n, d, dim_weights, leaf_size, eta, t->H, err, -1, true, adm_half)) {
        delete t;
        return fail(DWFMM_E_INVALID, err);
    }
    t->stage.reset(new (std::nothrow) TreeStage());
    if (!t->stage) {
        delete t;
        return fail(DWFMM_E_NOMEM, "host allocation failed");
    }
    TreeStage &S = *t->stage;
    const HostTree &H = t->H;
    const int dp = pad_dim(d);
    // SoA coordinates in tree order, zero rows up to dpad
    S.Xs.assign((size_t)dp * n, 0.0);
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < d; ++k) S.Xs[(size_t)k * n + i] = pts[(size_t)H.perm[i] * d + k];
    // reference-coordinate maps t = (x - lo) * sc + off (degenerate axes -> 1/2)
    S.clo = H.lo;
    S.csc.resize((size_t)H.ncl * d);
    S.coff.resize((size_t)H.ncl * d);
    for (size_t i = 0; i < S.csc.size(); ++i) {
        double w = H.hi[i] - H.lo[i];
        S.csc[i] = w > 0 ? 1.0 / w : 0.0;
        S.coff[i] = w > 0 ? 0.0 : 0.5;
    }
    std::vector<int32_t> &nsrc_local = S.nsrc_local, &nptr_leaf = S.nptr_leaf;
    nsrc_local.resize(H.Nsrc.size());
    nptr_leaf.resize(H.nleaf + 1);
    const int32_t lf = (int32_t)(H.nleaf - 1);
    for (size_t i = 0; i < H.Nsrc.size(); ++i) nsrc_local[i] = H.Nsrc[i] - lf;
    for (int64_t l = 0; l <= H.nleaf; ++l) nptr_leaf[l] = H.Nptr[lf + l];
    for (int64_t l = 0; l < H.nleaf; ++l) S.max_leaf = std::max(S.max_leaf, H.end[lf + l] - H.begin[lf + l]);
    // Symmetric nearfield: the self block is owned by its leaf; every other unordered pair
    // {t, s} goes to whichever leaf owns fewer blocks so far (ties to the smaller index).
    std::vector<std::pair<int32_t, int32_t>> owned;
    std::vector<int32_t> own_cnt(H.nleaf, 0);
    for (int32_t tl = 0; tl < (int32_t)H.nleaf; ++tl)
        for (int32_t q = nptr_leaf[tl]; q < nptr_leaf[tl + 1]; ++q) {
            const int32_t sl = nsrc_local[q];
            if (sl < tl) continue;
            int32_t o = tl, p = sl;
            if (sl != tl && own_cnt[sl] < own_cnt[tl]) std::swap(o, p);
            own_cnt[o]++;
            owned.push_back({o, p});
        }
    std::sort(owned.begin(), owned.end());
    t->own_total = (int64_t)owned.size();
    for (int64_t l = 0; l < H.nleaf; ++l) {
        t->own_max = std::max<int64_t>(t->own_max, own_cnt[l]);
        t->near_max = std::max<int64_t>(t->near_max, nptr_leaf[l + 1] - nptr_leaf[l]);
    }
    std::vector<int32_t> &own_ptr = S.own_ptr, &own_src = S.own_src, &inc_ptr = S.inc_ptr, &inc_blk = S.inc_blk;
    own_ptr.assign(H.nleaf + 1, 0);
    own_src.resize(owned.size());
    inc_ptr.assign(H.nleaf + 1, 0);
    for (auto &op : owned) own_ptr[op.first + 1]++;
    for (int64_t l = 0; l < H.nleaf; ++l) own_ptr[l + 1] += own_ptr[l];
    for (size_t b = 0; b < owned.size(); ++b) {
        own_src[b] = owned[b].second;
        if (owned[b].first != owned[b].second) inc_ptr[owned[b].second + 1]++;
    }
    for (int64_t l = 0; l < H.nleaf; ++l) inc_ptr[l + 1] += inc_ptr[l];
    inc_blk.resize(inc_ptr[H.nleaf]);
    {
        std::vector<int32_t> fill(inc_ptr.begin(), inc_ptr.end() - 1);
        for (size_t b = 0; b < owned.size(); ++b)
            if (owned[b].first != owned[b].second) inc_blk[fill[owned[b].second]++] = (int32_t)b;
    }
    {
        // nearfield work of each owner leaf (the entries of its owned blocks) and of each target
        // leaf of the several-rhs nearfield (the entries of its whole list), each plus one
        // 128-column chunk; each gives a launch order of 8 work-balanced segments (xcd_order)
        auto sz = [&](int32_t leaf) { return (double)(H.end[lf + leaf] - H.begin[lf + leaf]); };
        std::vector<double> lw(H.nleaf, 0.0), nw(H.nleaf, 0.0);
        for (auto &op : owned) lw[op.first] += sz(op.first) * sz(op.second);
        for (int32_t l = 0; l < (int32_t)H.nleaf; ++l) {
            lw[l] += 128.0 * sz(l);
            double ns = 0.0;
            for (int32_t q = nptr_leaf[l]; q < nptr_leaf[l + 1]; ++q) ns += sz(nsrc_local[q]);
            nw[l] = sz(l) * (ns + 128.0);
        }
        t->leaf_work = lw;
        S.leaf_order = xcd_order(lw);
        S.near_order = xcd_order(nw);
        S.near_order_seq = xcd_order(nw, false);
    }
    std::vector<double> &center = S.center, rad(H.nleaf, 0.0);
    center.assign((size_t)H.nleaf * dp, 0.0);
    for (int64_t l = 0; l < H.nleaf; ++l) {
        double r2 = 0.0;
        for (int k = 0; k < d; ++k) {
            const double lo = H.lo[(size_t)(lf + l) * d + k], hi = H.hi[(size_t)(lf + l) * d + k];
            center[(size_t)l * dp + k] = 0.5 * (lo + hi);
            r2 += 0.25 * (hi - lo) * (hi - lo);
        }
        rad[l] = std::sqrt(r2);
    }
    double reach2 = 0.0;
    for (int64_t l = 0; l < H.nleaf; ++l)
        for (int32_t q = nptr_leaf[l]; q < nptr_leaf[l + 1]; ++q) {
            const int32_t s2 = nsrc_local[q];
            double dc = 0.0;
            for (int k = 0; k < d; ++k) {
                const double dd = center[(size_t)s2 * dp + k] - center[(size_t)l * dp + k];
                dc += dd * dd;
            }
            const double reach = rad[l] + std::sqrt(dc) + rad[s2];
            reach2 = std::max(reach2, reach * reach);
        }
    t->near_reach2 = reach2;
    *out = t;
    return DWFMM_OK;
}

// Device bytes the upload of a staged tree allocates (what its arena will report).
static size_t tree_stage_bytes(const dwfmm_tree t)
{
    const TreeStage &S = *t->stage;
    const HostTree &H = t->H;
    size_t b = sizeof(double) * (S.Xs.size() + S.clo.size() + S.csc.size() + S.coff.size() + S.center.size());
    b += sizeof(int32_t) * (H.perm.size() + H.begin.size() + H.end.size() + H.Fptr.size() + H.Fsrc.size() +
                            S.nptr_leaf.size() + S.nsrc_local.size() + S.own_ptr.size() + S.own_src.size() +
                            S.inc_ptr.size() + S.inc_blk.size() + S.leaf_order.size() + S.near_order.size() +
                            S.near_order_seq.size());
    return b;
}

static dwfmm_status tree_upload(dwfmm_tree t, hipStream_t st)
{
    (void)hipGetDevice(&t->device);
    const HostTree &H = t->H;
    TreeStage &S = *t->stage;
    DevTree &D = t->D;
    auto up = [&](auto **dst, const auto &v) { return t->arena.upload(dst, v, st); };
    hipError_t e = hipSuccess;
    double *dXs;
    int32_t *dperm, *dcb, *dce, *dFp, *dFs, *dNp, *dNs, *dop, *dos, *dip, *dib, *dlo, *dno, *dnq;
    double *dcen;
    if ((e = up(&dXs, S.Xs)) != hipSuccess || (e = up(&dperm, H.perm)) != hipSuccess ||
        (e = up(&dlo, S.leaf_order)) != hipSuccess || (e = up(&dno, S.near_order)) != hipSuccess ||
        (e = up(&dnq, S.near_order_seq)) != hipSuccess ||
        (e = up(&dcb, H.begin)) != hipSuccess || (e = up(&dce, H.end)) != hipSuccess ||
        (e = up(&dFp, H.Fptr)) != hipSuccess || (e = up(&dFs, H.Fsrc)) != hipSuccess ||
        (e = up(&dNp, S.nptr_leaf)) != hipSuccess || (e = up(&dNs, S.nsrc_local)) != hipSuccess ||
        (e = up(&t->clo, S.clo)) != hipSuccess || (e = up(&t->csc, S.csc)) != hipSuccess ||
        (e = up(&t->coff, S.coff)) != hipSuccess || (e = up(&dop, S.own_ptr)) != hipSuccess ||
        (e = up(&dos, S.own_src)) != hipSuccess || (e = up(&dip, S.inc_ptr)) != hipSuccess ||
        (e = up(&dib, S.inc_blk)) != hipSuccess || (e = up(&dcen, S.center)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess) {
        t->arena.release();
        return fail(e == hipErrorOutOfMemory ? DWFMM_E_NOMEM : DWFMM_E_HIP,
                    std::string("tree upload: ") + hipGetErrorString(e));
    }
    D.n = (int)H.n;
    D.d = H.d;
    D.J = H.J;
    D.dpad = pad_dim(H.d);
    D.nleaf = (int)H.nleaf;
    D.ncl = (int)H.ncl;
    D.leaf_first = (int)(H.nleaf - 1);
    D.max_leaf = S.max_leaf;
    D.min_far_level = H.min_far_level;
    D.Xs = dXs;
    D.perm = dperm;
    D.cbeg = dcb;
    D.cend = dce;
    D.Fptr = dFp;
    D.Fsrc = dFs;
    D.Nptr = dNp;
    D.Nsrc = dNs;
    D.nblk = (int)S.own_src.size();
    D.own_ptr = dop;
    D.own_src = dos;
    D.inc_ptr = dip;
    D.inc_blk = dib;
    D.center = dcen;
    D.leaf_order = dlo;
    D.n_order = (int)S.leaf_order.size();
    D.near_order = dno;
    D.near_order_seq = dnq;
    D.n_near_order = (int)S.near_order.size();
    t->stage.reset();
    return DWFMM_OK;
}

static dwfmm_status tree_from_host(const std::vector<double> &pts, int64_t n, int32_t d, const double *dim_weights,
                                   int32_t leaf_size, double eta, hipStream_t st, dwfmm_tree *out, int adm_half)
{
    dwfmm_tree t = nullptr;
    dwfmm_status rc = tree_host(pts, n, d, dim_weights, leaf_size, eta, &t, adm_half);
    if (rc != DWFMM_OK) return rc;
    rc = tree_upload(t, st);
    if (rc != DWFMM_OK) {
        delete t;
        return rc;
    }
    *out = t;
    return DWFMM_OK;
}

extern "C" void dwfmm_tree_destroy(dwfmm_tree t)
{
    if (!t || t->destroyed) return;
    t->destroyed = true;
    tree_release(t);
}

// ============================================================== fmm_create
// BF16 several-rhs nearfield tile cache (dwfmm_opts.cache_near): kept when asked for with BF16 and
// max_nrhs > 1 on trees the several-rhs MFMA nearfield takes (leaves of at most 128 points, d <= 32).
static bool near_cache_on(const HostTree &H, const dwfmm_opts &o)
{
    if (!o.cache_near || o.precision != DWFMM_BF16 || o.max_nrhs < 2 || H.d > 32) return false;
    const int64_t lf = H.nleaf - 1;
    for (int64_t l = 0; l < H.nleaf; ++l)
        if (H.end[lf + l] - H.begin[lf + l] > 128) return false;
    return true;
}

// Column tiles of each target leaf in the order the several-rhs nearfield streams its sources: the
// leaf's own block when listed, then per list segment of 256 entries the other leaves' points back
// to back, 16 columns a tile.  off[l] = first tile of leaf l, off[nleaf] = all tiles (4 KiB each).
static std::vector<int64_t> near_tile_offsets(const HostTree &H)
{
    const int64_t lf = H.nleaf - 1;
    std::vector<int64_t> off((size_t)H.nleaf + 1, 0);
    for (int64_t l = 0; l < H.nleaf; ++l) {
        const int64_t c = lf + l, nt = H.end[c] - H.begin[c], f0 = H.Nptr[c], f1 = H.Nptr[c + 1];
        int64_t t = 0;
        if (nt > 0) {
            bool diag = false;
            for (int64_t f = f0; f < f1; ++f) diag |= H.Nsrc[f] == c;
            if (diag) t += (nt + 15) / 16;
            for (int64_t fb = f0; fb < f1; fb += 256) {
                int64_t total = 0;
                for (int64_t f = fb; f < std::min<int64_t>(fb + 256, f1); ++f)
                    if (H.Nsrc[f] != c) total += H.end[H.Nsrc[f]] - H.begin[H.Nsrc[f]];
                t += (total + 15) / 16;
            }
        }
        off[(size_t)l + 1] = off[(size_t)l] + t;
    }
    return off;
}

extern "C" dwfmm_status dwfmm_fmm_create(dwfmm_tree tree, dwfmm_kernel kernel, double q, const dwfmm_opts *opts,
                                         void *stream, dwfmm_op *out)
{
    if (!out) return fail(DWFMM_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!tree || tree->destroyed) return fail(DWFMM_E_INVALID, "tree is NULL or destroyed");
    if (kernel.kind < 0 || kernel.kind > 3) return fail(DWFMM_E_INVALID, "unknown kernel kind");
    if (!(kernel.ell > 0.0) || !std::isfinite(kernel.ell)) return fail(DWFMM_E_INVALID, "kernel ell must be > 0");
    if (!(q >= 0.0) || !std::isfinite(q)) return fail(DWFMM_E_INVALID, "q must be finite and >= 0");
    dwfmm_opts o{};
    o.weight_rule = DWFMM_W_R1;
    o.precision = DWFMM_FP64;
    o.max_nrhs = 1;
    o.check_every = 1;
    o.ir_max_outer = 30;
    if (opts) {
        o = *opts;
        if (o.max_nrhs == 0) o.max_nrhs = 1;
        if (o.check_every == 0) o.check_every = 1;
        if (o.ir_max_outer == 0) o.ir_max_outer = 30;
    }
    if (o.max_nrhs < 1 || o.max_nrhs > 32) return fail(DWFMM_E_INVALID, "max_nrhs must be in [1, 32]");
    if (o.check_every < 1) return fail(DWFMM_E_INVALID, "check_every must be >= 1");
    if (o.precision < 0 || o.precision > 2) return fail(DWFMM_E_INVALID, "unknown precision");
    if (o.node_rule < 0 || o.node_rule > 1 || o.afp_candidates < 0)
        return fail(DWFMM_E_INVALID, "unknown node rule or negative candidate count");
    if (o.index_rule < 0 || o.index_rule > 1) return fail(DWFMM_E_INVALID, "unknown index rule");
    if (o.ir_max_inner < 0) return fail(DWFMM_E_INVALID, "ir_max_inner must be >= 0");
    if (o.cache_near && (o.precision != DWFMM_BF16 || o.max_nrhs < 2))
        return fail(DWFMM_E_INVALID, "cache_near needs BF16 precision and max_nrhs > 1");
    const HostTree &H = tree->H;
    hipStream_t st = (hipStream_t)stream;

    dwfmm_op op = new (std::nothrow) dwfmm_op_s();
    if (!op) return fail(DWFMM_E_NOMEM, "host allocation failed");
    std::string err;
    std::vector<double> omega(H.d);
    if (!compute_weights(o.weight_rule, H.d, H.b.data(), H.eta, o.omega, omega.data(), err) ||
        !build_basis(H.d, omega.data(), q, op->B, err, o.node_rule, o.afp_candidates, o.index_rule)) {
        delete op;
        return fail(DWFMM_E_INVALID, err);
    }
    const HostBasis &B = op->B;
    const int nx = B.nx, dp = tree->D.dpad;
    if (nx > 128 || nx * dp > 3072) {
        delete op;
        return fail(DWFMM_E_INVALID, "index set too large for the GPU kernels (n_x <= 128, n_x * d <= 3072)");
    }
    std::vector<double> nodes, nodes_p((size_t)H.ncl * nx * dp, 0.0), E;
    box_nodes(H, B, nodes);
    for (int64_t c = 0; c < H.ncl; ++c)
        for (int a = 0; a < nx; ++a)
            for (int k = 0; k < H.d; ++k)
                nodes_p[((size_t)c * nx + a) * dp + k] = nodes[((size_t)c * nx + a) * H.d + k];
    // axis-major zero-padded copy for the MFMA coupling kernel, and squared node norms
    const int dk = (H.d + 3) / 4 * 4, nxp = (nx + 15) / 16 * 16;
    std::vector<double> nodesT((size_t)H.ncl * dk * nxp, 0.0), nnorm((size_t)H.ncl * nxp, 0.0);
    for (int64_t c = 0; c < H.ncl; ++c)
        for (int a = 0; a < nx; ++a) {
            double s = 0.0;
            for (int k = 0; k < H.d; ++k) {
                const double v = nodes[((size_t)c * nx + a) * H.d + k];
                nodesT[((size_t)c * dk + k) * nxp + a] = v;
                s += v * v;
            }
            nnorm[(size_t)c * nxp + a] = s;
        }
    transfer_matrices(H, B, E);
    // Legendre slots (axis, degree >= 1) and, per basis function, the slots whose product it is
    std::vector<int32_t> leg_axis, leg_deg;
    std::vector<std::vector<int>> slot(H.d);
    for (int k = 0; k < H.d; ++k) {
        slot[k].assign(B.mk[k] + 1, -1);
        for (int m = 1; m <= B.mk[k]; ++m) {
            slot[k][m] = (int)leg_axis.size();
            leg_axis.push_back(k);
            leg_deg.push_back(m);
        }
    }
    int nnz_max = 1;
    for (int a = 0; a < nx; ++a) {
        int c = 0;
        for (int k = 0; k < H.d; ++k) c += B.alpha[(size_t)a * H.d + k] != 0;
        nnz_max = std::max(nnz_max, c);
    }
    std::vector<int32_t> lidx((size_t)nx * nnz_max, -1);
    for (int a = 0; a < nx; ++a) {
        int j = 0;
        for (int k = 0; k < H.d; ++k) {
            int m = B.alpha[(size_t)a * H.d + k];
            if (m) lidx[(size_t)a * nnz_max + j++] = slot[k][m];
        }
    }
    if (leg_axis.size() > 128) {
        delete op;
        return fail(DWFMM_E_INVALID, "too many Legendre slots");
    }
    if (leg_axis.empty()) {  // keep device arrays non-empty
        leg_axis.push_back(0);
        leg_deg.push_back(0);
    }

    auto up = [&](auto **dst, const auto &v) { return op->arena.upload(dst, v, st); };
    const size_t n = (size_t)H.n, R = (size_t)o.max_nrhs;
    double *dnodes, *dE, *dVinv, *dLb, *dxt, *dM, *dL;
    __bf16 *dxtb = nullptr;
    int32_t *dlidx, *dla, *dld;
    hipError_t e = hipSuccess;
    double *dnodesT, *dnnorm;
    if ((e = up(&dnodes, nodes_p)) != hipSuccess || (e = up(&dE, E)) != hipSuccess ||
        (e = up(&dnodesT, nodesT)) != hipSuccess || (e = up(&dnnorm, nnorm)) != hipSuccess ||
        (e = up(&dVinv, B.Vinv)) != hipSuccess || (e = up(&dlidx, lidx)) != hipSuccess ||
        (e = up(&dla, leg_axis)) != hipSuccess || (e = up(&dld, leg_deg)) != hipSuccess ||
        (e = op->arena.alloc((void **)&dLb, sizeof(double) * nx * n)) != hipSuccess ||
        (e = op->arena.alloc((void **)&dxt, sizeof(double) * n * R)) != hipSuccess ||
        (R > 1 && (e = op->arena.alloc((void **)&dxtb, sizeof(__bf16) * n * R)) != hipSuccess) ||
        (e = op->arena.alloc((void **)&dM, sizeof(double) * H.ncl * nx * R)) != hipSuccess ||
        (e = op->arena.alloc((void **)&dL, sizeof(double) * H.ncl * nx * R)) != hipSuccess ||
        (e = op->arena.alloc((void **)&op->D.rowbuf, sizeof(double) * 128 * H.nleaf)) != hipSuccess ||
        (e = op->arena.alloc((void **)&op->D.colbuf, sizeof(double) * 128 * (size_t)tree->D.nblk)) != hipSuccess ||
        (e = op->arena.alloc((void **)&op->r, sizeof(double) * n * R)) != hipSuccess ||
        (e = op->arena.alloc((void **)&op->p, sizeof(double) * n * R)) != hipSuccess ||
        (e = op->arena.alloc((void **)&op->q, sizeof(double) * n * R)) != hipSuccess ||
        (o.precision != DWFMM_FP64 &&
         ((e = op->arena.alloc((void **)&op->ir_r, sizeof(double) * n * R)) != hipSuccess ||
          (e = op->arena.alloc((void **)&op->ir_d, sizeof(double) * n * R)) != hipSuccess)) ||
        (e = op->arena.alloc((void **)&op->partial, sizeof(double) * 2 * kDotBlocks * R)) != hipSuccess ||
        (e = op->arena.alloc((void **)&op->scal, sizeof(double) * 16 * R)) != hipSuccess ||
        (e = op->arena.alloc((void **)&op->state, sizeof(int32_t) * 4 * R)) != hipSuccess ||
        (e = hipMemsetAsync(dM, 0, sizeof(double) * H.ncl * nx * R, st)) != hipSuccess ||
        (e = hipMemsetAsync(dL, 0, sizeof(double) * H.ncl * nx * R, st)) != hipSuccess ||
        (e = launch_basis(tree->D, nx, tree->clo, tree->csc, tree->coff, dlidx, nnz_max, dVinv,
                          (int)leg_axis.size(), dla, dld, dLb, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess) {
        op->arena.release();
        delete op;
        return fail(e == hipErrorOutOfMemory ? DWFMM_E_NOMEM : DWFMM_E_HIP,
                    std::string("operator setup: ") + hipGetErrorString(e));
    }
    if (near_cache_on(H, o)) {
        const std::vector<int64_t> toff = near_tile_offsets(H);
        int64_t *dtoff = nullptr;
        if ((e = op->arena.alloc((void **)&op->D.near_tiles, 4096 * (size_t)toff.back())) != hipSuccess ||
            (e = up(&dtoff, toff)) != hipSuccess || (e = hipStreamSynchronize(st)) != hipSuccess) {
            op->arena.release();
            delete op;
            return fail(e == hipErrorOutOfMemory ? DWFMM_E_NOMEM : DWFMM_E_HIP,
                        std::string("nearfield tile cache: ") + hipGetErrorString(e));
        }
        op->D.near_tile_off = dtoff;
        op->D.near_filled = &op->near_filled;
    }
    DevOp &D = op->D;
    D.kind = kernel.kind;
    D.ell = kernel.ell;
    D.gauss_split = kernel.kind == DWFMM_GAUSSIAN && tree->near_reach2 / kernel.ell <= 600.0;
    D.gauss_split32 = kernel.kind == DWFMM_GAUSSIAN && tree->near_reach2 / kernel.ell <= 80.0;
    {
        // every |x - c| and |y - c| of a nearfield entry is at most the reach (c the target leaf's midpoint)
        const double reach = std::sqrt(tree->near_reach2);
        // (the exponent held to [-60, 60] so that the kernel's 1 / hscale^2 stays a finite float)
        const int e = reach > 0.0 && std::isfinite(reach) ? std::clamp((int)std::ceil(std::log2(reach)), -60, 60) : 0;
        D.hscale = (float)std::ldexp(1.0, -e);
    }
    D.matern_in_range = kernel.kind == DWFMM_MATERN32 &&
                        std::sqrt(tree->near_reach2) * (1.7320508075688772 * 1.4426950408889634) / kernel.ell <= 1000.0;
    D.nx = nx;
    D.max_nrhs = o.max_nrhs;
    D.nodes = dnodes;
    D.nxp = nxp;
    D.nodesT = dnodesT;
    D.nnorm = dnnorm;
    D.E = dE;
    D.Lb = dLb;
    D.xt = dxt;
    D.xtb = dxtb;
    D.M = dM;
    D.L = dL;
    op->precision = o.precision;
    op->max_nrhs = o.max_nrhs;
    op->check_every = o.check_every;
    op->ir_inner_rtol = o.ir_inner_rtol;
    op->ir_max_outer = o.ir_max_outer;
    op->ir_max_inner = o.ir_max_inner;
    op->progress = o.progress;
    op->progress_ctx = o.progress_ctx;
    op->b_lidx = dlidx;
    op->b_la = dla;
    op->b_ld = dld;
    op->b_Vinv = dVinv;
    op->b_nnz = nnz_max;
    op->b_nleg = (int)leg_axis.size();
    if ((e = hipStreamCreateWithFlags(&op->fork.side, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&op->fork.forked, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&op->fork.joined, hipEventDisableTiming)) != hipSuccess) {
        op->arena.release();
        delete op;
        return fail(DWFMM_E_HIP, std::string("operator streams: ") + hipGetErrorString(e));
    }
    op->tree = tree;
    tree->refs++;
    *out = op;
    return DWFMM_OK;
}

// Device bytes dwfmm_fmm_create allocates for an operator with basis B and workspace for R
// right-hand sides on a tree with these sizes (what the operator's arena reports).
static size_t op_device_bytes(const HostTree &H, int64_t nblk, const HostBasis &B, int R, int precision)
{
    const size_t nx = (size_t)B.nx, dp = (size_t)pad_dim(H.d), dk = (size_t)(H.d + 3) / 4 * 4;
    const size_t nxp = (nx + 15) / 16 * 16, ncl = (size_t)H.ncl, n = (size_t)H.n;
    size_t nleg = 0, nnz_max = 1;
    for (int k = 0; k < H.d; ++k) nleg += (size_t)B.mk[k];
    for (size_t a = 0; a < nx; ++a) {
        size_t c = 0;
        for (int k = 0; k < H.d; ++k) c += B.alpha[a * H.d + k] != 0;
        nnz_max = std::max(nnz_max, c);
    }
    nleg = std::max<size_t>(nleg, 1);
    size_t b = 8 * (ncl * nx * dp + ncl * nx * nx + ncl * dk * nxp + ncl * nxp + nx * nx);  // nodes, E, nodesT, norms, V^-1
    b += 4 * (nx * nnz_max + 2 * nleg);                                                     // Legendre slot tables
    b += 8 * (nx * n + n * R + 2 * ncl * nx * R);                                          // basis cache, xt, M, L
    if (R > 1) b += 2 * n * R;                                                              // xtb
    b += 8 * 128 * ((size_t)H.nleaf + (size_t)nblk);                                       // row and column sums
    b += 8 * n * R * (precision != DWFMM_FP64 ? 5 : 3);                                    // r, p, q (, ir_r, ir_d)
    b += 8 * (2 * (size_t)kDotBlocks * R + 16 * (size_t)R) + 4 * 4 * (size_t)R;            // partial, scal, state
    return b;
}

extern "C" size_t dwfmm_op_bytes_for(dwfmm_tree tree, double q, const dwfmm_opts *opts)
{
    if (!tree || tree->destroyed || !(q >= 0.0) || !std::isfinite(q)) return 0;
    dwfmm_opts o{};
    o.weight_rule = DWFMM_W_R1;
    o.max_nrhs = 1;
    if (opts) {
        o = *opts;
        if (o.max_nrhs == 0) o.max_nrhs = 1;
    }
    if (o.max_nrhs < 1 || o.max_nrhs > 32 || o.precision < 0 || o.precision > 2) return 0;
    const HostTree &H = tree->H;
    std::string err;
    std::vector<double> omega(H.d);
    HostBasis B;
    if (!compute_weights(o.weight_rule, H.d, H.b.data(), H.eta, o.omega, omega.data(), err) ||
        !build_basis(H.d, omega.data(), q, B, err, o.node_rule, o.afp_candidates, o.index_rule))
        return 0;
    const int64_t nblk = tree->stage ? (int64_t)tree->stage->own_src.size() : (int64_t)tree->D.nblk;
    const size_t tb = tree->stage ? tree_stage_bytes(tree) : tree->arena.total;
    size_t cache = 0;
    if (near_cache_on(H, o)) cache = 4096 * (size_t)near_tile_offsets(H).back() + 8 * ((size_t)H.nleaf + 1);
    return tb + op_device_bytes(H, nblk, B, o.max_nrhs, o.precision) + cache;
}

extern "C" void dwfmm_op_destroy(dwfmm_op op)
{
    if (!op) return;
    op->arena.release();
    dwfmm_tree t = op->tree;
    delete op;
    if (t) tree_release(t);
}

// ============================================================== matvec
extern "C" dwfmm_status dwfmm_fmm_matvec_parts(dwfmm_op op, const double *x, double *y, int32_t nrhs, int32_t parts,
                                               int32_t precision, void *stream)
{
    if (!op) return fail(DWFMM_E_INVALID, "op is NULL");
    if (!x || !y) return fail(DWFMM_E_INVALID, "x or y is NULL");
    if (x == y) return fail(DWFMM_E_INVALID, "x and y must be distinct");
    if (nrhs < 1 || nrhs > op->max_nrhs) return fail(DWFMM_E_INVALID, "nrhs must be in [1, max_nrhs]");
    if (parts < 0 || parts > 3) return fail(DWFMM_E_INVALID, "parts must be in [0, 3]");
    if (precision < 0 || precision > 2) return fail(DWFMM_E_INVALID, "unknown precision");
    const KernelTimer *tm = nullptr;
    if (op->timing) {
        if (op->timers_used == op->timers.size()) {
            KernelTimer k;
            HIP_TRY(hipEventCreate(&k.p2p_start));
            HIP_TRY(hipEventCreate(&k.p2p_stop));
            HIP_TRY(hipEventCreate(&k.m2l_start));
            HIP_TRY(hipEventCreate(&k.m2l_stop));
            op->timers.push_back(k);
        }
        tm = &op->timers[op->timers_used++];
    }
    HIP_TRY(launch_matvec(op->tree->D, op->D, x, y, nrhs, parts, precision, (hipStream_t)stream, tm, &op->fork));
    return DWFMM_OK;
}

extern "C" dwfmm_status dwfmm_op_timing(dwfmm_op op, int32_t enable, double *out)
{
    if (!op) return fail(DWFMM_E_INVALID, "op is NULL");
    if (out) {
        double p2p = 0.0, m2l = 0.0;
        for (size_t i = 0; i < op->timers_used; ++i) {
            float ms = 0.0f;
            HIP_TRY(hipEventSynchronize(op->timers[i].p2p_stop));
            HIP_TRY(hipEventElapsedTime(&ms, op->timers[i].p2p_start, op->timers[i].p2p_stop));
            p2p += ms;
            if (hipEventQuery(op->timers[i].m2l_stop) == hipSuccess &&
                hipEventElapsedTime(&ms, op->timers[i].m2l_start, op->timers[i].m2l_stop) == hipSuccess)
                m2l += ms;
        }
        out[0] = p2p;
        out[1] = m2l;
        out[2] = (double)op->timers_used;
    }
    op->timing = enable != 0;
    op->timers_used = 0;
    return DWFMM_OK;
}

extern "C" dwfmm_status dwfmm_fmm_matvec(dwfmm_op op, const double *x, double *y, int32_t nrhs, void *stream)
{
    if (!op) return fail(DWFMM_E_INVALID, "op is NULL");
    return dwfmm_fmm_matvec_parts(op, x, y, nrhs, 3, op->precision, stream);
}

// ============================================================== allocation-free matvec
// The per-call workspace of a matvec (charges in tree order, moments, locals, nearfield row and
// column sums) taken from one file-scope device array instead of the operator's buffers.  Each
// GPU holds its own copy of the array; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device (the array's name is no device address on the host).
namespace {
constexpr size_t kStaticScratchBytes = DWFMM_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

size_t align256(size_t b) { return (b + 255) / 256 * 256; }
}  // namespace

// The device address of this GPU's scratch array, looked up once per device (with that device
// current, as the caller's device is here).
static dwfmm_status static_scratch(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(DWFMM_E_INVALID, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(DWFMM_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return DWFMM_OK;
}

// Workspace bytes of one allocation-free matvec: every part starts at a multiple of 256 bytes.
static size_t static_scratch_need(dwfmm_op op, int32_t nrhs)
{
    const DevTree &T = op->tree->D;
    const size_t n = (size_t)T.n, nx = (size_t)op->D.nx, r = (size_t)nrhs;
    size_t b = align256(sizeof(double) * n * r) + 2 * align256(sizeof(double) * (size_t)T.ncl * nx * r);
    if (nrhs > 1) b += align256(sizeof(__bf16) * n * r);
    if (nrhs == 1) b += align256(sizeof(double) * 128 * (size_t)T.nleaf) + align256(sizeof(double) * 128 * (size_t)T.nblk);
    return b;
}

extern "C" dwfmm_status dwfmm_fmm_matvec_static(dwfmm_op op, const double *x, double *y, int32_t nrhs, void *stream)
{
    if (!op) return fail(DWFMM_E_INVALID, "op is NULL");
    if (!x || !y) return fail(DWFMM_E_INVALID, "x or y is NULL");
    if (x == y) return fail(DWFMM_E_INVALID, "x and y must be distinct");
    if (nrhs < 1 || nrhs > 32) return fail(DWFMM_E_INVALID, "nrhs must be in [1, 32]");
    const size_t need = static_scratch_need(op, nrhs);
    if (need > kStaticScratchBytes)
        return fail(DWFMM_E_INVALID, "workspace of " + std::to_string(need) + " bytes exceeds the static scratch of " +
                                         std::to_string(kStaticScratchBytes) + " bytes");
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != op->tree->device) return fail(DWFMM_E_INVALID, "the operator's device must be current");
    void *base = nullptr;
    const dwfmm_status s = static_scratch(dev, &base);
    if (s != DWFMM_OK) return s;
    const DevTree &T = op->tree->D;
    const size_t n = (size_t)T.n, nx = (size_t)op->D.nx, r = (size_t)nrhs;
    unsigned char *p = (unsigned char *)base;
    DevOp O = op->D;  // the operator's tables, this call's workspace
    O.xt = (double *)p;
    p += align256(sizeof(double) * n * r);
    O.M = (double *)p;
    p += align256(sizeof(double) * (size_t)T.ncl * nx * r);
    O.L = (double *)p;
    p += align256(sizeof(double) * (size_t)T.ncl * nx * r);
    O.xtb = nullptr;
    if (nrhs > 1) {
        O.xtb = (__bf16 *)p;
        p += align256(sizeof(__bf16) * n * r);
    }
    if (nrhs == 1) {
        O.rowbuf = (double *)p;
        p += align256(sizeof(double) * 128 * (size_t)T.nleaf);
        O.colbuf = (double *)p;
    } else {
        O.rowbuf = O.colbuf = nullptr;  // only the one-rhs symmetric nearfield uses them
    }
    O.max_nrhs = nrhs;
    HIP_TRY(launch_matvec(T, O, x, y, nrhs, 3, op->precision, (hipStream_t)stream, nullptr, &op->fork));
    return DWFMM_OK;
}

// ============================================================== CG
namespace {

// scal layout per column c (stride nrhs): [0] rr, [1] |f|^2, [2] pq, [3] rr_new, [4] a, [5] beta
// state layout: [0] status (0 active, 1 converged, 2 breakdown), [1] iters, [2] neg curvature
__global__ void cg_check_kernel(double *scal, int32_t *state, int nrhs, double rtol)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nrhs) return;
    const double rr = scal[c], ff = scal[nrhs + c];
    if (state[c] == 0 && sqrt(rr) <= rtol * sqrt(ff)) state[c] = 1;
}

__global__ void cg_alpha_kernel(double *scal, int32_t *state, int nrhs)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nrhs) return;
    double a = 0.0;
    if (state[c] == 0) {
        const double pq = scal[2 * nrhs + c];
        if (!isfinite(pq) || fabs(pq) <= 1e-300) {
            state[c] = 2;
        } else {
            if (pq < 0.0) state[2 * nrhs + c] += 1;
            a = scal[c] / pq;
        }
    }
    scal[4 * nrhs + c] = a;
}

__global__ void cg_beta_kernel(double *scal, int32_t *state, int nrhs)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nrhs) return;
    double b = 0.0;
    if (state[c] == 0) {
        b = scal[3 * nrhs + c] / scal[c];
        scal[c] = scal[3 * nrhs + c];
        state[nrhs + c] += 1;
    }
    scal[5 * nrhs + c] = b;
}

// v = a + s * b  (s per column from scal[slot], applied where state == 0 if masked)
__global__ void axpy_kernel(double *out, const double *a, const double *b,
                            const double *__restrict__ scal, int slot, double sign, const int32_t *__restrict__ state,
                            int masked, size_t total, int nrhs)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % nrhs);
        if (masked && state[c] != 0) continue;
        out[i] = a[i] + sign * scal[slot * nrhs + c] * b[i];
    }
}

// out = a + lam * b   (adds the ridge term)
__global__ void ridge_kernel(double *__restrict__ out, const double *__restrict__ b, double lam, size_t total)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x)
        out[i] = fma(lam, b[i], out[i]);
}

// out = f - a
__global__ void sub_kernel(double *out, const double *f, const double *a,
                           size_t total)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x)
        out[i] = f[i] - a[i];
}

__global__ void copy_kernel(double *__restrict__ out, const double *__restrict__ a, size_t total)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x)
        out[i] = a[i];
}

constexpr int kEwBlocks = 1024;

}  // namespace

namespace {

// The CG descriptor of a one-rhs problem on its operator's workspace.
CgItem cg_item(dwfmm_op op, double lambda, const double *b, double *x, double rtol, int max_it)
{
    CgItem it{};
    it.x = x;
    it.r = op->r;
    it.p = op->p;
    it.q = op->q;
    it.b = b;
    it.partial = op->partial;
    it.scal = op->scal;
    it.state = op->state;
    it.lambda = lambda;
    it.rtol = rtol;
    it.n = op->tree->D.n;
    it.nblk = cg_blocks(it.n);
    it.chunk = (it.n + it.nblk - 1) / it.nblk;
    it.max_it = max_it;
    return it;
}

// CG on (K~ + lambda I) x = b with one rhs: the matvec, then the vector steps of launch_cg.
hipError_t cg_run1(dwfmm_op op, double lambda, const double *b, double *x, double rtol, int max_iter, int precision,
                   hipStream_t st, std::vector<int32_t> &hstate, std::vector<double> &hrr)
{
    const DevTree &T = op->tree->D;
    const CgItem it = cg_item(op, lambda, b, x, rtol, max_iter);
    hipError_t e;
    if ((e = launch_matvec(T, op->D, x, op->q, 1, 3, precision, st, nullptr, &op->fork)) != hipSuccess ||
        (e = launch_cg(CG_START, nullptr, 0, 0, it, st)) != hipSuccess ||
        (e = launch_cg(CG_START_SUM, nullptr, 0, 0, it, st)) != hipSuccess)
        return e;
    hstate.assign(3, 0);
    hrr.assign(2, 0.0);
    for (int k = 0; k < max_iter; ++k) {
        if (k % op->check_every == 0) {
            if ((e = hipMemcpyAsync(hstate.data(), op->state, sizeof(int32_t), hipMemcpyDeviceToHost, st)) !=
                    hipSuccess ||
                (op->progress &&
                 (e = hipMemcpyAsync(hrr.data(), op->scal, sizeof(double) * 2, hipMemcpyDeviceToHost, st)) !=
                     hipSuccess) ||
                (e = hipStreamSynchronize(st)) != hipSuccess)
                return e;
            if (op->progress) {
                const double rel = hrr[1] > 0 ? std::sqrt(hrr[0] / hrr[1]) : std::sqrt(hrr[0]);
                op->progress(op->progress_ctx, k, 1, &rel);
            }
            if (hstate[0] != 0) break;
        }
        if ((e = launch_matvec(T, op->D, op->p, op->q, 1, 3, precision, st, nullptr, &op->fork)) != hipSuccess)
            return e;
        for (int step : {CG_PQ, CG_ALPHA, CG_XR, CG_BETA, CG_P})
            if ((e = launch_cg(step, nullptr, 0, 0, it, st)) != hipSuccess) return e;
    }
    if ((e = hipMemcpyAsync(hrr.data(), op->scal, sizeof(double) * 2, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipMemcpyAsync(hstate.data(), op->state, sizeof(int32_t) * 3, hipMemcpyDeviceToHost, st)) != hipSuccess)
        return e;
    return hipStreamSynchronize(st);
}

// CG on (K~ + lambda I) x = b in the given matvec precision, x holding the start vector.
// Vectors, inner products and scalars are FP64 on the device; the host reads the column
// states every check_every iterations.  On return hstate[0..3n) = state (0 active,
// 1 converged, 2 breakdown), iterations, negative-curvature steps; hrr[0..2n) = |r|^2, |b|^2.
hipError_t cg_run(dwfmm_op op, double lambda, const double *b, double *x, int nrhs, double rtol, int max_iter,
                  int precision, hipStream_t st, std::vector<int32_t> &hstate, std::vector<double> &hrr)
{
    if (nrhs == 1) return cg_run1(op, lambda, b, x, rtol, max_iter, precision, st, hstate, hrr);
    const DevTree &T = op->tree->D;
    const size_t total = (size_t)T.n * nrhs;
    const int nb = (nrhs + 63) / 64;
    double *r = op->r, *p = op->p, *q = op->q, *scal = op->scal;
    int32_t *state = op->state;
    hipError_t e;
    auto matvecA = [&](const double *v, double *out) -> hipError_t {
        hipError_t e2 = launch_matvec(T, op->D, v, out, nrhs, 3, precision, st, nullptr, &op->fork);
        if (e2 != hipSuccess) return e2;
        if (lambda != 0.0) hipLaunchKernelGGL(ridge_kernel, dim3(kEwBlocks), dim3(256), 0, st, out, v, lambda, total);
        return hipGetLastError();
    };
    if ((e = hipMemsetAsync(state, 0, sizeof(int32_t) * 3 * nrhs, st)) != hipSuccess) return e;
    if ((e = matvecA(x, q)) != hipSuccess) return e;
    hipLaunchKernelGGL(sub_kernel, dim3(kEwBlocks), dim3(256), 0, st, r, b, q, total);
    hipLaunchKernelGGL(copy_kernel, dim3(kEwBlocks), dim3(256), 0, st, p, r, total);
    if ((e = launch_dot(r, r, T.n, nrhs, op->partial, scal, st)) != hipSuccess) return e;
    if ((e = launch_dot(b, b, T.n, nrhs, op->partial, scal + nrhs, st)) != hipSuccess) return e;
    hstate.assign(3 * nrhs, 0);
    hrr.assign(2 * nrhs, 0.0);
    for (int it = 0; it < max_iter; ++it) {
        hipLaunchKernelGGL(cg_check_kernel, dim3(nb), dim3(64), 0, st, scal, state, nrhs, rtol);
        if (it % op->check_every == 0) {
            if ((e = hipMemcpyAsync(hstate.data(), state, sizeof(int32_t) * nrhs, hipMemcpyDeviceToHost, st)) !=
                hipSuccess)
                return e;
            if (op->progress && (e = hipMemcpyAsync(hrr.data(), scal, sizeof(double) * 2 * nrhs,
                                                    hipMemcpyDeviceToHost, st)) != hipSuccess)
                return e;
            if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
            if (op->progress) {
                std::vector<double> rel(nrhs);
                for (int c = 0; c < nrhs; ++c)
                    rel[c] = hrr[nrhs + c] > 0 ? std::sqrt(hrr[c] / hrr[nrhs + c]) : std::sqrt(hrr[c]);
                op->progress(op->progress_ctx, it, nrhs, rel.data());
            }
            bool active = false;
            for (int c = 0; c < nrhs; ++c) active |= hstate[c] == 0;
            if (!active) break;
        }
        if ((e = matvecA(p, q)) != hipSuccess) return e;
        if ((e = launch_dot(p, q, T.n, nrhs, op->partial, scal + 2 * nrhs, st)) != hipSuccess) return e;
        hipLaunchKernelGGL(cg_alpha_kernel, dim3(nb), dim3(64), 0, st, scal, state, nrhs);
        // x += a p ; r -= a q  (a = 0 for inactive columns)
        hipLaunchKernelGGL(axpy_kernel, dim3(kEwBlocks), dim3(256), 0, st, x, x, p, scal, 4, 1.0, state, 0, total, nrhs);
        hipLaunchKernelGGL(axpy_kernel, dim3(kEwBlocks), dim3(256), 0, st, r, r, q, scal, 4, -1.0, state, 0, total,
                           nrhs);
        if ((e = launch_dot(r, r, T.n, nrhs, op->partial, scal + 3 * nrhs, st)) != hipSuccess) return e;
        hipLaunchKernelGGL(cg_beta_kernel, dim3(nb), dim3(64), 0, st, scal, state, nrhs);
        // p = r + beta p on active columns
        hipLaunchKernelGGL(axpy_kernel, dim3(kEwBlocks), dim3(256), 0, st, p, r, p, scal, 5, 1.0, state, 1, total,
                           nrhs);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(cg_check_kernel, dim3(nb), dim3(64), 0, st, scal, state, nrhs, rtol);
    hrr.assign(2 * nrhs, 0.0);
    if ((e = hipMemcpyAsync(hrr.data(), scal, sizeof(double) * 2 * nrhs, hipMemcpyDeviceToHost, st)) != hipSuccess)
        return e;
    if ((e = hipMemcpyAsync(hstate.data(), state, sizeof(int32_t) * 3 * nrhs, hipMemcpyDeviceToHost, st)) !=
        hipSuccess)
        return e;
    return hipStreamSynchronize(st);
}

// out = f - (K~_64 + lambda I) v in FP64; |out|^2 per column into host res.
hipError_t residual64(dwfmm_op op, double lambda, const double *f, const double *v, double *out, int nrhs,
                      hipStream_t st, std::vector<double> &res)
{
    const DevTree &T = op->tree->D;
    const size_t total = (size_t)T.n * nrhs;
    hipError_t e = launch_matvec(T, op->D, v, out, nrhs, 3, DWFMM_FP64, st, nullptr, &op->fork);
    if (e != hipSuccess) return e;
    if (nrhs == 1) {
        CgItem it = cg_item(op, lambda, nullptr, nullptr, 0.0, 0);
        it.f = f;
        it.v = v;
        it.out = out;
        res.assign(1, 0.0);
        if ((e = launch_cg(CG_RES, nullptr, 0, 0, it, st)) != hipSuccess ||
            (e = launch_cg(CG_RES_SUM, nullptr, 0, 0, it, st)) != hipSuccess ||
            (e = hipMemcpyAsync(res.data(), op->scal + 8, sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess)
            return e;
        return hipStreamSynchronize(st);
    }
    if (lambda != 0.0) hipLaunchKernelGGL(ridge_kernel, dim3(kEwBlocks), dim3(256), 0, st, out, v, lambda, total);
    hipLaunchKernelGGL(sub_kernel, dim3(kEwBlocks), dim3(256), 0, st, out, f, out, total);
    if ((e = launch_dot(out, out, T.n, nrhs, op->partial, op->scal + 8 * nrhs, st)) != hipSuccess) return e;
    res.assign(nrhs, 0.0);
    if ((e = hipMemcpyAsync(res.data(), op->scal + 8 * nrhs, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st)) !=
        hipSuccess)
        return e;
    return hipStreamSynchronize(st);
}

}  // namespace

extern "C" dwfmm_status dwfmm_fmm_solve(dwfmm_op op, double lambda, const double *f, double *alpha, int32_t nrhs,
                                        double rtol, int32_t max_iter, void *stream, dwfmm_solve_info *info)
{
    if (!op) return fail(DWFMM_E_INVALID, "op is NULL");
    if (!f || !alpha || !info) return fail(DWFMM_E_INVALID, "f, alpha or info is NULL");
    if (nrhs < 1 || nrhs > op->max_nrhs) return fail(DWFMM_E_INVALID, "nrhs must be in [1, max_nrhs]");
    if (!std::isfinite(lambda) || lambda < 0.0) return fail(DWFMM_E_INVALID, "lambda must be finite and >= 0");
    if (!(rtol > 0.0) || max_iter < 0) return fail(DWFMM_E_INVALID, "rtol must be > 0 and max_iter >= 0");
    hipStream_t st = (hipStream_t)stream;
    const DevTree &T = op->tree->D;
    const size_t total = (size_t)T.n * nrhs;
    std::vector<int32_t> hstate;
    std::vector<double> hrr, res, fn2;
    HIP_TRY(launch_dot(f, f, T.n, nrhs, op->partial, op->scal + 9 * nrhs, st));
    fn2.assign(nrhs, 0.0);
    HIP_TRY(hipMemcpyAsync(fn2.data(), op->scal + 9 * nrhs, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    auto den = [&](int c) { return fn2[c] > 0 ? std::sqrt(fn2[c]) : 1.0; };
    dwfmm_status worst = DWFMM_OK;
    auto record = [&](dwfmm_status s) {
        if (s == DWFMM_E_BREAKDOWN) worst = DWFMM_E_BREAKDOWN;
        else if (s == DWFMM_E_NOT_CONVERGED && worst == DWFMM_OK) worst = DWFMM_E_NOT_CONVERGED;
    };

    if (op->precision == DWFMM_FP64) {
        HIP_TRY(cg_run(op, lambda, f, alpha, nrhs, rtol, max_iter, DWFMM_FP64, st, hstate, hrr));
        HIP_TRY(residual64(op, lambda, f, alpha, op->q, nrhs, st, res));
        for (int c = 0; c < nrhs; ++c) {
            dwfmm_solve_info &I = info[c];
            I.iters = hstate[nrhs + c];
            I.neg_curvature_steps = hstate[2 * nrhs + c];
            I.refine_steps = 0;
            I.rel_res_recursive = std::sqrt(hrr[c]) / den(c);
            I.rel_res_true = std::sqrt(res[c]) / den(c);
            I.status = hstate[c] == 1 ? DWFMM_OK : (hstate[c] == 2 ? DWFMM_E_BREAKDOWN : DWFMM_E_NOT_CONVERGED);
            record((dwfmm_status)I.status);
        }
    } else {
        // Iterative refinement: FP64 residual, reduced-precision inner CG, alpha += delta.
        const double rtol_in =
            op->ir_inner_rtol > 0 ? op->ir_inner_rtol : (op->precision == DWFMM_FP32 ? 1e-4 : 1e-2);
        std::vector<int32_t> iters(nrhs, 0), neg(nrhs, 0), stall(nrhs, 0), done(nrhs, 0), broke(nrhs, 0), steps(nrhs, 0);
        std::vector<double> best;
        HIP_TRY(residual64(op, lambda, f, alpha, op->ir_r, nrhs, st, res));
        best = res;
        int used = 0;
        for (int c = 0; c < nrhs; ++c) done[c] = std::sqrt(res[c]) <= rtol * den(c);
        for (int outer = 0; outer < op->ir_max_outer && used < max_iter; ++outer) {
            bool any = false;
            for (int c = 0; c < nrhs; ++c) any |= !done[c] && stall[c] < 3;
            if (!any) break;
            // mask: 0 = update this column
            std::vector<int32_t> mask(nrhs);
            for (int c = 0; c < nrhs; ++c) mask[c] = (!done[c] && stall[c] < 3) ? 0 : 1;
            HIP_TRY(hipMemcpyAsync(op->state + 3 * op->max_nrhs, mask.data(), sizeof(int32_t) * nrhs,
                                   hipMemcpyHostToDevice, st));
            HIP_TRY(hipMemsetAsync(op->ir_d, 0, sizeof(double) * total, st));
            const int inner = op->ir_max_inner > 0 ? std::min(op->ir_max_inner, max_iter - used) : max_iter - used;
            HIP_TRY(cg_run(op, lambda, op->ir_r, op->ir_d, nrhs, rtol_in, inner, op->precision, st, hstate, hrr));
            int most = 0;
            for (int c = 0; c < nrhs; ++c) {
                if (mask[c]) continue;
                iters[c] += hstate[nrhs + c];
                neg[c] += hstate[2 * nrhs + c];
                most = std::max(most, hstate[nrhs + c]);
                if (hstate[c] == 2 && hstate[nrhs + c] == 0) broke[c] = 1;
                steps[c]++;
            }
            used += std::max(most, 1);
            // alpha += delta on the columns being refined (scale slot 10 holds 1.0)
            if (nrhs == 1) {
                CgItem it = cg_item(op, lambda, nullptr, op->ir_d, 0.0, 0);
                it.acc = alpha;
                it.frozen = mask[0];
                HIP_TRY(launch_cg(CG_ADD, nullptr, 0, 0, it, st));
            } else {
                std::vector<double> one(nrhs, 1.0);
                HIP_TRY(hipMemcpyAsync(op->scal + 10 * nrhs, one.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice,
                                       st));
                hipLaunchKernelGGL(axpy_kernel, dim3(kEwBlocks), dim3(256), 0, st, alpha, alpha, op->ir_d, op->scal, 10,
                                   1.0, op->state + 3 * op->max_nrhs, 1, total, nrhs);
                HIP_TRY(hipGetLastError());
            }
            HIP_TRY(residual64(op, lambda, f, alpha, op->ir_r, nrhs, st, res));
            std::vector<int32_t> keep(nrhs, 1);  // 0: take the correction back
            bool undo = false;
            for (int c = 0; c < nrhs; ++c) {
                if (mask[c]) continue;
                if (std::sqrt(res[c]) <= rtol * den(c)) done[c] = 1;
                else if (res[c] > best[c]) {
                    keep[c] = 0;
                    undo = true;
                    stall[c] = 3;
                } else if (res[c] == best[c]) stall[c]++;
                else { best[c] = res[c]; stall[c] = 0; }
                if (broke[c]) stall[c] = 3;
            }
            if (undo) {
                // a correction that raised the FP64 residual is taken back and the column stops
                // at the lowest residual it reached
                if (nrhs == 1) {
                    CgItem it = cg_item(op, lambda, nullptr, op->ir_d, 0.0, 0);
                    it.acc = alpha;
                    HIP_TRY(launch_cg(CG_SUB, nullptr, 0, 0, it, st));
                } else {
                    std::vector<double> one(nrhs, 1.0);
                    HIP_TRY(hipMemcpyAsync(op->state + 3 * op->max_nrhs, keep.data(), sizeof(int32_t) * nrhs,
                                           hipMemcpyHostToDevice, st));
                    HIP_TRY(hipMemcpyAsync(op->scal + 10 * nrhs, one.data(), sizeof(double) * nrhs,
                                           hipMemcpyHostToDevice, st));
                    hipLaunchKernelGGL(axpy_kernel, dim3(kEwBlocks), dim3(256), 0, st, alpha, alpha, op->ir_d, op->scal,
                                       10, -1.0, op->state + 3 * op->max_nrhs, 1, total, nrhs);
                    HIP_TRY(hipGetLastError());
                }
                std::vector<double> res2;
                HIP_TRY(residual64(op, lambda, f, alpha, op->ir_r, nrhs, st, res2));
                for (int c = 0; c < nrhs; ++c)
                    if (!keep[c]) res[c] = res2[c];
            }
        }
        for (int c = 0; c < nrhs; ++c) {
            dwfmm_solve_info &I = info[c];
            I.iters = iters[c];
            I.neg_curvature_steps = neg[c];
            I.refine_steps = steps[c];
            I.rel_res_recursive = std::sqrt(res[c]) / den(c);
            I.rel_res_true = std::sqrt(res[c]) / den(c);
            I.status = done[c] ? DWFMM_OK : (broke[c] ? DWFMM_E_BREAKDOWN : DWFMM_E_NOT_CONVERGED);
            record((dwfmm_status)I.status);
        }
    }
    if (worst != DWFMM_OK) g_err = worst == DWFMM_E_BREAKDOWN ? "CG breakdown" : "CG did not converge";
    return worst;
}

// ============================================================== batches of problems
struct dwfmm_batch_s {
    std::vector<dwfmm_op> ops;        // all problems, in caller order
    std::vector<int> item_of;         // op index -> batch item, or -1 (run on its own)
    std::vector<BatchItem> items;
    Arena arena;
    BatchPlan plan;
    const double **d_xs = nullptr;
    double **d_ys = nullptr;
    std::vector<const double *> h_xs;  // staged pointer arrays (pinned by the vectors)
    std::vector<double *> h_ys;
    std::vector<BatchItem> h_items;    // host sources of the set-up uploads, kept until destruction
    std::vector<int2> h_work;
    std::vector<double> m2l_ms;        // tuned M2L times, [launch][4, 2, 1 waves], -1 = not timed
    std::vector<double> m2l_ms_pers;   // the same in the persistent layout
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int flags = 0;
    int force_prec = -1;              // >= 0: every problem runs in this precision (the FP64 companion)
    dwfmm_batch b64 = nullptr;        // FP64 companion plan for the refinement residuals of a solve
    CgItem *d_cg = nullptr;           // solve: CG descriptors and status mirror, one per problem
    double *d_mirror = nullptr;
    StreamFork fork;                  // eager calls: the farfield beside the nearfield
    bool own_fork = false;            // the fork was created for this batch (else a caller's, shared)
    ~dwfmm_batch_s()
    {
        if (own_fork) {
            if (fork.forked) (void)hipEventDestroy(fork.forked);
            if (fork.joined) (void)hipEventDestroy(fork.joined);
            if (fork.side) (void)hipStreamDestroy(fork.side);
        }
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

namespace {

bool batch_eligible(dwfmm_op op)
{
    const DevTree &T = op->tree->D;
    return op->D.kind <= 2 && T.max_leaf <= 128 && T.d <= 32 && op->D.nxp <= 64 && T.dpad == (T.d + 3) / 4 * 4;
}

}  // namespace

// Batch plan for a set of operators.  With sync == false the uploads stay queued on `st`
// (their host sources live in the batch object), for callers that only use the batch on `st`.
static dwfmm_status batch_build(const dwfmm_op *ops, int32_t count, int32_t flags, hipStream_t st, bool sync,
                                dwfmm_batch *out, int force_prec = -1, const StreamFork *shared_fork = nullptr);

extern "C" dwfmm_status dwfmm_batch_create(const dwfmm_op *ops, int32_t count, int32_t flags, void *stream,
                                           dwfmm_batch *out)
{
    return batch_build(ops, count, flags, (hipStream_t)stream, true, out);
}

static dwfmm_status batch_build(const dwfmm_op *ops, int32_t count, int32_t flags, hipStream_t st, bool sync,
                                dwfmm_batch *out, int force_prec, const StreamFork *shared_fork)
{
    if (!out) return fail(DWFMM_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!ops || count < 1) return fail(DWFMM_E_INVALID, "ops is NULL or count < 1");
    for (int i = 0; i < count; ++i)
        if (!ops[i]) return fail(DWFMM_E_INVALID, "ops contains NULL");
    const int forced = (flags >> 4) & 7;
    if ((flags & ~(DWFMM_BATCH_GRAPH | DWFMM_BATCH_TUNE | DWFMM_BATCH_M2L_PERSISTENT | DWFMM_BATCH_M2L_WAVES(7))) !=
            0 ||
        (forced != 0 && forced != 1 && forced != 2 && forced != 4))
        return fail(DWFMM_E_INVALID, "unknown batch flags");
    dwfmm_batch b = new (std::nothrow) dwfmm_batch_s();
    if (!b) return fail(DWFMM_E_NOMEM, "host allocation failed");
    b->ops.assign(ops, ops + count);
    b->item_of.assign(count, -1);
    b->flags = flags;
    b->force_prec = force_prec;
    std::vector<const HostTree *> item_tree;  // host tree of each batch item
    std::vector<const std::vector<double> *> item_work;  // nearfield work per leaf of each item
    for (int i = 0; i < count; ++i) {
        if (!batch_eligible(ops[i])) continue;
        const DevTree &T = ops[i]->tree->D;
        BatchItem it{};
        it.T = T;
        it.O = ops[i]->D;
        it.far = T.min_far_level <= T.J;
        it.precision = force_prec >= 0 ? force_prec : ops[i]->precision;
        b->item_of[i] = (int)b->items.size();
        b->items.push_back(it);
        item_tree.push_back(&ops[i]->tree->H);
        item_work.push_back(&ops[i]->tree->leaf_work);
    }
    // work lists: leaves, per level M2M / L2L, and one slice per kernel variant for M2L and P2P
    std::vector<int2> work;
    BatchPlan &P = b->plan;
    P.leaf_off = 0;
    for (int it = 0; it < (int)b->items.size(); ++it)
        for (int l = 0; l < b->items[it].T.nleaf; ++l) work.push_back(make_int2(it, l));
    P.leaf_cnt = (int)work.size();
    int maxJ = 0;
    for (auto &it : b->items) maxJ = std::max(maxJ, it.T.J);
    for (int j = maxJ - 1; j >= 0; --j) {
        const int off = (int)work.size();
        for (int it = 0; it < (int)b->items.size(); ++it) {
            const BatchItem &I = b->items[it];
            if (!I.far || j < I.T.min_far_level || j >= I.T.J) continue;
            for (int c = (1 << j) - 1; c < (1 << (j + 1)) - 1; ++c) work.push_back(make_int2(it, c));
        }
        if ((int)work.size() > off) P.m2m.push_back({off, (int)work.size() - off});
    }
    for (int j = 1; j <= maxJ; ++j) {
        const int off = (int)work.size();
        for (int it = 0; it < (int)b->items.size(); ++it) {
            const BatchItem &I = b->items[it];
            if (!I.far || j < I.T.min_far_level + 1 || j > I.T.J) continue;
            for (int c = (1 << j) - 1; c < (1 << (j + 1)) - 1; ++c) work.push_back(make_int2(it, c));
        }
        if ((int)work.size() > off) P.l2l.push_back({off, (int)work.size() - off});
    }
    auto key = [&](const BatchItem &I, bool far_list) {
        // the FP64 nearfield of a split Gaussian runs its own kernel variant (kind 4), the FP64
        // nearfield of a Matern kernel within the exponent range its unclamped variant (kind 5)
        const int kind = !far_list && I.O.kind == DWFMM_GAUSSIAN &&
                                 (I.precision == 0 ? I.O.gauss_split : I.O.gauss_split32)
                             ? 4
                             : (!far_list && I.O.kind == DWFMM_MATERN32 && I.precision == 0 && I.O.matern_in_range
                                    ? 5
                                    : I.O.kind);
        return std::vector<int>{kind, (I.T.d + 3) / 4 * 4, far_list ? I.O.nxp / 16 : 0, I.precision != 0};
    };
    std::vector<std::vector<int>> keys;
    for (auto &it : b->items) {
        for (int fl = 0; fl < 2; ++fl) {
            if (fl && !it.far) continue;
            auto k = key(it, fl);
            k.push_back(fl);
            if (std::find(keys.begin(), keys.end(), k) == keys.end()) keys.push_back(k);
        }
    }
    for (auto &k : keys) {
        const bool far_list = k[4];
        std::vector<int2> lst;
        for (int it = 0; it < (int)b->items.size(); ++it) {
            const BatchItem &I = b->items[it];
            auto ki = key(I, far_list);
            ki.push_back(far_list);
            if (ki != k) continue;
            if (far_list) {
                if (!I.far) continue;
                for (int c = (1 << I.T.min_far_level) - 1; c < I.T.ncl; ++c) lst.push_back(make_int2(it, c));
            } else {
                for (int l = 0; l < I.T.nleaf; ++l) lst.push_back(make_int2(it, l));
            }
        }
        if (lst.empty()) continue;
        if (far_list) {
            // longest farfield lists first (ties in list order): the costly clusters start early,
            // and a persistent grid striding over the list takes a balanced mix of them
            // (the list lengths are gathered once: looking them up in the trees inside the sort's
            // comparisons cost most of a plan rebuild)
            std::vector<std::pair<int64_t, int64_t>> kv(lst.size());  // (-list length, position)
            for (size_t i = 0; i < lst.size(); ++i) {
                const HostTree &H = *item_tree[lst[i].x];
                kv[i] = {-(int64_t)(H.Fptr[lst[i].y + 1] - H.Fptr[lst[i].y]), (int64_t)i};
            }
            std::sort(kv.begin(), kv.end());
            std::vector<int2> sorted(lst.size());
            for (size_t i = 0; i < lst.size(); ++i) sorted[i] = lst[kv[i].second];
            lst.swap(sorted);
        }
        if (!far_list) {
            // Workgroup q runs on XCD q % 8.  The list is cut into 8 contiguous segments of equal
            // nearfield work (consecutive leaves of a problem share source points in the XCD's
            // L2), segment k dealt to XCD k and padded to the longest: the leaves of different
            // problems differ several-fold in work, so equal counts per XCD would leave most
            // XCDs idle while one finishes.  Work per leaf: its tree's owned-block entries.
            std::vector<double> wk(lst.size());
            double total = 0.0;
            for (size_t i = 0; i < lst.size(); ++i) {
                wk[i] = (*item_work[lst[i].x])[lst[i].y];
                total += wk[i];
            }
            std::vector<size_t> cut(9, lst.size());
            cut[0] = 0;
            double acc = 0.0;
            for (size_t i = 0, k = 1; i < lst.size() && k < 8; ++i) {
                acc += wk[i];
                while (k < 8 && acc >= total * k / 8.0) cut[k++] = i + 1;
            }
            size_t longest = 0;
            for (int k = 0; k < 8; ++k) longest = std::max(longest, cut[k + 1] - cut[k]);
            std::vector<int2> perm(8 * longest, make_int2(-1, 0));
            for (int k = 0; k < 8; ++k) {
                // the costliest leaves of the segment first (ties in list order), so it ends on short ones
                std::vector<std::pair<double, size_t>> seg;
                for (size_t j = cut[k]; j < cut[k + 1]; ++j) seg.push_back({-wk[j], j});
                std::sort(seg.begin(), seg.end());
                for (size_t j = 0; j < seg.size(); ++j) perm[8 * j + k] = lst[seg[j].second];
            }
            lst.swap(perm);
        }
        BatchLaunch L{k[0], k[1], k[2], k[3], (int)work.size(), (int)lst.size()};
        work.insert(work.end(), lst.begin(), lst.end());
        (far_list ? P.m2l : P.p2p).push_back(L);
    }
    if (work.empty()) work.push_back(make_int2(-1, 0));
    const int nitems = std::max<int>(1, (int)b->items.size());
    BatchItem *d_items;
    int2 *d_work;
    hipError_t e;
    b->h_items = b->items;
    if (b->h_items.empty()) b->h_items.resize(1);
    b->h_work.swap(work);
    if ((e = b->arena.upload(&d_items, b->h_items, st)) != hipSuccess ||
        (e = b->arena.upload(&d_work, b->h_work, st)) != hipSuccess ||
        (e = b->arena.alloc((void **)&b->d_xs, sizeof(double *) * nitems)) != hipSuccess ||
        (e = b->arena.alloc((void **)&b->d_ys, sizeof(double *) * nitems)) != hipSuccess ||
        (sync && (e = hipStreamSynchronize(st)) != hipSuccess)) {
        b->arena.release();
        delete b;
        return fail(e == hipErrorOutOfMemory ? DWFMM_E_NOMEM : DWFMM_E_HIP, std::string("batch setup: ") + hipGetErrorString(e));
    }
    P.items = d_items;
    P.work = d_work;
    P.xs = b->d_xs;
    P.ys = b->d_ys;
    b->h_xs.resize(nitems);
    b->h_ys.resize(nitems);
    b->m2l_ms.assign(3 * P.m2l.size(), -1.0);
    b->m2l_ms_pers.assign(3 * P.m2l.size(), -1.0);
    for (auto &L : P.m2l) {
        if (forced && m2l_wpc_available(L.nxt, forced)) L.wpc = forced;
        if (flags & DWFMM_BATCH_M2L_PERSISTENT) L.grid = kM2lPersistentGrid;
    }
    if ((flags & DWFMM_BATCH_TUNE) && !P.m2l.empty()) {
        // time each compiled shape of every M2L launch on this batch in both layouts (one
        // warm-up, three timed launches) and keep the fastest
        hipEvent_t e0 = nullptr, e1 = nullptr;
        e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        const int shapes[3] = {4, 2, 1};
        for (size_t i = 0; i < P.m2l.size() && e == hipSuccess; ++i) {
            BatchLaunch &L = P.m2l[i];
            float best = -1.0f;
            for (int lay = 0; lay < 2 && e == hipSuccess; ++lay)
                for (int j = 0; j < 3 && e == hipSuccess; ++j) {
                    if (!m2l_wpc_available(L.nxt, shapes[j])) continue;
                    BatchLaunch c = L;
                    c.wpc = shapes[j];
                    c.grid = lay ? kM2lPersistentGrid : 0;
                    float ms = 0.0f;
                    if ((e = launch_batch_m2l(P, c, st)) != hipSuccess || (e = hipEventRecord(e0, st)) != hipSuccess)
                        break;
                    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) e = launch_batch_m2l(P, c, st);
                    if (e == hipSuccess) e = hipEventRecord(e1, st);
                    if (e == hipSuccess) e = hipEventSynchronize(e1);
                    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                    if (e != hipSuccess) break;
                    (lay ? b->m2l_ms_pers : b->m2l_ms)[3 * i + j] = ms / 3.0;
                    if (best < 0.0f || ms < best) {
                        best = ms;
                        L.wpc = c.wpc;
                        L.grid = c.grid;
                    }
                }
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (e != hipSuccess) {
            dwfmm_status s = fail(DWFMM_E_HIP, std::string("batch tuning: ") + hipGetErrorString(e));
            b->arena.release();
            delete b;
            return s;
        }
    }
    // eager batches run the farfield on a side stream: a caller's (plans rebuilt often share one)
    // or one of their own
    if (!(flags & DWFMM_BATCH_GRAPH) && !b->items.empty() && shared_fork && shared_fork->side)
        b->fork = *shared_fork;
    else if (!(flags & DWFMM_BATCH_GRAPH) && !b->items.empty() &&
        (b->own_fork = true,
         (e = hipStreamCreateWithFlags(&b->fork.side, hipStreamNonBlocking)) != hipSuccess ||
         (e = hipEventCreateWithFlags(&b->fork.forked, hipEventDisableTiming)) != hipSuccess ||
         (e = hipEventCreateWithFlags(&b->fork.joined, hipEventDisableTiming)) != hipSuccess)) {
        b->arena.release();
        delete b;
        return fail(DWFMM_E_HIP, std::string("batch streams: ") + hipGetErrorString(e));
    }
    if ((flags & DWFMM_BATCH_GRAPH) && !b->items.empty()) {
        // capture the batched matvec once (its stages in order on one stream); each call refreshes
        // the x/y pointer arrays, then replays it
        hipStream_t cs;
        if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) == hipSuccess) {
            e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                hipError_t el = launch_batch_matvec(P, cs);
                e = hipStreamEndCapture(cs, &b->graph);
                if (el != hipSuccess) e = el;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
            (void)hipStreamDestroy(cs);
        }
        if (e != hipSuccess) {
            dwfmm_status s = fail(DWFMM_E_HIP, std::string("batch graph capture: ") + hipGetErrorString(e));
            b->arena.release();
            delete b;
            return s;
        }
    }
    *out = b;
    return DWFMM_OK;
}

extern "C" dwfmm_status dwfmm_batch_m2l_shapes(dwfmm_batch b, int32_t *wpc, double *ms, int32_t cap, int32_t *count)
{
    if (!b || !count || cap < 0 || (cap > 0 && !wpc)) return fail(DWFMM_E_INVALID, "bad argument");
    const auto &m2l = b->plan.m2l;
    *count = (int32_t)m2l.size();
    for (int i = 0; i < std::min<int>(cap, (int)m2l.size()); ++i) {
        wpc[i] = m2l[i].wpc;
        if (ms)
            for (int j = 0; j < 3; ++j) ms[3 * i + j] = b->m2l_ms[3 * i + j];
    }
    return DWFMM_OK;
}

extern "C" dwfmm_status dwfmm_batch_m2l_layout(dwfmm_batch b, int32_t *grid, double *ms, int32_t cap, int32_t *count)
{
    if (!b || !count || cap < 0 || (cap > 0 && !grid)) return fail(DWFMM_E_INVALID, "bad argument");
    const auto &m2l = b->plan.m2l;
    *count = (int32_t)m2l.size();
    for (int i = 0; i < std::min<int>(cap, (int)m2l.size()); ++i) {
        grid[i] = m2l[i].grid;
        if (ms)
            for (int j = 0; j < 3; ++j) ms[3 * i + j] = b->m2l_ms_pers[3 * i + j];
    }
    return DWFMM_OK;
}

extern "C" dwfmm_status dwfmm_batch_matvec(dwfmm_batch b, const double *const *xs, double *const *ys, void *stream)
{
    if (!b) return fail(DWFMM_E_INVALID, "batch is NULL");
    if (!xs || !ys) return fail(DWFMM_E_INVALID, "xs or ys is NULL");
    hipStream_t st = (hipStream_t)stream;
    for (size_t i = 0; i < b->ops.size(); ++i) {
        if (!xs[i] || !ys[i] || xs[i] == ys[i]) return fail(DWFMM_E_INVALID, "bad x/y pointer in batch");
        const int it = b->item_of[i];
        if (it >= 0) {
            b->h_xs[it] = xs[i];
            b->h_ys[it] = ys[i];
        }
    }
    if (!b->items.empty()) {
        HIP_TRY(hipMemcpyAsync(b->d_xs, b->h_xs.data(), sizeof(double *) * b->items.size(), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(b->d_ys, b->h_ys.data(), sizeof(double *) * b->items.size(), hipMemcpyHostToDevice, st));
        if (b->exec)
            HIP_TRY(hipGraphLaunch(b->exec, st));
        else
            HIP_TRY(launch_batch_matvec(b->plan, st, &b->fork));
    }
    for (size_t i = 0; i < b->ops.size(); ++i) {
        if (b->item_of[i] >= 0) continue;
        dwfmm_op op = b->ops[i];
        HIP_TRY(launch_matvec(op->tree->D, op->D, xs[i], ys[i], 1, 3, b->force_prec >= 0 ? b->force_prec : op->precision,
                              st));
    }
    return DWFMM_OK;
}

extern "C" void dwfmm_batch_destroy(dwfmm_batch b)
{
    if (!b) return;
    if (b->b64) dwfmm_batch_destroy(b->b64);
    b->arena.release();
    delete b;
}

namespace {

// The batched matvec of a solve over the problems still iterating: a plan over a subset of the
// batch's operators (the whole batch at first), rebuilt when the subset halves.  Batched and
// single-problem kernels give the same bits, so the subset never changes a result.
struct SolvePlan {
    dwfmm_batch full = nullptr;  // the batch (or its FP64 companion)
    dwfmm_batch sub = nullptr;   // owned plan over idx, or NULL while idx is the whole batch
    std::vector<int> idx;        // problem index of each operator of the current plan
    std::vector<const double *> xs;
    std::vector<double *> ys;
    ~SolvePlan()
    {
        if (sub) dwfmm_batch_destroy(sub);
    }
    void reset(dwfmm_batch b)
    {
        if (sub) dwfmm_batch_destroy(sub);
        sub = nullptr;
        full = b;
        idx.resize(b->ops.size());
        for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
    }
    // call only after the stream has drained (the old plan may still be referenced by queued work)
    dwfmm_status shrink(const std::vector<int> &keep, hipStream_t st)
    {
        if (keep.empty() || keep.size() * 2 > idx.size()) return DWFMM_OK;
        std::vector<dwfmm_op> ops;
        for (int i : keep) ops.push_back(full->ops[i]);
        dwfmm_batch nb = nullptr;
        dwfmm_status rc = batch_build(ops.data(), (int)ops.size(), full->flags & DWFMM_BATCH_GRAPH, st, true, &nb,
                                      full->force_prec, &full->fork);
        if (rc != DWFMM_OK) return rc;
        if (sub) dwfmm_batch_destroy(sub);
        sub = nb;
        idx = keep;
        return DWFMM_OK;
    }
    dwfmm_status matvec(const std::vector<const double *> &src, const std::vector<double *> &dst, hipStream_t st)
    {
        xs.resize(idx.size());
        ys.resize(idx.size());
        for (size_t k = 0; k < idx.size(); ++k) {
            xs[k] = src[idx[k]];
            ys[k] = dst[idx[k]];
        }
        return dwfmm_batch_matvec(sub ? sub : full, xs.data(), ys.data(), st);
    }
};

}  // namespace

extern "C" dwfmm_status dwfmm_batch_solve(dwfmm_batch b, double lambda, const double *const *fs,
                                          double *const *alphas, double rtol, int32_t max_iter, int32_t check_every,
                                          void *stream, dwfmm_solve_info *infos)
{
    if (!b) return fail(DWFMM_E_INVALID, "batch is NULL");
    if (!fs || !alphas || !infos) return fail(DWFMM_E_INVALID, "fs, alphas or infos is NULL");
    if (!std::isfinite(lambda) || lambda < 0.0) return fail(DWFMM_E_INVALID, "lambda must be finite and >= 0");
    if (!(rtol > 0.0) || max_iter < 0 || check_every < 1)
        return fail(DWFMM_E_INVALID, "rtol must be > 0, max_iter >= 0 and check_every >= 1");
    if (b->force_prec >= 0) return fail(DWFMM_E_INVALID, "not a batch from dwfmm_batch_create");
    const int P = (int)b->ops.size();
    const int prec = b->ops[0]->precision;
    for (int i = 0; i < P; ++i) {
        if (b->ops[i]->precision != prec) return fail(DWFMM_E_INVALID, "the batch's operators differ in precision");
        if (!fs[i] || !alphas[i] || (const double *)alphas[i] == fs[i])
            return fail(DWFMM_E_INVALID, "bad f/alpha pointer in batch");
    }
    hipStream_t st = (hipStream_t)stream;
    if (!b->d_cg) {
        HIP_TRY(b->arena.alloc((void **)&b->d_cg, sizeof(CgItem) * P));
        HIP_TRY(b->arena.alloc((void **)&b->d_mirror, sizeof(double) * 8 * P));
    }
    std::vector<CgItem> items(P);
    std::vector<double> mir(8 * (size_t)P);
    std::vector<const double *> src(P);
    std::vector<double *> dst(P);
    int nblocks = 0;
    auto set_items = [&](auto fill) -> hipError_t {
        // the previous upload from `items` may still be queued
        hipError_t e0 = hipStreamSynchronize(st);
        if (e0 != hipSuccess) return e0;
        nblocks = 0;
        for (int i = 0; i < P; ++i) {
            items[i] = CgItem{};
            fill(i, items[i]);
            items[i].blk0 = nblocks;
            items[i].mirror = b->d_mirror + 8 * (size_t)i;
            nblocks += items[i].nblk;
        }
        return hipMemcpyAsync(b->d_cg, items.data(), sizeof(CgItem) * P, hipMemcpyHostToDevice, st);
    };
    auto step = [&](int s) { return launch_cg(s, b->d_cg, P, nblocks, items[0], st); };
    auto read_mirror = [&]() -> hipError_t {
        hipError_t e = step(CG_MIRROR);
        if (e == hipSuccess) e = hipMemcpyAsync(mir.data(), b->d_mirror, sizeof(double) * 8 * P, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        return e;
    };
    // CG iterations on the current items until no problem steps; matvecs on `plan`, which
    // shrinks to the stepping problems
    SolvePlan plan;
    auto iterate = [&](dwfmm_batch lo, int cap) -> dwfmm_status {
        plan.reset(lo);
        for (int i = 0; i < P; ++i) {
            src[i] = items[i].p;
            dst[i] = items[i].q;
        }
        for (int k = 0; k < cap; ++k) {
            if (k % check_every == 0) {
                HIP_TRY(read_mirror());
                std::vector<int> keep;
                for (int i = 0; i < P; ++i)
                    if (mir[8 * (size_t)i] == 0.0 && mir[8 * (size_t)i + 1] < items[i].max_it) keep.push_back(i);
                if (keep.empty()) break;
                dwfmm_status rc = plan.shrink(keep, st);
                if (rc != DWFMM_OK) return rc;
            }
            dwfmm_status rc = plan.matvec(src, dst, st);
            if (rc != DWFMM_OK) return rc;
            for (int sstep : {CG_PQ, CG_ALPHA, CG_XR, CG_BETA, CG_P}) HIP_TRY(step(sstep));
        }
        HIP_TRY(read_mirror());
        return DWFMM_OK;
    };
    // res[i] = |f_i - (K~_64 + lambda I) alpha_i|^2 for the problems with include[i]
    dwfmm_batch full64 = b;
    std::vector<double> res(P, 0.0);
    auto residual = [&](const std::vector<int> &include) -> dwfmm_status {
        for (int i = 0; i < P; ++i) {
            src[i] = alphas[i];
            dst[i] = prec == DWFMM_FP64 ? b->ops[i]->q : b->ops[i]->ir_r;
        }
        SolvePlan rp;
        rp.reset(full64);
        std::vector<int> keep;
        for (int i = 0; i < P; ++i)
            if (include[i]) keep.push_back(i);
        dwfmm_status rc = rp.shrink(keep, st);
        if (rc != DWFMM_OK) return rc;
        rc = rp.matvec(src, dst, st);
        if (rc != DWFMM_OK) return rc;
        HIP_TRY(set_items([&](int i, CgItem &it) {
            it = cg_item(b->ops[i], lambda, nullptr, nullptr, 0.0, 0);
            it.f = fs[i];
            it.v = alphas[i];
            it.out = dst[i];
            it.frozen = !include[i];
        }));
        HIP_TRY(step(CG_RES));
        HIP_TRY(step(CG_RES_SUM));
        HIP_TRY(read_mirror());
        for (int i = 0; i < P; ++i)
            if (include[i]) res[i] = mir[8 * (size_t)i + 5];
        return DWFMM_OK;
    };
    std::vector<double> den(P, 1.0);
    dwfmm_status worst = DWFMM_OK;
    auto record = [&](dwfmm_status s2) {
        if (s2 == DWFMM_E_BREAKDOWN) worst = DWFMM_E_BREAKDOWN;
        else if (s2 == DWFMM_E_NOT_CONVERGED && worst == DWFMM_OK) worst = DWFMM_E_NOT_CONVERGED;
    };
    const std::vector<int> all(P, 1);

    if (prec == DWFMM_FP64) {
        for (int i = 0; i < P; ++i) {
            src[i] = alphas[i];
            dst[i] = b->ops[i]->q;
        }
        plan.reset(b);
        dwfmm_status rc = plan.matvec(src, dst, st);
        if (rc != DWFMM_OK) return rc;
        HIP_TRY(set_items([&](int i, CgItem &it) { it = cg_item(b->ops[i], lambda, fs[i], alphas[i], rtol, max_iter); }));
        HIP_TRY(step(CG_START));
        HIP_TRY(step(CG_START_SUM));
        rc = iterate(b, max_iter);
        if (rc != DWFMM_OK) return rc;
        std::vector<double> m(mir);
        rc = residual(all);
        if (rc != DWFMM_OK) return rc;
        for (int i = 0; i < P; ++i) {
            const double *mi = m.data() + 8 * (size_t)i;
            const double dn = mi[4] > 0 ? std::sqrt(mi[4]) : 1.0;
            dwfmm_solve_info &I = infos[i];
            I.iters = (int32_t)mi[1];
            I.neg_curvature_steps = (int32_t)mi[2];
            I.refine_steps = 0;
            I.rel_res_recursive = std::sqrt(mi[3]) / dn;
            I.rel_res_true = std::sqrt(res[i]) / dn;
            I.status = mi[0] == 1.0 ? DWFMM_OK : (mi[0] == 2.0 ? DWFMM_E_BREAKDOWN : DWFMM_E_NOT_CONVERGED);
            record((dwfmm_status)I.status);
        }
    } else {
        // iterative refinement per problem, its outer steps taken together: FP64 residual on
        // the FP64 companion plan, inner CG on the batch's own (reduced) matvec, alpha += delta
        if (!b->b64) {
            dwfmm_status rc =
                batch_build(b->ops.data(), P, b->flags & DWFMM_BATCH_GRAPH, st, true, &b->b64, DWFMM_FP64, &b->fork);
            if (rc != DWFMM_OK) return rc;
        }
        full64 = b->b64;
        for (int i = 0; i < P; ++i) {
            dwfmm_op op = b->ops[i];
            HIP_TRY(launch_dot(fs[i], fs[i], op->tree->D.n, 1, op->partial, op->scal + 9, st));
        }
        dwfmm_status rc = residual(all);
        if (rc != DWFMM_OK) return rc;
        std::vector<int32_t> iters(P, 0), neg(P, 0), stall(P, 0), done(P, 0), broke(P, 0), steps(P, 0), used(P, 0);
        std::vector<double> best(res);
        for (int i = 0; i < P; ++i) {
            const double ff = mir[8 * (size_t)i + 6];
            den[i] = ff > 0 ? std::sqrt(ff) : 1.0;
            done[i] = std::sqrt(res[i]) <= rtol * den[i];
        }
        for (int outer = 0;; ++outer) {
            std::vector<int> run(P, 0);
            bool any = false;
            for (int i = 0; i < P; ++i) {
                run[i] = !done[i] && stall[i] < 3 && outer < b->ops[i]->ir_max_outer && used[i] < max_iter;
                any |= run[i] != 0;
            }
            if (!any) break;
            int cap = 0;
            HIP_TRY(set_items([&](int i, CgItem &it) {
                dwfmm_op op = b->ops[i];
                const double rtol_in =
                    op->ir_inner_rtol > 0 ? op->ir_inner_rtol : (op->precision == DWFMM_FP32 ? 1e-4 : 1e-2);
                const int inner =
                    op->ir_max_inner > 0 ? std::min(op->ir_max_inner, max_iter - used[i]) : max_iter - used[i];
                it = cg_item(op, lambda, op->ir_r, op->ir_d, rtol_in, run[i] ? inner : 0);
                it.zero_x = 1;
                it.frozen = !run[i];
                if (run[i]) cap = std::max(cap, inner);
            }));
            HIP_TRY(step(CG_START));
            HIP_TRY(step(CG_START_SUM));
            rc = iterate(b, cap);
            if (rc != DWFMM_OK) return rc;
            for (int i = 0; i < P; ++i) {
                if (!run[i]) continue;
                const double *mi = mir.data() + 8 * (size_t)i;
                const int it_i = (int)mi[1];
                iters[i] += it_i;
                neg[i] += (int)mi[2];
                used[i] += std::max(it_i, 1);
                if (mi[0] == 2.0 && it_i == 0) broke[i] = 1;
                steps[i]++;
            }
            // alpha += delta on the problems being refined
            HIP_TRY(set_items([&](int i, CgItem &it) {
                it = cg_item(b->ops[i], lambda, nullptr, b->ops[i]->ir_d, 0.0, 0);
                it.acc = alphas[i];
                it.frozen = !run[i];
            }));
            HIP_TRY(step(CG_ADD));
            rc = residual(run);
            if (rc != DWFMM_OK) return rc;
            std::vector<int> back(P, 0);
            bool undo = false;
            for (int i = 0; i < P; ++i) {
                if (!run[i]) continue;
                if (std::sqrt(res[i]) <= rtol * den[i]) done[i] = 1;
                else if (res[i] > best[i]) {
                    back[i] = 1;
                    undo = true;
                    stall[i] = 3;
                } else if (res[i] == best[i]) stall[i]++;
                else {
                    best[i] = res[i];
                    stall[i] = 0;
                }
                if (broke[i]) stall[i] = 3;
            }
            if (undo) {
                // as alone: a correction that raised the residual is taken back, the problem stops
                HIP_TRY(set_items([&](int i, CgItem &it) {
                    it = cg_item(b->ops[i], lambda, nullptr, b->ops[i]->ir_d, 0.0, 0);
                    it.acc = alphas[i];
                    it.frozen = !back[i];
                }));
                HIP_TRY(step(CG_SUB));
                rc = residual(back);
                if (rc != DWFMM_OK) return rc;
            }
        }
        for (int i = 0; i < P; ++i) {
            dwfmm_solve_info &I = infos[i];
            I.iters = iters[i];
            I.neg_curvature_steps = neg[i];
            I.refine_steps = steps[i];
            I.rel_res_recursive = std::sqrt(res[i]) / den[i];
            I.rel_res_true = std::sqrt(res[i]) / den[i];
            I.status = done[i] ? DWFMM_OK : (broke[i] ? DWFMM_E_BREAKDOWN : DWFMM_E_NOT_CONVERGED);
            record((dwfmm_status)I.status);
        }
    }
    if (worst != DWFMM_OK) g_err = worst == DWFMM_E_BREAKDOWN ? "CG breakdown" : "CG did not converge";
    return worst;
}

// ============================================================== solve server (continuous batching)
namespace {

struct ServerRequest {
    int64_t id = 0;
    int64_t n = 0;
    int d = 0, leaf = 0, max_iter = 0, precision = 0;
    double eta = 0, q = 0, lambda = 0, rtol = 0;
    dwfmm_kernel kernel{};
    std::vector<double> pts, b, f;  // host copies of the inputs
    size_t need = 0;                // device bytes counted against the budget from hand-off to retirement
    dwfmm_tree tree = nullptr;      // device state from preparation to retirement
    dwfmm_op op = nullptr;
    double *d_alpha = nullptr, *d_f = nullptr;
    dwfmm_status prep = DWFMM_OK;   // outcome of the preparation and its message
    std::string prep_err;
    size_t exact = 0;               // device bytes from the host-built tree (0 until it is built)
    bool more = false;              // handed back: exact exceeds the bytes reserved at hand-off
    int iters = 0;
    std::vector<double> alpha;      // result
    dwfmm_solve_info info{};
    double t_submit = 0, t_handoff = 0, t_active = 0, t_retired = 0;  // seconds since the server's creation
};

constexpr int kServerWorkers = 4;

}  // namespace

struct dwfmm_server_s {
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
    size_t budget = 0, held = 0;
    int max_active = 0, check_every = 1, device = 0;
    hipStream_t st = nullptr;
    std::deque<ServerRequest *> queue;  // submitted, waiting for budget and a slot (FIFO)
    int preparing = 0;                  // handed to the workers, not yet active
    std::vector<ServerRequest *> active;
    std::vector<ServerRequest *> finished;
    int64_t next_id = 0, ticks = 0;
    dwfmm_batch batch = nullptr;
    std::vector<dwfmm_batch> old_batches;  // replaced plans, freed at the next synchronisation
    bool dirty = true;
    std::vector<const double *> xs;
    std::vector<double *> ys;
    // CG descriptors of the active requests (rebuilt with the batch plan) and their status mirror
    CgItem *d_cg = nullptr;
    double *d_mirror = nullptr;
    std::vector<CgItem> h_cg;
    std::vector<std::vector<CgItem>> old_cg;  // host sources of queued uploads, freed at the next synchronisation
    std::vector<double> h_mirror;
    int cg_nblocks = 0;
    StreamFork fork;  // the batched farfield beside the nearfield, shared by every plan of the server
    // host-side accounting: ticks, plan rebuilds, seconds rebuilding plans, launching a tick's
    // work, waiting for the device at checks, retiring requests
    int64_t n_rebuilds = 0;
    double t_rebuild = 0, t_launch = 0, t_wait = 0, t_retire = 0;
    // preparation workers: each builds tree, operator and CG start on a stream of its own
    std::mutex mu;
    std::condition_variable cv_todo, cv_ready;
    std::deque<ServerRequest *> todo, ready;
    bool stop = false;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> worker_streams;
    ~dwfmm_server_s();
};

namespace {

void free_request_device(ServerRequest *r)
{
    if (r->op) dwfmm_op_destroy(r->op);
    if (r->tree) dwfmm_tree_destroy(r->tree);
    if (r->d_alpha) (void)hipFree(r->d_alpha);
    if (r->d_f) (void)hipFree(r->d_f);
    r->op = nullptr;
    r->tree = nullptr;
    r->d_alpha = r->d_f = nullptr;
}

void release_request(ServerRequest *r, size_t &held)
{
    free_request_device(r);
    held -= std::min(held, r->need);
    r->need = 0;
    std::vector<double>().swap(r->pts);
    std::vector<double>().swap(r->f);
}

// Device bytes a request will hold: the operator estimate with its index-set size, plus alpha and f.
size_t request_bytes(const ServerRequest &r)
{
    std::vector<double> om(r.d);
    std::string err;
    HostBasis B;
    int nx = 64;
    if (compute_weights(DWFMM_W_R1, r.d, r.b.data(), r.eta, nullptr, om.data(), err) &&
        build_basis(r.d, om.data(), r.q, B, err))
        nx = B.nx;
    return dwfmm_estimate_bytes(r.n, r.d, r.leaf, nx, 1) + 2 * (size_t)r.n * sizeof(double);
}

// First phase of a request's preparation, host only: the tree and the exact device bytes the
// request will hold (tree, operator, alpha and f).
dwfmm_status prepare_host(ServerRequest *r)
{
    dwfmm_status rc = tree_host(r->pts, r->n, r->d, r->b.data(), r->leaf, r->eta, &r->tree, 0);
    if (rc != DWFMM_OK) return rc;
    dwfmm_opts o{};
    o.precision = r->precision;
    o.max_nrhs = 1;
    const size_t ob = dwfmm_op_bytes_for(r->tree, r->q, &o);
    if (ob == 0) return fail(DWFMM_E_INVALID, "index set of the request cannot be built");
    r->exact = ob + 2 * sizeof(double) * (size_t)r->n;
    return DWFMM_OK;
}

// Second phase: upload the tree, build the operator, alpha = 0 and the CG start r = p = f,
// with its scalars.  Runs on a worker thread and its stream; returns once the stream has
// drained, so the main stream may use the request without waiting on it.
dwfmm_status prepare_request(ServerRequest *r, hipStream_t ws)
{
    dwfmm_status rc = tree_upload(r->tree, ws);
    if (rc != DWFMM_OK) return rc;
    dwfmm_opts o{};
    o.precision = r->precision;
    o.max_nrhs = 1;
    o.check_every = 1;
    rc = dwfmm_fmm_create(r->tree, r->kernel, r->q, &o, ws, &r->op);
    if (rc != DWFMM_OK) return rc;
    const size_t nb = sizeof(double) * r->n;
    HIP_TRY(hipMalloc(&r->d_alpha, nb));
    HIP_TRY(hipMalloc(&r->d_f, nb));
    HIP_TRY(hipMemcpyAsync(r->d_f, r->f.data(), nb, hipMemcpyHostToDevice, ws));
    // alpha = 0, so A alpha = 0: the start step clears both instead of running a matvec
    CgItem it = cg_item(r->op, r->lambda, r->d_f, r->d_alpha, r->rtol, r->max_iter);
    it.zero_x = 1;
    HIP_TRY(launch_cg(CG_START, nullptr, 0, 0, it, ws));
    HIP_TRY(launch_cg(CG_START_SUM, nullptr, 0, 0, it, ws));
    HIP_TRY(hipStreamSynchronize(ws));
    return DWFMM_OK;
}

void worker_main(dwfmm_server s, int w)
{
    (void)hipSetDevice(s->device);
    hipStream_t ws = s->worker_streams[w];
    for (;;) {
        ServerRequest *r;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_todo.wait(lk, [&] { return s->stop || !s->todo.empty(); });
            if (s->stop) return;
            r = s->todo.front();
            s->todo.pop_front();
        }
        if (!r->tree) {
            r->prep = prepare_host(r);
            if (r->prep == DWFMM_OK && r->exact > r->need) {
                // reserved too little: back to the main thread, which re-queues it with its exact bytes
                r->more = true;
                {
                    std::lock_guard<std::mutex> lk(s->mu);
                    s->ready.push_back(r);
                }
                s->cv_ready.notify_one();
                continue;
            }
        }
        if (r->prep == DWFMM_OK) r->prep = prepare_request(r, ws);
        if (r->prep != DWFMM_OK) {
            r->prep_err = g_err;
            (void)hipStreamSynchronize(ws);  // nothing of the failed request stays in flight
        }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->ready.push_back(r);
        }
        s->cv_ready.notify_one();
    }
}

// Hand waiting requests to the workers while slots and budget allow, first come first served
// (a request is always taken when nothing else holds memory).  Its bytes count from here.
void hand_off(dwfmm_server s)
{
    bool any = false;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        while (!s->queue.empty() && (int)s->active.size() + s->preparing < s->max_active) {
            ServerRequest *r = s->queue.front();
            const bool idle = s->active.empty() && s->preparing == 0;
            if (!idle && s->held + r->need > s->budget) break;
            s->queue.pop_front();
            s->held += r->need;
            s->preparing++;
            r->t_handoff = s->now();
            s->todo.push_back(r);
            any = true;
        }
    }
    if (any) s->cv_todo.notify_all();
}

// Prepared requests join the active set (a failed preparation finishes the request with its
// status); with `wait`, block until at least one is ready.
void admit_ready(dwfmm_server s, bool wait)
{
    std::deque<ServerRequest *> got;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        if (wait) s->cv_ready.wait(lk, [&] { return !s->ready.empty(); });
        got.swap(s->ready);
    }
    for (ServerRequest *r : got) {
        s->preparing--;
        if (r->more) {
            // its host tree is built; it waits at the front of the queue for its exact bytes
            r->more = false;
            s->held -= std::min(s->held, r->need);
            r->need = r->exact;
            s->queue.push_front(r);
            continue;
        }
        if (r->prep != DWFMM_OK) {
            release_request(r, s->held);
            r->info.status = r->prep;
            r->t_active = r->t_retired = s->now();
            s->finished.push_back(r);
            continue;
        }
        const size_t actual = dwfmm_op_bytes(r->op) + 2 * sizeof(double) * (size_t)r->n;
        s->held = s->held - std::min(s->held, r->need) + actual;
        r->need = actual;
        r->iters = 0;
        r->t_active = s->now();
        s->active.push_back(r);
        s->dirty = true;
    }
}

// Finish a request: true FP64 residual, alpha to the host, release device memory.
dwfmm_status retire(dwfmm_server s, ServerRequest *r, int32_t state)
{
    hipStream_t st = s->st;
    dwfmm_op op = r->op;
    std::vector<double> res, sc(2);
    std::vector<int32_t> hs(3);
    HIP_TRY(hipMemcpyAsync(sc.data(), op->scal, sizeof(double) * 2, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hs.data(), op->state, sizeof(int32_t) * 3, hipMemcpyDeviceToHost, st));
    HIP_TRY(residual64(op, r->lambda, r->d_f, r->d_alpha, op->q, 1, st, res));
    r->alpha.resize(r->n);
    HIP_TRY(hipMemcpyAsync(r->alpha.data(), r->d_alpha, sizeof(double) * r->n, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const double den = sc[1] > 0 ? std::sqrt(sc[1]) : 1.0;
    r->info.iters = hs[1];
    r->info.neg_curvature_steps = hs[2];
    r->info.refine_steps = 0;
    r->info.rel_res_recursive = std::sqrt(sc[0]) / den;
    r->info.rel_res_true = std::sqrt(res[0]) / den;
    r->info.status = state == 1 ? DWFMM_OK : (state == 2 ? DWFMM_E_BREAKDOWN : DWFMM_E_NOT_CONVERGED);
    // a reduced-precision request converges on its own operator; it has met its tolerance only if the
    // FP64 residual has too
    if (r->info.status == DWFMM_OK && r->precision != DWFMM_FP64 && !(r->info.rel_res_true <= r->rtol))
        r->info.status = DWFMM_E_NOT_CONVERGED;
    release_request(r, s->held);
    r->t_retired = s->now();
    return DWFMM_OK;
}

}  // namespace

dwfmm_server_s::~dwfmm_server_s()
{
    {
        std::lock_guard<std::mutex> lk(mu);
        stop = true;
    }
    cv_todo.notify_all();
    for (auto &t : workers) t.join();
    (void)hipStreamSynchronize(st);
    if (batch) dwfmm_batch_destroy(batch);
    for (dwfmm_batch b : old_batches) dwfmm_batch_destroy(b);
    for (auto *v : {&queue, &todo, &ready})
        for (ServerRequest *r : *v) {
            free_request_device(r);
            delete r;
        }
    for (auto *v : {&active, &finished})
        for (ServerRequest *r : *v) {
            free_request_device(r);
            delete r;
        }
    for (hipStream_t w : worker_streams) (void)hipStreamDestroy(w);
    if (d_cg) (void)hipFree(d_cg);
    if (d_mirror) (void)hipFree(d_mirror);
    if (fork.forked) (void)hipEventDestroy(fork.forked);
    if (fork.joined) (void)hipEventDestroy(fork.joined);
    if (fork.side) (void)hipStreamDestroy(fork.side);
}

extern "C" dwfmm_status dwfmm_server_create(size_t budget_bytes, int32_t max_active, int32_t check_every,
                                            void *stream, dwfmm_server *out)
{
    if (!out) return fail(DWFMM_E_INVALID, "out is NULL");
    *out = nullptr;
    if (budget_bytes == 0 || max_active < 1 || check_every < 1)
        return fail(DWFMM_E_INVALID, "budget must be > 0, max_active and check_every >= 1");
    dwfmm_server s = new (std::nothrow) dwfmm_server_s();
    if (!s) return fail(DWFMM_E_NOMEM, "host allocation failed");
    s->budget = budget_bytes;
    s->max_active = max_active;
    s->check_every = check_every;
    s->st = (hipStream_t)stream;
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipMalloc(&s->d_cg, sizeof(CgItem) * max_active);
    if (e == hipSuccess) e = hipMalloc(&s->d_mirror, sizeof(double) * 8 * max_active);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->fork.side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->fork.forked, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->fork.joined, hipEventDisableTiming);
    for (int w = 0; w < kServerWorkers && e == hipSuccess; ++w) {
        hipStream_t ws = nullptr;
        e = hipStreamCreateWithFlags(&ws, hipStreamNonBlocking);
        if (e == hipSuccess) s->worker_streams.push_back(ws);
    }
    if (e != hipSuccess) {
        delete s;
        return fail(DWFMM_E_HIP, std::string("server set-up: ") + hipGetErrorString(e));
    }
    try {
        for (int w = 0; w < kServerWorkers; ++w) s->workers.emplace_back(worker_main, s, w);
    } catch (...) {
        delete s;
        return fail(DWFMM_E_NOMEM, "could not start the preparation threads");
    }
    *out = s;
    return DWFMM_OK;
}

extern "C" dwfmm_status dwfmm_server_submit(dwfmm_server s, const dwfmm_request *req, int64_t *id)
{
    if (!s || !req || !id) return fail(DWFMM_E_INVALID, "NULL argument");
    const dwfmm_request &q = *req;
    if (!q.points || !q.dim_weights || !q.f) return fail(DWFMM_E_INVALID, "points, dim_weights or f is NULL");
    if (q.n < 1 || q.n > (int64_t)1 << 30 || q.d < 1 || q.d > kMaxDim || q.leaf_size < 1 || q.leaf_size > 1024 ||
        !(q.eta > 0.0) || !(q.q >= 0.0) || !(q.lambda >= 0.0) || !(q.rtol > 0.0) || q.max_iter < 0 ||
        q.kernel.kind < 0 || q.kernel.kind > 3 || !(q.kernel.ell > 0.0) || q.precision < 0 || q.precision > 2)
        return fail(DWFMM_E_INVALID, "request argument out of range");
    for (int k = 0; k < q.d; ++k)
        if (!(q.dim_weights[k] > 0.0) || !std::isfinite(q.dim_weights[k]))
            return fail(DWFMM_E_INVALID, "dim_weights must be finite and > 0");
    ServerRequest *r = new (std::nothrow) ServerRequest();
    if (!r) return fail(DWFMM_E_NOMEM, "host allocation failed");
    r->id = s->next_id++;
    r->n = q.n;
    r->d = q.d;
    r->leaf = q.leaf_size;
    r->eta = q.eta;
    r->q = q.q;
    r->lambda = q.lambda;
    r->rtol = q.rtol;
    r->max_iter = q.max_iter;
    r->precision = q.precision;
    r->kernel = q.kernel;
    r->pts.assign(q.points, q.points + (size_t)q.n * q.d);
    r->b.assign(q.dim_weights, q.dim_weights + q.d);
    r->f.assign(q.f, q.f + q.n);
    r->need = request_bytes(*r);
    r->t_submit = s->now();
    s->queue.push_back(r);
    *id = r->id;
    hand_off(s);
    return DWFMM_OK;
}

extern "C" dwfmm_status dwfmm_server_tick(dwfmm_server s, int32_t *n_active, int32_t *n_queued)
{
    if (!s) return fail(DWFMM_E_INVALID, "server is NULL");
    hipStream_t st = s->st;
    hand_off(s);
    admit_ready(s, s->active.empty() && s->preparing > 0);
    if (!s->active.empty()) {
        // one batched matvec q = K~ p over all active requests
        double tm = s->now();
        if (s->dirty) {
            s->n_rebuilds++;
            if (s->batch) s->old_batches.push_back(s->batch);
            s->batch = nullptr;
            std::vector<dwfmm_op> ops;
            for (ServerRequest *r : s->active) ops.push_back(r->op);
            dwfmm_status rc = batch_build(ops.data(), (int)ops.size(), 0, st, false, &s->batch, -1, &s->fork);
            if (rc != DWFMM_OK) return rc;
            s->old_cg.push_back(std::move(s->h_cg));
            s->h_cg.clear();
            s->cg_nblocks = 0;
            for (ServerRequest *r : s->active) {
                CgItem it = cg_item(r->op, r->lambda, r->d_f, r->d_alpha, r->rtol, r->max_iter);
                it.blk0 = s->cg_nblocks;
                it.mirror = s->d_mirror + 8 * s->h_cg.size();
                s->cg_nblocks += it.nblk;
                s->h_cg.push_back(it);
            }
            HIP_TRY(hipMemcpyAsync(s->d_cg, s->h_cg.data(), sizeof(CgItem) * s->h_cg.size(), hipMemcpyHostToDevice,
                                   st));
            s->dirty = false;
            const double t1 = s->now();
            s->t_rebuild += t1 - tm;
            tm = t1;
        }
        s->xs.clear();
        s->ys.clear();
        for (ServerRequest *r : s->active) {
            s->xs.push_back(r->op->p);
            s->ys.push_back(r->op->q);
        }
        dwfmm_status rc = dwfmm_batch_matvec(s->batch, s->xs.data(), s->ys.data(), st);
        if (rc != DWFMM_OK) return rc;
        // the CG update of every active request (FP64, its own scalars on the device): each step
        // is one launch over all of them
        const int nact = (int)s->active.size();
        for (int step : {CG_PQ, CG_ALPHA, CG_XR, CG_BETA, CG_P})
            HIP_TRY(launch_cg(step, s->d_cg, nact, s->cg_nblocks, s->h_cg[0], st));
        for (ServerRequest *r : s->active) r->iters++;
        s->ticks++;
        s->t_launch += s->now() - tm;
        // every check_every ticks (and when a request reaches max_iter): retire finished requests.
        // This is the only place the tick waits for the device.
        bool due = s->ticks % s->check_every == 0;
        for (ServerRequest *r : s->active) due |= r->iters >= r->max_iter;
        if (due) {
            s->h_mirror.resize(8 * (size_t)nact);
            HIP_TRY(launch_cg(CG_MIRROR, s->d_cg, nact, s->cg_nblocks, s->h_cg[0], st));
            HIP_TRY(hipMemcpyAsync(s->h_mirror.data(), s->d_mirror, sizeof(double) * 8 * nact, hipMemcpyDeviceToHost,
                                   st));
            tm = s->now();
            HIP_TRY(hipStreamSynchronize(st));
            const double tw = s->now();
            s->t_wait += tw - tm;
            std::vector<int32_t> flags(nact);
            for (int i = 0; i < nact; ++i) flags[i] = (int32_t)s->h_mirror[8 * (size_t)i];
            for (dwfmm_batch b : s->old_batches) dwfmm_batch_destroy(b);
            s->old_batches.clear();
            s->old_cg.clear();
            std::vector<ServerRequest *> keep;
            for (size_t i = 0; i < s->active.size(); ++i) {
                ServerRequest *r = s->active[i];
                if (flags[i] != 0 || r->iters >= r->max_iter) {
                    dwfmm_status rc = retire(s, r, flags[i]);
                    if (rc != DWFMM_OK) return rc;
                    s->finished.push_back(r);
                    s->dirty = true;
                } else {
                    keep.push_back(r);
                }
            }
            s->active.swap(keep);
            hand_off(s);
            s->t_retire += s->now() - tw;
        }
    }
    if (n_active) *n_active = (int32_t)s->active.size();
    if (n_queued) *n_queued = (int32_t)(s->queue.size() + s->preparing);
    return DWFMM_OK;
}

extern "C" dwfmm_status dwfmm_server_result(dwfmm_server s, int64_t id, double *alpha, dwfmm_solve_info *info,
                                            double *times, int32_t *done)
{
    if (!s || !done) return fail(DWFMM_E_INVALID, "NULL argument");
    *done = 0;
    for (size_t i = 0; i < s->finished.size(); ++i) {
        ServerRequest *r = s->finished[i];
        if (r->id != id) continue;
        if (alpha) std::copy(r->alpha.begin(), r->alpha.end(), alpha);
        if (info) *info = r->info;
        if (times) {
            times[0] = r->t_submit;
            times[1] = r->t_handoff;
            times[2] = r->t_active;
            times[3] = r->t_retired;
        }
        *done = 1;
        s->finished.erase(s->finished.begin() + i);
        delete r;
        return DWFMM_OK;
    }
    return DWFMM_OK;
}

extern "C" dwfmm_status dwfmm_server_finished(dwfmm_server s, int64_t *ids, int32_t cap, int32_t *count)
{
    if (!s || !count || cap < 0 || (cap > 0 && !ids)) return fail(DWFMM_E_INVALID, "bad argument");
    *count = (int32_t)s->finished.size();
    for (int i = 0; i < std::min<int>(cap, (int)s->finished.size()); ++i) ids[i] = s->finished[i]->id;
    return DWFMM_OK;
}

extern "C" dwfmm_status dwfmm_server_stats(dwfmm_server s, double *out)
{
    if (!s || !out) return fail(DWFMM_E_INVALID, "NULL argument");
    out[0] = (double)s->ticks;
    out[1] = (double)s->n_rebuilds;
    out[2] = s->t_rebuild;
    out[3] = s->t_launch;
    out[4] = s->t_wait;
    out[5] = s->t_retire;
    return DWFMM_OK;
}

extern "C" size_t dwfmm_server_bytes(dwfmm_server s) { return s ? s->held : 0; }

extern "C" void dwfmm_server_destroy(dwfmm_server s) { delete s; }

// ============================================================== evaluation at new points
struct dwfmm_eval_s {
    dwfmm_op op = nullptr;  // the source operator (must outlive the plan)
    HostTree H;             // target tree
    DevTree D{};
    DevOp O{};
    Arena arena;
    int64_t nF = 0, nN = 0;
};

extern "C" dwfmm_status dwfmm_eval_create(dwfmm_op op, const double *targets, int64_t m, void *stream,
                                          dwfmm_eval *out)
{
    if (!out) return fail(DWFMM_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!op || !targets) return fail(DWFMM_E_INVALID, "op or targets is NULL");
    if (m < 1 || m > (int64_t)1 << 30) return fail(DWFMM_E_INVALID, "m must be in [1, 2^30]");
    const dwfmm_tree src = op->tree;
    const HostTree &Hs = src->H;
    const int d = Hs.d, dp = src->D.dpad, nx = op->B.nx;
    hipStream_t st = (hipStream_t)stream;
    std::vector<double> pts((size_t)m * d);
    HIP_TRY(hipMemcpyAsync(pts.data(), targets, pts.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (double v : pts)
        if (!std::isfinite(v)) return fail(DWFMM_E_NONFINITE, "targets contain NaN or Inf");
    dwfmm_eval ev = new (std::nothrow) dwfmm_eval_s();
    if (!ev) return fail(DWFMM_E_NOMEM, "host allocation failed");
    ev->op = op;
    std::string err;
    // target tree of the source tree's depth, same rules; cross partition with the same admissibility
    if (!build_tree(pts.data(), m, d, Hs.b.data(), Hs.leaf, Hs.eta, ev->H, err, Hs.J, false)) {
        delete ev;
        return fail(DWFMM_E_INVALID, err);
    }
    HostTree &H = ev->H;
    partition_pairs(H, Hs, Hs.eta, H.Fptr, H.Fsrc, H.Nptr, H.Nsrc, H.min_far_level);
    ev->nF = (int64_t)H.Fsrc.size();
    ev->nN = (int64_t)H.Nsrc.size();
    const int32_t lf = (int32_t)(H.nleaf - 1);
    std::vector<double> Xs((size_t)dp * m, 0.0);
    for (int64_t i = 0; i < m; ++i)
        for (int k = 0; k < d; ++k) Xs[(size_t)k * m + i] = pts[(size_t)H.perm[i] * d + k];
    std::vector<double> clo(H.lo), csc((size_t)H.ncl * d), coff((size_t)H.ncl * d);
    for (size_t i = 0; i < csc.size(); ++i) {
        const double w = H.hi[i] - H.lo[i];
        csc[i] = w > 0 ? 1.0 / w : 0.0;
        coff[i] = w > 0 ? 0.0 : 0.5;
    }
    // nearfield lists per target leaf, naming source leaves leaf-locally
    std::vector<int32_t> nptr_leaf(H.nleaf + 1), nsrc_local(H.Nsrc.size());
    for (int64_t l = 0; l <= H.nleaf; ++l) nptr_leaf[l] = H.Nptr[lf + l];
    for (size_t i = 0; i < H.Nsrc.size(); ++i) nsrc_local[i] = H.Nsrc[i] - lf;
    int max_leaf = 0;
    for (int64_t l = 0; l < H.nleaf; ++l) max_leaf = std::max(max_leaf, H.end[lf + l] - H.begin[lf + l]);
    // launch order of the cross nearfield: 8 segments of equal work (target points x listed source
    // points), costliest target leaf first within a segment
    std::vector<int32_t> near_order;
    {
        std::vector<double> nw(H.nleaf, 0.0);
        for (int64_t l = 0; l < H.nleaf; ++l) {
            double ns = 0.0;
            for (int32_t q = nptr_leaf[l]; q < nptr_leaf[l + 1]; ++q) ns += Hs.end[H.Nsrc[q]] - Hs.begin[H.Nsrc[q]];
            nw[l] = (double)(H.end[lf + l] - H.begin[lf + l]) * (ns + 128.0);
        }
        near_order = xcd_order(nw);
    }
    std::vector<double> nodes, nodes_p((size_t)H.ncl * nx * dp, 0.0), E;
    box_nodes(H, op->B, nodes);
    for (int64_t c = 0; c < H.ncl; ++c)
        for (int a = 0; a < nx; ++a)
            for (int k = 0; k < d; ++k)
                nodes_p[((size_t)c * nx + a) * dp + k] = nodes[((size_t)c * nx + a) * d + k];
    // axis-major zero-padded nodes and squared node norms for the MFMA coupling (as for the operator)
    const int dkx = (d + 3) / 4 * 4, nxp = op->D.nxp;
    std::vector<double> nodesT((size_t)H.ncl * dkx * nxp, 0.0), nnorm((size_t)H.ncl * nxp, 0.0);
    for (int64_t c = 0; c < H.ncl; ++c)
        for (int a = 0; a < nx; ++a) {
            double sq = 0.0;
            for (int k = 0; k < d; ++k) {
                const double v = nodes[((size_t)c * nx + a) * d + k];
                nodesT[((size_t)c * dkx + k) * nxp + a] = v;
                sq += v * v;
            }
            nnorm[(size_t)c * nxp + a] = sq;
        }
    transfer_matrices(H, op->B, E);

    auto up = [&](auto **dst, const auto &v) { return ev->arena.upload(dst, v, st); };
    hipError_t e = hipSuccess;
    double *dXs, *dclo, *dcsc, *dcoff, *dnodes, *dE, *dLb, *dL, *dnodesT = nullptr, *dnnorm = nullptr;
    int32_t *dperm, *dcb, *dce, *dFp, *dFs, *dNp, *dNs, *dno;
    const size_t R = (size_t)op->max_nrhs;
    if ((e = up(&dXs, Xs)) != hipSuccess || (e = up(&dperm, H.perm)) != hipSuccess ||
        (e = up(&dno, near_order)) != hipSuccess ||
        (e = up(&dcb, H.begin)) != hipSuccess || (e = up(&dce, H.end)) != hipSuccess ||
        (e = up(&dFp, H.Fptr)) != hipSuccess || (e = up(&dFs, H.Fsrc)) != hipSuccess ||
        (e = up(&dNp, nptr_leaf)) != hipSuccess || (e = up(&dNs, nsrc_local)) != hipSuccess ||
        (e = up(&dclo, clo)) != hipSuccess || (e = up(&dcsc, csc)) != hipSuccess ||
        (e = up(&dcoff, coff)) != hipSuccess || (e = up(&dnodes, nodes_p)) != hipSuccess ||
        (e = up(&dE, E)) != hipSuccess || (e = up(&dnodesT, nodesT)) != hipSuccess ||
        (e = up(&dnnorm, nnorm)) != hipSuccess ||
        (e = ev->arena.alloc((void **)&dLb, sizeof(double) * nx * (size_t)m)) != hipSuccess ||
        (e = ev->arena.alloc((void **)&dL, sizeof(double) * H.ncl * nx * R)) != hipSuccess) {
        ev->arena.release();
        delete ev;
        return fail(e == hipErrorOutOfMemory ? DWFMM_E_NOMEM : DWFMM_E_HIP,
                    std::string("evaluation setup: ") + hipGetErrorString(e));
    }
    DevTree &D = ev->D;
    D.n = (int)m;
    D.d = d;
    D.J = H.J;
    D.dpad = dp;
    D.nleaf = (int)H.nleaf;
    D.ncl = (int)H.ncl;
    D.leaf_first = lf;
    D.max_leaf = max_leaf;
    D.min_far_level = H.min_far_level;
    D.Xs = dXs;
    D.perm = dperm;
    D.cbeg = dcb;
    D.cend = dce;
    D.Fptr = dFp;
    D.Fsrc = dFs;
    D.Nptr = dNp;
    D.Nsrc = dNs;
    D.near_order = dno;
    D.n_near_order = (int)near_order.size();
    DevOp &O = ev->O;
    O.kind = op->D.kind;
    O.ell = op->D.ell;
    O.nx = nx;
    O.max_nrhs = op->max_nrhs;
    O.nodes = dnodes;
    O.E = dE;
    O.Lb = dLb;
    O.L = dL;
    O.nxp = op->D.nxp;
    O.nodesT = op->D.nodesT ? dnodesT : nullptr;  // the MFMA coupling needs both sides' layouts
    O.nnorm = op->D.nnorm ? dnnorm : nullptr;
    // Split Gaussian in the cross nearfield, exp(-|x-c|^2/ell) exp(-|y-c|^2/ell) exp(2 (x-c).(y-c)/ell)
    // with c the target leaf's first point: |x - c| <= 2 r_t and |y - c| <= r_t + |m_t - m_s| + r_s
    // (r: half box diagonals, m: box midpoints), so with B = 2 r_t + |m_t - m_s| + r_s over all cross
    // near pairs, B^2 / ell <= 300 keeps every exponent within 600.
    {
        const int32_t lfs = src->D.leaf_first;
        auto half_diag = [d](const HostTree &T, int64_t c, double *mid) {
            double r2 = 0.0;
            for (int k = 0; k < d; ++k) {
                const double lo = T.lo[(size_t)c * d + k], hi = T.hi[(size_t)c * d + k];
                mid[k] = 0.5 * (lo + hi);
                r2 += 0.25 * (hi - lo) * (hi - lo);
            }
            return std::sqrt(r2);
        };
        std::vector<double> mt(d), ms(d);
        double bmax2 = 0.0;
        for (int64_t l = 0; l < H.nleaf; ++l) {
            if (nptr_leaf[l] == nptr_leaf[l + 1]) continue;
            const double rt = half_diag(H, lf + l, mt.data());
            for (int32_t q = nptr_leaf[l]; q < nptr_leaf[l + 1]; ++q) {
                const double rs = half_diag(Hs, lfs + nsrc_local[q], ms.data());
                double dc = 0.0;
                for (int k = 0; k < d; ++k) dc += (mt[k] - ms[k]) * (mt[k] - ms[k]);
                const double B = 2.0 * rt + std::sqrt(dc) + rs;
                bmax2 = std::max(bmax2, B * B);
            }
        }
        O.gauss_split = O.kind == DWFMM_GAUSSIAN && bmax2 / O.ell <= 300.0;
    }
    if ((e = hipMemsetAsync(dL, 0, sizeof(double) * H.ncl * nx * R, st)) != hipSuccess ||
        (e = launch_basis(D, nx, dclo, dcsc, dcoff, op->b_lidx, op->b_nnz, op->b_Vinv, op->b_nleg, op->b_la, op->b_ld,
                          dLb, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess) {
        ev->arena.release();
        delete ev;
        return fail(DWFMM_E_HIP, std::string("evaluation setup: ") + hipGetErrorString(e));
    }
    *out = ev;
    return DWFMM_OK;
}

extern "C" dwfmm_status dwfmm_eval_apply(dwfmm_eval ev, const double *x, double *y, int32_t nrhs, void *stream)
{
    if (!ev) return fail(DWFMM_E_INVALID, "evaluation plan is NULL");
    if (!x || !y) return fail(DWFMM_E_INVALID, "x or y is NULL");
    if (nrhs < 1 || nrhs > ev->op->max_nrhs) return fail(DWFMM_E_INVALID, "nrhs must be in [1, max_nrhs]");
    HIP_TRY(launch_eval(ev->D, ev->O, ev->op->tree->D, ev->op->D, x, y, nrhs, (hipStream_t)stream));
    return DWFMM_OK;
}

extern "C" dwfmm_status dwfmm_eval_info(dwfmm_eval ev, int64_t *out)
{
    if (!ev || !out) return fail(DWFMM_E_INVALID, "NULL argument");
    out[0] = ev->D.n;
    out[1] = ev->D.J;
    out[2] = ev->D.ncl;
    out[3] = ev->nF;
    out[4] = ev->nN;
    return DWFMM_OK;
}

extern "C" dwfmm_status dwfmm_eval_tree_get(dwfmm_eval ev, int64_t *perm, int64_t *begin, int64_t *end, double *lo,
                                            double *hi, int64_t *Fptr, int64_t *Fsrc, int64_t *Nptr, int64_t *Nsrc)
{
    if (!ev) return fail(DWFMM_E_INVALID, "evaluation plan is NULL");
    const HostTree &H = ev->H;
    if (perm) std::copy(H.perm.begin(), H.perm.end(), perm);
    if (begin) std::copy(H.begin.begin(), H.begin.end(), begin);
    if (end) std::copy(H.end.begin(), H.end.end(), end);
    if (lo) std::copy(H.lo.begin(), H.lo.end(), lo);
    if (hi) std::copy(H.hi.begin(), H.hi.end(), hi);
    if (Fptr) std::copy(H.Fptr.begin(), H.Fptr.end(), Fptr);
    if (Fsrc) std::copy(H.Fsrc.begin(), H.Fsrc.end(), Fsrc);
    if (Nptr) std::copy(H.Nptr.begin(), H.Nptr.end(), Nptr);
    if (Nsrc) std::copy(H.Nsrc.begin(), H.Nsrc.end(), Nsrc);
    return DWFMM_OK;
}

extern "C" void dwfmm_eval_destroy(dwfmm_eval ev)
{
    if (!ev) return;
    ev->arena.release();
    delete ev;
}

// ============================================================== sizes and introspection
extern "C" size_t dwfmm_estimate_bytes(int64_t n, int32_t d, int32_t leaf_size, int32_t n_x, int32_t nrhs)
{
    if (n < 1 || d < 1 || leaf_size < 1 || n_x < 1 || nrhs < 1) return 0;
    int J = 0;
    while ((n + ((int64_t)1 << J) - 1) >> J > leaf_size) ++J;
    const size_t ncl = ((size_t)1 << (J + 1)) - 1;
    const size_t dp = (size_t)pad_dim(d);
    size_t b = 0;
    b += dp * n * 8 + 4 * (size_t)n;                 // coordinates, permutation
    b += ncl * (8 + 3 * 8 * (size_t)d);              // ranges, box maps
    b += ncl * 64 * 4 * 2;                           // lists (estimate: 64 entries per cluster)
    b += ncl * n_x * dp * 8 + ncl * n_x * n_x * 8;   // nodes, transfer matrices
    b += (size_t)n_x * n * 8;                        // basis cache
    b += (size_t)n * nrhs * 8 * 4;                   // xt, r, p, q
    b += 2 * ncl * n_x * nrhs * 8;                   // moments, locals
    const size_t nleaf = ((size_t)1 << J);
    b += 128 * 8 * nleaf * (1 + 128);                // nearfield row sums, column sums (estimate: 128 owned blocks per leaf)
    return b;
}

extern "C" size_t dwfmm_op_bytes(dwfmm_op op)
{
    if (!op) return 0;
    return op->arena.total + op->tree->arena.total;
}

extern "C" const char *dwfmm_last_error(void) { return g_err.c_str(); }

extern "C" dwfmm_status dwfmm_tree_info(dwfmm_tree t, int64_t *out)
{
    if (!t || !out) return fail(DWFMM_E_INVALID, "NULL argument");
    const HostTree &H = t->H;
    out[0] = H.n;
    out[1] = H.d;
    out[2] = H.J;
    out[3] = H.ncl;
    out[4] = (int64_t)H.Fsrc.size();
    out[5] = (int64_t)H.Nsrc.size();
    out[6] = H.nleaf;
    out[7] = H.leaf;
    return DWFMM_OK;
}

extern "C" dwfmm_status dwfmm_tree_stats(dwfmm_tree t, int64_t *out)
{
    if (!t || !out) return fail(DWFMM_E_INVALID, "NULL argument");
    out[0] = t->own_max;
    out[1] = t->near_max;
    out[2] = t->own_total;
    return DWFMM_OK;
}

extern "C" dwfmm_status dwfmm_tree_leaf_order(dwfmm_tree t, int32_t *order, double *work, int32_t cap,
                                             int32_t *count)
{
    if (!t || t->destroyed || !count || cap < 0) return fail(DWFMM_E_INVALID, "bad argument");
    *count = t->D.n_order;
    if (order && cap > 0 && t->D.leaf_order) {
        const int m = std::min<int>(cap, t->D.n_order);
        HIP_TRY(hipMemcpy(order, t->D.leaf_order, sizeof(int32_t) * m, hipMemcpyDeviceToHost));
    }
    if (work)
        for (size_t l = 0; l < t->leaf_work.size(); ++l) work[l] = t->leaf_work[l];
    return DWFMM_OK;
}

extern "C" dwfmm_status dwfmm_tree_get(dwfmm_tree t, int64_t *perm, int64_t *begin, int64_t *end, double *lo,
                                       double *hi, int64_t *Fptr, int64_t *Fsrc, int64_t *Nptr, int64_t *Nsrc)
{
    if (!t) return fail(DWFMM_E_INVALID, "NULL tree");
    const HostTree &H = t->H;
    if (perm) std::copy(H.perm.begin(), H.perm.end(), perm);
    if (begin) std::copy(H.begin.begin(), H.begin.end(), begin);
    if (end) std::copy(H.end.begin(), H.end.end(), end);
    if (lo) std::copy(H.lo.begin(), H.lo.end(), lo);
    if (hi) std::copy(H.hi.begin(), H.hi.end(), hi);
    if (Fptr) std::copy(H.Fptr.begin(), H.Fptr.end(), Fptr);
    if (Fsrc) std::copy(H.Fsrc.begin(), H.Fsrc.end(), Fsrc);
    if (Nptr) std::copy(H.Nptr.begin(), H.Nptr.end(), Nptr);
    if (Nsrc) std::copy(H.Nsrc.begin(), H.Nsrc.end(), Nsrc);
    return DWFMM_OK;
}

extern "C" dwfmm_status dwfmm_op_info(dwfmm_op op, int64_t *out)
{
    if (!op || !out) return fail(DWFMM_E_INVALID, "NULL argument");
    out[0] = op->B.nx;
    out[1] = op->max_nrhs;
    out[2] = op->precision;
    out[3] = (int64_t)dwfmm_op_bytes(op);
    out[4] = op->D.gauss_split;
    out[5] = op->D.gauss_split32;
    out[6] = !op->D.near_tiles ? 0 : op->near_filled ? 2 : 1;
    return DWFMM_OK;
}

extern "C" dwfmm_status dwfmm_op_basis(dwfmm_op op, uint8_t *alpha, double *xi, double *Vinv, double *omega)
{
    if (!op) return fail(DWFMM_E_INVALID, "NULL op");
    const HostBasis &B = op->B;
    if (alpha) std::copy(B.alpha.begin(), B.alpha.end(), alpha);
    if (xi) std::copy(B.xi.begin(), B.xi.end(), xi);
    if (Vinv) std::copy(B.Vinv.begin(), B.Vinv.end(), Vinv);
    if (omega) std::copy(B.omega.begin(), B.omega.end(), omega);
    return DWFMM_OK;
}

extern "C" dwfmm_status dwfmm_op_lebesgue(dwfmm_op op, int64_t n_samples, double *out)
{
    if (!op || !out) return fail(DWFMM_E_INVALID, "NULL op or out");
    if (n_samples < 0 || n_samples > 100000000) return fail(DWFMM_E_INVALID, "n_samples must be in [0, 1e8]");
    *out = lebesgue_sampled(op->B, n_samples);
    return DWFMM_OK;
}

extern "C" dwfmm_status dwfmm_op_moments(dwfmm_op op, double *moments, double *locals, int32_t nrhs)
{
    if (!op) return fail(DWFMM_E_INVALID, "NULL op");
    if (nrhs < 1 || nrhs > op->max_nrhs) return fail(DWFMM_E_INVALID, "bad nrhs");
    const size_t cnt = (size_t)op->tree->H.ncl * op->B.nx * nrhs;
    if (moments) HIP_TRY(hipMemcpy(moments, op->D.M, cnt * sizeof(double), hipMemcpyDeviceToHost));
    if (locals) HIP_TRY(hipMemcpy(locals, op->D.L, cnt * sizeof(double), hipMemcpyDeviceToHost));
    return DWFMM_OK;
}
