/*
 * dwfmm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of the dimension weighted fast
 * multipole method (Harbrecht, Multerer, Quizi, "The dimension weighted fast
 * multipole method for scattered data approximation", arXiv 2402.09531).
 * It exists to check the GPU library; only tests/, the smoke entry point and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header or table with the GPU library.
 *
 * Every step follows the paper's notation:
 *   weights            omega_k               Thm 4.6, Sec 6.2 (and the R1/R2 readings)
 *   index set          Lambda_{omega,q,d}    Sec 4 (weighted total degree index sets)
 *   Legendre basis     p_j, p_alpha          Sec 5.2 (orthonormal on [0,1], tensorised)
 *   Vandermonde        V = [p_a'(xi_a)]      Sec 5.2, eq. (Vandermonde)
 *   cluster tree       balanced binary tree  Sec 5.1, Def 5.1/5.2 (longest-edge median split)
 *   admissibility      dist >= eta max diam  Sec 5.2, eq. (admissibility)
 *                      (or eta dist >= max diam / 2, the half-diagonal reading)
 *   farfield block     P_nu V^-1 S V^-T P_nu'^T           Sec 5.2, eq. (LowRankBlock)
 *   nested bases       T_child = V^-1 [p^nu_a'(a_child(xi_a))]  Sec 5.2 (two-scale relation)
 *   solver             CG on (K + lambda I) alpha = y      Sec 2, eq. (LGS); Sec 6.2
 *
 * The farfield is evaluated in the paper's own (Legendre-coefficient) form:
 * leaf moments P_nu^T x, upward with T_c^T, coupling with C = V^-1 S V^-T
 * formed explicitly per block, downward with T_c, and P_nu at the leaves.
 * The nearfield is the plain kernel sum over inadmissible leaf pairs.
 *
 * Readings of places where the paper is silent or garbled (each also listed in
 * the design notes): tree stopping depth J = min{j : ceil(N/2^j) <= leaf},
 * left child takes ceil(n/2), split order (coordinate, original index);
 * farfield = admissible blocks whose parent block is not admissible;
 * admissibility uses the full box diagonal and is inclusive (compared squared);
 * Chebyshev first-kind nodes per axis, Leja ordered; degenerate box axes map
 * to the reference midpoint.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXD 64

enum { ORC_MATERN32 = 0, ORC_GAUSSIAN = 1, ORC_EXPONENTIAL = 2, ORC_POLY = 3 };
enum { ORC_W_R1 = 0, ORC_W_R2 = 1, ORC_W_R3 = 2, ORC_W_EXPLICIT = 3, ORC_W_THM = 4 };

/* ------------------------------------------------------------------ */
/* Kernel functions (Sec 6.2 exponential kernel; Matern-3/2 and Gaussian
 * as used by the workloads; a polynomial test kernel).                 */
/* ------------------------------------------------------------------ */
double orc_kernel(int kind, double ell, int d, const double *x, const double *y)
{
    double r2 = 0.0;
    for (int k = 0; k < d; ++k) {
        double t = x[k] - y[k];
        r2 += t * t;
    }
    switch (kind) {
    case ORC_MATERN32: {
        double s = sqrt(3.0) * sqrt(r2) / ell;
        return (1.0 + s) * exp(-s);
    }
    case ORC_GAUSSIAN:
        return exp(-r2 / ell);
    case ORC_EXPONENTIAL:
        return exp(-sqrt(r2) / ell);
    case ORC_POLY: {
        /* 1 + sum_{k < p} x_k y_k + (x_0 y_0)^2 with p = (int) ell axes. */
        int p = (int)ell;
        double v = 1.0;
        for (int k = 0; k < p && k < d; ++k) v += x[k] * y[k];
        v += (x[0] * y[0]) * (x[0] * y[0]);
        return v;
    }
    }
    return NAN;
}

/* ------------------------------------------------------------------ */
/* Dimension weights.                                                  */
/* ------------------------------------------------------------------ */
static double g_rho(double tau) { return 2.0 * tau + sqrt(1.0 + 4.0 * tau * tau); }

/* rule R1: omega_k = max(1, log2(b_max / b_k))
 * rule R2: omega_k = 1 + log2(b_max / b_k)
 * rule R3: Sec 6.2, tau_k = 1/(eta b_k), rho_k = e g(tau_k)/g(tau_1), omega_k = log rho_k
 * rule THM: Thm 4.6, omega_k = log(g(tau_k)) with tau given in aux
 * rule EXPLICIT: omega given in aux                                   */
int orc_weights(int rule, int d, const double *b, double eta, const double *aux, double *omega)
{
    if (d < 1 || d > ORC_MAXD) return -1;
    double bmax = 0.0;
    if (b)
        for (int k = 0; k < d; ++k) bmax = b[k] > bmax ? b[k] : bmax;
    for (int k = 0; k < d; ++k) {
        switch (rule) {
        case ORC_W_R1: {
            double w = log2(bmax / b[k]);
            omega[k] = w > 1.0 ? w : 1.0;
            break;
        }
        case ORC_W_R2:
            omega[k] = 1.0 + log2(bmax / b[k]);
            break;
        case ORC_W_R3: {
            double t1 = 1.0 / (eta * b[0]), tk = 1.0 / (eta * b[k]);
            omega[k] = log(exp(1.0) * g_rho(tk) / g_rho(t1));
            break;
        }
        case ORC_W_THM:
            omega[k] = log(g_rho(aux[k]));
            break;
        case ORC_W_EXPLICIT:
            omega[k] = aux[k];
            break;
        default:
            return -1;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Weighted total degree index set (Sec 4):
 *   Lambda = { alpha >= 0 : sum_k omega_k alpha_k <= q }  (+1e-9 slack)
 * box_rule != 0 gives the tensor set { max_k alpha_k <= q } instead.
 * Enumerated depth-first; then sorted by (weighted degree, colex).     */
/* ------------------------------------------------------------------ */
typedef struct {
    int d;
    const double *omega;
    double q;
    int box;
    long count, cap;
    unsigned char *out;
    unsigned char cur[ORC_MAXD];
} enum_ctx;

static void enum_rec(enum_ctx *c, int k, double rem)
{
    if (k == c->d) {
        if (c->out && c->count < c->cap) memcpy(c->out + c->count * c->d, c->cur, c->d);
        c->count++;
        return;
    }
    for (int a = 0; a < 256; ++a) {
        if (c->box) {
            if (a > (int)c->q) break;
            c->cur[k] = (unsigned char)a;
            enum_rec(c, k + 1, rem);
        } else {
            double used = c->omega[k] * a;
            if (used > rem + 1e-9) break;
            c->cur[k] = (unsigned char)a;
            enum_rec(c, k + 1, rem - used);
            if (c->omega[k] <= 0.0) break; /* zero weight: unbounded axis, keep alpha_k = 0 */
        }
    }
    c->cur[k] = 0;
}

typedef struct {
    double w;
    const unsigned char *a;
    int d;
} sort_item;

static int cmp_items(const void *pa, const void *pb)
{
    const sort_item *x = (const sort_item *)pa, *y = (const sort_item *)pb;
    if (x->w < y->w) return -1;
    if (x->w > y->w) return 1;
    for (int k = x->d - 1; k >= 0; --k) {
        if (x->a[k] != y->a[k]) return x->a[k] < y->a[k] ? -1 : 1;
    }
    return 0;
}

long orc_index_set(int d, const double *omega, double q, int box_rule, unsigned char *out, long cap)
{
    if (d < 1 || d > ORC_MAXD) return -1;
    enum_ctx c;
    memset(&c, 0, sizeof c);
    c.d = d;
    c.omega = omega;
    c.q = q;
    c.box = box_rule;
    c.out = out;
    c.cap = out ? cap : 0;
    enum_rec(&c, 0, q);
    if (out && c.count <= cap) {
        long n = c.count;
        sort_item *it = (sort_item *)malloc(sizeof(sort_item) * (size_t)n);
        unsigned char *copy = (unsigned char *)malloc((size_t)n * d);
        memcpy(copy, out, (size_t)n * d);
        for (long i = 0; i < n; ++i) {
            double w = 0.0;
            for (int k = 0; k < d; ++k) w += omega ? omega[k] * copy[i * d + k] : copy[i * d + k];
            it[i].w = w;
            it[i].a = copy + i * d;
            it[i].d = d;
        }
        qsort(it, (size_t)n, sizeof(sort_item), cmp_items);
        for (long i = 0; i < n; ++i) memcpy(out + i * d, it[i].a, d);
        free(it);
        free(copy);
    }
    return c.count;
}

/* ------------------------------------------------------------------ */
/* Interpolation nodes per axis: the m+1 Chebyshev points of the first
 * kind on [0,1], put in Leja order (start nearest 1/2; each next point
 * maximises the product of distances to the points already chosen;
 * ties within relative 1e-9 go to the smaller point).                 */
/* ------------------------------------------------------------------ */
void orc_axis_nodes(int m, double *z)
{
    const double pi = 3.14159265358979323846;
    if (m == 0) {
        z[0] = 0.5;
        return;
    }
    int n = m + 1;
    double t[256];
    int used[256];
    for (int j = 0; j < n; ++j) {
        t[j] = (1.0 - cos((2.0 * j + 1.0) * pi / (2.0 * n))) / 2.0;
        used[j] = 0;
    }
    /* first: nearest 1/2 */
    int best = -1;
    for (int j = 0; j < n; ++j) {
        if (best < 0) { best = j; continue; }
        double dj = fabs(t[j] - 0.5), db = fabs(t[best] - 0.5);
        if (dj < db - 1e-9 * (db > 0 ? db : 1.0)) best = j;
        else if (fabs(dj - db) <= 1e-9 * (db > 0 ? db : 1.0) && t[j] < t[best]) best = j;
    }
    z[0] = t[best];
    used[best] = 1;
    for (int i = 1; i < n; ++i) {
        int bj = -1;
        double bv = -1.0;
        for (int j = 0; j < n; ++j) {
            if (used[j]) continue;
            double p = 1.0;
            for (int l = 0; l < i; ++l) p *= fabs(t[j] - z[l]);
            if (bj < 0 || p > bv * (1.0 + 1e-9)) { bj = j; bv = p; }
            else if (fabs(p - bv) <= 1e-9 * bv && t[j] < t[bj]) { bj = j; bv = p; }
        }
        z[i] = t[bj];
        used[bj] = 1;
    }
}

/* ------------------------------------------------------------------ */
/* Orthonormal Legendre polynomials on [0,1] (Sec 5.2):
 *   p_j(t) = sqrt(2j+1) P_j(2t-1), P by the three-term recurrence.     */
/* ------------------------------------------------------------------ */
double orc_legendre(int j, double t)
{
    double s = 2.0 * t - 1.0;
    double p0 = 1.0, p1 = s;
    if (j == 0) return 1.0;
    for (int n = 1; n < j; ++n) {
        double p2 = ((2.0 * n + 1.0) * s * p1 - n * p0) / (n + 1.0);
        p0 = p1;
        p1 = p2;
    }
    return sqrt(2.0 * j + 1.0) * p1;
}

/* p_alpha(t) = prod_k p_{alpha_k}(t_k) */
static double leg_tensor(int d, const unsigned char *alpha, const double *t)
{
    double v = 1.0;
    for (int k = 0; k < d; ++k)
        if (alpha[k]) v *= orc_legendre(alpha[k], t[k]);
    return v;
}

/* Gauss-Jordan inverse with partial pivoting (row-major n x n). */
static int invert(int n, const double *A, double *Ainv)
{
    double *M = (double *)malloc(sizeof(double) * (size_t)n * 2 * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < 2 * n; ++j)
            M[i * 2 * n + j] = j < n ? A[i * n + j] : (j - n == i ? 1.0 : 0.0);
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(M[r * 2 * n + c]) > fabs(M[p * 2 * n + c])) p = r;
        if (M[p * 2 * n + c] == 0.0) { free(M); return -1; }
        if (p != c)
            for (int j = 0; j < 2 * n; ++j) {
                double t = M[c * 2 * n + j];
                M[c * 2 * n + j] = M[p * 2 * n + j];
                M[p * 2 * n + j] = t;
            }
        double piv = M[c * 2 * n + c];
        for (int j = 0; j < 2 * n; ++j) M[c * 2 * n + j] /= piv;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            double f = M[r * 2 * n + c];
            if (f == 0.0) continue;
            for (int j = 0; j < 2 * n; ++j) M[r * 2 * n + j] -= f * M[c * 2 * n + j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Ainv[i * n + j] = M[i * 2 * n + n + j];
    free(M);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Approximate Fekete points (Sec 5.4): a greedy column-pivoted QR of  */
/* the Vandermonde matrix over candidate points of the Halton sequence. */
/* ------------------------------------------------------------------ */

/* Radical inverse of i in base p (the Halton coordinate), exactly: the
 * digits of i reversed behind the radix point, formed as an integer over
 * p^(number of digits) and divided once. */
double orc_radical_inverse(long i, int p)
{
    long num = 0, den = 1;
    while (i > 0) {
        num = num * p + i % p;
        den *= p;
        i /= p;
    }
    return (double)num / (double)den;
}

static int nth_prime(int r)
{
    int count = -1;
    for (int c = 2;; ++c) {
        int prime = 1;
        for (int f = 2; f * f <= c; ++f)
            if (c % f == 0) { prime = 0; break; }
        if (prime && ++count == r) return c;
    }
}

/* Candidate j (j = 0..M-1) is Halton point j+1 over the axes with m_k > 0
 * (the r-th such axis in base prime r); the other coordinates are 1/2. */
void orc_halton_candidates(int d, const int *mk, long M, double *Y)
{
    for (long j = 0; j < M; ++j) {
        int r = 0;
        for (int k = 0; k < d; ++k)
            Y[j * d + k] = mk[k] > 0 ? orc_radical_inverse(j + 1, nth_prime(r++)) : 0.5;
    }
}

/* Select nx of the M candidates Y: A = [p_b(y_j)] (basis b by row, candidate
 * j by column) is reduced by Householder reflections; step k takes the column
 * whose remaining part (rows k..nx-1) has the largest norm, a norm within
 * relative 1e-12 of the largest going to the lowest candidate index.  The
 * norms are recomputed from the reduced matrix at every step.  chosen[k] is
 * the candidate taken at step k.  Returns 0, or -1 if a step finds no column
 * with a non-zero remaining part. */
int orc_afp_select(int d, long nx, const unsigned char *alpha, long M, const double *Y, long *chosen)
{
    double *A = (double *)malloc(sizeof(double) * (size_t)nx * M);
    long *id = (long *)malloc(sizeof(long) * (size_t)M);
    double *v = (double *)malloc(sizeof(double) * (size_t)nx);
    for (long j = 0; j < M; ++j) {
        id[j] = j;
        for (long b = 0; b < nx; ++b) A[b * M + j] = leg_tensor(d, alpha + b * d, Y + j * d);
    }
    int rc = 0;
    for (long k = 0; k < nx; ++k) {
        double best = -1.0;
        for (long j = k; j < M; ++j) {
            double s = 0.0;
            for (long r = k; r < nx; ++r) s += A[r * M + j] * A[r * M + j];
            if (s > best) best = s;
        }
        if (!(best > 0.0)) { rc = -1; break; }
        long jp = -1;
        for (long j = k; j < M; ++j) {
            double s = 0.0;
            for (long r = k; r < nx; ++r) s += A[r * M + j] * A[r * M + j];
            if (s >= best * (1.0 - 1e-12) && (jp < 0 || id[j] < id[jp])) jp = j;
        }
        if (jp != k) {
            for (long r = 0; r < nx; ++r) {
                double t = A[r * M + k];
                A[r * M + k] = A[r * M + jp];
                A[r * M + jp] = t;
            }
            long t = id[k];
            id[k] = id[jp];
            id[jp] = t;
        }
        chosen[k] = id[k];
        /* reflector H = I - 2 v v^T / (v^T v) mapping column k (rows k..) onto a multiple of e_k */
        double nrm = 0.0;
        for (long r = k; r < nx; ++r) nrm += A[r * M + k] * A[r * M + k];
        nrm = sqrt(nrm);
        double a0 = A[k * M + k];
        double alpha_k = a0 >= 0.0 ? -nrm : nrm;
        for (long r = k; r < nx; ++r) v[r] = A[r * M + k];
        v[k] = a0 - alpha_k;
        double vv = 0.0;
        for (long r = k; r < nx; ++r) vv += v[r] * v[r];
        if (vv == 0.0) continue;
        for (long j = k; j < M; ++j) {
            double dot = 0.0;
            for (long r = k; r < nx; ++r) dot += v[r] * A[r * M + j];
            double f = 2.0 * dot / vv;
            for (long r = k; r < nx; ++r) A[r * M + j] -= f * v[r];
        }
    }
    free(A);
    free(id);
    free(v);
    return rc;
}

/* Default number of candidates for nx nodes. */
long orc_afp_candidates(long nx) { return nx * 50 > 2000 ? nx * 50 : 2000; }

/* ------------------------------------------------------------------ */
/* The plan: tree, partition, index set, nodes, V, V^-1, T matrices.   */
/* ------------------------------------------------------------------ */
typedef struct {
    long n;
    int d, leaf, J, kind, nx;
    double eta, ell, q;
    int adm_half;   /* admissibility against half the box diagonal */
    long ncl;
    double *X;      /* n*d, original order */
    long *perm;     /* tree position -> original index */
    long *cb, *ce;  /* cluster point range in tree order */
    double *lo, *hi; /* ncl*d tight boxes */
    double omega[ORC_MAXD];
    int mk[ORC_MAXD];
    unsigned char *alpha; /* nx*d */
    double *xi;     /* nx*d reference nodes */
    double *V, *Vinv;
    double *T;      /* ncl*nx*nx; T[c] for c >= 1 */
    /* farfield and nearfield lists, CSR by target cluster */
    long nF, nN;
    long *Fptr, *Fsrc; /* Fptr: ncl+1 */
    long *Nptr, *Nsrc; /* Nptr: ncl+1 (only leaves non-empty) */
    int *flevel_count;
} orc_plan;

static long cl_level_first(int j) { return (1L << j) - 1; }
static int cl_level(long c)
{
    int j = 0;
    while ((1L << (j + 1)) - 1 <= c) ++j;
    return j;
}

static const double *g_sortX;
static int g_sortd, g_sorta;
static int cmp_pts(const void *pa, const void *pb)
{
    long a = *(const long *)pa, b = *(const long *)pb;
    double xa = g_sortX[a * g_sortd + g_sorta], xb = g_sortX[b * g_sortd + g_sorta];
    if (xa < xb) return -1;
    if (xa > xb) return 1;
    return a < b ? -1 : (a > b ? 1 : 0);
}

static void box_of(orc_plan *P, long c)
{
    int d = P->d;
    double *lo = P->lo + c * d, *hi = P->hi + c * d;
    for (int k = 0; k < d; ++k) { lo[k] = INFINITY; hi[k] = -INFINITY; }
    for (long i = P->cb[c]; i < P->ce[c]; ++i) {
        const double *x = P->X + P->perm[i] * d;
        for (int k = 0; k < d; ++k) {
            if (x[k] < lo[k]) lo[k] = x[k];
            if (x[k] > hi[k]) hi[k] = x[k];
        }
    }
}

/* Sec 5.1: cardinality balanced clustering, split along the longest edge
 * of the tight bounding box so that both halves hold (nearly) equally
 * many points. */
static void build_tree_depth(orc_plan *P, int J);

static void build_tree(orc_plan *P)
{
    int J = 0;
    while ((P->n + (1L << J) - 1) / (1L << J) > P->leaf) ++J;
    build_tree_depth(P, J);
}

/* The tree of Sec 5.1 with a given depth J (clusters may be empty when n < 2^J). */
static void build_tree_depth(orc_plan *P, int J)
{
    long n = P->n;
    int d = P->d;
    P->J = J;
    P->ncl = (1L << (J + 1)) - 1;
    P->perm = (long *)malloc(sizeof(long) * (size_t)n);
    for (long i = 0; i < n; ++i) P->perm[i] = i;
    P->cb = (long *)malloc(sizeof(long) * (size_t)P->ncl);
    P->ce = (long *)malloc(sizeof(long) * (size_t)P->ncl);
    P->lo = (double *)malloc(sizeof(double) * (size_t)P->ncl * d);
    P->hi = (double *)malloc(sizeof(double) * (size_t)P->ncl * d);
    P->cb[0] = 0;
    P->ce[0] = n;
    g_sortX = P->X;
    g_sortd = d;
    for (int j = 0; j <= J; ++j) {
        for (long c = cl_level_first(j); c < cl_level_first(j + 1); ++c) {
            box_of(P, c);
            if (j == J) continue;
            long b = P->cb[c], e = P->ce[c], m = e - b;
            int a = 0;
            double best = -1.0;
            for (int k = 0; k < d; ++k) {
                double ext = m > 0 ? P->hi[c * d + k] - P->lo[c * d + k] : 0.0;
                if (ext > best) { best = ext; a = k; }
            }
            g_sorta = a;
            if (m > 1) qsort(P->perm + b, (size_t)m, sizeof(long), cmp_pts);
            long half = (m + 1) / 2;
            P->cb[2 * c + 1] = b;
            P->ce[2 * c + 1] = b + half;
            P->cb[2 * c + 2] = b + half;
            P->ce[2 * c + 2] = e;
        }
    }
}

/* eq. (admissibility): dist(B, B') >= eta max{diam B, diam B'}, compared squared; with
 * adm_half the diameter is half the box diagonal: eta dist >= max diag / 2, i.e.
 * (2 eta)^2 dist^2 >= max diag^2. */
static int adm_test(double dist2, double dm, double eta, int half)
{
    if (half) return (2.0 * eta) * (2.0 * eta) * dist2 >= dm;
    return dist2 >= eta * eta * dm;
}

static int admissible(const orc_plan *P, long a, long b)
{
    int d = P->d;
    const double *la = P->lo + a * d, *ha = P->hi + a * d, *lb = P->lo + b * d, *hb = P->hi + b * d;
    double dist2 = 0.0, da2 = 0.0, db2 = 0.0;
    for (int k = 0; k < d; ++k) {
        double g1 = lb[k] - ha[k], g2 = la[k] - hb[k];
        double g = g1 > g2 ? g1 : g2;
        if (g < 0.0) g = 0.0;
        dist2 += g * g;
        da2 += (ha[k] - la[k]) * (ha[k] - la[k]);
        db2 += (hb[k] - lb[k]) * (hb[k] - lb[k]);
    }
    double dm = da2 > db2 ? da2 : db2;
    return adm_test(dist2, dm, P->eta, P->adm_half);
}

typedef struct {
    long n, cap;
    long *t, *s;
} pairlist;
static void pl_push(pairlist *L, long t, long s)
{
    if (L->n == L->cap) {
        L->cap = L->cap ? 2 * L->cap : 1024;
        L->t = (long *)realloc(L->t, sizeof(long) * (size_t)L->cap);
        L->s = (long *)realloc(L->s, sizeof(long) * (size_t)L->cap);
    }
    L->t[L->n] = t;
    L->s[L->n] = s;
    L->n++;
}

static void partition_rec(const orc_plan *P, long a, long b, int level, pairlist *F, pairlist *N)
{
    if (P->ce[a] == P->cb[a] || P->ce[b] == P->cb[b]) return;
    if (admissible(P, a, b)) { pl_push(F, a, b); return; }
    if (level < P->J) {
        for (int i = 1; i <= 2; ++i)
            for (int j = 1; j <= 2; ++j) partition_rec(P, 2 * a + i, 2 * b + j, level + 1, F, N);
        return;
    }
    pl_push(N, a, b);
}

static void to_csr(long ncl, const pairlist *L, long **ptr, long **src)
{
    long *p = (long *)calloc((size_t)ncl + 1, sizeof(long));
    long *s = (long *)malloc(sizeof(long) * (size_t)(L->n > 0 ? L->n : 1));
    for (long i = 0; i < L->n; ++i) p[L->t[i] + 1]++;
    for (long c = 0; c < ncl; ++c) p[c + 1] += p[c];
    long *fill = (long *)malloc(sizeof(long) * (size_t)ncl);
    for (long c = 0; c < ncl; ++c) fill[c] = p[c];
    for (long i = 0; i < L->n; ++i) s[fill[L->t[i]]++] = L->s[i];
    free(fill);
    *ptr = p;
    *src = s;
}

/* a_nu(xi)_k = lo_k + xi_k (hi_k - lo_k); degenerate axis -> lo_k */
static void map_to_box(int d, const double *lo, const double *hi, const double *xi, double *x)
{
    for (int k = 0; k < d; ++k) x[k] = hi[k] > lo[k] ? lo[k] + xi[k] * (hi[k] - lo[k]) : lo[k];
}
/* a_nu^-1(x)_k = (x_k - lo_k)/(hi_k - lo_k); degenerate axis -> 1/2 */
static void map_from_box(int d, const double *lo, const double *hi, const double *x, double *t)
{
    for (int k = 0; k < d; ++k) t[k] = hi[k] > lo[k] ? (x[k] - lo[k]) / (hi[k] - lo[k]) : 0.5;
}

void orc_destroy(orc_plan *P)
{
    if (!P) return;
    free(P->X); free(P->perm); free(P->cb); free(P->ce); free(P->lo); free(P->hi);
    free(P->alpha); free(P->xi); free(P->V); free(P->Vinv); free(P->T);
    free(P->Fptr); free(P->Fsrc); free(P->Nptr); free(P->Nsrc);
    free(P);
}

/* Build everything the matvec needs.  points: n*d row-major, original order. */
orc_plan *orc_create_ex(const double *points, long n, int d, const double *b, int leaf, double eta,
                        int kind, double ell, double q, int weight_rule, const double *weight_aux,
                        int node_rule, long n_candidates, int index_rule, int adm_half);

orc_plan *orc_create(const double *points, long n, int d, const double *b, int leaf, double eta,
                     int kind, double ell, double q, int weight_rule, const double *weight_aux)
{
    return orc_create_ex(points, n, d, b, leaf, eta, kind, ell, q, weight_rule, weight_aux, 0, 0, 0, 0);
}

/* node_rule 0: per-axis Chebyshev-Leja nodes; 1: approximate Fekete points from
 * n_candidates Halton candidates (0 = the default count).  index_rule 0: weighted
 * total degree set; 1: the tensor set max_k alpha_k <= q (Sec 6.1, TPI).  adm_half:
 * admissibility against half the box diagonal. */
orc_plan *orc_create_ex(const double *points, long n, int d, const double *b, int leaf, double eta,
                        int kind, double ell, double q, int weight_rule, const double *weight_aux,
                        int node_rule, long n_candidates, int index_rule, int adm_half)
{
    if (n < 1 || d < 1 || d > ORC_MAXD || leaf < 1 || !(eta > 0)) return NULL;
    orc_plan *P = (orc_plan *)calloc(1, sizeof(orc_plan));
    P->n = n; P->d = d; P->leaf = leaf; P->eta = eta; P->kind = kind; P->ell = ell; P->q = q;
    P->adm_half = adm_half != 0;
    P->X = (double *)malloc(sizeof(double) * (size_t)n * d);
    memcpy(P->X, points, sizeof(double) * (size_t)n * d);
    if (orc_weights(weight_rule, d, b, eta, weight_aux, P->omega) != 0) { orc_destroy(P); return NULL; }
    long nx = orc_index_set(d, P->omega, q, index_rule, NULL, 0);
    P->nx = (int)nx;
    P->alpha = (unsigned char *)malloc((size_t)nx * d);
    orc_index_set(d, P->omega, q, index_rule, P->alpha, nx);
    for (int k = 0; k < d; ++k) {
        P->mk[k] = 0;
        for (long a = 0; a < nx; ++a)
            if (P->alpha[a * d + k] > P->mk[k]) P->mk[k] = P->alpha[a * d + k];
    }
    P->xi = (double *)malloc(sizeof(double) * (size_t)nx * d);
    if (node_rule == 0) {
        /* nodes xi_alpha = (z^(1)_{alpha_1}, ..., z^(d)_{alpha_d}) */
        for (int k = 0; k < d; ++k) {
            double z[256];
            orc_axis_nodes(P->mk[k], z);
            for (long a = 0; a < nx; ++a) P->xi[a * d + k] = z[P->alpha[a * d + k]];
        }
    } else {
        long M = n_candidates > 0 ? n_candidates : orc_afp_candidates(nx);
        if (M < nx) { orc_destroy(P); return NULL; }
        double *Y = (double *)malloc(sizeof(double) * (size_t)M * d);
        long *chosen = (long *)malloc(sizeof(long) * (size_t)nx);
        orc_halton_candidates(d, P->mk, M, Y);
        int rc = orc_afp_select(d, nx, P->alpha, M, Y, chosen);
        if (rc == 0)
            for (long a = 0; a < nx; ++a) memcpy(P->xi + a * d, Y + chosen[a] * d, sizeof(double) * d);
        free(Y);
        free(chosen);
        if (rc != 0) { orc_destroy(P); return NULL; }
    }
    /* eq. (Vandermonde): V[alpha][alpha'] = p_alpha'(xi_alpha) */
    P->V = (double *)malloc(sizeof(double) * (size_t)nx * nx);
    P->Vinv = (double *)malloc(sizeof(double) * (size_t)nx * nx);
    for (long a = 0; a < nx; ++a)
        for (long b2 = 0; b2 < nx; ++b2) P->V[a * nx + b2] = leg_tensor(d, P->alpha + b2 * d, P->xi + a * d);
    if (invert((int)nx, P->V, P->Vinv) != 0) { orc_destroy(P); return NULL; }

    build_tree(P);

    pairlist F = {0, 0, NULL, NULL}, N = {0, 0, NULL, NULL};
    partition_rec(P, 0, 0, 0, &F, &N);
    P->nF = F.n;
    P->nN = N.n;
    to_csr(P->ncl, &F, &P->Fptr, &P->Fsrc);
    to_csr(P->ncl, &N, &P->Nptr, &P->Nsrc);
    free(F.t); free(F.s); free(N.t); free(N.s);

    /* Transfer matrices T_c = V^-1 M_c, M_c[alpha][alpha'] = p_alpha'(a_nu^-1(a_c(xi_alpha))) */
    P->T = (double *)calloc((size_t)P->ncl * nx * nx, sizeof(double));
    double *M = (double *)malloc(sizeof(double) * (size_t)nx * nx);
    double xc[ORC_MAXD], t[ORC_MAXD];
    for (long c = 1; c < P->ncl; ++c) {
        long pa = (c - 1) / 2;
        if (P->ce[c] == P->cb[c]) continue;
        for (long a = 0; a < nx; ++a) {
            map_to_box(d, P->lo + c * d, P->hi + c * d, P->xi + a * d, xc);
            map_from_box(d, P->lo + pa * d, P->hi + pa * d, xc, t);
            for (long b2 = 0; b2 < nx; ++b2) M[a * nx + b2] = leg_tensor(d, P->alpha + b2 * d, t);
        }
        double *Tc = P->T + c * nx * nx;
        for (long a = 0; a < nx; ++a)
            for (long b2 = 0; b2 < nx; ++b2) {
                double s = 0.0;
                for (long g = 0; g < nx; ++g) s += P->Vinv[a * nx + g] * M[g * nx + b2];
                Tc[a * nx + b2] = s;
            }
    }
    free(M);
    return P;
}

/* ------------------------------------------------------------------ */
/* Matvec y = K~ x (x, y: n x nrhs row-major, original order).
 * parts: bit 0 nearfield, bit 1 farfield.  If leaf_lo < leaf_hi only
 * targets in leaves [leaf_lo, leaf_hi) (leaf index within level J) are
 * computed; other rows of y are left zero.
 * moments_out / locals_out (optional, ncl*nx*nrhs) receive the Legendre
 * moments P_nu^T x_nu and the accumulated Legendre locals.            */
/* ------------------------------------------------------------------ */
void orc_matvec_ex(const orc_plan *P, const double *x, double *y, int nrhs, int parts, long leaf_lo,
                   long leaf_hi, double *moments_out, double *locals_out)
{
    long n = P->n, ncl = P->ncl;
    int d = P->d, nx = P->nx, J = P->J;
    long L0 = cl_level_first(J), nleaf = 1L << J;
    if (!(leaf_lo < leaf_hi)) { leaf_lo = 0; leaf_hi = nleaf; }
    memset(y, 0, sizeof(double) * (size_t)n * nrhs);
    /* which clusters feed a requested target leaf */
    char *want = (char *)calloc((size_t)ncl, 1);
    for (long l = leaf_lo; l < leaf_hi; ++l)
        for (long c = L0 + l;; c = (c - 1) / 2) {
            want[c] = 1;
            if (c == 0) break;
        }

    if (parts & 2) {
        size_t msz = (size_t)ncl * nx * nrhs;
        double *mom = (double *)calloc(msz, sizeof(double));
        double *loc = (double *)calloc(msz, sizeof(double));
        /* leaf moments: mhat_nu = P_nu^T x_nu */
#pragma omp parallel for schedule(dynamic, 4)
        for (long c = L0; c < ncl; ++c) {
            double t[ORC_MAXD];
            for (long i = P->cb[c]; i < P->ce[c]; ++i) {
                long oi = P->perm[i];
                map_from_box(d, P->lo + c * d, P->hi + c * d, P->X + oi * d, t);
                for (int a = 0; a < nx; ++a) {
                    double p = leg_tensor(d, P->alpha + a * d, t);
                    for (int r = 0; r < nrhs; ++r) mom[(c * nx + a) * nrhs + r] += p * x[oi * nrhs + r];
                }
            }
        }
        /* upward: mhat_nu = sum_c T_c^T mhat_c (two-scale relation) */
        for (int j = J - 1; j >= 0; --j) {
#pragma omp parallel for schedule(dynamic, 4)
            for (long c = cl_level_first(j); c < cl_level_first(j + 1); ++c) {
                for (long ch = 2 * c + 1; ch <= 2 * c + 2; ++ch) {
                    const double *Tc = P->T + ch * nx * nx;
                    for (int b2 = 0; b2 < nx; ++b2)
                        for (int a = 0; a < nx; ++a)
                            for (int r = 0; r < nrhs; ++r)
                                mom[(c * nx + b2) * nrhs + r] += Tc[a * nx + b2] * mom[(ch * nx + a) * nrhs + r];
                }
            }
        }
        /* coupling: lhat_nu += C_{nu,nu'} mhat_nu', C = V^-1 S V^-T */
#pragma omp parallel
        {
            double *S = (double *)malloc(sizeof(double) * (size_t)nx * nx);
            double *W = (double *)malloc(sizeof(double) * (size_t)nx * nx);
            double *C = (double *)malloc(sizeof(double) * (size_t)nx * nx);
            double *xa = (double *)malloc(sizeof(double) * (size_t)nx * d);
            double *xb = (double *)malloc(sizeof(double) * (size_t)nx * d);
#pragma omp for schedule(dynamic, 1)
            for (long c = 0; c < ncl; ++c) {
                if (!want[c] || P->Fptr[c] == P->Fptr[c + 1]) continue;
                for (int a = 0; a < nx; ++a) map_to_box(d, P->lo + c * d, P->hi + c * d, P->xi + a * d, xa + a * d);
                for (long f = P->Fptr[c]; f < P->Fptr[c + 1]; ++f) {
                    long s = P->Fsrc[f];
                    for (int a = 0; a < nx; ++a) map_to_box(d, P->lo + s * d, P->hi + s * d, P->xi + a * d, xb + a * d);
                    for (int a = 0; a < nx; ++a)
                        for (int b2 = 0; b2 < nx; ++b2)
                            S[a * nx + b2] = orc_kernel(P->kind, P->ell, d, xa + a * d, xb + b2 * d);
                    /* W = V^-1 S ; C = W V^-T */
                    for (int a = 0; a < nx; ++a)
                        for (int b2 = 0; b2 < nx; ++b2) {
                            double sum = 0.0;
                            for (int g = 0; g < nx; ++g) sum += P->Vinv[a * nx + g] * S[g * nx + b2];
                            W[a * nx + b2] = sum;
                        }
                    for (int a = 0; a < nx; ++a)
                        for (int b2 = 0; b2 < nx; ++b2) {
                            double sum = 0.0;
                            for (int g = 0; g < nx; ++g) sum += W[a * nx + g] * P->Vinv[b2 * nx + g];
                            C[a * nx + b2] = sum;
                        }
                    for (int a = 0; a < nx; ++a)
                        for (int b2 = 0; b2 < nx; ++b2)
                            for (int r = 0; r < nrhs; ++r)
                                loc[(c * nx + a) * nrhs + r] += C[a * nx + b2] * mom[(s * nx + b2) * nrhs + r];
                }
            }
            free(S); free(W); free(C); free(xa); free(xb);
        }
        /* downward: lhat_c += T_c lhat_nu */
        for (int j = 0; j < J; ++j) {
#pragma omp parallel for schedule(dynamic, 4)
            for (long c = cl_level_first(j); c < cl_level_first(j + 1); ++c) {
                for (long ch = 2 * c + 1; ch <= 2 * c + 2; ++ch) {
                    if (!want[ch]) continue;
                    const double *Tc = P->T + ch * nx * nx;
                    for (int a = 0; a < nx; ++a)
                        for (int b2 = 0; b2 < nx; ++b2)
                            for (int r = 0; r < nrhs; ++r)
                                loc[(ch * nx + a) * nrhs + r] += Tc[a * nx + b2] * loc[(c * nx + b2) * nrhs + r];
                }
            }
        }
        /* leaves: y_nu += P_nu lhat_nu */
#pragma omp parallel for schedule(dynamic, 4)
        for (long l = leaf_lo; l < leaf_hi; ++l) {
            long c = L0 + l;
            double t[ORC_MAXD];
            for (long i = P->cb[c]; i < P->ce[c]; ++i) {
                long oi = P->perm[i];
                map_from_box(d, P->lo + c * d, P->hi + c * d, P->X + oi * d, t);
                for (int a = 0; a < nx; ++a) {
                    double p = leg_tensor(d, P->alpha + a * d, t);
                    for (int r = 0; r < nrhs; ++r) y[oi * nrhs + r] += p * loc[(c * nx + a) * nrhs + r];
                }
            }
        }
        if (moments_out) memcpy(moments_out, mom, msz * sizeof(double));
        if (locals_out) memcpy(locals_out, loc, msz * sizeof(double));
        free(mom);
        free(loc);
    }
    if (parts & 1) {
        /* nearfield: y_i += sum_{nu' near nu} sum_{j in nu'} K(x_i, x_j) x_j */
#pragma omp parallel for schedule(dynamic, 1)
        for (long l = leaf_lo; l < leaf_hi; ++l) {
            long c = L0 + l;
            for (long f = P->Nptr[c]; f < P->Nptr[c + 1]; ++f) {
                long s = P->Nsrc[f];
                for (long i = P->cb[c]; i < P->ce[c]; ++i) {
                    long oi = P->perm[i];
                    for (long jj = P->cb[s]; jj < P->ce[s]; ++jj) {
                        long oj = P->perm[jj];
                        double k = orc_kernel(P->kind, P->ell, d, P->X + oi * d, P->X + oj * d);
                        for (int r = 0; r < nrhs; ++r) y[oi * nrhs + r] += k * x[oj * nrhs + r];
                    }
                }
            }
        }
    }
    free(want);
}

void orc_matvec(const orc_plan *P, const double *x, double *y, int nrhs)
{
    orc_matvec_ex(P, x, y, nrhs, 3, 0, 0, NULL, NULL);
}

/* ------------------------------------------------------------------ */
/* Conjugate gradients on (K~ + lambda I) alpha = f (eq. (LGS)), one
 * independent iteration per right-hand side column.  Stops a column when
 * ||r|| <= rtol ||f|| (recursive residual); a non-positive curvature step
 * p^T A p < 0 is taken and counted; |p^T A p| <= 1e-300 or a non-finite
 * value is a breakdown.  alpha holds the start vector on entry.
 * info (per column, 5 doubles): iters, neg_curv, rel_res_recursive,
 * rel_res_true, status (0 ok, 1 not converged, 2 breakdown).          */
/* ------------------------------------------------------------------ */
static void apply_A(const orc_plan *P, double lambda, const double *v, double *out, int nrhs)
{
    orc_matvec(P, v, out, nrhs);
    for (long i = 0; i < P->n * nrhs; ++i) out[i] += lambda * v[i];
}

int orc_cg(const orc_plan *P, double lambda, const double *f, double *alpha, int nrhs, double rtol,
           int max_iter, double *info)
{
    long n = P->n;
    size_t sz = (size_t)n * nrhs;
    double *r = (double *)malloc(sz * sizeof(double));
    double *p = (double *)malloc(sz * sizeof(double));
    double *qv = (double *)malloc(sz * sizeof(double));
    double *rr = (double *)calloc((size_t)nrhs, sizeof(double));
    double *fn = (double *)calloc((size_t)nrhs, sizeof(double));
    int *state = (int *)calloc((size_t)nrhs, sizeof(int)); /* 0 active, 1 converged, 2 breakdown */
    int *iters = (int *)calloc((size_t)nrhs, sizeof(int));
    int *neg = (int *)calloc((size_t)nrhs, sizeof(int));
    apply_A(P, lambda, alpha, qv, nrhs);
    for (size_t i = 0; i < sz; ++i) { r[i] = f[i] - qv[i]; p[i] = r[i]; }
    for (long i = 0; i < n; ++i)
        for (int c = 0; c < nrhs; ++c) {
            rr[c] += r[i * nrhs + c] * r[i * nrhs + c];
            fn[c] += f[i * nrhs + c] * f[i * nrhs + c];
        }
    for (int c = 0; c < nrhs; ++c) fn[c] = sqrt(fn[c]);
    for (int it = 0; it < max_iter; ++it) {
        int active = 0;
        for (int c = 0; c < nrhs; ++c) {
            if (state[c] == 0 && sqrt(rr[c]) <= rtol * fn[c]) state[c] = 1;
            if (state[c] == 0) active = 1;
        }
        if (!active) break;
        apply_A(P, lambda, p, qv, nrhs);
        for (int c = 0; c < nrhs; ++c) {
            if (state[c] != 0) continue;
            double pq = 0.0;
            for (long i = 0; i < n; ++i) pq += p[i * nrhs + c] * qv[i * nrhs + c];
            if (!isfinite(pq) || fabs(pq) <= 1e-300) { state[c] = 2; continue; }
            if (pq < 0.0) neg[c]++;
            double a = rr[c] / pq, rn = 0.0;
            for (long i = 0; i < n; ++i) {
                alpha[i * nrhs + c] += a * p[i * nrhs + c];
                r[i * nrhs + c] -= a * qv[i * nrhs + c];
                rn += r[i * nrhs + c] * r[i * nrhs + c];
            }
            double beta = rn / rr[c];
            for (long i = 0; i < n; ++i) p[i * nrhs + c] = r[i * nrhs + c] + beta * p[i * nrhs + c];
            rr[c] = rn;
            iters[c]++;
        }
    }
    for (int c = 0; c < nrhs; ++c)
        if (state[c] == 0 && sqrt(rr[c]) <= rtol * fn[c]) state[c] = 1;
    /* true residual */
    apply_A(P, lambda, alpha, qv, nrhs);
    int worst = 0;
    for (int c = 0; c < nrhs; ++c) {
        double tr = 0.0;
        for (long i = 0; i < n; ++i) {
            double e = f[i * nrhs + c] - qv[i * nrhs + c];
            tr += e * e;
        }
        double den = fn[c] > 0 ? fn[c] : 1.0;
        int st = state[c] == 1 ? 0 : (state[c] == 2 ? 2 : 1);
        info[c * 5 + 0] = iters[c];
        info[c * 5 + 1] = neg[c];
        info[c * 5 + 2] = sqrt(rr[c]) / den;
        info[c * 5 + 3] = sqrt(tr) / den;
        info[c * 5 + 4] = st;
        if (st > worst) worst = st;
    }
    free(r); free(p); free(qv); free(rr); free(fn); free(state); free(iters); free(neg);
    return worst;
}

/* ------------------------------------------------------------------ */
/* Accessors for tests.                                                */
/* ------------------------------------------------------------------ */
void orc_sizes(const orc_plan *P, long *out)
{
    /* n, d, J, ncl, nx, nF, nN */
    out[0] = P->n; out[1] = P->d; out[2] = P->J; out[3] = P->ncl; out[4] = P->nx; out[5] = P->nF; out[6] = P->nN;
}
void orc_get_tree(const orc_plan *P, long *perm, long *cb, long *ce, double *lo, double *hi)
{
    if (perm) memcpy(perm, P->perm, sizeof(long) * (size_t)P->n);
    if (cb) memcpy(cb, P->cb, sizeof(long) * (size_t)P->ncl);
    if (ce) memcpy(ce, P->ce, sizeof(long) * (size_t)P->ncl);
    if (lo) memcpy(lo, P->lo, sizeof(double) * (size_t)P->ncl * P->d);
    if (hi) memcpy(hi, P->hi, sizeof(double) * (size_t)P->ncl * P->d);
}
void orc_get_lists(const orc_plan *P, long *Fptr, long *Fsrc, long *Nptr, long *Nsrc)
{
    if (Fptr) memcpy(Fptr, P->Fptr, sizeof(long) * (size_t)(P->ncl + 1));
    if (Fsrc) memcpy(Fsrc, P->Fsrc, sizeof(long) * (size_t)P->nF);
    if (Nptr) memcpy(Nptr, P->Nptr, sizeof(long) * (size_t)(P->ncl + 1));
    if (Nsrc) memcpy(Nsrc, P->Nsrc, sizeof(long) * (size_t)P->nN);
}
void orc_get_basis(const orc_plan *P, unsigned char *alpha, double *xi, double *V, double *Vinv, double *omega)
{
    int nx = P->nx, d = P->d;
    if (alpha) memcpy(alpha, P->alpha, (size_t)nx * d);
    if (xi) memcpy(xi, P->xi, sizeof(double) * (size_t)nx * d);
    if (V) memcpy(V, P->V, sizeof(double) * (size_t)nx * nx);
    if (Vinv) memcpy(Vinv, P->Vinv, sizeof(double) * (size_t)nx * nx);
    if (omega) memcpy(omega, P->omega, sizeof(double) * (size_t)d);
}
/* Sampled Lebesgue constant (Sec 5.4): the largest sum_a |l_a(t)| over the corners
 * t = (0,...,0), (1,...,1) and the Halton candidates 1..M, with the Lagrange basis
 * l_a(t) = sum_g (V^-1)[g][a] p_g(t) (so that l_a(xi_b) = delta_ab). */
double orc_lebesgue(const orc_plan *P, long M)
{
    int nx = P->nx, d = P->d;
    double *Y = (double *)malloc(sizeof(double) * (size_t)(M + 2) * d);
    for (int k = 0; k < d; ++k) {
        Y[k] = 0.0;
        Y[d + k] = 1.0;
    }
    orc_halton_candidates(d, P->mk, M, Y + 2 * d);
    double *p = (double *)malloc(sizeof(double) * (size_t)nx);
    double best = 0.0;
    for (long j = 0; j < M + 2; ++j) {
        const double *t = Y + j * d;
        for (int g = 0; g < nx; ++g) p[g] = leg_tensor(d, P->alpha + (size_t)g * d, t);
        double sum = 0.0;
        for (int a = 0; a < nx; ++a) {
            double l = 0.0;
            for (int g = 0; g < nx; ++g) l += P->Vinv[(size_t)g * nx + a] * p[g];
            sum += fabs(l);
        }
        if (sum > best) best = sum;
    }
    free(p);
    free(Y);
    return best;
}

/* Near-field entry count E_N = sum over near blocks of |nu||nu'|. */
double orc_near_entries(const orc_plan *P)
{
    double s = 0.0;
    for (long c = 0; c < P->ncl; ++c)
        for (long f = P->Nptr[c]; f < P->Nptr[c + 1]; ++f) {
            long src = P->Nsrc[f];
            s += (double)(P->ce[c] - P->cb[c]) * (double)(P->ce[src] - P->cb[src]);
        }
    return s;
}
/* Thread count for the following calls (n >= 1; timing runs only). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Evaluation at new points: y_i = sum_j K~(t_i, x_j) x_j for targets t_i  */
/* that are not the data sites.  The targets get a tree of the source      */
/* tree's depth built by the same rules (Sec 5.1); target and source        */
/* clusters of equal level are paired as in Sec 5.2 with the same           */
/* admissibility (a block is farfield when admissible and its parent pair   */
/* is not, nearfield when an inadmissible pair of leaves); farfield blocks  */
/* are interpolated in both variables exactly as in eq. (LowRankBlock),     */
/* with the target clusters' own boxes, nodes and transfer matrices.        */
/* ------------------------------------------------------------------ */
typedef struct {
    orc_plan T;              /* target tree: X, n, d, J, ncl, perm, cb, ce, lo, hi, T (transfer) */
    const orc_plan *S;       /* the source plan */
    long nF, nN;
    long *Fptr, *Fsrc, *Nptr, *Nsrc;   /* CSR over target clusters of source clusters */
} orc_eval;

static int admissible_cross(const orc_plan *A, long a, const orc_plan *B, long b, double eta)
{
    int d = A->d;
    const double *la = A->lo + a * d, *ha = A->hi + a * d, *lb = B->lo + b * d, *hb = B->hi + b * d;
    double dist2 = 0.0, da2 = 0.0, db2 = 0.0;
    for (int k = 0; k < d; ++k) {
        double g1 = lb[k] - ha[k], g2 = la[k] - hb[k];
        double g = g1 > g2 ? g1 : g2;
        if (g < 0.0) g = 0.0;
        dist2 += g * g;
        da2 += (ha[k] - la[k]) * (ha[k] - la[k]);
        db2 += (hb[k] - lb[k]) * (hb[k] - lb[k]);
    }
    double dm = da2 > db2 ? da2 : db2;
    return adm_test(dist2, dm, eta, B->adm_half);
}

static void partition_cross(const orc_plan *A, const orc_plan *B, long a, long b, int level, pairlist *F,
                            pairlist *N)
{
    if (A->ce[a] == A->cb[a] || B->ce[b] == B->cb[b]) return;
    if (admissible_cross(A, a, B, b, B->eta)) { pl_push(F, a, b); return; }
    if (level < B->J) {
        for (int i = 1; i <= 2; ++i)
            for (int j = 1; j <= 2; ++j) partition_cross(A, B, 2 * a + i, 2 * b + j, level + 1, F, N);
        return;
    }
    pl_push(N, a, b);
}

orc_eval *orc_eval_create(const orc_plan *S, const double *targets, long m)
{
    if (!S || m < 1) return NULL;
    orc_eval *E = (orc_eval *)calloc(1, sizeof(orc_eval));
    orc_plan *T = &E->T;
    int d = S->d, nx = S->nx;
    E->S = S;
    T->n = m; T->d = d; T->leaf = S->leaf; T->eta = S->eta; T->nx = nx; T->adm_half = S->adm_half;
    T->X = (double *)malloc(sizeof(double) * (size_t)m * d);
    memcpy(T->X, targets, sizeof(double) * (size_t)m * d);
    build_tree_depth(T, S->J);
    pairlist F = {0, 0, NULL, NULL}, N = {0, 0, NULL, NULL};
    partition_cross(T, S, 0, 0, 0, &F, &N);
    E->nF = F.n;
    E->nN = N.n;
    to_csr(T->ncl, &F, &E->Fptr, &E->Fsrc);
    to_csr(T->ncl, &N, &E->Nptr, &E->Nsrc);
    free(F.t); free(F.s); free(N.t); free(N.s);
    /* target transfer matrices T_c = V^-1 M_c, M_c[alpha][alpha'] = p_alpha'(a_par^-1(a_c(xi_alpha))) */
    T->T = (double *)calloc((size_t)T->ncl * nx * nx, sizeof(double));
    double *M = (double *)malloc(sizeof(double) * (size_t)nx * nx);
    double xc[ORC_MAXD], t[ORC_MAXD];
    for (long c = 1; c < T->ncl; ++c) {
        long pa = (c - 1) / 2;
        if (T->ce[c] == T->cb[c]) continue;
        for (long a = 0; a < nx; ++a) {
            map_to_box(d, T->lo + c * d, T->hi + c * d, S->xi + a * d, xc);
            map_from_box(d, T->lo + pa * d, T->hi + pa * d, xc, t);
            for (long b2 = 0; b2 < nx; ++b2) M[a * nx + b2] = leg_tensor(d, S->alpha + b2 * d, t);
        }
        double *Tc = T->T + c * nx * nx;
        for (long a = 0; a < nx; ++a)
            for (long b2 = 0; b2 < nx; ++b2) {
                double sum = 0.0;
                for (long g = 0; g < nx; ++g) sum += S->Vinv[a * nx + g] * M[g * nx + b2];
                Tc[a * nx + b2] = sum;
            }
    }
    free(M);
    return E;
}

void orc_eval_destroy(orc_eval *E)
{
    if (!E) return;
    orc_plan *T = &E->T;
    free(T->X); free(T->perm); free(T->cb); free(T->ce); free(T->lo); free(T->hi); free(T->T);
    free(E->Fptr); free(E->Fsrc); free(E->Nptr); free(E->Nsrc);
    free(E);
}

/* y (m x nrhs, target order) = K~(targets, sources) x (n x nrhs, source order) */
void orc_eval_apply(const orc_eval *E, const double *x, double *y, int nrhs)
{
    const orc_plan *S = E->S, *T = &E->T;
    int d = S->d, nx = S->nx, J = S->J;
    long m = T->n, L0 = cl_level_first(J);
    memset(y, 0, sizeof(double) * (size_t)m * nrhs);
    size_t msz = (size_t)S->ncl * nx * nrhs, lsz = (size_t)T->ncl * nx * nrhs;
    double *mom = (double *)calloc(msz, sizeof(double));
    double *loc = (double *)calloc(lsz, sizeof(double));
    /* source leaf moments mhat = P^T x, upward with T_c^T (Sec 5.2) */
#pragma omp parallel for schedule(dynamic, 4)
    for (long c = L0; c < S->ncl; ++c) {
        double t[ORC_MAXD];
        for (long i = S->cb[c]; i < S->ce[c]; ++i) {
            long oi = S->perm[i];
            map_from_box(d, S->lo + c * d, S->hi + c * d, S->X + oi * d, t);
            for (int a = 0; a < nx; ++a) {
                double p = leg_tensor(d, S->alpha + a * d, t);
                for (int r = 0; r < nrhs; ++r) mom[(c * nx + a) * nrhs + r] += p * x[oi * nrhs + r];
            }
        }
    }
    for (int j = J - 1; j >= 0; --j) {
#pragma omp parallel for schedule(dynamic, 4)
        for (long c = cl_level_first(j); c < cl_level_first(j + 1); ++c)
            for (long ch = 2 * c + 1; ch <= 2 * c + 2; ++ch) {
                const double *Tc = S->T + ch * nx * nx;
                for (int b2 = 0; b2 < nx; ++b2)
                    for (int a = 0; a < nx; ++a)
                        for (int r = 0; r < nrhs; ++r)
                            mom[(c * nx + b2) * nrhs + r] += Tc[a * nx + b2] * mom[(ch * nx + a) * nrhs + r];
            }
    }
    /* coupling of target cluster c with its farfield source clusters: C = V^-1 S V^-T */
#pragma omp parallel
    {
        double *Sm = (double *)malloc(sizeof(double) * (size_t)nx * nx);
        double *W = (double *)malloc(sizeof(double) * (size_t)nx * nx);
        double *C = (double *)malloc(sizeof(double) * (size_t)nx * nx);
        double *xa = (double *)malloc(sizeof(double) * (size_t)nx * d);
        double *xb = (double *)malloc(sizeof(double) * (size_t)nx * d);
#pragma omp for schedule(dynamic, 1)
        for (long c = 0; c < T->ncl; ++c) {
            if (E->Fptr[c] == E->Fptr[c + 1]) continue;
            for (int a = 0; a < nx; ++a) map_to_box(d, T->lo + c * d, T->hi + c * d, S->xi + a * d, xa + a * d);
            for (long f = E->Fptr[c]; f < E->Fptr[c + 1]; ++f) {
                long s = E->Fsrc[f];
                for (int a = 0; a < nx; ++a) map_to_box(d, S->lo + s * d, S->hi + s * d, S->xi + a * d, xb + a * d);
                for (int a = 0; a < nx; ++a)
                    for (int b2 = 0; b2 < nx; ++b2) Sm[a * nx + b2] = orc_kernel(S->kind, S->ell, d, xa + a * d, xb + b2 * d);
                for (int a = 0; a < nx; ++a)
                    for (int b2 = 0; b2 < nx; ++b2) {
                        double sum = 0.0;
                        for (int g = 0; g < nx; ++g) sum += S->Vinv[a * nx + g] * Sm[g * nx + b2];
                        W[a * nx + b2] = sum;
                    }
                for (int a = 0; a < nx; ++a)
                    for (int b2 = 0; b2 < nx; ++b2) {
                        double sum = 0.0;
                        for (int g = 0; g < nx; ++g) sum += W[a * nx + g] * S->Vinv[b2 * nx + g];
                        C[a * nx + b2] = sum;
                    }
                for (int a = 0; a < nx; ++a)
                    for (int b2 = 0; b2 < nx; ++b2)
                        for (int r = 0; r < nrhs; ++r)
                            loc[(c * nx + a) * nrhs + r] += C[a * nx + b2] * mom[(s * nx + b2) * nrhs + r];
            }
        }
        free(Sm); free(W); free(C); free(xa); free(xb);
    }
    /* downward on the target tree: lhat_c += T_c lhat_parent */
    for (int j = 0; j < J; ++j) {
#pragma omp parallel for schedule(dynamic, 4)
        for (long c = cl_level_first(j); c < cl_level_first(j + 1); ++c)
            for (long ch = 2 * c + 1; ch <= 2 * c + 2; ++ch) {
                if (T->ce[ch] == T->cb[ch]) continue;
                const double *Tc = T->T + ch * nx * nx;
                for (int a = 0; a < nx; ++a)
                    for (int b2 = 0; b2 < nx; ++b2)
                        for (int r = 0; r < nrhs; ++r)
                            loc[(ch * nx + a) * nrhs + r] += Tc[a * nx + b2] * loc[(c * nx + b2) * nrhs + r];
            }
    }
    /* target leaves: y_i += p(a_leaf^-1 t_i)^T lhat_leaf, plus the direct nearfield */
#pragma omp parallel for schedule(dynamic, 1)
    for (long c = L0; c < T->ncl; ++c) {
        double t[ORC_MAXD];
        for (long i = T->cb[c]; i < T->ce[c]; ++i) {
            long oi = T->perm[i];
            map_from_box(d, T->lo + c * d, T->hi + c * d, T->X + oi * d, t);
            for (int a = 0; a < nx; ++a) {
                double p = leg_tensor(d, S->alpha + a * d, t);
                for (int r = 0; r < nrhs; ++r) y[oi * nrhs + r] += p * loc[(c * nx + a) * nrhs + r];
            }
            for (long f = E->Nptr[c]; f < E->Nptr[c + 1]; ++f) {
                long s = E->Nsrc[f];
                for (long jj = S->cb[s]; jj < S->ce[s]; ++jj) {
                    long oj = S->perm[jj];
                    double k = orc_kernel(S->kind, S->ell, d, T->X + oi * d, S->X + oj * d);
                    for (int r = 0; r < nrhs; ++r) y[oi * nrhs + r] += k * x[oj * nrhs + r];
                }
            }
        }
    }
    free(mom);
    free(loc);
}

void orc_eval_sizes(const orc_eval *E, long *out)
{
    out[0] = E->T.n; out[1] = E->T.J; out[2] = E->T.ncl; out[3] = E->nF; out[4] = E->nN;
}

void orc_eval_get(const orc_eval *E, long *perm, long *cb, long *ce, double *lo, double *hi, long *Fptr, long *Fsrc,
                  long *Nptr, long *Nsrc)
{
    const orc_plan *T = &E->T;
    long ncl = T->ncl;
    if (perm) memcpy(perm, T->perm, sizeof(long) * (size_t)T->n);
    if (cb) memcpy(cb, T->cb, sizeof(long) * (size_t)ncl);
    if (ce) memcpy(ce, T->ce, sizeof(long) * (size_t)ncl);
    if (lo) memcpy(lo, T->lo, sizeof(double) * (size_t)ncl * T->d);
    if (hi) memcpy(hi, T->hi, sizeof(double) * (size_t)ncl * T->d);
    if (Fptr) memcpy(Fptr, E->Fptr, sizeof(long) * (size_t)(ncl + 1));
    if (Fsrc) memcpy(Fsrc, E->Fsrc, sizeof(long) * (size_t)E->nF);
    if (Nptr) memcpy(Nptr, E->Nptr, sizeof(long) * (size_t)(ncl + 1));
    if (Nsrc) memcpy(Nsrc, E->Nsrc, sizeof(long) * (size_t)E->nN);
}
