// Host-side setup of the dimension weighted FMM (arXiv 2402.09531):
//   weights (Thm 4.6, Sec 6.2), index set (Sec 4), Legendre basis and
//   Vandermonde inverse (Sec 5.2), cluster tree (Sec 5.1), admissibility and
//   block partition (Sec 5.2), nested transfer matrices (Sec 5.2).
#include "setup.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <thread>

namespace dwfmm {

// ------------------------------------------------------------------ weights
bool compute_weights(int rule, int d, const double *b, double eta, const double *explicit_omega, double *omega,
                     std::string &err)
{
    double bmax = 0.0;
    for (int k = 0; k < d; ++k) bmax = std::max(bmax, b[k]);
    auto g = [](double t) { return 2.0 * t + std::sqrt(1.0 + 4.0 * t * t); };
    for (int k = 0; k < d; ++k) {
        switch (rule) {
        case 0:  // R1
            omega[k] = std::max(1.0, std::log2(bmax / b[k]));
            break;
        case 1:  // R2
            omega[k] = 1.0 + std::log2(bmax / b[k]);
            break;
        case 2: {  // R3, Sec 6.2 normalisation omega_1 = 1
            double t1 = 1.0 / (eta * b[0]), tk = 1.0 / (eta * b[k]);
            omega[k] = std::log(std::exp(1.0) * g(tk) / g(t1));
            break;
        }
        case 3:
            if (!explicit_omega) {
                err = "explicit weight rule needs opts.omega";
                return false;
            }
            omega[k] = explicit_omega[k];
            break;
        default:
            err = "unknown weight rule";
            return false;
        }
        if (!(omega[k] > 0.0) || !std::isfinite(omega[k])) {
            err = "dimension weight omega_k must be finite and > 0";
            return false;
        }
    }
    return true;
}

// ------------------------------------------------------------------ Legendre
void legendre01(int m, double t, double *out)
{
    // P_j(s), s = 2t - 1, by (j+1) P_{j+1} = (2j+1) s P_j - j P_{j-1}; scaled by sqrt(2j+1).
    const double s = 2.0 * t - 1.0;
    double pm1 = 1.0, p = s;
    out[0] = 1.0;
    if (m >= 1) out[1] = std::sqrt(3.0) * s;
    for (int j = 1; j < m; ++j) {
        double pn = ((2.0 * j + 1.0) * s * p - j * pm1) / (j + 1.0);
        pm1 = p;
        p = pn;
        out[j + 1] = std::sqrt(2.0 * (j + 1) + 1.0) * pn;
    }
}

// ------------------------------------------------------------------ nodes
// m+1 first-kind Chebyshev points on [0,1], ordered as a Leja sequence that
// starts at the point nearest 1/2 (ties within 1e-9 go to the smaller point).
static std::vector<double> leja_chebyshev(int m)
{
    if (m == 0) return {0.5};
    const int n = m + 1;
    const double pi = 3.14159265358979323846;
    std::vector<double> pts(n);
    for (int j = 0; j < n; ++j) pts[j] = (1.0 - std::cos((2.0 * j + 1.0) * pi / (2.0 * n))) / 2.0;
    std::vector<double> seq;
    std::vector<bool> taken(n, false);
    // start
    int s = 0;
    for (int j = 1; j < n; ++j) {
        double dj = std::fabs(pts[j] - 0.5), ds = std::fabs(pts[s] - 0.5);
        double tol = 1e-9 * (ds > 0 ? ds : 1.0);
        if (dj < ds - tol || (std::fabs(dj - ds) <= tol && pts[j] < pts[s])) s = j;
    }
    seq.push_back(pts[s]);
    taken[s] = true;
    while ((int)seq.size() < n) {
        int best = -1;
        double bv = 0.0;
        for (int j = 0; j < n; ++j) {
            if (taken[j]) continue;
            double prod = 1.0;
            for (double z : seq) prod *= std::fabs(pts[j] - z);
            if (best < 0 || prod > bv * (1.0 + 1e-9) || (std::fabs(prod - bv) <= 1e-9 * bv && pts[j] < pts[best])) {
                best = j;
                bv = prod;
            }
        }
        seq.push_back(pts[best]);
        taken[best] = true;
    }
    return seq;
}

// LU factorisation with partial pivoting, then inverse column by column.
static bool lu_inverse(int n, const std::vector<double> &A, std::vector<double> &inv)
{
    std::vector<double> LU(A);
    std::vector<int> piv(n);
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i)
            if (std::fabs(LU[i * n + k]) > std::fabs(LU[p * n + k])) p = i;
        if (LU[p * n + k] == 0.0) return false;
        piv[k] = p;
        if (p != k)
            for (int j = 0; j < n; ++j) std::swap(LU[k * n + j], LU[p * n + j]);
        for (int i = k + 1; i < n; ++i) {
            LU[i * n + k] /= LU[k * n + k];
            for (int j = k + 1; j < n; ++j) LU[i * n + j] -= LU[i * n + k] * LU[k * n + j];
        }
    }
    inv.assign((size_t)n * n, 0.0);
    std::vector<double> col(n);
    for (int c = 0; c < n; ++c) {
        std::fill(col.begin(), col.end(), 0.0);
        col[c] = 1.0;
        for (int k = 0; k < n; ++k)
            if (piv[k] != k) std::swap(col[k], col[piv[k]]);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < i; ++j) col[i] -= LU[i * n + j] * col[j];
        for (int i = n - 1; i >= 0; --i) {
            for (int j = i + 1; j < n; ++j) col[i] -= LU[i * n + j] * col[j];
            col[i] /= LU[i * n + i];
        }
        for (int i = 0; i < n; ++i) inv[(size_t)i * n + c] = col[i];
    }
    return true;
}

// ------------------------------------------------------------------ basis
// Basis values p_b(t), b in canonical order, through the parent recursion of the index set.
static void basis_values(const HostBasis &B, const double *t, std::vector<std::vector<double>> &axv, double *pv)
{
    for (int k = 0; k < B.d; ++k) legendre01(B.mk[k], t[k], axv[k].data());
    pv[0] = 1.0;
    for (int j = 1; j < B.nx; ++j) pv[j] = pv[B.par[j]] * axv[B.pax[j]][B.pdeg[j]];
}

// Approximate Fekete points (Sec 5.4).  Candidates: Halton points 1..M over the axes with
// m_k > 0 (the r-th active axis in the r-th prime base; the radical inverse is formed as an
// integer over a power of the base, so it is exact up to one rounding), 1/2 elsewhere.
// Selection: greedy volume maximisation over the candidates' basis-value vectors c_j --
// step k takes the candidate whose component orthogonal to the vectors already taken is
// longest (relative 1e-12 ties to the lowest index), which is the pivot order of a
// column-pivoted QR of the Vandermonde matrix.  The orthogonal components are kept by
// modified Gram-Schmidt, projecting each new direction out twice.
// Halton points 1..M over the axes with m_k > 0 (the r-th active axis in the r-th prime base),
// 1/2 on the others: Y[j][k], j < M.
static void halton_points(const HostBasis &B, int64_t M, std::vector<double> &Y)
{
    const int d = B.d;
    std::vector<int> primes;
    for (int c = 2; (int)primes.size() < d; ++c) {
        bool pr = true;
        for (int f : primes) {
            if (f * f > c) break;
            if (c % f == 0) { pr = false; break; }
        }
        if (pr) primes.push_back(c);
    }
    Y.assign((size_t)M * d, 0.5);
    for (int64_t j = 0; j < M; ++j) {
        int r = 0;
        for (int k = 0; k < d; ++k) {
            if (B.mk[k] == 0) continue;
            const uint64_t base = (uint64_t)primes[r++];
            uint64_t i = (uint64_t)j + 1, num = 0, den = 1;
            for (; i > 0; i /= base) {
                num = num * base + i % base;
                den *= base;
            }
            Y[(size_t)j * d + k] = (double)num / (double)den;
        }
    }
}

static bool afp_nodes(HostBasis &B, int64_t M, std::string &err)
{
    const int d = B.d, nx = B.nx;
    if (M < nx) {
        err = "fewer AFP candidates than nodes";
        return false;
    }
    std::vector<double> Y;
    halton_points(B, M, Y);
    // residual vectors, candidate-major
    std::vector<double> R((size_t)M * nx), qv(nx);
    std::vector<std::vector<double>> axv(d);
    for (int k = 0; k < d; ++k) axv[k].resize(B.mk[k] + 1);
    for (int64_t j = 0; j < M; ++j) basis_values(B, &Y[(size_t)j * d], axv, &R[(size_t)j * nx]);
    std::vector<char> taken(M, 0);
    std::vector<double> nrm2(M);
    B.xi.assign((size_t)nx * d, 0.0);
    for (int k = 0; k < nx; ++k) {
        double top = 0.0;
        for (int64_t j = 0; j < M; ++j) {
            if (taken[j]) continue;
            double s = 0.0;
            for (int b = 0; b < nx; ++b) s += R[(size_t)j * nx + b] * R[(size_t)j * nx + b];
            nrm2[j] = s;
            top = std::max(top, s);
        }
        if (!(top > 0.0)) {
            err = "AFP candidates do not span the polynomial space";
            return false;
        }
        int64_t pick = -1;
        for (int64_t j = 0; j < M && pick < 0; ++j)
            if (!taken[j] && nrm2[j] >= top * (1.0 - 1e-12)) pick = j;
        taken[pick] = 1;
        std::copy(&Y[(size_t)pick * d], &Y[(size_t)pick * d] + d, &B.xi[(size_t)k * d]);
        const double inv = 1.0 / std::sqrt(nrm2[pick]);
        for (int b = 0; b < nx; ++b) qv[b] = R[(size_t)pick * nx + b] * inv;
        for (int pass = 0; pass < 2; ++pass)
            for (int64_t j = 0; j < M; ++j) {
                if (taken[j]) continue;
                double *rj = &R[(size_t)j * nx];
                double dot = 0.0;
                for (int b = 0; b < nx; ++b) dot += qv[b] * rj[b];
                for (int b = 0; b < nx; ++b) rj[b] -= dot * qv[b];
            }
    }
    return true;
}

double lebesgue_sampled(const HostBasis &B, int64_t n_samples)
{
    const int d = B.d, nx = B.nx;
    std::vector<double> Y;
    halton_points(B, n_samples, Y);
    std::vector<double> corner0(d, 0.0), corner1(d, 1.0);
    std::vector<std::vector<double>> axv(d);
    for (int k = 0; k < d; ++k) axv[k].resize(B.mk[k] + 1);
    std::vector<double> pv(nx);
    auto lebesgue_at = [&](const double *t) {
        basis_values(B, t, axv, pv.data());
        double sum = 0.0;
        for (int a = 0; a < nx; ++a) {
            double l = 0.0;  // l_a(t) = sum_g (V^-1)[g][a] p_g(t)
            for (int g = 0; g < nx; ++g) l += B.Vinv[(size_t)g * nx + a] * pv[g];
            sum += std::fabs(l);
        }
        return sum;
    };
    double best = std::max(lebesgue_at(corner0.data()), lebesgue_at(corner1.data()));
    for (int64_t j = 0; j < n_samples; ++j) best = std::max(best, lebesgue_at(&Y[(size_t)j * d]));
    return best;
}

bool build_basis(int d, const double *omega, double q, HostBasis &B, std::string &err, int node_rule,
                 int64_t n_cand, int index_rule)
{
    B = HostBasis();
    B.d = d;
    B.omega.assign(omega, omega + d);
    // enumerate {alpha : sum_k omega_k alpha_k <= q} with an odometer over axes
    std::vector<std::vector<uint8_t>> set;
    std::vector<int> a(d, 0);
    const double slack = 1e-9;
    for (;;) {
        bool inside;
        if (index_rule == 1) {
            int top = 0;
            for (int k = 0; k < d; ++k) top = std::max(top, a[k]);
            inside = top <= q + slack;
        } else {
            double used = 0.0;
            for (int k = 0; k < d; ++k) used += omega[k] * a[k];
            inside = used <= q + slack;
        }
        if (inside) {
            set.emplace_back(a.begin(), a.end());
            if (set.size() > 4096) {
                err = "index set larger than 4096 entries";
                return false;
            }
            a[0]++;  // advance the fastest axis
            continue;
        }
        // overflow: reset the lowest non-zero axis and carry
        int k = 0;
        while (k < d && a[k] == 0) ++k;
        if (k >= d - 1) break;
        a[k] = 0;
        a[k + 1]++;
    }
    // canonical order: weighted degree (summed over axes in order), then colex
    std::vector<double> key(set.size());
    for (size_t i = 0; i < set.size(); ++i) {
        double w = 0.0;
        for (int k = 0; k < d; ++k) w += omega[k] * set[i][k];
        key[i] = w;
    }
    std::vector<size_t> ord(set.size());
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](size_t x, size_t y) {
        if (key[x] != key[y]) return key[x] < key[y];
        for (int k = d - 1; k >= 0; --k)
            if (set[x][k] != set[y][k]) return set[x][k] < set[y][k];
        return false;
    });
    const int nx = (int)set.size();
    B.nx = nx;
    B.alpha.resize((size_t)nx * d);
    for (int i = 0; i < nx; ++i)
        for (int k = 0; k < d; ++k) B.alpha[(size_t)i * d + k] = set[ord[i]][k];
    B.mk.assign(d, 0);
    for (int i = 0; i < nx; ++i)
        for (int k = 0; k < d; ++k) B.mk[k] = std::max<int>(B.mk[k], B.alpha[(size_t)i * d + k]);
    // parent structure: beta = parent + beta_k e_k with k the last non-zero axis
    B.par.assign(nx, -1);
    B.pax.assign(nx, 0);
    B.pdeg.assign(nx, 0);
    for (int i = 1; i < nx; ++i) {
        int k = d - 1;
        while (B.alpha[(size_t)i * d + k] == 0) --k;
        std::vector<uint8_t> p(B.alpha.begin() + (size_t)i * d, B.alpha.begin() + (size_t)(i + 1) * d);
        p[k] = 0;
        int found = -1;
        for (int j = 0; j < i; ++j)
            if (std::equal(p.begin(), p.end(), B.alpha.begin() + (size_t)j * d)) { found = j; break; }
        if (found < 0) {
            err = "index set is not a lower set";
            return false;
        }
        B.par[i] = found;
        B.pax[i] = k;
        B.pdeg[i] = B.alpha[(size_t)i * d + k];
    }
    int off = 0;
    for (int k = 0; k < d; ++k)
        if (B.mk[k] > 0) {
            B.act_axis.push_back(k);
            B.act_off.push_back(off);
            B.act_m.push_back(B.mk[k]);
            off += B.mk[k] + 1;
        }
    B.nleg = off;
    if (node_rule == 0) {
        // per-axis nodes; xi_alpha = (z^(1)_{alpha_1}, ..., z^(d)_{alpha_d})
        B.xi.resize((size_t)nx * d);
        for (int k = 0; k < d; ++k) {
            std::vector<double> z = leja_chebyshev(B.mk[k]);
            for (int i = 0; i < nx; ++i) B.xi[(size_t)i * d + k] = z[B.alpha[(size_t)i * d + k]];
        }
    } else if (!afp_nodes(B, n_cand > 0 ? n_cand : std::max<int64_t>(2000, 50 * (int64_t)nx), err)) {
        return false;
    }
    // Vandermonde V[a][b] = p_b(xi_a) and its inverse
    std::vector<double> V((size_t)nx * nx);
    std::vector<double> leg(256);
    for (int i = 0; i < nx; ++i) {
        std::vector<double> pv(nx);
        pv[0] = 1.0;
        std::vector<std::vector<double>> axv(d);
        for (int k = 0; k < d; ++k) {
            axv[k].resize(B.mk[k] + 1);
            legendre01(B.mk[k], B.xi[(size_t)i * d + k], axv[k].data());
        }
        for (int j = 1; j < nx; ++j) pv[j] = pv[B.par[j]] * axv[B.pax[j]][B.pdeg[j]];
        for (int j = 0; j < nx; ++j) V[(size_t)i * nx + j] = pv[j];
    }
    if (!lu_inverse(nx, V, B.Vinv)) {
        err = "Vandermonde matrix is singular";
        return false;
    }
    return true;
}

// ------------------------------------------------------------------ tree
bool build_tree(const double *pts, int64_t n, int d, const double *b, int leaf, double eta, HostTree &T,
                std::string &err, int forced_J, bool with_partition, int adm_half)
{
    T = HostTree();
    T.n = n;
    T.d = d;
    T.leaf = leaf;
    T.eta = eta;
    T.adm_half = adm_half;
    T.b.assign(b, b + d);
    int J = 0;
    if (forced_J >= 0)
        J = forced_J;
    else
        while ((n + ((int64_t)1 << J) - 1) >> J > leaf) ++J;
    if (J > 30) {
        err = "tree too deep";
        return false;
    }
    T.J = J;
    T.ncl = ((int64_t)1 << (J + 1)) - 1;
    T.nleaf = (int64_t)1 << J;
    T.perm.resize(n);
    std::iota(T.perm.begin(), T.perm.end(), 0);
    T.begin.assign(T.ncl, 0);
    T.end.assign(T.ncl, 0);
    T.lo.assign((size_t)T.ncl * d, 0.0);
    T.hi.assign((size_t)T.ncl * d, 0.0);
    T.begin[0] = 0;
    T.end[0] = (int32_t)n;
    // Working copy of the coordinates kept in the current tree order (SoA), so that boxes and
    // median selections read contiguous memory; the clusters of a level are independent and
    // are processed by parallel threads.
    std::vector<double> W((size_t)d * n);
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < d; ++k) W[(size_t)k * n + i] = pts[(size_t)i * d + k];
    auto cluster = [&](int64_t c, int j, std::vector<std::pair<double, int32_t>> &key, std::vector<double> &tmp,
                       std::vector<int32_t> &itmp) {
        const int32_t bgn = T.begin[c], e = T.end[c], m = e - bgn;
        double *lo = &T.lo[(size_t)c * d], *hi = &T.hi[(size_t)c * d];
        for (int k = 0; k < d && m > 0; ++k) {
            const double *w = &W[(size_t)k * n + bgn];
            double a = w[0], z = w[0];
            for (int32_t i = 1; i < m; ++i) {
                a = std::min(a, w[i]);
                z = std::max(z, w[i]);
            }
            lo[k] = a;
            hi[k] = z;
        }
        std::vector<int32_t> order;
        if (j == J) {
            // canonical order inside a leaf: by original index
            key.resize(m);
            for (int32_t i = 0; i < m; ++i) key[i] = {(double)T.perm[bgn + i], i};
            std::sort(key.begin(), key.end());
        } else {
            int axis = 0;
            double ext = -1.0;
            for (int k = 0; k < d; ++k) {
                const double w = m > 0 ? hi[k] - lo[k] : 0.0;
                if (w > ext) {
                    ext = w;
                    axis = k;
                }
            }
            const int32_t half = (m + 1) / 2;
            T.begin[2 * c + 1] = bgn;
            T.end[2 * c + 1] = bgn + half;
            T.begin[2 * c + 2] = bgn + half;
            T.end[2 * c + 2] = e;
            if (m <= 1) return;
            // order by (coordinate, original index); the left child takes the first ceil(m/2)
            key.resize(m);
            const double *w = &W[(size_t)axis * n + bgn];
            for (int32_t i = 0; i < m; ++i) key[i] = {w[i], i};
            const int32_t *pid = &T.perm[bgn];
            std::nth_element(key.begin(), key.begin() + half, key.end(),
                             [&](const std::pair<double, int32_t> &u, const std::pair<double, int32_t> &v) {
                                 return u.first < v.first || (u.first == v.first && pid[u.second] < pid[v.second]);
                             });
        }
        // apply the new order to the working coordinates (not needed below the leaves) and the permutation
        tmp.resize(m);
        itmp.resize(m);
        for (int k = 0; k < d && j < J; ++k) {
            double *w = &W[(size_t)k * n + bgn];
            for (int32_t i = 0; i < m; ++i) tmp[i] = w[key[i].second];
            std::copy(tmp.begin(), tmp.end(), w);
        }
        for (int32_t i = 0; i < m; ++i) itmp[i] = T.perm[bgn + key[i].second];
        std::copy(itmp.begin(), itmp.end(), T.perm.begin() + bgn);
    };
    const int nthreads = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    for (int j = 0; j <= J; ++j) {
        const int64_t first = ((int64_t)1 << j) - 1, last = ((int64_t)1 << (j + 1)) - 1;
        const int64_t cnt = last - first;
        const int nt = (int)std::min<int64_t>(nthreads, cnt);
        auto work = [&](int t) {
            std::vector<std::pair<double, int32_t>> key;
            std::vector<double> tmp;
            std::vector<int32_t> itmp;
            for (int64_t c = first + t; c < last; c += nt) cluster(c, j, key, tmp, itmp);
        };
        if (nt <= 1 || (int64_t)n < 50000) {
            for (int t = 0; t < nt; ++t) work(t);
        } else {
            std::vector<std::thread> pool;
            for (int t = 0; t < nt; ++t) pool.emplace_back(work, t);
            for (auto &th : pool) th.join();
        }
    }
    if (with_partition) partition_pairs(T, T, eta, T.Fptr, T.Fsrc, T.Nptr, T.Nsrc, T.min_far_level);
    else T.min_far_level = J + 1;
    return true;
}

// ------------------------------------------------------------------ transfer
void partition_pairs(const HostTree &A, const HostTree &B, double eta, std::vector<int32_t> &Fptr,
                     std::vector<int32_t> &Fsrc, std::vector<int32_t> &Nptr, std::vector<int32_t> &Nsrc,
                     int &min_far_level)
{
    const int d = A.d, J = B.J;
    std::vector<std::pair<int32_t, int32_t>> far, near;
    // full diagonal: dist^2 >= eta^2 D^2; half diagonal: eta dist >= D / 2, i.e. (2 eta)^2 dist^2 >= D^2
    const bool half = B.adm_half != 0;
    const double lhs_scale = half ? (2.0 * eta) * (2.0 * eta) : 1.0, rhs_scale = half ? 1.0 : eta * eta;
    auto admissible = [&](int64_t u, int64_t v) {
        const double *lu = &A.lo[(size_t)u * d], *hu = &A.hi[(size_t)u * d];
        const double *lv = &B.lo[(size_t)v * d], *hv = &B.hi[(size_t)v * d];
        double dist2 = 0.0, du = 0.0, dv = 0.0;
        for (int k = 0; k < d; ++k) {
            double gap = std::max(std::max(lv[k] - hu[k], lu[k] - hv[k]), 0.0);
            dist2 += gap * gap;
            du += (hu[k] - lu[k]) * (hu[k] - lu[k]);
            dv += (hv[k] - lv[k]) * (hv[k] - lv[k]);
        }
        return lhs_scale * dist2 >= rhs_scale * std::max(du, dv);
    };
    struct Item { int32_t u, v; int lev; };
    std::vector<Item> stack{{0, 0, 0}};
    while (!stack.empty()) {
        Item it = stack.back();
        stack.pop_back();
        if (A.end[it.u] == A.begin[it.u] || B.end[it.v] == B.begin[it.v]) continue;
        if (admissible(it.u, it.v)) {
            far.push_back({it.u, it.v});
        } else if (it.lev < J) {
            // reverse push so that children pop in (1,1),(1,2),(2,1),(2,2) order
            for (int i = 2; i >= 1; --i)
                for (int k = 2; k >= 1; --k) stack.push_back({2 * it.u + i, 2 * it.v + k, it.lev + 1});
        } else {
            near.push_back({it.u, it.v});
        }
    }
    auto csr = [&](std::vector<std::pair<int32_t, int32_t>> &pairs, std::vector<int32_t> &ptr,
                   std::vector<int32_t> &src) {
        std::stable_sort(pairs.begin(), pairs.end(),
                         [](const std::pair<int32_t, int32_t> &x, const std::pair<int32_t, int32_t> &y) {
                             return x.first < y.first || (x.first == y.first && x.second < y.second);
                         });
        ptr.assign(A.ncl + 1, 0);
        src.resize(pairs.size());
        for (auto &p : pairs) ptr[p.first + 1]++;
        for (int64_t c = 0; c < A.ncl; ++c) ptr[c + 1] += ptr[c];
        for (size_t i = 0; i < pairs.size(); ++i) src[i] = pairs[i].second;
    };
    csr(far, Fptr, Fsrc);
    csr(near, Nptr, Nsrc);
    min_far_level = J + 1;
    for (auto &p : far) {
        int lev = 0;
        while ((((int64_t)1 << (lev + 1)) - 1) <= p.first) ++lev;
        min_far_level = std::min(min_far_level, lev);
    }
}

static void ref_coords(const double *lo, const double *hi, const double *x, int d, double *t)
{
    for (int k = 0; k < d; ++k) t[k] = hi[k] > lo[k] ? (x[k] - lo[k]) / (hi[k] - lo[k]) : 0.5;
}

void box_nodes(const HostTree &T, const HostBasis &B, std::vector<double> &nodes)
{
    const int d = T.d, nx = B.nx;
    nodes.assign((size_t)T.ncl * nx * d, 0.0);
    for (int64_t c = 0; c < T.ncl; ++c) {
        const double *lo = &T.lo[(size_t)c * d], *hi = &T.hi[(size_t)c * d];
        for (int a = 0; a < nx; ++a)
            for (int k = 0; k < d; ++k) {
                double w = hi[k] - lo[k];
                nodes[((size_t)c * nx + a) * d + k] = w > 0 ? lo[k] + B.xi[(size_t)a * d + k] * w : lo[k];
            }
    }
}

void transfer_matrices(const HostTree &T, const HostBasis &B, std::vector<double> &E)
{
    const int d = T.d, nx = B.nx;
    E.assign((size_t)T.ncl * nx * nx, 0.0);
    std::vector<double> x(d), t(d), pv(nx);
    std::vector<std::vector<double>> axv(d);
    for (int k = 0; k < d; ++k) axv[k].resize(B.mk[k] + 1);
    for (int64_t c = 1; c < T.ncl; ++c) {
        if (T.end[c] == T.begin[c]) continue;
        const int64_t p = (c - 1) / 2;
        const double *lc = &T.lo[(size_t)c * d], *hc = &T.hi[(size_t)c * d];
        const double *lp = &T.lo[(size_t)p * d], *hp = &T.hi[(size_t)p * d];
        for (int a = 0; a < nx; ++a) {
            for (int k = 0; k < d; ++k) {
                double w = hc[k] - lc[k];
                x[k] = w > 0 ? lc[k] + B.xi[(size_t)a * d + k] * w : lc[k];
            }
            ref_coords(lp, hp, x.data(), d, t.data());
            for (int k = 0; k < d; ++k) legendre01(B.mk[k], t[k], axv[k].data());
            pv[0] = 1.0;
            for (int j = 1; j < nx; ++j) pv[j] = pv[B.par[j]] * axv[B.pax[j]][B.pdeg[j]];
            // l_b(t) = sum_g (V^-1)[g][b] p_g(t)
            for (int bb = 0; bb < nx; ++bb) {
                double s = 0.0;
                for (int g = 0; g < nx; ++g) s += B.Vinv[(size_t)g * nx + bb] * pv[g];
                E[((size_t)c * nx + a) * nx + bb] = s;
            }
        }
    }
}

}  // namespace dwfmm
