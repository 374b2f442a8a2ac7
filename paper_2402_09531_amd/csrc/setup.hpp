// Host-side construction of the FMM structure: cluster tree, block partition,
// index set, interpolation nodes, V^-1 and transfer matrices.  The data built
// here is uploaded once; the matvec itself runs in HIP kernels.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace dwfmm {

constexpr int kMaxDim = 64;

// Balanced binary cluster tree with heap numbering: cluster t of level j has id
// 2^j - 1 + t, children 2c+1 and 2c+2.  Points are stored in tree order.
struct HostTree {
    int64_t n = 0;
    int d = 0, leaf = 0, J = 0;
    double eta = 0.0;
    int adm_half = 0;                    // admissibility against the half box diagonal
    int64_t ncl = 0, nleaf = 0;
    std::vector<double> b;               // box side lengths b_k (dimension weights)
    std::vector<int32_t> perm;           // tree position -> original index
    std::vector<int32_t> begin, end;     // point range of each cluster
    std::vector<double> lo, hi;          // tight boxes, [ncl][d]
    std::vector<int32_t> Fptr, Fsrc;     // farfield CSR over target clusters
    std::vector<int32_t> Nptr, Nsrc;     // nearfield CSR over target clusters (leaves only)
    int min_far_level = 0;               // first level holding a farfield block (J+1 if none)
};

// Index set Lambda_{omega,q,d}, nodes and Vandermonde inverse.
struct HostBasis {
    int d = 0, nx = 0;
    std::vector<double> omega;           // [d]
    std::vector<uint8_t> alpha;          // [nx][d], canonical order
    std::vector<int> mk;                 // max_alpha alpha_k per axis
    std::vector<double> xi;              // reference nodes [nx][d]
    std::vector<double> Vinv;            // [nx][nx], row-major, (V^-1)[g][b]
    // p_beta = p_{par[beta]} * p_{pdeg[beta]}(t_{pax[beta]}) for beta > 0
    std::vector<int32_t> par, pax, pdeg;
    // active axes (mk > 0), and offsets of their 1-D Legendre value blocks
    std::vector<int32_t> act_axis, act_off, act_m;
    int nleg = 0;                        // sum over active axes of (mk + 1)
};

// forced_J >= 0 builds a tree of that depth (clusters may be empty); with_partition = false
// skips the block partition (Fptr/Fsrc/Nptr/Nsrc stay empty).  adm_half selects the
// admissibility eta dist >= max half diagonal instead of dist >= eta max diagonal.
bool build_tree(const double *pts_host, int64_t n, int d, const double *b, int leaf, double eta, HostTree &T,
                std::string &err, int forced_J = -1, bool with_partition = true, int adm_half = 0);

// Level-wise block partition of (target cluster, source cluster) pairs of two trees of equal
// depth with the admissibility of Sec 5.2 (against the full or, when B.adm_half is set, the
// half box diagonal): CSR over target clusters of source clusters; nearfield entries are leaf
// pairs.  min_far_level: first level with a farfield block (J+1 if none).  With A = B it is
// the square partition of build_tree.
void partition_pairs(const HostTree &A, const HostTree &B, double eta, std::vector<int32_t> &Fptr,
                     std::vector<int32_t> &Fsrc, std::vector<int32_t> &Nptr, std::vector<int32_t> &Nsrc,
                     int &min_far_level);

// Sampled Lebesgue constant (Sec 5.4): the largest sum_a |l_a(t)| of the Lagrange basis
// l(t) = V^-T p(t) over the corners t = 0 and t = 1 and the Halton points 1..n_samples of the
// AFP candidate sequence (a lower bound of the constant over [0,1]^d).
double lebesgue_sampled(const HostBasis &B, int64_t n_samples);

// node_rule 0: per-axis Chebyshev-Leja nodes; 1: approximate Fekete points from n_cand
// Halton candidates (0 = max(2000, 50 n_x)).  index_rule 0: weighted total degree set;
// 1: tensor set max_k alpha_k <= q.
bool build_basis(int d, const double *omega, double q, HostBasis &B, std::string &err, int node_rule = 0,
                 int64_t n_cand = 0, int index_rule = 0);

bool compute_weights(int rule, int d, const double *b, double eta, const double *explicit_omega, double *omega,
                     std::string &err);

// Lagrange transfer matrices E_c[a][b] = l^parent_b(a_parent^-1(a_c(xi_a))), c >= 1.
void transfer_matrices(const HostTree &T, const HostBasis &B, std::vector<double> &E);

// Interpolation nodes of every box: nodes[c][a][k] = a_c(xi_a)_k.
void box_nodes(const HostTree &T, const HostBasis &B, std::vector<double> &nodes);

// Orthonormal Legendre values p_0..p_m at t on [0,1].
void legendre01(int m, double t, double *out);

}  // namespace dwfmm
