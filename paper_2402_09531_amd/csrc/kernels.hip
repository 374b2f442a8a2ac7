// HIP kernels (gfx950) for one dimension weighted FMM matvec, arXiv 2402.09531 Sec 5.2:
//   P2M  leaf moments      m_nu = L_nu^T x_nu  (Lagrange basis of the leaf box)
//   M2M  upward            m_nu = sum_c E_c^T m_c                 (two-scale relation)
//   M2L  coupling          l_nu += S_{nu,nu'} m_nu',  S = [K(a_nu(xi_a), a_nu'(xi_b))]
//   L2L  downward          l_c += E_c l_nu
//   L2P  leaf evaluation   y_nu += L_nu l_nu
//   P2P  nearfield         y_nu += K_{nu,nu'} x_nu' over inadmissible leaf pairs
// The Lagrange form L = P V^-1 of the paper's Legendre cluster basis P is used
// throughout: it is the same operator, K~_{nu,nu'} = P_nu V^-1 S V^-T P_nu'^T.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "device.hpp"

namespace dwfmm {

namespace {

constexpr int kMaxNx = 128;
constexpr int kMaxNodeWords = 3072;  // nx * dpad bound of the generic M2L node tiles
constexpr int kM2lRows = 16;         // coupling rows the generic M2L forms at a time
typedef double dbl4 __attribute__((ext_vector_type(4)));  // accumulator of v_mfma_f64_16x16x4f64

// e^x in FP64 for |x| <= 708 without special-case branches: Cody-Waite reduction
// x = n ln2 + r, |r| <= ln2/2, with a two-part ln2, then a degree-10 polynomial
// for e^r (coefficients: the interpolant of e^r at 11 first-kind Chebyshev points
// of [-ln2/2, ln2/2], from csrc/gen_exp_coeffs.py; 2.9e-16 relative interpolation
// error), scaled by 2^n.
__device__ __forceinline__ double exp_bounded(double x)
{
    const double n = rint(x * 1.4426950408889634);
    double r = fma(-n, 0.6931471805599453, x);
    r = fma(-n, 2.3201926491189795e-17, r);
    double p = 2.7626373407076024e-07;
    p = fma(p, r, 2.764018103268004e-06);
    p = fma(p, r, 2.480150429736007e-05);
    p = fma(p, r, 0.00019841170269600702);
    p = fma(p, r, 0.0013888888932537785);
    p = fma(p, r, 0.008333333385668792);
    p = fma(p, r, 0.04166666666657299);
    p = fma(p, r, 0.166666666665544);
    p = fma(p, r, 0.5000000000000006);
    p = fma(p, r, 1.0000000000000067);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)n);
}

// 2^f for f in [-1/2, 1/2]: the degree-10 interpolant of 2^f at 11 first-kind Chebyshev points
// of [-1/2, 1/2] (csrc/gen_exp_coeffs.py; 2.9e-16 relative).
__device__ __forceinline__ double exp2_frac(double f)
{
    double p = 7.072587226569927e-09;
    p = fma(p, f, 1.0208690586037056e-07);
    p = fma(p, f, 1.3215442576793237e-06);
    p = fma(p, f, 1.5252657258547322e-05);
    p = fma(p, f, 0.00015403530441763784);
    p = fma(p, f, 0.001333355823016814);
    p = fma(p, f, 0.00961812910760687);
    p = fma(p, f, 0.055504108664447695);
    p = fma(p, f, 0.24022650695910097);
    p = fma(p, f, 0.69314718055995);
    return fma(p, f, 1.0);
}

// 2^t in FP64 for |t| <= 1020: t = n + f with n = rint(t) and f = t - n in [-1/2, 1/2]
// (exact), then 2^f by exp2_frac, scaled by 2^n.  Two operations fewer than exp_bounded
// where the caller can fold log2(e) into its own operands.
__device__ __forceinline__ double exp2_bounded(double t)
{
    const double n = rint(t);
    return ldexp(exp2_frac(t - n), (int)n);
}

// 2^t for t <= 0: arguments below -1075 (where 2^t underflows to zero) are clamped.
__device__ __forceinline__ double exp2_nonpos(double t) { return exp2_bounded(fmax(t, -1075.0)); }

// sqrt(x) for x >= 1e-300 (callers clamp; below that the kernels are 1 to double precision):
// with y the hardware reciprocal square root and g = x y, e = 1 - g y is small (about twice
// the seed's relative error) and sqrt(x) = g (1 - e)^(-1/2) = g (1 + e/2 + 3e^2/8 + ...).
// Two terms of the series leave 5e^3/16, below 2^-58 for a seed within 2^-20 (the device
// builtin is far better), so the result is within one unit in the last place.  No scaling of
// tiny arguments and no special values, unlike the library square root.
__device__ __forceinline__ double sqrt_pos(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double g = x * y;
    const double e = fma(-g, y, 1.0);
    const double w = g * e;
    return fma(w, fma(e, 0.375, 0.5), g);
}

// Kernel value from the squared distance, with the branch-free exponential.  r2 may be slightly
// negative from rounding in the Gram form; the kernels that take its square root clamp it.
// The exponentials are taken as 2^t with log2(e) folded into the scale of the argument.
template <int KIND>
__device__ __forceinline__ double kernel_fast(double r2, double inv_ell)
{
    constexpr double kLog2e = 1.4426950408889634, kSqrt3 = 1.7320508075688772;
    if constexpr (KIND == 0) {
        const double r = sqrt_pos(fmax(r2, 1e-300));
        const double s = r * (kSqrt3 * inv_ell);
        const double e = exp2_nonpos(r * (-kSqrt3 * kLog2e * inv_ell));
        return fma(s, e, e);
    } else if constexpr (KIND == 1) {
        return exp2_nonpos(r2 * (-kLog2e * inv_ell));
    } else {
        return exp2_nonpos(sqrt_pos(fmax(r2, 1e-300)) * (-kLog2e * inv_ell));
    }
}

// Matern-3/2 (1 + s) e^-s from s^2 = 3 r^2 / ell^2, for callers whose coordinates are already
// scaled by sqrt(3) / ell: one multiplication fewer than kernel_fast<0>.  Without CLAMP the
// caller guarantees s log2(e) <= 1000, and 2^(-s log2(e)) is split by the round-to-integer
// constant 1.5 2^52: m = -s log2(e) + 1.5 2^52 rounded once (an FMA) has unit spacing, so
// n = m - 1.5 2^52 is the nearest integer to -s log2(e) (exact subtraction), its two's complement
// sits in the low 32 bits of m, and f = -s log2(e) - n lies in [-1/2, 1/2] -- the multiplication,
// rounding and conversion of exp2_bounded in two operations.
template <bool CLAMP>
__device__ __forceinline__ double matern_s2(double s2)
{
    constexpr double kLog2e = 1.4426950408889634, kRound = 6755399441055744.0;  // 1.5 2^52
    // |s2| + 1e-300 keeps the square root's argument positive (s2 may be a rounding below zero)
    // in one addition, where a clamp by fmax would first canonicalise an MFMA result
    const double s = sqrt_pos(fabs(s2) + 1e-300);
    if constexpr (CLAMP) {
        const double e = exp2_nonpos(s * -kLog2e);
        return fma(s, e, e);
    } else {
        const double m = fma(s, -kLog2e, kRound);
        const double n = m - kRound;
        const double e = ldexp(exp2_frac(fma(s, -kLog2e, -n)), __double2loint(m));
        return fma(s, e, e);
    }
}

template <int KIND>
__device__ __forceinline__ double kernel_val(double r2, double inv_ell)
{
    if constexpr (KIND == 0) {
        double s = 1.7320508075688772 * sqrt(r2) * inv_ell;
        return (1.0 + s) * exp(-s);
    } else if constexpr (KIND == 1) {
        return exp(-r2 * inv_ell);
    } else {
        return exp(-sqrt(r2) * inv_ell);
    }
}

// POLY_TEST kernel 1 + sum_{k<p} x_k y_k + (x_0 y_0)^2
__device__ __forceinline__ double poly_kernel(const double *a, const double *b, int p)
{
    double v = 1.0;
    for (int k = 0; k < p; ++k) v += a[k] * b[k];
    double t = a[0] * b[0];
    return v + t * t;
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// ---------------------------------------------------------------- basis cache
// Lb[a][i] = l_a(t_i) = sum_g Vinv[g][a] p_g(t_i), t_i = reference coordinates of
// point i in its leaf box.  lidx[g][j] lists the Legendre slots whose product is p_g.
__global__ void basis_kernel(DevTree T, int nx, const double *__restrict__ clo, const double *__restrict__ csc,
                             const double *__restrict__ coff, const int32_t *__restrict__ lidx, int nnz_max,
                             const double *__restrict__ Vinv, int nleg, const int32_t *__restrict__ leg_axis,
                             const int32_t *__restrict__ leg_deg, double *__restrict__ Lb)
{
    const int c = T.leaf_first + blockIdx.x;
    const int cb = T.cbeg[c], ce = T.cend[c];
    for (int i = cb + (int)threadIdx.x; i < ce; i += blockDim.x) {
        double leg[128];
        double p[kMaxNx];
        for (int s = 0; s < nleg; ++s) {
            const int k = leg_axis[s], m = leg_deg[s];
            const double t = (T.Xs[(size_t)k * T.n + i] - clo[(size_t)c * T.d + k]) * csc[(size_t)c * T.d + k] +
                             coff[(size_t)c * T.d + k];
            // orthonormal Legendre p_m(t) = sqrt(2m+1) P_m(2t-1)
            const double u = 2.0 * t - 1.0;
            double p0 = 1.0, p1 = u;
            double v = 1.0;
            if (m >= 1) {
                for (int j = 1; j < m; ++j) {
                    double p2 = ((2.0 * j + 1.0) * u * p1 - j * p0) / (j + 1.0);
                    p0 = p1;
                    p1 = p2;
                }
                v = sqrt(2.0 * m + 1.0) * p1;
            }
            leg[s] = v;
        }
        for (int g = 0; g < nx; ++g) {
            double v = 1.0;
            for (int j = 0; j < nnz_max; ++j) {
                const int s = lidx[g * nnz_max + j];
                if (s >= 0) v *= leg[s];
            }
            p[g] = v;
        }
        for (int a = 0; a < nx; ++a) {
            double v = 0.0;
            for (int g = 0; g < nx; ++g) v += Vinv[g * nx + a] * p[g];
            Lb[(size_t)a * T.n + i] = v;
        }
    }
}

// ---------------------------------------------------------------- P2M (+ gather of x into tree order)
// Kernel bodies are __device__ functions of (tree, operator, block index) so that a single
// problem and a batch of problems run the same code.
__device__ __forceinline__ void p2m_body(const DevTree &T, const DevOp &O, int l, const double *__restrict__ x,
                                         int nrhs, int do_far, double *xl)
{
    const int c = T.leaf_first + l;
    const int cb = T.cbeg[c], ce = T.cend[c], np = ce - cb;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int r = 0; r < nrhs; ++r) {
        for (int i = threadIdx.x; i < np; i += blockDim.x) {
            const double v = x[(size_t)T.perm[cb + i] * nrhs + r];
            xl[i] = v;
            O.xt[(size_t)(cb + i) * nrhs + r] = v;
            if (O.xtb) O.xtb[(size_t)(cb + i) * nrhs + r] = (__bf16)(float)v;
        }
        __syncthreads();
        if (do_far) {
            for (int a = wave; a < O.nx; a += blockDim.x >> 6) {
                double s = 0.0;
                for (int i = lane; i < np; i += 64) s += O.Lb[(size_t)a * T.n + cb + i] * xl[i];
                s = wave_sum(s);
                if (lane == 0) O.M[((size_t)c * O.nx + a) * nrhs + r] = s;
            }
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void p2m_kernel(DevTree T, DevOp O, const double *__restrict__ x, int nrhs,
                                                  int do_far)
{
    extern __shared__ double xl[];  // [max_leaf]
    p2m_body(T, O, blockIdx.x, x, nrhs, do_far, xl);
}

// P2M for several rhs: the leaf's whole block of charges is staged once (rows of nrhs
// doubles, read and written in order), then every (node, rhs) moment sums over the leaf's
// points from LDS, in point order.  For leaves of at most 4096 / nrhs points.
__global__ __launch_bounds__(256) void p2m_multi_kernel(DevTree T, DevOp O, const double *__restrict__ x, int nrhs,
                                                        int do_far)
{
    extern __shared__ double xl[];  // [np][nrhs]
    const int l = blockIdx.x, c = T.leaf_first + l;
    const int cb = T.cbeg[c], np = T.cend[c] - cb;
    for (int e = threadIdx.x; e < np * nrhs; e += blockDim.x) {
        const int i = e / nrhs, r = e - i * nrhs;
        const double v = x[(size_t)T.perm[cb + i] * nrhs + r];
        xl[e] = v;
        O.xt[(size_t)cb * nrhs + e] = v;
        if (O.xtb) O.xtb[(size_t)cb * nrhs + e] = (__bf16)(float)v;
    }
    if (!do_far) return;  // uniform over the workgroup
    __syncthreads();
    const int nx = O.nx;
    for (int p = threadIdx.x; p < nx * nrhs; p += blockDim.x) {
        const int a = p / nrhs, r = p - a * nrhs;
        const double *lb = O.Lb + (size_t)a * T.n + cb;
        double s = 0.0;
        for (int i = 0; i < np; ++i) s = fma(lb[i], xl[i * nrhs + r], s);
        O.M[((size_t)c * nx + a) * nrhs + r] = s;
    }
}

// ---------------------------------------------------------------- M2M, one level
__device__ __forceinline__ void m2m_body(const DevTree &T, const DevOp &O, int c, int nrhs)
{
    const int nx = O.nx;
    for (int p = threadIdx.x; p < nx * nrhs; p += blockDim.x) {
        const int a = p / nrhs, r = p % nrhs;
        double s = 0.0;
        for (int ch = 2 * c + 1; ch <= 2 * c + 2; ++ch) {
            const double *E = O.E + (size_t)ch * nx * nx;
            const double *m = O.M + (size_t)ch * nx * nrhs;
            for (int b = 0; b < nx; ++b) s += E[b * nx + a] * m[b * nrhs + r];
        }
        O.M[((size_t)c * nx + a) * nrhs + r] = s;
    }
}

__global__ __launch_bounds__(64) void m2m_kernel(DevTree T, DevOp O, int first, int nrhs)
{
    m2m_body(T, O, first + blockIdx.x, nrhs);
}

// ---------------------------------------------------------------- M2L, all farfield levels at once
// General kernel (any kernel kind, n_x <= 128, up to 32 rhs): one workgroup per target
// cluster, node coordinates of the target and of each farfield source in LDS, the coupling
// matrix S formed kM2lRows rows at a time and applied to the source moments.
// Ot/Os: target and source side (the same operator for the matvec; for evaluation at new
// points the target side holds the target tree's nodes and locals).  T: the target tree,
// whose Fptr/Fsrc name source clusters.
template <int KIND>
__device__ __forceinline__ void m2l_general_body(const DevTree &T, const DevOp &O, const DevOp &Os, int c, int nrhs)
{
    __shared__ double tn[kMaxNodeWords];
    __shared__ double sn[kMaxNodeWords];
    __shared__ double S[kM2lRows * kMaxNx];
    const int nx = O.nx, dp = T.dpad;
    const int f0 = T.Fptr[c], f1 = T.Fptr[c + 1];
    const double inv_ell = 1.0 / O.ell;
    constexpr int kAcc = (kMaxNx * 32 + 255) / 256;
    double acc[kAcc];
#pragma unroll
    for (int k = 0; k < kAcc; ++k) acc[k] = 0.0;
    if (f0 < f1) {
        for (int q = threadIdx.x; q < nx * dp; q += blockDim.x) tn[q] = O.nodes[(size_t)c * nx * dp + q];
        for (int f = f0; f < f1; ++f) {
            const int s = T.Fsrc[f];
            const double *m = Os.M + (size_t)s * nx * nrhs;
            for (int q = threadIdx.x; q < nx * dp; q += blockDim.x) sn[q] = Os.nodes[(size_t)s * nx * dp + q];
            for (int a0 = 0; a0 < nx; a0 += kM2lRows) {
                const int rows = min(kM2lRows, nx - a0);
                __syncthreads();  // sn staged / the previous chunk consumed
                for (int q = threadIdx.x; q < rows * nx; q += blockDim.x) {
                    const int a = a0 + q / nx, b = q % nx;
                    double v;
                    if constexpr (KIND == 3) {
                        v = poly_kernel(&tn[a * dp], &sn[b * dp], (int)O.ell);
                    } else {
                        double r2 = 0.0;
                        for (int k = 0; k < dp; ++k) {
                            const double t = tn[a * dp + k] - sn[b * dp + k];
                            r2 += t * t;
                        }
                        v = kernel_val<KIND>(r2, inv_ell);
                    }
                    S[q] = v;
                }
                __syncthreads();
#pragma unroll
                for (int k = 0; k < kAcc; ++k) {
                    const int p = threadIdx.x + 256 * k;
                    const int a = p / nrhs, r = p % nrhs;
                    if (p < nx * nrhs && a >= a0 && a < a0 + rows) {
                        double v = 0.0;
                        for (int b = 0; b < nx; ++b) v += S[(a - a0) * nx + b] * m[b * nrhs + r];
                        acc[k] += v;
                    }
                }
            }
            __syncthreads();  // before the next source overwrites sn
        }
    }
#pragma unroll
    for (int k = 0; k < kAcc; ++k) {
        const int p = threadIdx.x + 256 * k;
        if (p < nx * nrhs) O.L[(size_t)c * nx * nrhs + p] = acc[k];
    }
}

template <int KIND>
__global__ __launch_bounds__(256) void m2l_kernel(DevTree T, DevOp O, int first, int nrhs)
{
    m2l_general_body<KIND>(T, O, O, first + blockIdx.x, nrhs);
}

template <int KIND>
__global__ __launch_bounds__(256) void m2l_cross_kernel(DevTree T, DevOp Ot, DevOp Os, int first, int nrhs)
{
    m2l_general_body<KIND>(T, Ot, Os, first + blockIdx.x, nrhs);
}

// ---------------------------------------------------------------- M2L on MFMA (one rhs)
// l_c[a] = sum over farfield sources s of sum_b K(t_a, s_b) m_s[b]: the node-pair
// distances take their cross term from FP64 MFMA 16x16x4 tiles (NXT x NXT tiles
// per block pair), the kernel values and the product with the moments run on the
// vector ALU.  The farfield list of a cluster is split into four classes
// f = Fptr[c] + k (mod 4); each class is summed in list order in its own
// accumulators and the four class sums are added in a fixed order.  WPC waves carry
// one cluster (4 / WPC classes each, 4 / WPC clusters per 256-thread workgroup); the
// result is bitwise the same for every WPC.  part: this cluster's [4][NXP] slice of LDS;
// every wave reaches the barrier (an idle slot passes valid = false).
template <int KIND, int DK, int NXT, int WPC>
__device__ __forceinline__ void m2l_mfma_body(const DevTree &T, const DevOp &O, const DevOp &Os, int c, bool valid,
                                              double *part)
{
    constexpr int NKC = DK / 4, NXP = 16 * NXT, RPW = 4 / WPC;
    const int nx = O.nx;
    const int tid = threadIdx.x, lane = tid & 63, wi = (tid >> 6) % WPC, lt = tid % (64 * WPC);
    const int li = lane & 15, lg = lane >> 4;
    const int f0 = valid ? T.Fptr[c] : 0, f1 = valid ? T.Fptr[c + 1] : 0;
    const double inv_ell = 1.0 / O.ell;
    const double *tnode = O.nodesT + (size_t)(valid ? c : 0) * DK * NXP;
    double A[NXT][NKC], tn[NXT][4], racc[RPW][NXT][4];
#pragma unroll
    for (int rt = 0; rt < NXT; ++rt) {
#pragma unroll
        for (int kc = 0; kc < NKC; ++kc) A[rt][kc] = tnode[(4 * kc + lg) * NXP + 16 * rt + li];
#pragma unroll
        for (int v = 0; v < 4; ++v) tn[rt][v] = O.nnorm[(size_t)(valid ? c : 0) * NXP + 16 * rt + 4 * v + lg];
    }
#pragma unroll
    for (int k = 0; k < RPW; ++k)
#pragma unroll
        for (int rt = 0; rt < NXT; ++rt)
#pragma unroll
            for (int v = 0; v < 4; ++v) racc[k][rt][v] = 0.0;
    for (int base = f0 + wi; base < f1; base += 4) {
#pragma unroll
        for (int k = 0; k < RPW; ++k) {
            const int f = base + k * WPC;  // class wi + k WPC
            if (f >= f1) break;            // uniform over the wave
            const int s = T.Fsrc[f];
            const double *snode = Os.nodesT + (size_t)s * DK * NXP;
#pragma unroll
            for (int ct = 0; ct < NXT; ++ct) {
                const int b = 16 * ct + li;
                double B[NKC];
#pragma unroll
                for (int kc = 0; kc < NKC; ++kc) B[kc] = snode[(4 * kc + lg) * NXP + b];
                const double nb = Os.nnorm[(size_t)s * NXP + b];
                const double mb = b < nx ? Os.M[(size_t)s * nx + b] : 0.0;
#pragma unroll
                for (int rt = 0; rt < NXT; ++rt) {
                    dbl4 G = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int kc = 0; kc < NKC; ++kc) G = __builtin_amdgcn_mfma_f64_16x16x4f64(A[rt][kc], B[kc], G, 0, 0, 0);
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const double r2 = fmax(fma(-2.0, G[v], tn[rt][v] + nb), 0.0);
                        racc[k][rt][v] = fma(kernel_fast<KIND>(r2, inv_ell), mb, racc[k][rt][v]);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < RPW; ++k)
#pragma unroll
        for (int rt = 0; rt < NXT; ++rt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double s = racc[k][rt][v];
                s += __shfl_xor(s, 1, 64);
                s += __shfl_xor(s, 2, 64);
                s += __shfl_xor(s, 4, 64);
                s += __shfl_xor(s, 8, 64);
                if (li == 0) part[(wi + k * WPC) * NXP + 16 * rt + 4 * v + lg] = s;
            }
    __syncthreads();
    if (valid && lt < nx)
        O.L[(size_t)c * nx + lt] = ((part[lt] + part[NXP + lt]) + part[2 * NXP + lt]) + part[3 * NXP + lt];
}

template <int KIND, int DK, int NXT>
__global__ __launch_bounds__(256) void m2l_mfma_kernel(DevTree T, DevOp O, int first)
{
    __shared__ double part[4 * 16 * NXT];
    m2l_mfma_body<KIND, DK, NXT, 4>(T, O, O, first + blockIdx.x, true, part);
}

// The coupling of an evaluation: target clusters of the target tree (its cross farfield lists
// name source clusters), source nodes and moments from the source operator.
template <int KIND, int DK, int NXT>
__global__ __launch_bounds__(256) void m2l_cross_mfma_kernel(DevTree Tt, DevOp Ot, DevOp Os, int first)
{
    __shared__ double part[4 * 16 * NXT];
    m2l_mfma_body<KIND, DK, NXT, 4>(Tt, Ot, Os, first + blockIdx.x, true, part);
}

template <int KIND, int DK>
void launch_m2l_cross_mfma_d(const DevTree &Tt, const DevOp &Ot, const DevOp &Os, int first, int cnt, hipStream_t st)
{
    switch (Os.nxp / 16) {
    case 1: hipLaunchKernelGGL((m2l_cross_mfma_kernel<KIND, DK, 1>), dim3(cnt), dim3(256), 0, st, Tt, Ot, Os, first); break;
    case 2: hipLaunchKernelGGL((m2l_cross_mfma_kernel<KIND, DK, 2>), dim3(cnt), dim3(256), 0, st, Tt, Ot, Os, first); break;
    case 3: hipLaunchKernelGGL((m2l_cross_mfma_kernel<KIND, DK, 3>), dim3(cnt), dim3(256), 0, st, Tt, Ot, Os, first); break;
    default: hipLaunchKernelGGL((m2l_cross_mfma_kernel<KIND, DK, 4>), dim3(cnt), dim3(256), 0, st, Tt, Ot, Os, first); break;
    }
}

template <int KIND>
void launch_m2l_cross_mfma_k(const DevTree &Tt, const DevOp &Ot, const DevOp &Os, int first, int cnt, hipStream_t st)
{
    switch ((Tt.d + 3) / 4 * 4) {
    case 4: launch_m2l_cross_mfma_d<KIND, 4>(Tt, Ot, Os, first, cnt, st); break;
    case 8: launch_m2l_cross_mfma_d<KIND, 8>(Tt, Ot, Os, first, cnt, st); break;
    case 12: launch_m2l_cross_mfma_d<KIND, 12>(Tt, Ot, Os, first, cnt, st); break;
    case 16: launch_m2l_cross_mfma_d<KIND, 16>(Tt, Ot, Os, first, cnt, st); break;
    case 20: launch_m2l_cross_mfma_d<KIND, 20>(Tt, Ot, Os, first, cnt, st); break;
    case 24: launch_m2l_cross_mfma_d<KIND, 24>(Tt, Ot, Os, first, cnt, st); break;
    case 28: launch_m2l_cross_mfma_d<KIND, 28>(Tt, Ot, Os, first, cnt, st); break;
    default: launch_m2l_cross_mfma_d<KIND, 32>(Tt, Ot, Os, first, cnt, st); break;
    }
}

template <int KIND, int DK>
void launch_m2l_mfma_d(const DevTree &T, const DevOp &O, int first, int cnt, hipStream_t st)
{
    switch (O.nxp / 16) {
    case 1: hipLaunchKernelGGL((m2l_mfma_kernel<KIND, DK, 1>), dim3(cnt), dim3(256), 0, st, T, O, first); break;
    case 2: hipLaunchKernelGGL((m2l_mfma_kernel<KIND, DK, 2>), dim3(cnt), dim3(256), 0, st, T, O, first); break;
    case 3: hipLaunchKernelGGL((m2l_mfma_kernel<KIND, DK, 3>), dim3(cnt), dim3(256), 0, st, T, O, first); break;
    default: hipLaunchKernelGGL((m2l_mfma_kernel<KIND, DK, 4>), dim3(cnt), dim3(256), 0, st, T, O, first); break;
    }
}

template <int KIND>
void launch_m2l_mfma_k(const DevTree &T, const DevOp &O, int first, int cnt, hipStream_t st)
{
    switch ((T.d + 3) / 4 * 4) {
    case 4: launch_m2l_mfma_d<KIND, 4>(T, O, first, cnt, st); break;
    case 8: launch_m2l_mfma_d<KIND, 8>(T, O, first, cnt, st); break;
    case 12: launch_m2l_mfma_d<KIND, 12>(T, O, first, cnt, st); break;
    case 16: launch_m2l_mfma_d<KIND, 16>(T, O, first, cnt, st); break;
    case 20: launch_m2l_mfma_d<KIND, 20>(T, O, first, cnt, st); break;
    case 24: launch_m2l_mfma_d<KIND, 24>(T, O, first, cnt, st); break;
    case 28: launch_m2l_mfma_d<KIND, 28>(T, O, first, cnt, st); break;
    default: launch_m2l_mfma_d<KIND, 32>(T, O, first, cnt, st); break;
    }
}

// ---------------------------------------------------------------- L2L, one level
__device__ __forceinline__ void l2l_body(const DevTree &T, const DevOp &O, int c, int nrhs)
{
    const int par = (c - 1) / 2;
    const int nx = O.nx;
    const double *E = O.E + (size_t)c * nx * nx;
    const double *lp = O.L + (size_t)par * nx * nrhs;
    for (int p = threadIdx.x; p < nx * nrhs; p += blockDim.x) {
        const int a = p / nrhs, r = p % nrhs;
        double s = 0.0;
        for (int b = 0; b < nx; ++b) s += E[a * nx + b] * lp[b * nrhs + r];
        O.L[((size_t)c * nx + a) * nrhs + r] += s;
    }
}

__global__ __launch_bounds__(64) void l2l_kernel(DevTree T, DevOp O, int first, int nrhs)
{
    l2l_body(T, O, first + blockIdx.x, nrhs);
}

// ---------------------------------------------------------------- P2P + L2P + scatter to original order
constexpr int kP2PThreads = 128;

// T/O: target tree and target side; Ts/xs: source tree and the charges in source tree order
// (the same tree and O.xt for the matvec).  T's nearfield lists name source leaves.
template <int KIND, int DP>
__device__ __forceinline__ void p2p_general_body(const DevTree &T, const DevOp &O, const DevTree &Ts,
                                                 const double *__restrict__ xs, double *__restrict__ y, int nrhs,
                                                 int do_near, int do_far)
{
    // source points staged per pass; fewer for wide points so that LDS stays below 32 KB
    constexpr int SCH = DP <= 32 ? kP2PThreads : kP2PThreads / 2;
    __shared__ double sx[SCH * DP];
    __shared__ double sq[SCH];
    const int l = blockIdx.x, c = T.leaf_first + l;
    const int cb = T.cbeg[c], ce = T.cend[c];
    const double inv_ell = 1.0 / O.ell;
    const int n = T.n, ns_all = Ts.n;
    for (int t0 = cb; t0 < ce; t0 += kP2PThreads) {
        const int i = t0 + (int)threadIdx.x;
        const bool active = i < ce;
        double xt[DP];
#pragma unroll
        for (int k = 0; k < DP; ++k) xt[k] = active ? T.Xs[(size_t)k * n + i] : 0.0;
        for (int r = 0; r < nrhs; ++r) {
            double acc = 0.0;
            if (do_near) {
                for (int f = T.Nptr[l]; f < T.Nptr[l + 1]; ++f) {
                    const int s = Ts.leaf_first + T.Nsrc[f];
                    const int sb = Ts.cbeg[s], se = Ts.cend[s];
                    for (int s0 = sb; s0 < se; s0 += SCH) {
                        __syncthreads();
                        const int j = s0 + (int)threadIdx.x;
                        if ((int)threadIdx.x < SCH && j < se) {
#pragma unroll
                            for (int k = 0; k < DP; ++k) sx[threadIdx.x * DP + k] = Ts.Xs[(size_t)k * ns_all + j];
                            sq[threadIdx.x] = xs[(size_t)j * nrhs + r];
                        }
                        __syncthreads();
                        const int m = min(SCH, se - s0);
                        for (int jj = 0; jj < m; ++jj) {
                            double kv;
                            if constexpr (KIND == 3) {
                                kv = poly_kernel(xt, &sx[jj * DP], (int)O.ell);
                            } else {
                                double r2 = 0.0;
#pragma unroll
                                for (int k = 0; k < DP; ++k) {
                                    const double t = xt[k] - sx[jj * DP + k];
                                    r2 = fma(t, t, r2);
                                }
                                kv = kernel_val<KIND>(r2, inv_ell);
                            }
                            acc = fma(kv, sq[jj], acc);
                        }
                    }
                }
            }
            if (do_far && active) {
                const double *lc = O.L + (size_t)c * O.nx * nrhs;
                for (int a = 0; a < O.nx; ++a) acc = fma(O.Lb[(size_t)a * n + i], lc[a * nrhs + r], acc);
            }
            if (active) y[(size_t)T.perm[i] * nrhs + r] = acc;
        }
    }
}

template <int KIND, int DP>
__global__ __launch_bounds__(kP2PThreads) void p2p_kernel(DevTree T, DevOp O, double *__restrict__ y, int nrhs,
                                                          int do_near, int do_far)
{
    p2p_general_body<KIND, DP>(T, O, T, O.xt, y, nrhs, do_near, do_far);
}

template <int KIND, int DP>
__global__ __launch_bounds__(kP2PThreads) void p2p_cross_kernel(DevTree T, DevOp Ot, DevTree Ts,
                                                                const double *__restrict__ xs, double *__restrict__ y,
                                                                int nrhs, int do_far)
{
    p2p_general_body<KIND, DP>(T, Ot, Ts, xs, y, nrhs, 1, do_far);
}

template <int KIND, int DP>
void launch_p2p_t(const DevTree &T, const DevOp &O, double *y, int nrhs, int near, int far, hipStream_t st)
{
    hipLaunchKernelGGL((p2p_kernel<KIND, DP>), dim3(T.nleaf), dim3(kP2PThreads), 0, st, T, O, y, nrhs, near, far);
}

template <int KIND, int DP>
void launch_p2p_cross_t(const DevTree &Tt, const DevOp &Ot, const DevTree &Ts, const double *xs, double *y, int nrhs,
                        int far, hipStream_t st)
{
    hipLaunchKernelGGL((p2p_cross_kernel<KIND, DP>), dim3(Tt.nleaf), dim3(kP2PThreads), 0, st, Tt, Ot, Ts, xs, y,
                       nrhs, far);
}

template <int KIND>
hipError_t launch_p2p_k(const DevTree &T, const DevOp &O, double *y, int nrhs, int near, int far, hipStream_t st)
{
    switch (T.dpad) {
#define DWFMM_CASE(D) \
    case D: launch_p2p_t<KIND, D>(T, O, y, nrhs, near, far, st); break;
        DWFMM_CASE(4) DWFMM_CASE(8) DWFMM_CASE(12) DWFMM_CASE(16) DWFMM_CASE(20) DWFMM_CASE(24)
        DWFMM_CASE(28) DWFMM_CASE(32) DWFMM_CASE(40) DWFMM_CASE(48) DWFMM_CASE(56) DWFMM_CASE(64)
#undef DWFMM_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int KIND>
hipError_t launch_p2p_cross_k(const DevTree &Tt, const DevOp &Ot, const DevTree &Ts, const double *xs, double *y,
                              int nrhs, int far, hipStream_t st)
{
    switch (Tt.dpad) {
#define DWFMM_CASE(D) \
    case D: launch_p2p_cross_t<KIND, D>(Tt, Ot, Ts, xs, y, nrhs, far, st); break;
        DWFMM_CASE(4) DWFMM_CASE(8) DWFMM_CASE(12) DWFMM_CASE(16) DWFMM_CASE(20) DWFMM_CASE(24)
        DWFMM_CASE(28) DWFMM_CASE(32) DWFMM_CASE(40) DWFMM_CASE(48) DWFMM_CASE(56) DWFMM_CASE(64)
#undef DWFMM_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- symmetric MFMA nearfield (one rhs)
// Owner leaf t evaluates each block K_{t,s} it owns once: the squared distance
// |x_i - y_j|^2 = |x_i|^2 + |y_j|^2 - 2 x_i.y_j takes the cross term from FP64
// MFMA 16x16x4 tiles (coordinates shifted to the owner leaf's box midpoint), the
// kernel value on the vector ALU.  Row sums K q_s stay in registers; column sums
// K^T q_t go to colbuf[block] and are added by the partner leaf in the combine
// pass, in a fixed order (no atomics, bitwise reproducible).  After the diagonal block
// the owner's other blocks are swept as one concatenated stream of source points, so a
// 16-wide column tile may hold the end of one block and the start of the next and only
// the stream's last tile carries padding.
// Lane layout of v_mfma_f64_16x16x4f64: A[i][k] in lane i + 16k, B[k][j] in lane
// j + 16k, D[i][j] in lane j + 16(i%4), element i/4 (checked with a probe).
constexpr int kSymLeaf = 128;
// Internal kernel variant of the symmetric FP64 nearfield: the Gaussian evaluated as
// exp(-|x-c|^2/ell) exp(-|y-c|^2/ell) exp(2 (x-c).(y-c)/ell) (operators with gauss_split set).
constexpr int kGaussSplit = 4;
// Internal kernel variant of the symmetric FP64 nearfield: the Matern kernel of an operator whose
// nearfield distances keep every exponent s log2(e) within 1000 (matern_in_range), evaluated
// without the underflow clamp.
constexpr int kMaternInRange = 5;
template <int KIND>
constexpr bool is_matern() { return KIND == 0 || KIND == kMaternInRange; }
constexpr int kSymSeg = 256;  // owned blocks per column-stream segment (= threads per workgroup)
// Row stride of the FP32 tile coordinates in LDS: a wave reads rows 4kc + g (g = 0..3) at 16
// consecutive columns; with 16 floats of padding the rows g and g + 1 fall on the two halves
// of the 32 banks instead of the same 16.
constexpr int kSX32 = 128 + 16;

// One leaf block, all 16x16 tiles of this wave's two row tiles.  DIAG: the block of a
// leaf with itself (i == j forced to distance 0, no column sums).  NK: the squared norms ride in
// two padding rows of the Gram operands (row operand |x|^2 and 1, column operand 1 and |y|^2), so
// the MFMA chain delivers the whole squared distance.
template <int KIND, int NKC, bool DIAG, bool NK>
__device__ __forceinline__ void sym_block(const double (&A)[2][NKC], const double (&rN)[2][4],
                                          const double (&rQ)[2][4], double (&racc)[2][4], const double *sX,
                                          const double *sN, const double *sQ, double *colpart, int ns, int ntiles,
                                          int w, int li, int lg, double inv_ell)
{
    const int rt[2] = {w, w + 4};
    const int nct = (ns + 15) / 16;
    for (int ct = 0; ct < nct; ++ct) {
        const int j = 16 * ct + li;
        const double nb = KIND == kGaussSplit || NK ? 0.0 : sN[j], qb = sQ[j];
        double Bf[NKC];
#pragma unroll
        for (int kc = 0; kc < NKC; ++kc) Bf[kc] = sX[(4 * kc + lg) * kSymLeaf + j];
        double cacc = 0.0;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (rt[u] >= ntiles) continue;  // uniform over the wave
            // A holds -2 (x - c): the MFMA chain starts from |x|^2 and adds -2 x.y, then |y|^2 is
            // added on the vector ALU (an ordinary add, so the clamp in kernel_fast needs no
            // canonicalisation of the MFMA result).
            // Split Gaussian: A holds (2 log2(e) / ell)(x - c) and the chain gives the base-2
            // exponent of the cross factor; the row and column factors sit in the charges.
            dbl4 G;
            if constexpr (KIND == kGaussSplit || NK)
                G = dbl4{0.0, 0.0, 0.0, 0.0};
            else
                G = dbl4{rN[u][0], rN[u][1], rN[u][2], rN[u][3]};
#pragma unroll
            for (int kc = 0; kc < NKC; ++kc) G = __builtin_amdgcn_mfma_f64_16x16x4f64(A[u][kc], Bf[kc], G, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double kv;
                if constexpr (KIND == kGaussSplit) {
                    kv = exp2_bounded(G[v]);  // the row operand carries log2(e)
                } else {
                    double r2 = NK ? G[v] : G[v] + nb;
                    if constexpr (DIAG) {
                        if (16 * rt[u] + 4 * v + lg == j) r2 = 0.0;
                    }
                    // Matern: the coordinates carry sqrt(3) / ell, so r2 is s^2
                    if constexpr (is_matern<KIND>())
                        kv = matern_s2<KIND == 0>(r2);
                    else
                        kv = kernel_fast<KIND>(r2, inv_ell);
                }
                racc[u][v] = fma(kv, qb, racc[u][v]);
                if constexpr (!DIAG) cacc = fma(kv, rQ[u][v], cacc);
            }
        }
        if constexpr (!DIAG) {
            cacc += __shfl_xor(cacc, 16, 64);
            cacc += __shfl_xor(cacc, 32, 64);
            if (lg == 0) colpart[w * kSymLeaf + j] = cacc;
        }
    }
}

template <int KIND, int DK>
__device__ __forceinline__ void p2p_sym_body(const DevTree &T, const DevOp &O, int l)
{
    constexpr int NKC = DK / 4;
    __shared__ double sX[DK * kSymLeaf];  // [k][j] shifted source coordinates
    // sN, colF and colJ alternate between two halves from chunk to chunk (nb): the column sums of one
    // chunk read them while the next chunk's staging writes the other half
    __shared__ double sN[2 * kSymLeaf], sQ[kSymLeaf], tN[kSymLeaf], tQ[kSymLeaf];
    __shared__ double colpart[4 * kSymLeaf];
    __shared__ double cen[DK];
    __shared__ int32_t sPre[kSymSeg + 1], sBlk[kSymSeg];  // owned-block segment: size prefix, block ids
    __shared__ int32_t sBeg[kSymSeg];                     // first source point of each block
    __shared__ int32_t colF[2 * kSymLeaf], colJ[2 * kSymLeaf];  // block and point of each stream column
    __shared__ int32_t sDiag;                             // the leaf owns its self block

    const int c = T.leaf_first + l;
    const int cb = T.cbeg[c], nt = T.cend[c] - cb;
    // the wave index is uniform: its row-tile tests below branch on scalars
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, lg = lane >> 4;
    const int n = T.n;
    const double inv_ell = 1.0 / O.ell;
    const int ntiles = (nt + 15) / 16;
    // Matern: shifted coordinates are scaled by sqrt(3) / ell, so the Gram tile gives s^2 = 3 r^2 / ell^2
    constexpr bool kMat = is_matern<KIND>();
    const double csc = kMat ? 1.7320508075688772 * inv_ell : 1.0;

    if (nt == 0) return;  // an empty leaf owns no block (uniform over the workgroup)
    // Coordinate rows k in [d, DK) are stored as zeros and cen[k] = 0 there, so every load
    // below is unconditional; point indices past the end of a leaf are clamped and masked.
    if (tid < DK) cen[tid] = T.center[(size_t)l * DK + tid];
    if (tid == 0) sDiag = 0;
    __syncthreads();
    // The self block is listed only when the leaf is not admissible with itself (a leaf whose
    // points all coincide has a zero-size box and takes its self block in the farfield).
    const int o0 = T.own_ptr[l], o1 = T.own_ptr[l + 1];
    for (int f = o0 + tid; f < o1; f += blockDim.x)
        if (T.own_src[f] == l) sDiag = 1;
    if (tid < kSymLeaf) {
        const bool ok = tid < nt;
        const int ii = cb + (ok ? tid : nt - 1);
        double xv[DK];
#pragma unroll
        for (int k = 0; k < DK; ++k) xv[k] = T.Xs[(size_t)k * n + ii];
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < DK; ++k) {
            const double v = kMat ? csc * (xv[k] - cen[k]) : xv[k] - cen[k];
            s = fma(v, v, s);
        }
        const double q = O.xt[ii];
        if constexpr (KIND == kGaussSplit) {
            const double a = exp_bounded(-s * inv_ell);  // row factor
            tN[tid] = ok ? a : 0.0;
            tQ[tid] = ok ? q * a : 0.0;
        } else {
            tN[tid] = ok ? s : 0.0;
            tQ[tid] = ok ? q : 0.0;
        }
    }
    const int rt[2] = {w, w + 4};
    double A[2][NKC];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int i = 16 * rt[u] + li;
        const bool ok = i < nt;
        const int ii = cb + (ok ? i : nt - 1);
        const double scale = KIND == kGaussSplit ? 2.0 * 1.4426950408889634 * inv_ell : (kMat ? -2.0 * csc : -2.0);
#pragma unroll
        for (int kc = 0; kc < NKC; ++kc) {
            const int k = 4 * kc + lg;
            const double v = T.Xs[(size_t)k * n + ii] - cen[k];
            A[u][kc] = ok ? scale * v : 0.0;
        }
    }
    __syncthreads();
    // Two padding rows free (d <= DK - 2): the squared norms go into the Gram operands
    const bool nk = KIND != kGaussSplit && T.d <= DK - 2;
    if (nk) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int i = 16 * rt[u] + li;
            const bool ok = i < nt;
#pragma unroll
            for (int kc = 0; kc < NKC; ++kc) {
                const int k = 4 * kc + lg;
                if (k == T.d) A[u][kc] = ok ? tN[i] : 0.0;
                else if (k == T.d + 1) A[u][kc] = ok ? 1.0 : 0.0;
            }
        }
    }
    double rN[2][4], rQ[2][4], racc[2][4];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = 16 * rt[u] + 4 * v + lg;
            rN[u][v] = KIND == kGaussSplit ? 0.0 : tN[i];  // split: the row factor is applied at the end
            rQ[u][v] = tQ[i];
            racc[u][v] = 0.0;
        }

    int nb = 0;  // the half of sN, colF and colJ this chunk uses
    // Column j of the tile arrays: point pidx shifted to the owner's midpoint, its squared norm
    // (split Gaussian: its column factor) and its charge; columns past the data are zero.
    auto stage = [&](int j, int pidx, bool ok) {
        double xv[DK];
#pragma unroll
        for (int k = 0; k < DK; ++k) xv[k] = T.Xs[(size_t)k * n + pidx];
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < DK; ++k) {
            const double v = ok ? (kMat ? csc * (xv[k] - cen[k]) : xv[k] - cen[k]) : 0.0;
            sX[k * kSymLeaf + j] = v;
            s = fma(v, v, s);
        }
        const double q = O.xt[pidx];
        if constexpr (KIND == kGaussSplit) {
            const double bfac = exp_bounded(-s * inv_ell);  // column factor
            sN[nb + j] = bfac;
            sQ[j] = ok ? q * bfac : 0.0;
        } else {
            sN[nb + j] = s;
            sQ[j] = ok ? q : 0.0;
            if (nk) {
                sX[T.d * kSymLeaf + j] = 1.0;
                sX[(T.d + 1) * kSymLeaf + j] = s;
            }
        }
    };
    // the tile loop with or without the norms in the Gram operands (uniform over the workgroup)
    auto block = [&](auto diag, int ns) {
        constexpr bool D = decltype(diag)::value;
        if constexpr (KIND != kGaussSplit) {
            if (nk) {
                sym_block<KIND, NKC, D, true>(A, rN, rQ, racc, sX, sN + nb, sQ, colpart, ns, ntiles, w, li, lg, inv_ell);
                return;
            }
        }
        sym_block<KIND, NKC, D, false>(A, rN, rQ, racc, sX, sN + nb, sQ, colpart, ns, ntiles, w, li, lg, inv_ell);
    };
    // 1) the leaf with itself (sDiag was set before the barrier that precedes rN)
    if (sDiag) {
        __syncthreads();
        if (tid < kSymLeaf) stage(tid, cb + (tid < nt ? tid : nt - 1), tid < nt);
        __syncthreads();
        block(std::true_type{}, nt);
    }
    // 2) the other owned blocks as one stream of source points, kSymLeaf columns at a time: a
    //    16-wide column tile may span two source leaves, so only the stream's last tile is padded.
    //    Owned blocks are taken kSymSeg at a time; sPre holds the prefix sums of their sizes.
    // The staging and column-sum threads alternate between waves 0-1 and 2-3 from chunk to chunk
    // (sid), so that the four SIMDs, which hold one wave of the workgroup each, share that work.
    int chunk = 0;
    for (int fb = o0; fb < o1; fb += kSymSeg) {
        const int fe = min(fb + kSymSeg, o1);
        __syncthreads();  // the previous segment's table is no longer read
        {
            int sz = 0, beg = 0;
            const int f = fb + tid;
            if (f < fe) {
                const int sl = T.own_src[f];
                beg = T.cbeg[T.leaf_first + sl];
                if (sl != l) sz = T.cend[T.leaf_first + sl] - beg;
            }
            sPre[tid + 1] = sz;
            sBlk[tid] = f;
            sBeg[tid] = beg;
            if (tid == 0) sPre[0] = 0;
        }
        __syncthreads();
        for (int off = 1; off < kSymSeg; off <<= 1) {  // inclusive scan of sPre[1..kSymSeg]
            const int add = tid >= off ? sPre[tid + 1 - off] : 0;
            __syncthreads();
            sPre[tid + 1] += add;
            __syncthreads();
        }
        const int total = sPre[kSymSeg];
        for (int c0 = 0; c0 < total; c0 += kSymLeaf, ++chunk) {
            const int ns = min(kSymLeaf, total - c0);
            const int sid = tid ^ ((chunk & 1) << 7);
            // no barrier here: the previous chunk's tiles ended at the barrier before its column sums,
            // which read only colpart and the other half of sN, colF and colJ; the barrier after this
            // staging keeps the next tiles (and colpart) behind every wave's column sums
            nb = (chunk & 1) * kSymLeaf;
            if (sid < kSymLeaf) {
                const int j = sid;
                const bool ok = j < ns;
                int pidx = cb, fblk = 0, jl = 0;
                if (ok) {
                    // the block holding stream column c0 + j: the largest k with sPre[k] <= c0 + j
                    // (it has a positive size, since sPre[k + 1] > c0 + j)
                    const int col = c0 + j;
                    int lo = 0, hi = kSymSeg;
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (sPre[mid] <= col) lo = mid;
                        else hi = mid - 1;
                    }
                    fblk = sBlk[lo];
                    jl = col - sPre[lo];
                    pidx = sBeg[lo] + jl;  // from LDS: only the coordinates are loaded from memory
                }
                stage(j, pidx, ok);
                colF[nb + j] = fblk;
                colJ[nb + j] = jl;
            }
            __syncthreads();
            block(std::false_type{}, ns);
            __syncthreads();
            if (sid < ns) {
                double cs = ((colpart[sid] + colpart[kSymLeaf + sid]) + colpart[2 * kSymLeaf + sid]) +
                            colpart[3 * kSymLeaf + sid];
                if constexpr (KIND == kGaussSplit) cs *= sN[nb + sid];
                O.colbuf[(size_t)colF[nb + sid] * kSymLeaf + colJ[nb + sid]] = cs;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            double s = racc[u][v];
            s += __shfl_xor(s, 1, 64);
            s += __shfl_xor(s, 2, 64);
            s += __shfl_xor(s, 4, 64);
            s += __shfl_xor(s, 8, 64);
            const int i = 16 * rt[u] + 4 * v + lg;
            if constexpr (KIND == kGaussSplit) s *= tN[i];  // row factor, from LDS
            if (li == 0 && i < nt) O.rowbuf[(size_t)l * kSymLeaf + i] = s;
        }
}

// Waves per SIMD (also for the batched variant): four for the split Gaussian and the Matern kernel
// up to d = 20 (128 registers; the few spills sit outside the tile loop; the extra wave beats the
// third by ~2% for both), three for the exponential kernel up to d = 20 (four were slower there),
// else what the registers allow.
template <int KIND, int DK>
constexpr int sym_waves() { return (KIND == kGaussSplit || is_matern<KIND>()) && DK <= 20 ? 4 : (DK <= 20 || (KIND != kGaussSplit && DK <= 24) ? 3 : 1); }

template <int KIND, int DK>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(sym_waves<KIND, DK>(), 8)))
void p2p_sym_kernel(DevTree T, DevOp O)
{
    const int l = T.leaf_order[blockIdx.x];
    if (l < 0) return;  // padding of a shorter XCD segment
    p2p_sym_body<KIND, DK>(T, O, l);
}

// ---------------------------------------------------------------- MFMA cross nearfield (new points, one rhs)
// Evaluation at new points: every (target leaf, source leaf) pair of the cross nearfield is its
// own block (no symmetry to use).  One workgroup per target leaf (at most kSymLeaf points): its
// rows, shifted to the leaf's first point, stay in registers as in the symmetric kernel; the
// source leaves of its nearfield list are swept as one stream of points, kSymLeaf columns at a
// time (sizes prefix-summed in LDS, a binary search per column); the Gram tile r^2 comes from
// FP64 MFMA, the kernel from kernel_fast.  The row sums get the farfield (L2P) added and are
// scattered to the caller's order.
template <int KIND, int NKC>
__device__ __forceinline__ void cross_block(const double (&A)[2][NKC], const double (&rN)[2][4], double (&racc)[2][4],
                                            const double *sX, const double *sN, const double *sQ, int ns, int ntiles,
                                            int w, int li, int lg, double inv_ell)
{
    const int rt[2] = {w, w + 4};
    const int nct = (ns + 15) / 16;
    for (int ct = 0; ct < nct; ++ct) {
        const int j = 16 * ct + li;
        const double nb = KIND == kGaussSplit ? 0.0 : sN[j], qb = sQ[j];
        double Bf[NKC];
#pragma unroll
        for (int kc = 0; kc < NKC; ++kc) Bf[kc] = sX[(4 * kc + lg) * kSymLeaf + j];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (rt[u] >= ntiles) continue;  // uniform over the wave
            // split Gaussian: A carries (2 log2(e) / ell)(x - c), the chain gives the base-2 exponent
            // of the cross factor, the column factor sits in the charge and the row factor (rN)
            // is applied to the row sums at the end
            dbl4 G;
            if constexpr (KIND == kGaussSplit)
                G = dbl4{0.0, 0.0, 0.0, 0.0};
            else
                G = dbl4{rN[u][0], rN[u][1], rN[u][2], rN[u][3]};
#pragma unroll
            for (int kc = 0; kc < NKC; ++kc) G = __builtin_amdgcn_mfma_f64_16x16x4f64(A[u][kc], Bf[kc], G, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double kv = KIND == kGaussSplit ? exp2_bounded(G[v]) : kernel_fast<KIND>(G[v] + nb, inv_ell);
                racc[u][v] = fma(kv, qb, racc[u][v]);
            }
        }
    }
}

template <int KIND, int DK>
__device__ __forceinline__ void p2p_cross_mfma_body(const DevTree &T, const DevOp &O, const DevTree &Ts,
                                                    const double *__restrict__ xs, double *__restrict__ y, int do_far,
                                                    int l)
{
    constexpr int NKC = DK / 4;
    __shared__ double sX[DK * kSymLeaf];
    __shared__ double sN[kSymLeaf], sQ[kSymLeaf], tN[kSymLeaf];
    __shared__ double cen[DK];
    __shared__ int32_t sPre[kSymSeg + 1], sBeg[kSymSeg];

    const int c = T.leaf_first + l;
    const int cb = T.cbeg[c], nt = T.cend[c] - cb;
    if (nt == 0) return;  // uniform over the workgroup
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int n = T.n, ns_all = Ts.n;
    const double inv_ell = 1.0 / O.ell;
    const int ntiles = (nt + 15) / 16;
    // rows k in [d, DK) of both trees' coordinates are zeros, so the shift is zero there
    if (tid < DK) cen[tid] = T.Xs[(size_t)tid * n + cb];
    __syncthreads();
    if (tid < kSymLeaf) {
        const bool ok = tid < nt;
        const int ii = cb + (ok ? tid : nt - 1);
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < DK; ++k) {
            const double v = T.Xs[(size_t)k * n + ii] - cen[k];
            s = fma(v, v, s);
        }
        if constexpr (KIND == kGaussSplit)
            tN[tid] = ok ? exp_bounded(-s * inv_ell) : 0.0;  // row factor
        else
            tN[tid] = ok ? s : 0.0;
    }
    const int rt[2] = {w, w + 4};
    double A[2][NKC];
    const double scale = KIND == kGaussSplit ? 2.0 * 1.4426950408889634 * inv_ell : -2.0;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int i = 16 * rt[u] + li;
        const bool ok = i < nt;
        const int ii = cb + (ok ? i : nt - 1);
#pragma unroll
        for (int kc = 0; kc < NKC; ++kc) {
            const int k = 4 * kc + lg;
            A[u][kc] = ok ? scale * (T.Xs[(size_t)k * n + ii] - cen[k]) : 0.0;
        }
    }
    __syncthreads();
    double rN[2][4], racc[2][4];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            rN[u][v] = tN[16 * rt[u] + 4 * v + lg];
            racc[u][v] = 0.0;
        }
    const int f0 = T.Nptr[l], f1 = T.Nptr[l + 1];
    int chunk = 0;  // the staging threads alternate between waves 0-1 and 2-3 (as in the symmetric kernel)
    for (int fb = f0; fb < f1; fb += kSymSeg) {
        const int fe = min(fb + kSymSeg, f1);
        __syncthreads();  // the previous segment's table is no longer read
        {
            int sz = 0, beg = 0;
            const int f = fb + tid;
            if (f < fe) {
                const int sc = Ts.leaf_first + T.Nsrc[f];
                beg = Ts.cbeg[sc];
                sz = Ts.cend[sc] - beg;
            }
            sPre[tid + 1] = sz;
            sBeg[tid] = beg;
            if (tid == 0) sPre[0] = 0;
        }
        __syncthreads();
        for (int off = 1; off < kSymSeg; off <<= 1) {  // inclusive scan of sPre[1..kSymSeg]
            const int add = tid >= off ? sPre[tid + 1 - off] : 0;
            __syncthreads();
            sPre[tid + 1] += add;
            __syncthreads();
        }
        const int total = sPre[kSymSeg];
        for (int c0 = 0; c0 < total; c0 += kSymLeaf, ++chunk) {
            const int ns = min(kSymLeaf, total - c0);
            const int sid = tid ^ ((chunk & 1) << 7);
            __syncthreads();  // the previous chunk's tiles are consumed
            if (sid < kSymLeaf) {
                const int j = sid;
                const bool ok = j < ns;
                int pidx = 0;  // any valid source point for the padding columns
                if (ok) {
                    // the list entry holding stream column c0 + j: the largest k with sPre[k] <= c0 + j
                    const int col = c0 + j;
                    int lo = 0, hi = kSymSeg;
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (sPre[mid] <= col) lo = mid;
                        else hi = mid - 1;
                    }
                    pidx = sBeg[lo] + (col - sPre[lo]);
                }
                double xv[DK];
#pragma unroll
                for (int k = 0; k < DK; ++k) xv[k] = Ts.Xs[(size_t)k * ns_all + pidx];
                double s = 0.0;
#pragma unroll
                for (int k = 0; k < DK; ++k) {
                    const double v = ok ? xv[k] - cen[k] : 0.0;
                    sX[k * kSymLeaf + j] = v;
                    s = fma(v, v, s);
                }
                sN[j] = s;
                if constexpr (KIND == kGaussSplit)
                    sQ[j] = ok ? xs[pidx] * exp_bounded(-s * inv_ell) : 0.0;  // charge times column factor
                else
                    sQ[j] = ok ? xs[pidx] : 0.0;
            }
            __syncthreads();
            cross_block<KIND, NKC>(A, rN, racc, sX, sN, sQ, ns, ntiles, w, li, lg, inv_ell);
        }
    }
    // row sums: reduce over the 16 column lanes, then farfield (L2P) and the scatter
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            double s = racc[u][v];
            s += __shfl_xor(s, 1, 64);
            s += __shfl_xor(s, 2, 64);
            s += __shfl_xor(s, 4, 64);
            s += __shfl_xor(s, 8, 64);
            if constexpr (KIND == kGaussSplit) s *= rN[u][v];  // row factor
            const int i = 16 * rt[u] + 4 * v + lg;
            if (li == 0) tN[i] = s;
        }
    __syncthreads();
    if (tid < nt) {
        double acc = tN[tid];
        if (do_far) {
            const double *lc = O.L + (size_t)c * O.nx;
            for (int a = 0; a < O.nx; ++a) acc = fma(O.Lb[(size_t)a * n + cb + tid], lc[a], acc);
        }
        y[T.perm[cb + tid]] = acc;
    }
}

template <int KIND, int DK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KIND == kGaussSplit && DK <= 20 ? 4 : (DK <= 24 ? 3 : 1), 8)))
void p2p_cross_mfma_kernel(DevTree T, DevOp O, DevTree Ts, const double *__restrict__ xs, double *__restrict__ y,
                           int do_far)
{
    const int l = T.near_order[blockIdx.x];
    if (l < 0) return;  // padding of a shorter XCD segment
    p2p_cross_mfma_body<KIND, DK>(T, O, Ts, xs, y, do_far, l);
}

template <int KIND>
hipError_t launch_cross_mfma_k(const DevTree &Tt, const DevOp &Ot, const DevTree &Ts, const double *xs, double *y,
                               int do_far, hipStream_t st)
{
    switch (Tt.dpad) {
#define DWFMM_XM(D)                                                                                        \
    case D:                                                                                                \
        hipLaunchKernelGGL((p2p_cross_mfma_kernel<KIND, D>), dim3(Tt.n_near_order), dim3(256), 0, st, Tt, Ot, Ts, xs, y, \
                           do_far);                                                                        \
        break;
        DWFMM_XM(4) DWFMM_XM(8) DWFMM_XM(12) DWFMM_XM(16) DWFMM_XM(20) DWFMM_XM(24) DWFMM_XM(28) DWFMM_XM(32)
#undef DWFMM_XM
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- MFMA nearfield, several rhs
// One workgroup per target leaf over all its nearfield source leaves.  The Gram tile is
// formed with the sources as the A operand: element v of lane (i + 16 g) then holds
// K[target i][source 4v + g], which is exactly the A operand of chunk v of
//   Y(16 targets x 16 rhs) += K(16 x 16) Q(16 sources x 16 rhs),
// so the kernel values feed the apply MFMAs without any lane exchange.  RB = number of
// 16-wide rhs tiles.  L2P and the scatter to caller order are fused at the end.  The split
// Gaussian variant (KIND kGaussSplit) starts each Gram chain from the sources' base-2 column
// factors and scales the finished sums by the targets' row factors.
// Staged charges [j][r] in rows of 16 RB doubles; with two rhs tiles the odd rows swap their
// halves (r ^ 16), so that the two lane groups of a half-wave (rows j and j + 1 of a tile
// column) read opposite halves of the 64 banks.  Coordinates [k][j] in rows of kSX64 doubles,
// 16 past the leaf size for the same reason.
template <int RB>
constexpr int q_stride() { return 16 * RB; }
template <int RB>
__device__ __forceinline__ int q_col(int j, int r) { return RB == 2 ? r ^ ((j & 1) << 4) : r; }
constexpr int kSX64 = kSymLeaf + 16;

template <int KIND, int DK, int RB, bool DIAG>
__device__ __forceinline__ void mrhs_block(const double (&Bt)[2][DK / 4], const double (&tn)[2], dbl4 (&Y)[2][RB],
                                           const double *sX, const double *sN, const double *sQ, int ns, int ntiles,
                                           int w, int li, int lg, double inv_ell)
{
    constexpr int NKC = DK / 4;
    const int rt[2] = {w, w + 4};
    const int nct = (ns + 15) / 16;
    for (int ct = 0; ct < nct; ++ct) {
        double Af[NKC];
#pragma unroll
        for (int kc = 0; kc < NKC; ++kc) Af[kc] = sX[(4 * kc + lg) * kSX64 + 16 * ct + li];
        double snv[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) snv[v] = sN[16 * ct + 4 * v + lg];
        double Qf[RB][4];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                Qf[rb][v] = sQ[(16 * ct + 4 * v + lg) * q_stride<RB>() + q_col<RB>(lg, 16 * rb + li)];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (rt[u] >= ntiles) continue;  // uniform over the wave
            // Split Gaussian: the target operand carries (2 log2(e) / ell)(x - c) and the chain
            // starts from the base-2 logarithm of each source's column factor (snv), so it delivers
            // the whole base-2 exponent of the entry but for the row factor, applied to the sums
            dbl4 G;
            if constexpr (KIND == kGaussSplit)
                G = dbl4{snv[0], snv[1], snv[2], snv[3]};
            else
                G = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kc = 0; kc < NKC; ++kc) G = __builtin_amdgcn_mfma_f64_16x16x4f64(Af[kc], Bt[u][kc], G, 0, 0, 0);
            double Kv[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                if constexpr (KIND == kGaussSplit) {
                    Kv[v] = exp2_bounded(G[v]);
                } else {
                    double r2 = fmax(fma(-2.0, G[v], tn[u] + snv[v]), 0.0);
                    if constexpr (DIAG) {
                        if (16 * rt[u] + li == 16 * ct + 4 * v + lg) r2 = 0.0;
                    }
                    Kv[v] = kernel_fast<KIND>(r2, inv_ell);
                }
            }
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int v = 0; v < 4; ++v) Y[u][rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(Kv[v], Qf[rb][v], Y[u][rb], 0, 0, 0);
        }
    }
}

template <int KIND, int DK, int RB>
__global__ __launch_bounds__(256) void p2p_mrhs_kernel(DevTree T, DevOp O, double *__restrict__ y, int nrhs,
                                                       int do_near, int do_far)
{
    constexpr int NKC = DK / 4;
    __shared__ double sX[DK * kSX64];
    __shared__ double sN[kSymLeaf];
    __shared__ double sQ[kSymLeaf * q_stride<RB>()];
    __shared__ double cen[DK];
    __shared__ int32_t sPre[kSymSeg + 1], sBeg[kSymSeg], colP[kSymLeaf], sDiag;
    constexpr bool kSplit = KIND == kGaussSplit;
    __shared__ double tF[kSplit ? kSymLeaf : 1];  // split Gaussian: row factors exp(-|x - c|^2 / ell)
    const int l = T.near_order[blockIdx.x];
    if (l < 0) return;  // padding of a shorter XCD segment
    const int c = T.leaf_first + l;
    const int cb = T.cbeg[c], nt = T.cend[c] - cb;
    if (nt == 0) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int n = T.n;
    const double inv_ell = 1.0 / O.ell;
    const int ntiles = (nt + 15) / 16;
    if (tid < DK) cen[tid] = T.center[(size_t)l * DK + tid];
    __syncthreads();
    // targets as the B operand: lane (i + 16 g) holds coordinate 4 kc + g of target i
    const int rt[2] = {w, w + 4};
    double Bt[2][NKC], tn[2];
    dbl4 Y[2][RB];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int i = 16 * rt[u] + li;
        const bool ok = i < nt;
        const int ii = cb + (ok ? i : nt - 1);
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < DK; ++k) {
            const double v = T.Xs[(size_t)k * n + ii] - cen[k];
            s = fma(v, v, s);
        }
        tn[u] = s;
        constexpr double kCross = 2.0 * 1.4426950408889634;
#pragma unroll
        for (int kc = 0; kc < NKC; ++kc) {
            const double v = T.Xs[(size_t)(4 * kc + lg) * n + ii] - cen[4 * kc + lg];
            Bt[u][kc] = kSplit ? (kCross * inv_ell) * v : v;
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) Y[u][rb] = dbl4{0.0, 0.0, 0.0, 0.0};
    }
    if constexpr (kSplit) {
        if (tid < kSymLeaf) {
            const int ii = cb + (tid < nt ? tid : nt - 1);
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < DK; ++k) {
                const double v = T.Xs[(size_t)k * n + ii] - cen[k];
                s = fma(v, v, s);
            }
            tF[tid] = exp_bounded(-s * inv_ell);
        }
    }
    if (do_near) {
        // the leaf's own block first (when listed), then the other source leaves as one stream of
        // points, kSymLeaf columns at a time (only the stream's last column tile is padded)
        const int f0 = T.Nptr[l], f1 = T.Nptr[l + 1];
        if (tid == 0) sDiag = 0;
        __syncthreads();
        for (int f = f0 + tid; f < f1; f += blockDim.x)
            if (T.Nsrc[f] == l) sDiag = 1;
        __syncthreads();
        // columns [c0, c0 + ns) of the current stream (or of the own block): colP holds each
        // column's point, set by the caller of stage_chunk before the barrier
        // sid: the 128 threads that stage the coordinates (waves 0-1 or 2-3, alternating by chunk)
        auto stage_chunk = [&](int ns, int sid) {
            if (sid < kSymLeaf) {
                const int j = sid;
                const bool ok = j < ns;
                const int jj = colP[j];
                double xv[DK];
#pragma unroll
                for (int k = 0; k < DK; ++k) xv[k] = T.Xs[(size_t)k * n + jj];
                double s = 0.0;
#pragma unroll
                for (int k = 0; k < DK; ++k) {
                    const double v = ok ? xv[k] - cen[k] : 0.0;
                    sX[k * kSX64 + j] = v;
                    s = fma(v, v, s);
                }
                // split Gaussian: the base-2 logarithm of the column factor exp(-|y - c|^2 / ell)
                sN[j] = kSplit ? s * (-1.4426950408889634 * inv_ell) : s;
            }
            // charges [j][r], zero beyond the stream and beyond nrhs: thread tid stages rhs
            // r = tid % 16RB of columns j0 + t * 256 / 16RB, every load issued before the first store
            constexpr int QPT = kSymLeaf * 16 * RB / 256;
            const int r = tid % (16 * RB), j0 = tid / (16 * RB);
            const int rr = r < nrhs ? r : 0;
            double qv[QPT];
#pragma unroll
            for (int t = 0; t < QPT; ++t) qv[t] = O.xt[(size_t)colP[j0 + t * (256 / (16 * RB))] * nrhs + rr];
#pragma unroll
            for (int t = 0; t < QPT; ++t) {
                const int j = j0 + t * (256 / (16 * RB));
                sQ[j * q_stride<RB>() + q_col<RB>(j, r)] = (j < ns && r < nrhs) ? qv[t] : 0.0;
            }
        };
        if (sDiag) {
            if (tid < kSymLeaf) colP[tid] = cb + (tid < nt ? tid : nt - 1);
            __syncthreads();
            stage_chunk(nt, tid);
            __syncthreads();
            mrhs_block<KIND, DK, RB, true>(Bt, tn, Y, sX, sN, sQ, nt, ntiles, w, li, lg, inv_ell);
        }
        int chunk = 0;  // the column search and coordinate staging alternate between waves 0-1 and 2-3
        for (int fb = f0; fb < f1; fb += kSymSeg) {
            const int fe = min(fb + kSymSeg, f1);
            __syncthreads();  // the previous tiles and table are consumed
            {
                int sz = 0, beg = 0;
                const int f = fb + tid;
                if (f < fe) {
                    const int sl = T.Nsrc[f];
                    beg = T.cbeg[T.leaf_first + sl];
                    if (sl != l) sz = T.cend[T.leaf_first + sl] - beg;
                }
                sPre[tid + 1] = sz;
                sBeg[tid] = beg;
                if (tid == 0) sPre[0] = 0;
            }
            __syncthreads();
            for (int off = 1; off < kSymSeg; off <<= 1) {  // inclusive scan of sPre[1..kSymSeg]
                const int add = tid >= off ? sPre[tid + 1 - off] : 0;
                __syncthreads();
                sPre[tid + 1] += add;
                __syncthreads();
            }
            const int total = sPre[kSymSeg];
            for (int c0 = 0; c0 < total; c0 += kSymLeaf, ++chunk) {
                const int ns = min(kSymLeaf, total - c0);
                const int sid = tid ^ ((chunk & 1) << 7);
                // no barrier here: the search writes only colP, which the previous chunk's tiles do not
                // read (its staging, which does, ended at the barrier before them), and the barrier after
                // the search keeps this chunk's staging behind every wave's previous tiles
                if (sid < kSymLeaf) {
                    int pidx = cb;  // any valid point for the padding columns
                    if (sid < ns) {
                        const int col = c0 + sid;  // the entry holding it: the largest k with sPre[k] <= col
                        int lo = 0, hi = kSymSeg;
                        while (lo < hi) {
                            const int mid = (lo + hi + 1) >> 1;
                            if (sPre[mid] <= col) lo = mid;
                            else hi = mid - 1;
                        }
                        pidx = sBeg[lo] + (col - sPre[lo]);
                    }
                    colP[sid] = pidx;
                }
                __syncthreads();
                stage_chunk(ns, sid);
                __syncthreads();
                mrhs_block<KIND, DK, RB, false>(Bt, tn, Y, sX, sN, sQ, ns, ntiles, w, li, lg, inv_ell);
            }
        }
    }
    if constexpr (kSplit) __syncthreads();  // tF is complete
    // Y[u][rb] element v of lane (r + 16 g) is output (target 16 rt + 4 v + g, rhs 16 rb + r)
    const double *lc = O.L + (size_t)c * O.nx * nrhs;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        if (rt[u] >= ntiles) continue;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const int r = 16 * rb + li;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * rt[u] + 4 * v + lg;
                double acc = Y[u][rb][v];
                if constexpr (kSplit) acc *= tF[i];  // the row factor
                if (do_far && i < nt && r < nrhs) {
                    // the farfield sum formed from zero and added once, as l2p_add_kernel does when
                    // the farfield ran beside this kernel: both orders give the same bits
                    double fs = 0.0;
                    for (int a = 0; a < O.nx; ++a) fs = fma(O.Lb[(size_t)a * n + cb + i], lc[a * nrhs + r], fs);
                    acc += fs;
                }
                if (i < nt && r < nrhs) y[(size_t)T.perm[cb + i] * nrhs + r] = acc;
            }
        }
    }
}

template <int KIND, int DK>
void launch_mrhs_d(const DevTree &T, const DevOp &O, double *y, int nrhs, int near, int far, hipStream_t st)
{
    if (nrhs <= 16)
        hipLaunchKernelGGL((p2p_mrhs_kernel<KIND, DK, 1>), dim3(T.n_near_order), dim3(256), 0, st, T, O, y, nrhs, near, far);
    else
        hipLaunchKernelGGL((p2p_mrhs_kernel<KIND, DK, 2>), dim3(T.n_near_order), dim3(256), 0, st, T, O, y, nrhs, near, far);
}

template <int KIND>
hipError_t launch_mrhs_k(const DevTree &T, const DevOp &O, double *y, int nrhs, int near, int far, hipStream_t st)
{
    switch ((T.d + 3) / 4 * 4) {
    case 4: launch_mrhs_d<KIND, 4>(T, O, y, nrhs, near, far, st); break;
    case 8: launch_mrhs_d<KIND, 8>(T, O, y, nrhs, near, far, st); break;
    case 12: launch_mrhs_d<KIND, 12>(T, O, y, nrhs, near, far, st); break;
    case 16: launch_mrhs_d<KIND, 16>(T, O, y, nrhs, near, far, st); break;
    case 20: launch_mrhs_d<KIND, 20>(T, O, y, nrhs, near, far, st); break;
    case 24: launch_mrhs_d<KIND, 24>(T, O, y, nrhs, near, far, st); break;
    case 28: launch_mrhs_d<KIND, 28>(T, O, y, nrhs, near, far, st); break;
    case 32: launch_mrhs_d<KIND, 32>(T, O, y, nrhs, near, far, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// y[perm] = owner row sums + received column sums (fixed order) + L2P
__device__ __forceinline__ void combine_body(const DevTree &T, const DevOp &O, int l, double *__restrict__ y,
                                             int do_near, int do_far)
{
    const int c = T.leaf_first + l;
    const int cb = T.cbeg[c], nt = T.cend[c] - cb;
    const int i = threadIdx.x;
    if (i >= nt) return;
    double acc = 0.0;
    if (do_near) {
        acc = O.rowbuf[(size_t)l * kSymLeaf + i];
        // eight column sums in flight at a time, added in list order
        const int q1 = T.inc_ptr[l + 1];
        int q = T.inc_ptr[l];
        for (; q + 8 <= q1; q += 8) {
            double v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = O.colbuf[(size_t)T.inc_blk[q + k] * kSymLeaf + i];
#pragma unroll
            for (int k = 0; k < 8; ++k) acc += v[k];
        }
        for (; q < q1; ++q) acc += O.colbuf[(size_t)T.inc_blk[q] * kSymLeaf + i];
    }
    if (do_far) {
        const double *lc = O.L + (size_t)c * O.nx;
        for (int a = 0; a < O.nx; ++a) acc = fma(O.Lb[(size_t)a * T.n + cb + i], lc[a], acc);
    }
    y[T.perm[cb + i]] = acc;
}

__global__ __launch_bounds__(kSymLeaf) void p2p_combine_kernel(DevTree T, DevOp O, double *__restrict__ y,
                                                               int do_near, int do_far)
{
    combine_body(T, O, blockIdx.x, y, do_near, do_far);
}

// Farfield evaluation (L2P) added to a several-rhs nearfield result that was computed beside the
// farfield: y[perm i][r] += sum_a l_a(x_i) L_c[a][r] for the points i of leaf blockIdx.x (the sum
// over a formed first, in order, then added once).  The leaf's locals sit in LDS (nx * nrhs
// doubles, dynamic); thread t keeps rhs t mod nrhs and walks the points t / nrhs, t / nrhs + per,
// ... (per = 256 / nrhs), so the nrhs threads of a point read one basis value and write one row.
__global__ __launch_bounds__(256) void l2p_add_kernel(DevTree T, DevOp O, double *__restrict__ y, int nrhs)
{
    extern __shared__ double sL[];  // [nx][nrhs]
    const int c = T.leaf_first + blockIdx.x;
    const int cb = T.cbeg[c], nt = T.cend[c] - cb;
    const int nx = O.nx;
    const double *lc = O.L + (size_t)c * nx * nrhs;
    for (int e = threadIdx.x; e < nx * nrhs; e += blockDim.x) sL[e] = lc[e];
    __syncthreads();
    const int per = blockDim.x / nrhs;
    const int r = threadIdx.x % nrhs, i0 = threadIdx.x / nrhs;
    if (i0 >= per) return;  // (no barrier follows)
    for (int i = i0; i < nt; i += per) {
        double acc = 0.0;
        for (int a = 0; a < nx; ++a) acc = fma(O.Lb[(size_t)a * T.n + cb + i], sL[a * nrhs + r], acc);
        y[(size_t)T.perm[cb + i] * nrhs + r] += acc;
    }
}

template <int KIND>
hipError_t launch_sym_k(const DevTree &T, const DevOp &O, hipStream_t st)
{
    const int dk = (T.d + 3) / 4 * 4;
    switch (dk) {
#define DWFMM_SYM(D) \
    case D: hipLaunchKernelGGL((p2p_sym_kernel<KIND, D>), dim3(T.n_order), dim3(256), 0, st, T, O); break;
        DWFMM_SYM(4) DWFMM_SYM(8) DWFMM_SYM(12) DWFMM_SYM(16) DWFMM_SYM(20) DWFMM_SYM(24) DWFMM_SYM(28)
        DWFMM_SYM(32)
#undef DWFMM_SYM
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- FP32 variants (reduced precision)
// Same algorithms in FP32 arithmetic: coordinates (shifted in FP64, then rounded),
// Gram tiles on v_mfma_f32_16x16x4f32, kernel values with the hardware exp2/sqrt,
// FP32 accumulation within a launch; results are stored as FP64.
// Lane layout of v_mfma_f32_16x16x4f32 (checked with a probe): A[i][k] in lane i + 16k,
// B[k][j] in lane j + 16k, D[i][j] in lane j + 16(i/4), element i%4.
typedef float flt4 __attribute__((ext_vector_type(4)));

template <int KIND>
__device__ __forceinline__ float kernel_f32(float r2, float inv_ell)
{
    // the products of constants are loop invariant in the callers and get hoisted
    constexpr float kLog2e = 1.4426950408889634f;
    if constexpr (KIND == 0) {
        const float s = __builtin_amdgcn_sqrtf(r2) * (1.7320508f * inv_ell);
        const float e = __builtin_amdgcn_exp2f(s * -kLog2e);
        return fmaf(s, e, e);
    } else if constexpr (KIND == 1) {
        return __builtin_amdgcn_exp2f(r2 * (inv_ell * -kLog2e));
    } else {
        return __builtin_amdgcn_exp2f(__builtin_amdgcn_sqrtf(r2) * (inv_ell * -kLog2e));
    }
}

template <int KIND, int NKC, bool DIAG>
__device__ __forceinline__ void sym_block32(const float (&A)[2][NKC], const float (&rN)[2][4], const float (&rQ)[2][4],
                                            float (&racc)[2][4], const float *sX, const float *sN, const float *sQ,
                                            float *colpart, int ns, int ntiles, int w, int li, int lg, float inv_ell)
{
    const int rt[2] = {w, w + 4};
    const int nct = (ns + 15) / 16;
    for (int ct = 0; ct < nct; ++ct) {
        const int j = 16 * ct + li;
        const float nb = KIND == kGaussSplit ? 0.0f : sN[j], qb = sQ[j];
        float Bf[NKC];
#pragma unroll
        for (int kc = 0; kc < NKC; ++kc) Bf[kc] = sX[(4 * kc + lg) * kSX32 + j];
        float cacc = 0.0f;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (rt[u] >= ntiles) continue;
            // A holds -2 (x - c): the chain starts from |x|^2 and adds -2 x.y, then |y|^2 is added
            // on the vector ALU (an ordinary add, so the clamp needs no canonicalisation of the
            // MFMA result).  Split Gaussian: A holds (2 log2(e) / ell)(x - c), the chain gives the
            // base-2 exponent of the cross factor; the row and column factors sit in the charges.
            flt4 G;
            if constexpr (KIND == kGaussSplit)
                G = flt4{0.0f, 0.0f, 0.0f, 0.0f};
            else
                G = flt4{rN[u][0], rN[u][1], rN[u][2], rN[u][3]};
#pragma unroll
            for (int kc = 0; kc < NKC; ++kc) G = __builtin_amdgcn_mfma_f32_16x16x4f32(A[u][kc], Bf[kc], G, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                float kv;
                if constexpr (KIND == kGaussSplit) {
                    kv = __builtin_amdgcn_exp2f(G[v]);
                } else {
                    const float g2 = G[v] + nb;
                    float r2 = KIND == 1 ? g2 : fmaxf(g2, 0.0f);
                    if constexpr (DIAG) {
                        if (16 * rt[u] + 4 * lg + v == j) r2 = 0.0f;
                    }
                    kv = kernel_f32<KIND>(r2, inv_ell);
                }
                racc[u][v] = fmaf(kv, qb, racc[u][v]);
                if constexpr (!DIAG) cacc = fmaf(kv, rQ[u][v], cacc);
            }
        }
        if constexpr (!DIAG) {
            cacc += __shfl_xor(cacc, 16, 64);
            cacc += __shfl_xor(cacc, 32, 64);
            if (lg == 0) colpart[w * kSymLeaf + j] = cacc;
        }
    }
}

template <int KIND, int DK>
__device__ __forceinline__ void p2p_sym32_body(const DevTree &T, const DevOp &O, int l)
{
    constexpr int NKC = DK / 4;
    __shared__ float sX[DK * kSX32];
    __shared__ float sN[kSymLeaf], sQ[kSymLeaf], tN[kSymLeaf], tQ[kSymLeaf];
    __shared__ float colpart[4 * kSymLeaf];
    __shared__ double cen[DK];
    __shared__ int32_t sPre[kSymSeg + 1], sBlk[kSymSeg], sBeg[kSymSeg];
    __shared__ int32_t colF[kSymLeaf], colJ[kSymLeaf];
    __shared__ int32_t sDiag;
    const int c = T.leaf_first + l;
    const int cb = T.cbeg[c], nt = T.cend[c] - cb;
    if (nt == 0) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int n = T.n;
    const float inv_ell = (float)(1.0 / O.ell);
    const int ntiles = (nt + 15) / 16;
    if (tid < DK) cen[tid] = T.center[(size_t)l * DK + tid];
    if (tid == 0) sDiag = 0;
    __syncthreads();
    const int o0 = T.own_ptr[l], o1 = T.own_ptr[l + 1];
    for (int f = o0 + tid; f < o1; f += blockDim.x)  // is the self block listed (as in FP64)
        if (T.own_src[f] == l) sDiag = 1;
    if (tid < kSymLeaf) {
        const bool ok = tid < nt;
        const int ii = cb + (ok ? tid : nt - 1);
        float s = 0.0f;
#pragma unroll
        for (int k = 0; k < DK; ++k) {
            const float v = (float)(T.Xs[(size_t)k * n + ii] - cen[k]);
            s = fmaf(v, v, s);
        }
        if constexpr (KIND == kGaussSplit) {
            const float a = __builtin_amdgcn_exp2f(s * (inv_ell * -1.4426950408889634f));  // row factor
            tN[tid] = ok ? a : 0.0f;
            tQ[tid] = ok ? (float)O.xt[ii] * a : 0.0f;
        } else {
            tN[tid] = ok ? s : 0.0f;
            tQ[tid] = ok ? (float)O.xt[ii] : 0.0f;
        }
    }
    const int rt[2] = {w, w + 4};
    float A[2][NKC];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int i = 16 * rt[u] + li;
        const bool ok = i < nt;
        const int ii = cb + (ok ? i : nt - 1);
        const float scale = KIND == kGaussSplit ? 2.0f * 1.4426950408889634f * inv_ell : -2.0f;
#pragma unroll
        for (int kc = 0; kc < NKC; ++kc) {
            const int k = 4 * kc + lg;
            const float v = (float)(T.Xs[(size_t)k * n + ii] - cen[k]);
            A[u][kc] = ok ? scale * v : 0.0f;
        }
    }
    __syncthreads();
    float rN[2][4], rQ[2][4], racc[2][4];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = 16 * rt[u] + 4 * lg + v;
            rN[u][v] = tN[i];
            rQ[u][v] = tQ[i];
            racc[u][v] = 0.0f;
        }
    // Tile column j: point pidx shifted to the owner's midpoint, its squared norm (split
    // Gaussian: its column factor) and its charge; columns past the data are zero.
    auto stage = [&](int j, int pidx, bool ok) {
        double xv[DK];
#pragma unroll
        for (int k = 0; k < DK; ++k) xv[k] = T.Xs[(size_t)k * n + pidx];
        float s = 0.0f;
#pragma unroll
        for (int k = 0; k < DK; ++k) {
            const float v = ok ? (float)(xv[k] - cen[k]) : 0.0f;
            sX[k * kSX32 + j] = v;
            s = fmaf(v, v, s);
        }
        const float q = (float)O.xt[pidx];
        if constexpr (KIND == kGaussSplit) {
            const float bfac = __builtin_amdgcn_exp2f(s * (inv_ell * -1.4426950408889634f));  // column factor
            sN[j] = bfac;
            sQ[j] = ok ? q * bfac : 0.0f;
        } else {
            sN[j] = s;
            sQ[j] = ok ? q : 0.0f;
        }
    };
    // the leaf with itself when listed, then the other owned blocks as one column stream (as in FP64)
    if (sDiag) {
        __syncthreads();
        if (tid < kSymLeaf) stage(tid, cb + (tid < nt ? tid : nt - 1), tid < nt);
        __syncthreads();
        sym_block32<KIND, NKC, true>(A, rN, rQ, racc, sX, sN, sQ, colpart, nt, ntiles, w, li, lg, inv_ell);
    }
    int chunk = 0;  // staging and column sums alternate between waves 0-1 and 2-3 (as in FP64)
    for (int fb = o0; fb < o1; fb += kSymSeg) {
        const int fe = min(fb + kSymSeg, o1);
        __syncthreads();
        {
            int sz = 0, beg = 0;
            const int f = fb + tid;
            if (f < fe) {
                const int sl = T.own_src[f];
                beg = T.cbeg[T.leaf_first + sl];
                if (sl != l) sz = T.cend[T.leaf_first + sl] - beg;
            }
            sPre[tid + 1] = sz;
            sBlk[tid] = f;
            sBeg[tid] = beg;
            if (tid == 0) sPre[0] = 0;
        }
        __syncthreads();
        for (int off = 1; off < kSymSeg; off <<= 1) {
            const int add = tid >= off ? sPre[tid + 1 - off] : 0;
            __syncthreads();
            sPre[tid + 1] += add;
            __syncthreads();
        }
        const int total = sPre[kSymSeg];
        for (int c0 = 0; c0 < total; c0 += kSymLeaf, ++chunk) {
            const int ns = min(kSymLeaf, total - c0);
            const int sid = tid ^ ((chunk & 1) << 7);
            __syncthreads();
            if (sid < kSymLeaf) {
                const int j = sid;
                const bool ok = j < ns;
                int pidx = cb, fblk = 0, jl = 0;
                if (ok) {
                    const int col = c0 + j;
                    int lo = 0, hi = kSymSeg;
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (sPre[mid] <= col) lo = mid;
                        else hi = mid - 1;
                    }
                    fblk = sBlk[lo];
                    jl = col - sPre[lo];
                    pidx = sBeg[lo] + jl;  // from LDS: only the coordinates are loaded from memory
                }
                stage(j, pidx, ok);
                colF[j] = fblk;
                colJ[j] = jl;
            }
            __syncthreads();
            sym_block32<KIND, NKC, false>(A, rN, rQ, racc, sX, sN, sQ, colpart, ns, ntiles, w, li, lg, inv_ell);
            __syncthreads();
            if (sid < ns) {
                float cs = ((colpart[sid] + colpart[kSymLeaf + sid]) + colpart[2 * kSymLeaf + sid]) +
                           colpart[3 * kSymLeaf + sid];
                if constexpr (KIND == kGaussSplit) cs *= sN[sid];
                O.colbuf[(size_t)colF[sid] * kSymLeaf + colJ[sid]] = (double)cs;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            float s = racc[u][v];
            s += __shfl_xor(s, 1, 64);
            s += __shfl_xor(s, 2, 64);
            s += __shfl_xor(s, 4, 64);
            s += __shfl_xor(s, 8, 64);
            const int i = 16 * rt[u] + 4 * lg + v;
            if constexpr (KIND == kGaussSplit) s *= rN[u][v];
            if (li == 0 && i < nt) O.rowbuf[(size_t)l * kSymLeaf + i] = (double)s;
        }
}

template <int KIND, int DK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(DK <= 12 ? 5 : 1, 8))) void p2p_sym32_kernel(DevTree T, DevOp O)
{
    const int l = T.leaf_order[blockIdx.x];
    if (l < 0) return;  // padding of a shorter XCD segment
    p2p_sym32_body<KIND, DK>(T, O, l);
}

template <int KIND>
hipError_t launch_sym32_k(const DevTree &T, const DevOp &O, hipStream_t st)
{
    switch ((T.d + 3) / 4 * 4) {
#define DWFMM_SYM(D) \
    case D: hipLaunchKernelGGL((p2p_sym32_kernel<KIND, D>), dim3(T.n_order), dim3(256), 0, st, T, O); break;
        DWFMM_SYM(4) DWFMM_SYM(8) DWFMM_SYM(12) DWFMM_SYM(16) DWFMM_SYM(20) DWFMM_SYM(24) DWFMM_SYM(28)
        DWFMM_SYM(32)
#undef DWFMM_SYM
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Nearfield for several rhs in reduced precision.  FP32 Gram tile with the sources as the
// A operand: element e of lane (i + 16 g) holds K[target i][source 4g + e].  BF16: that is the
// A operand of v_mfma_f32_16x16x16bf16_1k as is (A[i][k] in lane i + 16(k/4), element k%4),
// so Y(16 x 16 rhs) += K Q is one MFMA with FP32 accumulation.  FP32: element e is the A
// operand of chunk e (sources 4g + e) of four v_mfma_f32_16x16x4f32.
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float flt2v __attribute__((ext_vector_type(2)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
// Four floats rounded to BF16 (to nearest even) by two v_cvt_pk_bf16_f32: the pairs are joined
// through their 32-bit patterns (built element by element, a vector that feeds an MFMA compiles
// to four one-value conversions and two permutes).
__device__ __forceinline__ bf16x4 to_bf16x4(float a, float b, float c, float d)
{
    const uint32_t lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(flt2v{a, b}, bf16x2));
    const uint32_t hi = __builtin_bit_cast(uint32_t, __builtin_convertvector(flt2v{c, d}, bf16x2));
    return __builtin_bit_cast(bf16x4, u32x2{lo, hi});
}
// BF16 charges in the order the apply MFMA takes them: for column tile ct and rhs tile rb, lane
// li + 16 lg's four values (sources 16 ct + 4 lg ... + 3 of rhs 16 rb + li) at halves
// qt_slot = 4 (64 (RB ct + rb) + li + 16 lg): a wave reads 512 bytes in order, and a half-wave of
// the staging (16 rhs x 2 column groups) writes 256 bytes in order.  (Rows of 136 halves per rhs,
// read at words 68 li + 2 lg, still showed conflicts on about a sixth of the LDS cycles.)
template <int RB>
__device__ __forceinline__ int qt_slot(int ct, int rb, int lane) { return 4 * (64 * (RB * ct + rb) + lane); }
// BF16 mode's distances: each centred coordinate v (scaled by the operator's power of two, so
// |v| <= 1) is split into FP16 parts h = fp16(v) and l = fp16(2^11 (v - h)), and 2^11 times the Gram
// sum is formed on v_mfma_f32_16x16x32_f16 (FP32 accumulation) as sum h_x (2^11 h_y) + h_x l_y + l_x h_y
// in one accumulator (2^11 h is exact in FP16): three MFMAs of 16 cycles per 16 x 16 tile for up to
// 32 dimensions, against d / 4 of 32 cycles on v_mfma_f32_16x16x4f32.  The dropped terms are about 2^-22 |x_k y_k| each, far below the BF16
// rounding of the kernel values; the low parts carry the 2^11 so that they stay in FP16's normal
// range.  Sources sit in LDS in the order the MFMA takes them: for part p (0 high, 1 low) and
// column tile ct, lane li + 16 lg's eight values (source 16 ct + li, dimensions 8 lg ... 8 lg + 7)
// at halves 8 (64 (8 p + ct) + li + 16 lg), so a wave reads 1 KiB in order.  (Rows of 72 halves per
// column, read at words 36 li + 4 lg, showed LDS bank conflicts on most of their 16-byte reads.)
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ int gram_slot(int part, int ct, int lane) { return 8 * (64 * (8 * part + ct) + lane); }
template <int DK, bool BF16>
constexpr bool gram_f16() { return BF16 && DK >= 8; }
// FP32 charges stored [source][rhs]; rows of 16 RB + 4 floats put consecutive lane groups on
// the two halves of the banks
template <int RB>
constexpr int q_stride32() { return 16 * RB + 4; }

// A chunk's stored BF16 tiles for this wave (column tile ct, row tile w + 4u at tiles + ct * 512 +
// (w + 4u) * 64 + lane: 8 bytes per lane, one coalesced 512-byte row per wave), all loads issued at
// once so that they overlap each other and the chunk's charge staging; missing tiles read as zero.
__device__ __forceinline__ void load_tiles(uint2 (&pre)[8][2], const uint2 *tiles, int64_t tcap, int ns, int ntiles,
                                           int w, int lane)
{
    const int nct = (ns + 15) / 16;
#pragma unroll
    for (int ct = 0; ct < 8; ++ct)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int rt = w + 4 * u;
            // streamed once per apply: non-temporal, so that they do not push the charges out of L2
            pre[ct][u] = ct < nct && ct < tcap && rt < ntiles
                             ? __builtin_bit_cast(uint2, __builtin_nontemporal_load(reinterpret_cast<const uint64_t *>(
                                                             tiles + (size_t)ct * 512 + rt * 64 + lane)))
                             : make_uint2(0u, 0u);
        }
}

// The apply of a chunk from its stored tiles: Y += K Q on the BF16 MFMA, charges from LDS.
template <int RB>
__device__ __forceinline__ void apply_tiles(const uint2 (&pre)[8][2], flt4 (&Y)[2][RB], const __bf16 *sQt, int ns,
                                            int ntiles, int w, int li, int lg)
{
    const int nct = (ns + 15) / 16;
#pragma unroll
    for (int ct = 0; ct < 8; ++ct) {
        if (ct >= nct) break;
        bf16x4 Qb[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
            Qb[rb] = *reinterpret_cast<const bf16x4 *>(&sQt[qt_slot<RB>(ct, rb, li + 16 * lg)]);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (w + 4 * u >= ntiles) continue;
            const bf16x4 Ka = __builtin_bit_cast(bf16x4, pre[ct][u]);
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) Y[u][rb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(Ka, Qb[rb], Y[u][rb], 0, 0, 0);
        }
    }
}

// CM (BF16 only): 0 compute the kernel tiles, 1 compute them and also write them to `tiles`
// (column tile ct of this call at tiles + ct * 512, at most `tcap` column tiles).
// FP16 Gram (gram_f16): Th, Tl the targets' high and low parts and Th2 = 2^11 Th (lane (li, lg):
// target 16 rt + li, dimensions 8 lg ... 8 lg + 7), sXh the sources' rows; the exponent (split
// Gaussian) or r^2 is then gA G + (snv, or |x|^2 + |y|^2) with G = 2^11 times the Gram sum.
template <int KIND, int DK, int RB, bool BF16, bool DIAG, int CM = 0>
__device__ __forceinline__ void mrhs_block_lp(const float (&Bt)[2][DK / 4], const float (&tn)[2], flt4 (&Y)[2][RB],
                                              const float *sX, const float *sN, const float *sQ, const __bf16 *sQt,
                                              int ns, int ntiles, int w, int li, int lg, float inv_ell,
                                              const f16x8 (&Th)[2], const f16x8 (&Tl)[2], const f16x8 (&Th2)[2],
                                              const _Float16 *sXh, float gA, uint2 *tiles = nullptr,
                                              int64_t tcap = 0)
{
    static_assert(CM == 0 || (CM == 1 && BF16), "the tile cache holds BF16 tiles");
    constexpr int NKC = DK / 4;
    constexpr bool kH = gram_f16<DK, BF16>();
    const int rt[2] = {w, w + 4};
    [[maybe_unused]] const int lane = li + 16 * lg;
    const int nct = (ns + 15) / 16;
    for (int ct = 0; ct < nct; ++ct) {
        float Af[kH ? 1 : NKC], snv[4];
        f16x8 Ah, Al;
        if constexpr (kH) {
            Ah = *reinterpret_cast<const f16x8 *>(&sXh[gram_slot(0, ct, lane)]);
            Al = *reinterpret_cast<const f16x8 *>(&sXh[gram_slot(1, ct, lane)]);
        } else {
#pragma unroll
            for (int kc = 0; kc < NKC; ++kc) Af[kc] = sX[(4 * kc + lg) * kSX32 + 16 * ct + li];
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) snv[e] = sN[16 * ct + 4 * lg + e];
        // the charge operands of this column tile serve both row tiles
        bf16x4 Qb[BF16 ? RB : 1];
        if constexpr (BF16) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
                Qb[rb] = *reinterpret_cast<const bf16x4 *>(&sQt[qt_slot<RB>(ct, rb, li + 16 * lg)]);
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (rt[u] >= ntiles) continue;
            // split Gaussian as in the FP64 kernel: the chain starts from the sources' base-2 column
            // factors and delivers the entry's exponent but for the row factor
            flt4 G;
            if constexpr (kH) {
                // the small cross terms first, then the high parts' product
                G = flt4{0.0f, 0.0f, 0.0f, 0.0f};
                G = __builtin_amdgcn_mfma_f32_16x16x32_f16(Al, Th[u], G, 0, 0, 0);
                G = __builtin_amdgcn_mfma_f32_16x16x32_f16(Ah, Tl[u], G, 0, 0, 0);
                G = __builtin_amdgcn_mfma_f32_16x16x32_f16(Ah, Th2[u], G, 0, 0, 0);
            } else {
                if constexpr (KIND == kGaussSplit)
                    G = flt4{snv[0], snv[1], snv[2], snv[3]};
                else
                    G = flt4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int kc = 0; kc < NKC; ++kc) G = __builtin_amdgcn_mfma_f32_16x16x4f32(Af[kc], Bt[u][kc], G, 0, 0, 0);
            }
            float Kv[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if constexpr (KIND == kGaussSplit) {
                    Kv[e] = __builtin_amdgcn_exp2f(kH ? fmaf(gA, G[e], snv[e]) : G[e]);
                } else {
                    float r2 = fmaf(kH ? gA : -2.0f, G[e], tn[u] + snv[e]);
                    r2 = fmaxf(r2, 0.0f);
                    if constexpr (DIAG) {
                        if (16 * rt[u] + li == 16 * ct + 4 * lg + e) r2 = 0.0f;
                    }
                    Kv[e] = kernel_f32<KIND>(r2, inv_ell);
                }
            }
            if constexpr (BF16) {
                const bf16x4 Ka = to_bf16x4(Kv[0], Kv[1], Kv[2], Kv[3]);
                if constexpr (CM == 1) {
                    if (ct < tcap)
                        __builtin_nontemporal_store(__builtin_bit_cast(uint64_t, Ka),
                                                    reinterpret_cast<uint64_t *>(tiles + (size_t)ct * 512 + rt[u] * 64 + lane));
                }
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) Y[u][rb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(Ka, Qb[rb], Y[u][rb], 0, 0, 0);
            } else {
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        Y[u][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                            Kv[e], sQ[(16 * ct + 4 * lg + e) * q_stride32<RB>() + 16 * rb + li], Y[u][rb], 0, 0, 0);
            }
        }
    }
}

// Four waves per SIMD at d <= 20 (at most 128 VGPRs); reading stored tiles stages no coordinates,
// fits in 96 VGPRs and runs five, with more tile loads in flight (computing kernels at five waves
// spill in the staging and slow the farfield that runs beside them).
template <int KIND, int DK, int RB, bool BF16, int CM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CM == 2 && DK <= 20 ? 5 : DK <= 20 ? 4 : 1, 8))) void p2p_mrhs_lp_kernel(DevTree T, DevOp O, double *__restrict__ y, int nrhs,
                                                          int do_near, int do_far)
{
    constexpr int NKC = DK / 4;
    constexpr bool kH = gram_f16<DK, BF16>();
    // (reading stored tiles stages no coordinates)
    __shared__ float sX[kH || CM == 2 ? 1 : DK * kSX32];
    __shared__ __attribute__((aligned(16))) _Float16 sXh[kH && CM != 2 ? 2 * kSymLeaf * 32 : 8];
    __shared__ float sN[kSymLeaf];
    __shared__ float sQ[BF16 ? 1 : kSymLeaf * q_stride32<RB>()];
    __shared__ __attribute__((aligned(16))) __bf16 sQt[BF16 ? 16 * RB * kSymLeaf : 8];
    __shared__ double cen[DK];
    __shared__ int32_t sPre[kSymSeg + 1], sBeg[kSymSeg], colP[kSymLeaf], sDiag;
    constexpr bool kSplit = KIND == kGaussSplit;
    static_assert(CM == 0 || BF16, "the tile cache holds BF16 tiles");
    __shared__ float tF[kSplit ? kSymLeaf : 1];  // split Gaussian: row factors exp(-|x - c|^2 / ell)
    const int l = (CM == 2 ? T.near_order_seq : T.near_order)[blockIdx.x];
    if (l < 0) return;  // padding of a shorter XCD segment
    const int c = T.leaf_first + l;
    const int cb = T.cbeg[c], nt = T.cend[c] - cb;
    if (nt == 0) return;
    // the leaf's column tiles in the tile cache, taken in stream order (tb counts them)
    uint2 *ltiles = nullptr;
    int64_t lcount = 0, tb = 0;
    uint2 pre[CM == 2 ? 8 : 1][2];  // reading: the current chunk's tiles of this wave
    if constexpr (CM != 0) {
        ltiles = O.near_tiles + O.near_tile_off[l] * 512;
        lcount = O.near_tile_off[l + 1] - O.near_tile_off[l];
    }
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int n = T.n;
    const float inv_ell = (float)(1.0 / O.ell);
    const int ntiles = (nt + 15) / 16;
    if (tid < DK) cen[tid] = T.center[(size_t)l * DK + tid];
    __syncthreads();
    const int rt[2] = {w, w + 4};
    float Bt[2][NKC], tn[2];
    f16x8 Th[2], Tl[2], Th2[2];
    flt4 Y[2][RB];
    // FP16 Gram: the coordinates' power-of-two scale and the factor of its sum (which carries 2^11)
    const float hs = O.hscale;
    const float gA = (kSplit ? (float)(2.0 * 1.4426950408889634 / O.ell) / (hs * hs) : -2.0f / (hs * hs)) * 0x1p-11f;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int i = 16 * rt[u] + li;
        const bool ok = i < nt;
        const int ii = cb + (ok ? i : nt - 1);
        float s = 0.0f;
#pragma unroll
        for (int k = 0; k < DK; ++k) {
            const float v = (float)(T.Xs[(size_t)k * n + ii] - cen[k]);
            s = fmaf(v, v, s);
        }
        tn[u] = s;
        if constexpr (kH) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = 8 * lg + e;
                const float v = k < DK ? (float)(T.Xs[(size_t)k * n + ii] - cen[k]) * hs : 0.0f;
                const _Float16 h = (_Float16)v;
                Th[u][e] = h;
                Th2[u][e] = (_Float16)((float)h * 2048.0f);
                Tl[u][e] = (_Float16)((v - (float)h) * 2048.0f);
            }
        } else {
            const double csc = kSplit ? 2.0 * 1.4426950408889634 / O.ell : 1.0;
#pragma unroll
            for (int kc = 0; kc < NKC; ++kc) {
                const double v = T.Xs[(size_t)(4 * kc + lg) * n + ii] - cen[4 * kc + lg];
                Bt[u][kc] = (float)(kSplit ? csc * v : v);
            }
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) Y[u][rb] = flt4{0.0f, 0.0f, 0.0f, 0.0f};
    }
    if constexpr (kSplit) {
        if (tid < kSymLeaf) {
            const int ii = cb + (tid < nt ? tid : nt - 1);
            float s = 0.0f;
#pragma unroll
            for (int k = 0; k < DK; ++k) {
                const float v = (float)(T.Xs[(size_t)k * n + ii] - cen[k]);
                s = fmaf(v, v, s);
            }
            tF[tid] = __builtin_amdgcn_exp2f(s * (inv_ell * -1.4426950408889634f));
        }
    }
    if (do_near) {
        // the leaf's own block first (when listed), then the other source leaves as one stream of
        // points, kSymLeaf columns at a time (as in the FP64 kernel)
        const int f0 = T.Nptr[l], f1 = T.Nptr[l + 1];
        if (tid == 0) sDiag = 0;
        __syncthreads();
        for (int f = f0 + tid; f < f1; f += blockDim.x)
            if (T.Nsrc[f] == l) sDiag = 1;
        __syncthreads();
        // sid: the 128 threads that stage the coordinates (waves 0-1 or 2-3, alternating by chunk)
        auto stage_chunk = [&](int ns, int sid) {  // columns of colP[0..kSymLeaf), the first ns real
            if constexpr (CM != 2) if (sid < kSymLeaf) {  // (the coordinates are not needed to read stored tiles)
                const int j = sid;
                const bool ok = j < ns;
                const int jj = colP[j];
                double xv[DK];
#pragma unroll
                for (int k = 0; k < DK; ++k) xv[k] = T.Xs[(size_t)k * n + jj];
                float s = 0.0f;
#pragma unroll
                for (int k = 0; k < DK; ++k) {
                    const float v = ok ? (float)(xv[k] - cen[k]) : 0.0f;
                    if constexpr (!kH) sX[k * kSX32 + j] = v;
                    s = fmaf(v, v, s);
                }
                if constexpr (kH) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        f16x8 hv, lv;
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            const int k = 8 * q + e;
                            const float v = (k < DK && ok) ? (float)(xv[k < DK ? k : 0] - cen[k < DK ? k : 0]) * hs : 0.0f;
                            const _Float16 h = (_Float16)v;
                            hv[e] = h;
                            lv[e] = (_Float16)((v - (float)h) * 2048.0f);
                        }
                        *reinterpret_cast<f16x8 *>(&sXh[gram_slot(0, j >> 4, (j & 15) + 16 * q)]) = hv;
                        *reinterpret_cast<f16x8 *>(&sXh[gram_slot(1, j >> 4, (j & 15) + 16 * q)]) = lv;
                    }
                }
                // split Gaussian: the base-2 logarithm of the column factor exp(-|y - c|^2 / ell)
                sN[j] = kSplit ? s * (inv_ell * -1.4426950408889634f) : s;
            }
            // as in the FP64 kernel: every charge load of the thread issued before the first store
            constexpr int QPT = kSymLeaf * 16 * RB / 256, G = 256 / (16 * RB);
            // FP32: r = tid mod 16 RB.  BF16 (the 8-byte stores in the apply's order): a half-wave
            // takes 16 rhs x 2 neighbouring column groups, 32 consecutive slots
            const int r = BF16 ? (tid & 15) + 16 * ((tid >> 5) % RB) : tid % (16 * RB);
            const int j0 = BF16 ? (((tid >> 5) / RB) << 1) + ((tid >> 4) & 1) : tid / (16 * RB);
            const int rr = r < nrhs ? r : 0;
            if constexpr (BF16) {
                // charges of the BF16 copy P2M wrote (the values this path rounds the FP64 ones to,
                // a quarter of their bytes); columns 4 (j0 + G t) + e, e < 4: one 8-byte store of
                // four columns per t into the transposed tile (single 2-byte stores put rhs r and
                // r + 16 on one bank)
                __bf16 qb[QPT];
#pragma unroll
                for (int t = 0; t < QPT / 4; ++t)
#pragma unroll
                    for (int e = 0; e < 4; ++e) qb[4 * t + e] = O.xtb[(size_t)colP[4 * (j0 + G * t) + e] * nrhs + rr];
#pragma unroll
                for (int t = 0; t < QPT / 4; ++t) {
                    const int j = 4 * (j0 + G * t);
                    bf16x4 v;
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] = (j + e < ns && r < nrhs) ? qb[4 * t + e] : (__bf16)0.0f;
                    *reinterpret_cast<bf16x4 *>(&sQt[qt_slot<RB>(j >> 4, r >> 4, (r & 15) + 16 * ((j & 15) >> 2))]) = v;
                }
            } else {
                double qv[QPT];
#pragma unroll
                for (int t = 0; t < QPT; ++t) qv[t] = O.xt[(size_t)colP[j0 + t * G] * nrhs + rr];
#pragma unroll
                for (int t = 0; t < QPT; ++t) {
                    const int j = j0 + t * G;
                    sQ[j * q_stride32<RB>() + r] = (j < ns && r < nrhs) ? (float)qv[t] : 0.0f;
                }
            }
        };
        if (sDiag) {
            if constexpr (CM == 2) load_tiles(pre, ltiles, lcount, nt, ntiles, w, lane);
            if (tid < kSymLeaf) colP[tid] = cb + (tid < nt ? tid : nt - 1);
            __syncthreads();
            stage_chunk(nt, tid);
            __syncthreads();
            if constexpr (CM == 2) {
                apply_tiles<RB>(pre, Y, sQt, nt, ntiles, w, li, lg);
            } else {
                mrhs_block_lp<KIND, DK, RB, BF16, true, CM>(Bt, tn, Y, sX, sN, sQ, sQt, nt, ntiles, w, li, lg, inv_ell,
                                                           Th, Tl, Th2, sXh, gA, ltiles + tb * 512, lcount - tb);
            }
            tb += (nt + 15) / 16;
        }
        int chunk = 0;  // the column search and coordinate staging alternate between waves 0-1 and 2-3
        for (int fb = f0; fb < f1; fb += kSymSeg) {
            const int fe = min(fb + kSymSeg, f1);
            __syncthreads();  // the previous tiles and table are consumed
            {
                int sz = 0, beg = 0;
                const int f = fb + tid;
                if (f < fe) {
                    const int sl = T.Nsrc[f];
                    beg = T.cbeg[T.leaf_first + sl];
                    if (sl != l) sz = T.cend[T.leaf_first + sl] - beg;
                }
                sPre[tid + 1] = sz;
                sBeg[tid] = beg;
                if (tid == 0) sPre[0] = 0;
            }
            __syncthreads();
            for (int off = 1; off < kSymSeg; off <<= 1) {
                const int add = tid >= off ? sPre[tid + 1 - off] : 0;
                __syncthreads();
                sPre[tid + 1] += add;
                __syncthreads();
            }
            const int total = sPre[kSymSeg];
            for (int c0 = 0; c0 < total; c0 += kSymLeaf, ++chunk) {
                const int ns = min(kSymLeaf, total - c0);
                const int sid = tid ^ ((chunk & 1) << 7);
                if constexpr (CM == 2) load_tiles(pre, ltiles + tb * 512, lcount - tb, ns, ntiles, w, lane);
                // no barrier here, as in the FP64 kernel: the search writes only colP, which the previous
                // chunk's tiles do not read
                if (sid < kSymLeaf) {
                    int pidx = cb;
                    if (sid < ns) {
                        const int col = c0 + sid;
                        int lo = 0, hi = kSymSeg;
                        while (lo < hi) {
                            const int mid = (lo + hi + 1) >> 1;
                            if (sPre[mid] <= col) lo = mid;
                            else hi = mid - 1;
                        }
                        pidx = sBeg[lo] + (col - sPre[lo]);
                    }
                    colP[sid] = pidx;
                }
                __syncthreads();
                stage_chunk(ns, sid);
                __syncthreads();
                if constexpr (CM == 2) {
                    apply_tiles<RB>(pre, Y, sQt, ns, ntiles, w, li, lg);
                } else {
                    mrhs_block_lp<KIND, DK, RB, BF16, false, CM>(Bt, tn, Y, sX, sN, sQ, sQt, ns, ntiles, w, li, lg,
                                                                inv_ell, Th, Tl, Th2, sXh, gA, ltiles + tb * 512,
                                                                lcount - tb);
                }
                tb += (ns + 15) / 16;
            }
        }
    }
    if constexpr (kSplit) __syncthreads();  // tF is complete
    // Y[u][rb] element v of lane (r + 16 g) is output (target 16 rt + 4 g + v, rhs 16 rb + r)
    const double *lc = O.L + (size_t)c * O.nx * nrhs;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        if (rt[u] >= ntiles) continue;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const int r = 16 * rb + li;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * rt[u] + 4 * lg + v;
                double acc = (double)(kSplit ? Y[u][rb][v] * tF[i] : Y[u][rb][v]);
                if (do_far && i < nt && r < nrhs) {
                    // the farfield sum formed from zero and added once, as l2p_add_kernel does when
                    // the farfield ran beside this kernel: both orders give the same bits
                    double fs = 0.0;
                    for (int a = 0; a < O.nx; ++a) fs = fma(O.Lb[(size_t)a * n + cb + i], lc[a * nrhs + r], fs);
                    acc += fs;
                }
                if (i < nt && r < nrhs) y[(size_t)T.perm[cb + i] * nrhs + r] = acc;
            }
        }
    }
}

template <int KIND, int DK, bool BF16>
void launch_mrhs_lp_d(const DevTree &T, const DevOp &O, double *y, int nrhs, int near, int far, hipStream_t st)
{
#define DWFMM_LP(RB, CM)                                                                                   \
    hipLaunchKernelGGL((p2p_mrhs_lp_kernel<KIND, DK, RB, BF16, CM>), dim3(T.n_near_order), dim3(256), 0, st, T, O, y, \
                       nrhs, near, far)
    [[maybe_unused]] const int cm = BF16 ? O.near_cache_mode : 0;
    if constexpr (BF16) {
        if (cm == 1) {
            if (nrhs <= 16) DWFMM_LP(1, 1);
            else DWFMM_LP(2, 1);
            return;
        }
        if (cm == 2) {
            if (nrhs <= 16) DWFMM_LP(1, 2);
            else DWFMM_LP(2, 2);
            return;
        }
    }
    if (nrhs <= 16) DWFMM_LP(1, 0);
    else DWFMM_LP(2, 0);
#undef DWFMM_LP
}

template <int KIND, bool BF16>
hipError_t launch_mrhs_lp_k(const DevTree &T, const DevOp &O, double *y, int nrhs, int near, int far, hipStream_t st)
{
    switch ((T.d + 3) / 4 * 4) {
    case 4: launch_mrhs_lp_d<KIND, 4, BF16>(T, O, y, nrhs, near, far, st); break;
    case 8: launch_mrhs_lp_d<KIND, 8, BF16>(T, O, y, nrhs, near, far, st); break;
    case 12: launch_mrhs_lp_d<KIND, 12, BF16>(T, O, y, nrhs, near, far, st); break;
    case 16: launch_mrhs_lp_d<KIND, 16, BF16>(T, O, y, nrhs, near, far, st); break;
    case 20: launch_mrhs_lp_d<KIND, 20, BF16>(T, O, y, nrhs, near, far, st); break;
    case 24: launch_mrhs_lp_d<KIND, 24, BF16>(T, O, y, nrhs, near, far, st); break;
    case 28: launch_mrhs_lp_d<KIND, 28, BF16>(T, O, y, nrhs, near, far, st); break;
    case 32: launch_mrhs_lp_d<KIND, 32, BF16>(T, O, y, nrhs, near, far, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- M2L for several rhs on MFMA
// l_c[a][r] += sum_b S[a][b] m_s[b][r] over the farfield sources s of c.  As in the several-rhs
// nearfield, the Gram tile of node pairs is formed with the source nodes as the A operand so
// its elements are the A operand of the apply MFMAs.  PREC 0: FP64 throughout (element v of
// lane (a + 16 g) is S[a][4v + g]).  PREC 1: FP32 Gram/kernel/apply (element e of lane
// (a + 16 g) is S[a][4g + e], the A operand of chunk e of four v_mfma_f32_16x16x4f32).
// PREC 2: as PREC 1 up to the kernel values; the product S m then runs on BF16 MFMA with FP32
// accumulation: the four elements of a lane are the A operand of v_mfma_f32_16x16x16bf16_1k
// (A[a][k] in lane a + 16(k/4), element k%4, k = source node 4g + e) and the moments its B
// operand (lane r + 16g holds nodes 4g..4g+3 of rhs r).  Both operands are carried as BF16
// pairs hi + lo (lo the rounding remainder of hi), and the three products lo.hi, hi.lo, hi.hi
// are accumulated (the dropped lo.lo is below 2^-16 of the product): a single BF16 rounding
// of S and m costs ~7e-3 relative in the farfield through the interpolation's Lebesgue
// constant, enough to stall or reverse the FP64 refinement on small shifts.  nx <= 32 (two
// node tiles), up to 32 rhs (two rhs tiles); the four waves split the source list and their
// partial sums are added in wave order.
// v = hi + lo + O(2^-16 |v|) with hi, lo in BF16 (lo the BF16 rounding of v - hi)
__device__ __forceinline__ void bf16_pair(const float (&v)[4], bf16x4 &hi, bf16x4 &lo)
{
    hi = to_bf16x4(v[0], v[1], v[2], v[3]);
    float r[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) r[e] = v[e] - (float)hi[e];
    lo = to_bf16x4(r[0], r[1], r[2], r[3]);
}

template <int PREC>
struct m2l_types {
    typedef float T;
    typedef flt4 V;
};
template <>
struct m2l_types<0> {
    typedef double T;
    typedef dbl4 V;
};

template <int KIND, int DK, int PREC>
__global__ __launch_bounds__(256) void m2l_mrhs_kernel(DevTree T, DevOp O, int first, int nrhs)
{
    typedef typename m2l_types<PREC>::T R;
    typedef typename m2l_types<PREC>::V V4;
    constexpr bool LP = PREC != 0;
    constexpr int NKC = DK / 4;
    __shared__ double part[32 * 33];
    const int c = first + blockIdx.x;
    const int nx = O.nx, nxp = O.nxp;
    const int nxt = nxp / 16, nrb = (nrhs + 15) / 16;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int f0 = T.Fptr[c], f1 = T.Fptr[c + 1];
    const double inv_ell = 1.0 / O.ell;
    // target nodes as the B operand: lane (a + 16 g) holds coordinate 4 kc + g of node 16 rt + a
    const double *tnode = O.nodesT + (size_t)c * DK * nxp;
    R Bt[2][NKC], tn[2];
    V4 Y[2][2];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
        const int a = rt < nxt ? 16 * rt + li : li;
#pragma unroll
        for (int kc = 0; kc < NKC; ++kc) Bt[rt][kc] = (R)tnode[(4 * kc + lg) * nxp + a];
        tn[rt] = (R)O.nnorm[(size_t)c * nxp + a];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) Y[rt][rb] = V4{0, 0, 0, 0};
    }
    for (int f = f0 + w; f < f1; f += 4) {
        const int s = T.Fsrc[f];
        const double *snode = O.nodesT + (size_t)s * DK * nxp;
        const double *ms = O.M + (size_t)s * nx * nrhs;
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
            if (ct >= nxt) continue;
            R Af[NKC];
#pragma unroll
            for (int kc = 0; kc < NKC; ++kc) Af[kc] = (R)snode[(4 * kc + lg) * nxp + 16 * ct + li];
            R sn[4], Mq[2][4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int b = LP ? 16 * ct + 4 * lg + e : 16 * ct + 4 * e + lg;  // source node of element e
                sn[e] = (R)O.nnorm[(size_t)s * nxp + b];
#pragma unroll
                for (int rb = 0; rb < 2; ++rb) {
                    // B operand of chunk e: lane (r + 16 g) holds m_s[source node][rhs 16 rb + r]
                    const int r = 16 * rb + li;
                    Mq[rb][e] = (b < nx && r < nrhs && rb < nrb) ? (R)ms[(size_t)b * nrhs + r] : (R)0;
                }
            }
            bf16x4 Mh[2], Ml[2];  // PREC 2: the moments as BF16 pairs
            if constexpr (PREC == 2) {
#pragma unroll
                for (int rb = 0; rb < 2; ++rb) bf16_pair(Mq[rb], Mh[rb], Ml[rb]);
            }
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) {
                if (rt >= nxt) continue;
                V4 G = {0, 0, 0, 0};
                R Kv[4];
                if constexpr (LP) {
#pragma unroll
                    for (int kc = 0; kc < NKC; ++kc) G = __builtin_amdgcn_mfma_f32_16x16x4f32(Af[kc], Bt[rt][kc], G, 0, 0, 0);
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        Kv[e] = kernel_f32<KIND>(fmaxf(fmaf(-2.0f, G[e], tn[rt] + sn[e]), 0.0f), (float)inv_ell);
                } else {
#pragma unroll
                    for (int kc = 0; kc < NKC; ++kc) G = __builtin_amdgcn_mfma_f64_16x16x4f64(Af[kc], Bt[rt][kc], G, 0, 0, 0);
#pragma unroll
                    for (int e = 0; e < 4; ++e) Kv[e] = kernel_fast<KIND>(fmax(fma(-2.0, G[e], tn[rt] + sn[e]), 0.0), inv_ell);
                }
                if constexpr (PREC == 2) {
                    bf16x4 Kh, Kl;
                    bf16_pair(Kv, Kh, Kl);
#pragma unroll
                    for (int rb = 0; rb < 2; ++rb) {
                        if (rb >= nrb) continue;
                        // the two small cross terms first, then the leading product
                        Y[rt][rb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(Kl, Mh[rb], Y[rt][rb], 0, 0, 0);
                        Y[rt][rb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(Kh, Ml[rb], Y[rt][rb], 0, 0, 0);
                        Y[rt][rb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(Kh, Mh[rb], Y[rt][rb], 0, 0, 0);
                    }
                } else {
#pragma unroll
                    for (int rb = 0; rb < 2; ++rb) {
                        if (rb >= nrb) continue;
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            if constexpr (LP)
                                Y[rt][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(Kv[e], Mq[rb][e], Y[rt][rb], 0, 0, 0);
                            else
                                Y[rt][rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(Kv[e], Mq[rb][e], Y[rt][rb], 0, 0, 0);
                        }
                    }
                }
            }
        }
    }
    // output element v of lane (r + 16 g): target node 4g + v (PREC 1, 2) or 4v + g (FP64), rhs r
    for (int ww = 0; ww < 4; ++ww) {
        if (w == ww) {
#pragma unroll
            for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int a = 16 * rt + (LP ? 4 * lg + v : 4 * v + lg), r = 16 * rb + li;
                        const double val = (double)Y[rt][rb][v];
                        part[a * 33 + r] = ww == 0 ? val : part[a * 33 + r] + val;
                    }
        }
        __syncthreads();
    }
    for (int p = tid; p < nx * nrhs; p += 256) {
        const int a = p / nrhs, r = p % nrhs;
        O.L[(size_t)c * nx * nrhs + p] = part[a * 33 + r];
    }
}

template <int KIND, int PREC>
void launch_m2l_mrhs_k(const DevTree &T, const DevOp &O, int first, int cnt, int nrhs, hipStream_t st)
{
    switch ((T.d + 3) / 4 * 4) {
#define DWFMM_M2LR(D) \
    case D: hipLaunchKernelGGL((m2l_mrhs_kernel<KIND, D, PREC>), dim3(cnt), dim3(256), 0, st, T, O, first, nrhs); break;
        DWFMM_M2LR(4) DWFMM_M2LR(8) DWFMM_M2LR(12) DWFMM_M2LR(16) DWFMM_M2LR(20) DWFMM_M2LR(24) DWFMM_M2LR(28)
    default:
        DWFMM_M2LR(32)
#undef DWFMM_M2LR
    }
}

// M2L for one rhs in FP32: FP32 Gram tiles of the node pairs, FP32 kernel values and sums.
// Same list classes, WPC layout and fixed-order class sum as the FP64 version.
template <int KIND, int DK, int NXT, int WPC>
__device__ __forceinline__ void m2l_mfma32_body(const DevTree &T, const DevOp &O, int c, bool valid, float *part)
{
    constexpr int NKC = DK / 4, NXP = 16 * NXT, RPW = 4 / WPC;
    const int nx = O.nx;
    const int tid = threadIdx.x, lane = tid & 63, wi = (tid >> 6) % WPC, lt = tid % (64 * WPC);
    const int li = lane & 15, lg = lane >> 4;
    const int f0 = valid ? T.Fptr[c] : 0, f1 = valid ? T.Fptr[c + 1] : 0;
    const float inv_ell = (float)(1.0 / O.ell);
    const double *tnode = O.nodesT + (size_t)(valid ? c : 0) * DK * NXP;
    float A[NXT][NKC], tn[NXT][4], racc[RPW][NXT][4];
#pragma unroll
    for (int rt = 0; rt < NXT; ++rt) {
#pragma unroll
        for (int kc = 0; kc < NKC; ++kc) A[rt][kc] = (float)tnode[(4 * kc + lg) * NXP + 16 * rt + li];
#pragma unroll
        for (int v = 0; v < 4; ++v) tn[rt][v] = (float)O.nnorm[(size_t)(valid ? c : 0) * NXP + 16 * rt + 4 * lg + v];
    }
#pragma unroll
    for (int k = 0; k < RPW; ++k)
#pragma unroll
        for (int rt = 0; rt < NXT; ++rt)
#pragma unroll
            for (int v = 0; v < 4; ++v) racc[k][rt][v] = 0.0f;
    for (int base = f0 + wi; base < f1; base += 4) {
#pragma unroll
        for (int k = 0; k < RPW; ++k) {
            const int f = base + k * WPC;
            if (f >= f1) break;
            const int s = T.Fsrc[f];
            const double *snode = O.nodesT + (size_t)s * DK * NXP;
#pragma unroll
            for (int ct = 0; ct < NXT; ++ct) {
                const int b = 16 * ct + li;
                float B[NKC];
#pragma unroll
                for (int kc = 0; kc < NKC; ++kc) B[kc] = (float)snode[(4 * kc + lg) * NXP + b];
                const float nb = (float)O.nnorm[(size_t)s * NXP + b];
                const float mb = b < nx ? (float)O.M[(size_t)s * nx + b] : 0.0f;
#pragma unroll
                for (int rt = 0; rt < NXT; ++rt) {
                    flt4 G = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                    for (int kc = 0; kc < NKC; ++kc) G = __builtin_amdgcn_mfma_f32_16x16x4f32(A[rt][kc], B[kc], G, 0, 0, 0);
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const float r2 = fmaxf(fmaf(-2.0f, G[v], tn[rt][v] + nb), 0.0f);
                        racc[k][rt][v] = fmaf(kernel_f32<KIND>(r2, inv_ell), mb, racc[k][rt][v]);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < RPW; ++k)
#pragma unroll
        for (int rt = 0; rt < NXT; ++rt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                float s = racc[k][rt][v];
                s += __shfl_xor(s, 1, 64);
                s += __shfl_xor(s, 2, 64);
                s += __shfl_xor(s, 4, 64);
                s += __shfl_xor(s, 8, 64);
                if (li == 0) part[(wi + k * WPC) * NXP + 16 * rt + 4 * lg + v] = s;
            }
    __syncthreads();
    if (valid && lt < nx)
        O.L[(size_t)c * nx + lt] = (double)(((part[lt] + part[NXP + lt]) + part[2 * NXP + lt]) + part[3 * NXP + lt]);
}

template <int KIND, int DK, int NXT>
__global__ __launch_bounds__(256) void m2l_mfma32_kernel(DevTree T, DevOp O, int first)
{
    __shared__ float part[4 * 16 * NXT];
    m2l_mfma32_body<KIND, DK, NXT, 4>(T, O, first + blockIdx.x, true, part);
}

template <int KIND, int DK>
void launch_m2l32_d(const DevTree &T, const DevOp &O, int first, int cnt, hipStream_t st)
{
    switch (O.nxp / 16) {
    case 1: hipLaunchKernelGGL((m2l_mfma32_kernel<KIND, DK, 1>), dim3(cnt), dim3(256), 0, st, T, O, first); break;
    case 2: hipLaunchKernelGGL((m2l_mfma32_kernel<KIND, DK, 2>), dim3(cnt), dim3(256), 0, st, T, O, first); break;
    case 3: hipLaunchKernelGGL((m2l_mfma32_kernel<KIND, DK, 3>), dim3(cnt), dim3(256), 0, st, T, O, first); break;
    default: hipLaunchKernelGGL((m2l_mfma32_kernel<KIND, DK, 4>), dim3(cnt), dim3(256), 0, st, T, O, first); break;
    }
}

template <int KIND>
void launch_m2l32_k(const DevTree &T, const DevOp &O, int first, int cnt, hipStream_t st)
{
    switch ((T.d + 3) / 4 * 4) {
    case 4: launch_m2l32_d<KIND, 4>(T, O, first, cnt, st); break;
    case 8: launch_m2l32_d<KIND, 8>(T, O, first, cnt, st); break;
    case 12: launch_m2l32_d<KIND, 12>(T, O, first, cnt, st); break;
    case 16: launch_m2l32_d<KIND, 16>(T, O, first, cnt, st); break;
    case 20: launch_m2l32_d<KIND, 20>(T, O, first, cnt, st); break;
    case 24: launch_m2l32_d<KIND, 24>(T, O, first, cnt, st); break;
    case 28: launch_m2l32_d<KIND, 28>(T, O, first, cnt, st); break;
    default: launch_m2l32_d<KIND, 32>(T, O, first, cnt, st); break;
    }
}

// ---------------------------------------------------------------- batches of problems
// Every batched kernel reads (item, local block) from a work list and runs the same body
// as the single-problem kernel on that item's tree and operator.
__global__ __launch_bounds__(256) void p2m_batch_kernel(const BatchItem *items, const double *const *xs,
                                                        const int2 *work)
{
    __shared__ double xl[kSymLeaf];
    const int2 wk = work[blockIdx.x];
    if (wk.x < 0) return;
    const BatchItem &B = items[wk.x];
    p2m_body(B.T, B.O, wk.y, xs[wk.x], 1, B.far, xl);
}

__global__ __launch_bounds__(64) void m2m_batch_kernel(const BatchItem *items, const int2 *work)
{
    const int2 wk = work[blockIdx.x];
    if (wk.x < 0) return;
    m2m_body(items[wk.x].T, items[wk.x].O, wk.y, 1);
}

__global__ __launch_bounds__(64) void l2l_batch_kernel(const BatchItem *items, const int2 *work)
{
    const int2 wk = work[blockIdx.x];
    if (wk.x < 0) return;
    l2l_body(items[wk.x].T, items[wk.x].O, wk.y, 1);
}

// 4 / WPC clusters of the work list per workgroup and pass; slots past the end or on padding
// idle through the barrier.  A grid smaller than the list (the persistent layout) strides over
// it, the same for every thread of a workgroup; a barrier separates the passes, since a pass
// reuses the partial sums of the previous one.  Which workgroup takes an entry does not change
// its arithmetic, so both layouts give the same bits.
template <int KIND, int DK, int NXT, int WPC>
__global__ __launch_bounds__(256) void m2l_batch_kernel(const BatchItem *items, const int2 *work, int cnt)
{
    constexpr int CPB = 4 / WPC;
    __shared__ double part[CPB][4 * 16 * NXT];
    const int slot = (threadIdx.x >> 6) / WPC;
    for (int base = blockIdx.x * CPB; base < cnt; base += gridDim.x * CPB) {
        if (base != (int)blockIdx.x * CPB) __syncthreads();
        const int q = base + slot;
        const int2 wk = q < cnt ? work[q] : make_int2(-1, 0);
        const bool valid = wk.x >= 0;
        const BatchItem &I = items[valid ? wk.x : 0];
        m2l_mfma_body<KIND, DK, NXT, WPC>(I.T, I.O, I.O, wk.y, valid, part[slot]);
    }
}

template <int KIND, int DK, int NXT, int WPC>
__global__ __launch_bounds__(256) void m2l32_batch_kernel(const BatchItem *items, const int2 *work, int cnt)
{
    constexpr int CPB = 4 / WPC;
    __shared__ float part[CPB][4 * 16 * NXT];
    const int slot = (threadIdx.x >> 6) / WPC;
    for (int base = blockIdx.x * CPB; base < cnt; base += gridDim.x * CPB) {
        if (base != (int)blockIdx.x * CPB) __syncthreads();
        const int q = base + slot;
        const int2 wk = q < cnt ? work[q] : make_int2(-1, 0);
        const bool valid = wk.x >= 0;
        const BatchItem &I = items[valid ? wk.x : 0];
        m2l_mfma32_body<KIND, DK, NXT, WPC>(I.T, I.O, wk.y, valid, part[slot]);
    }
}

template <int KIND, int DK, bool FP32>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(FP32 ? (KIND == kGaussSplit && DK <= 20 ? 4 : (DK <= 20 || (KIND != kGaussSplit && DK <= 24) ? 3 : 1)) : sym_waves<KIND, DK>(), 8)))
void p2p_sym_batch_kernel(const BatchItem *items, const int2 *work)
{
    const int2 wk = work[blockIdx.x];
    if (wk.x < 0) return;
    if constexpr (FP32)
        p2p_sym32_body<KIND, DK>(items[wk.x].T, items[wk.x].O, wk.y);
    else
        p2p_sym_body<KIND, DK>(items[wk.x].T, items[wk.x].O, wk.y);
}

__global__ __launch_bounds__(kSymLeaf) void combine_batch_kernel(const BatchItem *items, double *const *ys,
                                                                 const int2 *work)
{
    const int2 wk = work[blockIdx.x];
    if (wk.x < 0) return;
    combine_body(items[wk.x].T, items[wk.x].O, wk.y, ys[wk.x], 1, items[wk.x].far);
}

template <int KIND, int DK, int NXT>
void launch_m2l_batch_x(const BatchPlan &P, const BatchLaunch &L, hipStream_t st)
{
    const int2 *w = P.work + L.off;
    // workgroups: one per 4 / W entries, or at most L.grid in the persistent layout
#define DWFMM_MW(W)                                                                                         \
    case W: {                                                                                               \
        const int groups = (L.cnt + 4 / W - 1) / (4 / W);                                                   \
        const int nwg = L.grid > 0 && L.grid < groups ? L.grid : groups;                                    \
        if (L.prec != 0)                                                                                    \
            hipLaunchKernelGGL((m2l32_batch_kernel<KIND, DK, NXT, W>), dim3(nwg), dim3(256), 0, st, P.items, \
                               w, L.cnt);                                                                   \
        else                                                                                                \
            hipLaunchKernelGGL((m2l_batch_kernel<KIND, DK, NXT, W>), dim3(nwg), dim3(256), 0, st, P.items,   \
                               w, L.cnt);                                                                   \
        break;                                                                                              \
    }
    if constexpr (NXT <= 2) {
        switch (L.wpc) {
            DWFMM_MW(1) DWFMM_MW(2)
        default:
            DWFMM_MW(4)
        }
    } else {
        switch (L.wpc) {
            DWFMM_MW(2)
        default:
            DWFMM_MW(4)
        }
    }
#undef DWFMM_MW
}

template <int KIND, int DK>
void launch_m2l_batch_d(const BatchPlan &P, const BatchLaunch &L, hipStream_t st)
{
    switch (L.nxt) {
    case 1: launch_m2l_batch_x<KIND, DK, 1>(P, L, st); break;
    case 2: launch_m2l_batch_x<KIND, DK, 2>(P, L, st); break;
    case 3: launch_m2l_batch_x<KIND, DK, 3>(P, L, st); break;
    default: launch_m2l_batch_x<KIND, DK, 4>(P, L, st); break;
    }
}

template <int KIND>
void launch_m2l_batch_k(const BatchPlan &P, const BatchLaunch &L, hipStream_t st)
{
    switch (L.dk) {
    case 4: launch_m2l_batch_d<KIND, 4>(P, L, st); break;
    case 8: launch_m2l_batch_d<KIND, 8>(P, L, st); break;
    case 12: launch_m2l_batch_d<KIND, 12>(P, L, st); break;
    case 16: launch_m2l_batch_d<KIND, 16>(P, L, st); break;
    case 20: launch_m2l_batch_d<KIND, 20>(P, L, st); break;
    case 24: launch_m2l_batch_d<KIND, 24>(P, L, st); break;
    case 28: launch_m2l_batch_d<KIND, 28>(P, L, st); break;
    default: launch_m2l_batch_d<KIND, 32>(P, L, st); break;
    }
}

template <int KIND, bool FP32>
void launch_p2p_batch_k(const BatchPlan &P, const BatchLaunch &L, hipStream_t st)
{
    const int2 *w = P.work + L.off;
    switch (L.dk) {
#define DWFMM_PB(D) \
    case D: hipLaunchKernelGGL((p2p_sym_batch_kernel<KIND, D, FP32>), dim3(L.cnt), dim3(256), 0, st, P.items, w); break;
        DWFMM_PB(4) DWFMM_PB(8) DWFMM_PB(12) DWFMM_PB(16) DWFMM_PB(20) DWFMM_PB(24) DWFMM_PB(28)
    default:
        DWFMM_PB(32)
#undef DWFMM_PB
    }
}

// ---------------------------------------------------------------- deterministic dot products
// Partial inner products of the columns of a and b (n rows of nrhs <= 32 values, row-major).
// Block blockIdx.x takes rows [i0, i1); thread t handles column r = t mod nrhs in the row group
// g = t / nrhs, rows i0 + g + G k, with G the largest power of two <= 256 / nrhs, so the G nrhs
// active threads of a block read consecutive addresses.  The G group sums of each column are
// added by a fixed pairwise tree in LDS: the result depends only on n, nrhs and the grid.
__global__ __launch_bounds__(256) void dot_partial_kernel(const double *__restrict__ a, const double *__restrict__ b,
                                                          int n, int nrhs, double *__restrict__ partial)
{
    __shared__ double red[256];
    int G = 1;
    while (2 * G * nrhs <= 256) G *= 2;
    const int t = threadIdx.x, r = t % nrhs, g = t / nrhs;
    const int chunk = (n + gridDim.x - 1) / gridDim.x;
    const int i0 = blockIdx.x * chunk, i1 = min(n, i0 + chunk);
    double s0 = 0.0, s1 = 0.0;
    if (g < G) {
        int i = i0 + g;
        for (; i + G < i1; i += 2 * G) {
            s0 = fma(a[(size_t)i * nrhs + r], b[(size_t)i * nrhs + r], s0);
            s1 = fma(a[(size_t)(i + G) * nrhs + r], b[(size_t)(i + G) * nrhs + r], s1);
        }
        if (i < i1) s0 = fma(a[(size_t)i * nrhs + r], b[(size_t)i * nrhs + r], s0);
    }
    red[t] = s0 + s1;
    for (int h = G / 2; h > 0; h >>= 1) {
        __syncthreads();
        if (g < h) red[t] += red[t + h * nrhs];
    }
    if (t < nrhs) partial[(size_t)blockIdx.x * nrhs + t] = red[t];
}

// out[r] = sum over blocks of partial[b][r]: one workgroup per column, thread t adds the blocks
// t, t + 256, ... in order, then a fixed pairwise tree over the 256 threads.
__global__ __launch_bounds__(256) void dot_final_kernel(const double *__restrict__ partial, int nblocks, int nrhs,
                                                        double *__restrict__ out)
{
    __shared__ double red[256];
    const int r = blockIdx.x, t = threadIdx.x;
    double s = 0.0;
    for (int b = t; b < nblocks; b += 256) s += partial[(size_t)b * nrhs + r];
    red[t] = s;
    for (int h = 128; h > 0; h >>= 1) {
        __syncthreads();
        if (t < h) red[t] += red[t + h];
    }
    if (t == 0) out[r] = red[0];
}

// ---------------------------------------------------------------- CG steps for one-rhs problems
// Sum of u_i v_i over rows [i0, i1) in the order of dot_partial_kernel with one column: thread t
// takes rows i0 + t + 256 k into two alternating accumulators, then a fixed pairwise tree over the
// 256 threads.  term(i, u, v) yields the factors of row i and may update vectors first (a row is
// visited by one thread only).  The sum is valid in thread 0.
template <class Term>
__device__ __forceinline__ double block_dot1(int i0, int i1, double *red, Term term)
{
    const int t = threadIdx.x;
    double s0 = 0.0, s1 = 0.0, u, v;
    int i = i0 + t;
    for (; i + 256 < i1; i += 512) {
        term(i, u, v);
        s0 = fma(u, v, s0);
        term(i + 256, u, v);
        s1 = fma(u, v, s1);
    }
    if (i < i1) {
        term(i, u, v);
        s0 = fma(u, v, s0);
    }
    red[t] = s0 + s1;
    for (int h = 128; h > 0; h >>= 1) {
        __syncthreads();
        if (t < h) red[t] += red[t + h];
    }
    return red[0];
}

// The blocks' partial sums of one problem, added as dot_final_kernel adds them (valid in thread 0).
__device__ __forceinline__ double final_dot1(const double *partial, int nblk, double *red)
{
    const int t = threadIdx.x;
    double s = 0.0;
    for (int b = t; b < nblk; b += 256) s += partial[b];
    red[t] = s;
    for (int h = 128; h > 0; h >>= 1) {
        __syncthreads();
        if (t < h) red[t] += red[t + h];
    }
    return red[0];
}

__global__ __launch_bounds__(256) void dot1_partial_kernel(const double *__restrict__ a, const double *__restrict__ b,
                                                           int n, double *__restrict__ partial)
{
    __shared__ double red[256];
    const int chunk = (n + gridDim.x - 1) / gridDim.x;
    const int i0 = blockIdx.x * chunk, i1 = min(n, i0 + chunk);
    const double s = block_dot1(i0, i1, red, [&](int i, double &u, double &v) {
        u = a[i];
        v = b[i];
    });
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__device__ __forceinline__ bool cg_stepping(const int32_t *state, int max_it)
{
    return state[0] == 0 && state[1] < max_it;
}

// Block steps: workgroup g takes block g - blk0 of the problem whose blocks contain g.
template <int STEP>
__global__ __launch_bounds__(256) void cg_block_kernel(const CgItem *__restrict__ items, int nitems, CgItem one)
{
    __shared__ double red[256];
    int k = 0;
    if (items) {
        int lo = 0, hi = nitems - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (items[mid].blk0 <= (int)blockIdx.x) lo = mid;
            else hi = mid - 1;
        }
        k = lo;
    }
    const CgItem &it = items ? items[k] : one;
    const int blk = (int)blockIdx.x - it.blk0;
    if (blk < 0 || blk >= it.nblk) return;
    const int i0 = blk * it.chunk, i1 = min(it.n, i0 + it.chunk);
    const double lam = it.lambda;
    double *x = it.x, *r = it.r, *p = it.p, *q = it.q;
    if (STEP == CG_START) {
        if (it.frozen) return;
        const double *b = it.b;
        if (it.zero_x)
            for (int i = i0 + threadIdx.x; i < i1; i += 256) {
                x[i] = 0.0;
                q[i] = 0.0;
            }
        const double s = block_dot1(i0, i1, red, [&](int i, double &u, double &v) {
            double qi = q[i];
            if (lam != 0.0) {
                qi = fma(lam, x[i], qi);
                q[i] = qi;
            }
            const double ri = b[i] - qi;
            r[i] = ri;
            p[i] = ri;
            u = ri;
            v = ri;
        });
        if (threadIdx.x == 0) it.partial[blk] = s;
        __syncthreads();
        const double s2 = block_dot1(i0, i1, red, [&](int i, double &u, double &v) {
            u = b[i];
            v = b[i];
        });
        if (threadIdx.x == 0) it.partial[kDotBlocks + blk] = s2;
    } else if (STEP == CG_PQ) {
        if (!cg_stepping(it.state, it.max_it)) return;
        const double s = block_dot1(i0, i1, red, [&](int i, double &u, double &v) {
            double qi = q[i];
            if (lam != 0.0) {
                qi = fma(lam, p[i], qi);
                q[i] = qi;
            }
            u = p[i];
            v = qi;
        });
        if (threadIdx.x == 0) it.partial[blk] = s;
    } else if (STEP == CG_XR) {
        if (!cg_stepping(it.state, it.max_it)) return;
        const double a = it.scal[4];
        const double s = block_dot1(i0, i1, red, [&](int i, double &u, double &v) {
            x[i] = fma(a, p[i], x[i]);
            const double ri = fma(-a, q[i], r[i]);
            r[i] = ri;
            u = ri;
            v = ri;
        });
        if (threadIdx.x == 0) it.partial[blk] = s;
    } else if (STEP == CG_P) {
        if (it.state[0] != 0) return;
        const double beta = it.scal[5];
        for (int i = i0 + threadIdx.x; i < i1; i += 256) p[i] = fma(beta, p[i], r[i]);
    } else if (STEP == CG_RES) {
        if (it.frozen) return;
        const double *f = it.f, *vv = it.v;
        double *out = it.out;
        const double s = block_dot1(i0, i1, red, [&](int i, double &u, double &v) {
            double o = out[i];
            if (lam != 0.0) o = fma(lam, vv[i], o);
            o = f[i] - o;
            out[i] = o;
            u = o;
            v = o;
        });
        if (threadIdx.x == 0) it.partial[blk] = s;
    } else if (STEP == CG_ADD) {
        if (it.frozen) return;
        double *acc = it.acc;
        for (int i = i0 + threadIdx.x; i < i1; i += 256) acc[i] = acc[i] + x[i];
    } else if (STEP == CG_SUB) {
        if (it.frozen) return;
        double *acc = it.acc;
        for (int i = i0 + threadIdx.x; i < i1; i += 256) acc[i] = acc[i] - x[i];
    }
}

// Problem steps: workgroup k takes problem k.
template <int STEP>
__global__ __launch_bounds__(256) void cg_item_kernel(const CgItem *__restrict__ items, CgItem one)
{
    __shared__ double red[256];
    const CgItem &it = items ? items[blockIdx.x] : one;
    double *scal = it.scal;
    int32_t *state = it.state;
    const int t = threadIdx.x;
    if (STEP == CG_START_SUM) {
        if (it.frozen) {
            if (t == 0) {
                state[0] = 3;
                state[1] = 0;
                state[2] = 0;
            }
            return;
        }
        const double rr = final_dot1(it.partial, it.nblk, red);
        __syncthreads();
        const double bb = final_dot1(it.partial + kDotBlocks, it.nblk, red);
        if (t == 0) {
            scal[0] = rr;
            scal[1] = bb;
            state[1] = 0;
            state[2] = 0;
            state[0] = sqrt(rr) <= it.rtol * sqrt(bb) ? 1 : 0;
        }
    } else if (STEP == CG_ALPHA) {
        if (!cg_stepping(state, it.max_it)) {
            if (t == 0) scal[4] = 0.0;
            return;
        }
        const double pq = final_dot1(it.partial, it.nblk, red);
        if (t == 0) {
            scal[2] = pq;
            double a = 0.0;
            if (!isfinite(pq) || fabs(pq) <= 1e-300) {
                state[0] = 2;
            } else {
                if (pq < 0.0) state[2] += 1;
                a = scal[0] / pq;
            }
            scal[4] = a;
        }
    } else if (STEP == CG_BETA) {
        if (!cg_stepping(state, it.max_it)) {
            if (t == 0) scal[5] = 0.0;
            return;
        }
        const double rrn = final_dot1(it.partial, it.nblk, red);
        if (t == 0) {
            scal[3] = rrn;
            scal[5] = rrn / scal[0];
            scal[0] = rrn;
            state[1] += 1;
            if (sqrt(rrn) <= it.rtol * sqrt(scal[1])) state[0] = 1;
        }
    } else if (STEP == CG_RES_SUM) {
        if (it.frozen) return;
        const double s = final_dot1(it.partial, it.nblk, red);
        if (t == 0) scal[8] = s;
    } else if (STEP == CG_MIRROR) {
        double *m = it.mirror;
        if (t < 3) m[t] = (double)state[t];
        else if (t == 3) m[3] = scal[0];
        else if (t == 4) m[4] = scal[1];
        else if (t == 5) m[5] = scal[8];
        else if (t == 6) m[6] = scal[9];
    }
}

}  // namespace

// The library compiles this file twice, in parallel: DWFMM_KERNELS_PART 1 holds the
// single-problem entry points, 2 the batched ones; each instantiates only the kernel
// templates it launches.  Without the macro both parts are compiled.
#if !defined(DWFMM_KERNELS_PART) || DWFMM_KERNELS_PART == 1
hipError_t launch_basis(const DevTree &T, int nx, const double *clo, const double *csc, const double *coff,
                        const int32_t *lidx, int nnz_max, const double *Vinv, int nleg, const int32_t *leg_axis,
                        const int32_t *leg_deg, double *Lb, hipStream_t stream)
{
    if (nx > kMaxNx || nleg > 128) return hipErrorInvalidValue;
    hipLaunchKernelGGL(basis_kernel, dim3(T.nleaf), dim3(64), 0, stream, T, nx, clo, csc, coff, lidx, nnz_max, Vinv,
                       nleg, leg_axis, leg_deg, Lb);
    return hipGetLastError();
}

hipError_t launch_matvec(const DevTree &T, const DevOp &O, const double *x, double *y, int nrhs, int parts,
                         int precision, hipStream_t main_st, const KernelTimer *timer, const StreamFork *fork)
{
    (void)precision;
    if (O.nx > kMaxNx || O.nx * T.dpad > kMaxNodeWords || nrhs > 32) return hipErrorInvalidValue;
    const int near = parts & 1;
    const int far = (parts & 2) && T.min_far_level <= T.J;
    // symmetric MFMA nearfield for one rhs, leaves <= 128 points, d <= 32, radial kernels
    const bool sym = nrhs == 1 && O.kind <= 2 && T.max_leaf <= kSymLeaf && T.d <= 32 && O.rowbuf && O.colbuf;
    // MFMA nearfield for several rhs (LDS of the FP64 kernel: at most 66 KB, at d <= 28 with two
    // 16-wide rhs tiles; gfx950 gives a workgroup up to 160 KB)
    const int dk = (T.d + 3) / 4 * 4;
    const bool mrhs = nrhs > 1 && O.kind <= 2 && T.max_leaf <= kSymLeaf && dk <= 32 && !(dk > 28 && nrhs > 16);
    if (nrhs > 1 && T.max_leaf * nrhs <= 4096)
        hipLaunchKernelGGL(p2m_multi_kernel, dim3(T.nleaf), dim3(256), sizeof(double) * T.max_leaf * nrhs, main_st, T,
                           O, x, nrhs, far);
    else
        hipLaunchKernelGGL(p2m_kernel, dim3(T.nleaf), dim3(256), sizeof(double) * T.max_leaf, main_st, T, O, x, nrhs,
                           far);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the symmetric nearfield does not read the locals, nor does the several-rhs one when its L2P
    // is left to a later kernel: the farfield may run beside it (not while the caller's stream is
    // being captured into a graph, which then holds the serial order)
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (fork && fork->side && hipStreamIsCapturing(main_st, &cap) != hipSuccess) return hipGetLastError();
    const bool split = far && near && (sym || mrhs) && fork && fork->side && cap == hipStreamCaptureStatusNone;
    hipStream_t st = main_st;
    if (split) {
        if ((e = hipEventRecord(fork->forked, main_st)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(fork->side, fork->forked, 0)) != hipSuccess) return e;
        st = fork->side;
    }
    if (far) {
        for (int j = T.J - 1; j >= T.min_far_level; --j)
            hipLaunchKernelGGL(m2m_kernel, dim3(1 << j), dim3(64), 0, st, T, O, (1 << j) - 1, nrhs);
        const int first = (1 << T.min_far_level) - 1;
        const int cnt = T.ncl - first;
        if (timer) (void)hipEventRecord(timer->m2l_start, st);
        const bool mfma = nrhs == 1 && O.kind <= 2 && T.d <= 32 && O.nxp <= 64 && O.nodesT && O.nnorm;
        const bool mfma_r = nrhs > 1 && O.kind <= 2 && T.d <= 32 && O.nxp <= 32 && O.nodesT && O.nnorm;
        if (mfma_r) {
#define DWFMM_M2LR_PREC(K)                                                      \
    (precision == 0   ? launch_m2l_mrhs_k<K, 0>(T, O, first, cnt, nrhs, st)     \
     : precision == 1 ? launch_m2l_mrhs_k<K, 1>(T, O, first, cnt, nrhs, st)     \
                      : launch_m2l_mrhs_k<K, 2>(T, O, first, cnt, nrhs, st))
            switch (O.kind) {
            case 0: DWFMM_M2LR_PREC(0); break;
            case 1: DWFMM_M2LR_PREC(1); break;
            default: DWFMM_M2LR_PREC(2); break;
            }
#undef DWFMM_M2LR_PREC
        } else if (mfma && precision != 0) {
            switch (O.kind) {
            case 0: launch_m2l32_k<0>(T, O, first, cnt, st); break;
            case 1: launch_m2l32_k<1>(T, O, first, cnt, st); break;
            default: launch_m2l32_k<2>(T, O, first, cnt, st); break;
            }
        } else if (mfma) {
            switch (O.kind) {
            case 0: launch_m2l_mfma_k<0>(T, O, first, cnt, st); break;
            case 1: launch_m2l_mfma_k<1>(T, O, first, cnt, st); break;
            default: launch_m2l_mfma_k<2>(T, O, first, cnt, st); break;
            }
        } else {
            switch (O.kind) {
            case 0: hipLaunchKernelGGL(m2l_kernel<0>, dim3(cnt), dim3(256), 0, st, T, O, first, nrhs); break;
            case 1: hipLaunchKernelGGL(m2l_kernel<1>, dim3(cnt), dim3(256), 0, st, T, O, first, nrhs); break;
            case 2: hipLaunchKernelGGL(m2l_kernel<2>, dim3(cnt), dim3(256), 0, st, T, O, first, nrhs); break;
            default: hipLaunchKernelGGL(m2l_kernel<3>, dim3(cnt), dim3(256), 0, st, T, O, first, nrhs); break;
            }
        }
        if (timer) (void)hipEventRecord(timer->m2l_stop, st);
        for (int j = T.min_far_level + 1; j <= T.J; ++j)
            hipLaunchKernelGGL(l2l_kernel, dim3(1 << j), dim3(64), 0, st, T, O, (1 << j) - 1, nrhs);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (split && (e = hipEventRecord(fork->joined, fork->side)) != hipSuccess) return e;
    }
    st = main_st;
    if (timer) (void)hipEventRecord(timer->p2p_start, st);
    if (sym) {
        if (near && precision == 0) {
            switch (O.kind) {
            case 0: e = O.matern_in_range ? launch_sym_k<kMaternInRange>(T, O, st) : launch_sym_k<0>(T, O, st); break;
            case 1: e = O.gauss_split ? launch_sym_k<kGaussSplit>(T, O, st) : launch_sym_k<1>(T, O, st); break;
            default: e = launch_sym_k<2>(T, O, st); break;
            }
            if (e != hipSuccess) return e;
        } else if (near) {  // FP32 (and BF16, whose single-rhs product has nothing to put on the BF16 MFMA)
            switch (O.kind) {
            case 0: e = launch_sym32_k<0>(T, O, st); break;
            case 1: e = O.gauss_split32 ? launch_sym32_k<kGaussSplit>(T, O, st) : launch_sym32_k<1>(T, O, st); break;
            default: e = launch_sym32_k<2>(T, O, st); break;
            }
            if (e != hipSuccess) return e;
        }
        if (timer) (void)hipEventRecord(timer->p2p_stop, st);
        if (split && (e = hipStreamWaitEvent(st, fork->joined, 0)) != hipSuccess) return e;
        hipLaunchKernelGGL(p2p_combine_kernel, dim3(T.nleaf), dim3(kSymLeaf), 0, st, T, O, y, near, far);
        return hipGetLastError();
    }
    if (mrhs) {
        // split: the nearfield kernel writes the near part only; L2P adds the farfield after the join
        const int nfar = split ? 0 : far;
        if (precision == 0) {
            switch (O.kind) {
            case 0: e = launch_mrhs_k<0>(T, O, y, nrhs, near, nfar, st); break;
            case 1:
                e = O.gauss_split ? launch_mrhs_k<kGaussSplit>(T, O, y, nrhs, near, nfar, st)
                                  : launch_mrhs_k<1>(T, O, y, nrhs, near, nfar, st);
                break;
            default: e = launch_mrhs_k<2>(T, O, y, nrhs, near, nfar, st); break;
            }
        } else if (precision == 1) {
            switch (O.kind) {
            case 0: e = launch_mrhs_lp_k<0, false>(T, O, y, nrhs, near, nfar, st); break;
            case 1:
                e = O.gauss_split32 ? launch_mrhs_lp_k<kGaussSplit, false>(T, O, y, nrhs, near, nfar, st)
                                    : launch_mrhs_lp_k<1, false>(T, O, y, nrhs, near, nfar, st);
                break;
            default: e = launch_mrhs_lp_k<2, false>(T, O, y, nrhs, near, nfar, st); break;
            }
        } else {
            if (near && !O.xtb) return hipErrorInvalidValue;  // the BF16 charges are staged from xtb
            // BF16 tile cache: the first nearfield launch writes the tiles, later ones read them (not
            // inside a graph capture, whose launches run later than the host flag would say)
            DevOp Oc = O;
            Oc.near_cache_mode = 0;
            if (O.near_tiles && near) {
                hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
                if ((e = hipStreamIsCapturing(st, &cs)) != hipSuccess) return e;
                if (cs == hipStreamCaptureStatusNone) Oc.near_cache_mode = *O.near_filled ? 2 : 1;
            }
            switch (O.kind) {
            case 0: e = launch_mrhs_lp_k<0, true>(T, Oc, y, nrhs, near, nfar, st); break;
            case 1:
                e = O.gauss_split32 ? launch_mrhs_lp_k<kGaussSplit, true>(T, Oc, y, nrhs, near, nfar, st)
                                    : launch_mrhs_lp_k<1, true>(T, Oc, y, nrhs, near, nfar, st);
                break;
            default: e = launch_mrhs_lp_k<2, true>(T, Oc, y, nrhs, near, nfar, st); break;
            }
            if (e == hipSuccess && Oc.near_cache_mode == 1) *O.near_filled = 1;
        }
        if (timer) (void)hipEventRecord(timer->p2p_stop, st);
        if (e != hipSuccess || !split) return e;
        if ((e = hipStreamWaitEvent(st, fork->joined, 0)) != hipSuccess) return e;
        hipLaunchKernelGGL(l2p_add_kernel, dim3(T.nleaf), dim3(256), sizeof(double) * O.nx * nrhs, st, T, O, y, nrhs);
        return hipGetLastError();
    }
    switch (O.kind) {
    case 0: e = launch_p2p_k<0>(T, O, y, nrhs, near, far, st); break;
    case 1: e = launch_p2p_k<1>(T, O, y, nrhs, near, far, st); break;
    case 2: e = launch_p2p_k<2>(T, O, y, nrhs, near, far, st); break;
    default: e = launch_p2p_k<3>(T, O, y, nrhs, near, far, st); break;
    }
    if (timer) (void)hipEventRecord(timer->p2p_stop, st);
    return e;
}

#endif

#if !defined(DWFMM_KERNELS_PART) || DWFMM_KERNELS_PART == 2
hipError_t launch_batch_m2l(const BatchPlan &P, const BatchLaunch &L, hipStream_t st)
{
    switch (L.kind) {
    case 0: launch_m2l_batch_k<0>(P, L, st); break;
    case 1: launch_m2l_batch_k<1>(P, L, st); break;
    default: launch_m2l_batch_k<2>(P, L, st); break;
    }
    return hipGetLastError();
}

hipError_t launch_batch_matvec(const BatchPlan &P, hipStream_t st, const StreamFork *fork)
{
    if (P.leaf_cnt == 0) return hipSuccess;
    hipLaunchKernelGGL(p2m_batch_kernel, dim3(P.leaf_cnt), dim3(256), 0, st, P.items, P.xs, P.work + P.leaf_off);
    // the farfield (moments, coupling, locals) only reads the charges P2M wrote and writes the
    // moments and locals, the nearfield only the row and column sums: with a fork the farfield
    // runs on the side stream beside the nearfield and is joined before the combine
    const bool forked = fork && fork->side && (!P.m2m.empty() || !P.m2l.empty() || !P.l2l.empty());
    hipStream_t fs = st;
    if (forked) {
        hipError_t e = hipEventRecord(fork->forked, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(fork->side, fork->forked, 0);
        if (e != hipSuccess) return e;
        fs = fork->side;
    }
    for (auto &lv : P.m2m)
        hipLaunchKernelGGL(m2m_batch_kernel, dim3(lv.second), dim3(64), 0, fs, P.items, P.work + lv.first);
    for (auto &L : P.m2l) (void)launch_batch_m2l(P, L, fs);
    for (auto &lv : P.l2l)
        hipLaunchKernelGGL(l2l_batch_kernel, dim3(lv.second), dim3(64), 0, fs, P.items, P.work + lv.first);
    if (forked) {
        hipError_t e = hipEventRecord(fork->joined, fs);
        if (e != hipSuccess) return e;
    }
    for (auto &L : P.p2p) {
        const bool lp = L.prec != 0;
        switch (L.kind) {
        case 0: lp ? launch_p2p_batch_k<0, true>(P, L, st) : launch_p2p_batch_k<0, false>(P, L, st); break;
        case 1: lp ? launch_p2p_batch_k<1, true>(P, L, st) : launch_p2p_batch_k<1, false>(P, L, st); break;
        case kGaussSplit:
            lp ? launch_p2p_batch_k<kGaussSplit, true>(P, L, st) : launch_p2p_batch_k<kGaussSplit, false>(P, L, st);
            break;
        case kMaternInRange:  // FP64 only (the reduced-precision plan keys Matern as kind 0)
            lp ? launch_p2p_batch_k<0, true>(P, L, st) : launch_p2p_batch_k<kMaternInRange, false>(P, L, st);
            break;
        default: lp ? launch_p2p_batch_k<2, true>(P, L, st) : launch_p2p_batch_k<2, false>(P, L, st); break;
        }
    }
    if (forked) {
        hipError_t e = hipStreamWaitEvent(st, fork->joined, 0);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(combine_batch_kernel, dim3(P.leaf_cnt), dim3(kSymLeaf), 0, st, P.items, P.ys,
                       P.work + P.leaf_off);
    return hipGetLastError();
}

#endif

#if !defined(DWFMM_KERNELS_PART) || DWFMM_KERNELS_PART == 1
hipError_t launch_eval(const DevTree &Tt, const DevOp &Ot, const DevTree &Ts, const DevOp &Os, const double *x,
                       double *y, int nrhs, hipStream_t st)
{
    if (Os.nx > kMaxNx || Os.nx * Ts.dpad > kMaxNodeWords || nrhs > 32 || Tt.dpad != Ts.dpad)
        return hipErrorInvalidValue;
    const int far = Tt.min_far_level <= Tt.J;
    // source side: charges into tree order and, if needed, moments up to the first cross-farfield level
    hipLaunchKernelGGL(p2m_kernel, dim3(Ts.nleaf), dim3(256), sizeof(double) * Ts.max_leaf, st, Ts, Os, x, nrhs, far);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (far) {
        for (int j = Ts.J - 1; j >= Tt.min_far_level; --j)
            hipLaunchKernelGGL(m2m_kernel, dim3(1 << j), dim3(64), 0, st, Ts, Os, (1 << j) - 1, nrhs);
        const int first = (1 << Tt.min_far_level) - 1;
        const int cnt = Tt.ncl - first;
        // one rhs, radial kernels, d <= 32, n_x <= 64: node-pair distances on FP64 MFMA
        const bool mfma = nrhs == 1 && Os.kind <= 2 && Tt.d <= 32 && Os.nxp <= 64 && Ot.nodesT && Ot.nnorm &&
                          Os.nodesT && Os.nnorm;
        if (mfma) switch (Os.kind) {
        case 0: launch_m2l_cross_mfma_k<0>(Tt, Ot, Os, first, cnt, st); break;
        case 1: launch_m2l_cross_mfma_k<1>(Tt, Ot, Os, first, cnt, st); break;
        default: launch_m2l_cross_mfma_k<2>(Tt, Ot, Os, first, cnt, st); break;
        }
        else switch (Os.kind) {
        case 0: hipLaunchKernelGGL(m2l_cross_kernel<0>, dim3(cnt), dim3(256), 0, st, Tt, Ot, Os, first, nrhs); break;
        case 1: hipLaunchKernelGGL(m2l_cross_kernel<1>, dim3(cnt), dim3(256), 0, st, Tt, Ot, Os, first, nrhs); break;
        case 2: hipLaunchKernelGGL(m2l_cross_kernel<2>, dim3(cnt), dim3(256), 0, st, Tt, Ot, Os, first, nrhs); break;
        default: hipLaunchKernelGGL(m2l_cross_kernel<3>, dim3(cnt), dim3(256), 0, st, Tt, Ot, Os, first, nrhs); break;
        }
        for (int j = Tt.min_far_level + 1; j <= Tt.J; ++j)
            hipLaunchKernelGGL(l2l_kernel, dim3(1 << j), dim3(64), 0, st, Tt, Ot, (1 << j) - 1, nrhs);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // one rhs, radial kernels, target leaves of at most kSymLeaf points, d <= 32: MFMA nearfield
    if (nrhs == 1 && Os.kind <= 2 && Tt.max_leaf <= kSymLeaf && Tt.dpad <= 32) {
        switch (Os.kind) {
        case 0: return launch_cross_mfma_k<0>(Tt, Ot, Ts, Os.xt, y, far, st);
        case 1:
            return Ot.gauss_split ? launch_cross_mfma_k<kGaussSplit>(Tt, Ot, Ts, Os.xt, y, far, st)
                                  : launch_cross_mfma_k<1>(Tt, Ot, Ts, Os.xt, y, far, st);
        default: return launch_cross_mfma_k<2>(Tt, Ot, Ts, Os.xt, y, far, st);
        }
    }
    switch (Os.kind) {
    case 0: return launch_p2p_cross_k<0>(Tt, Ot, Ts, Os.xt, y, nrhs, far, st);
    case 1: return launch_p2p_cross_k<1>(Tt, Ot, Ts, Os.xt, y, nrhs, far, st);
    case 2: return launch_p2p_cross_k<2>(Tt, Ot, Ts, Os.xt, y, nrhs, far, st);
    default: return launch_p2p_cross_k<3>(Tt, Ot, Ts, Os.xt, y, nrhs, far, st);
    }
}

hipError_t launch_dot(const double *a, const double *b, int n, int nrhs, double *partial, double *out,
                      hipStream_t stream)
{
    if (nrhs < 1 || nrhs > 256) return hipErrorInvalidValue;
    // at least 4096 values per block, at most kDotBlocks blocks (the partial buffer's rows)
    const int64_t vals = (int64_t)n * nrhs;
    const int nblk = (int)std::max<int64_t>(1, std::min<int64_t>(kDotBlocks, (vals + 4095) / 4096));
    if (nrhs == 1)
        hipLaunchKernelGGL(dot1_partial_kernel, dim3(nblk), dim3(256), 0, stream, a, b, n, partial);
    else
        hipLaunchKernelGGL(dot_partial_kernel, dim3(nblk), dim3(256), 0, stream, a, b, n, nrhs, partial);
    hipLaunchKernelGGL(dot_final_kernel, dim3(nrhs), dim3(256), 0, stream, partial, nblk, nrhs, out);
    return hipGetLastError();
}

hipError_t launch_cg(int step, const CgItem *items, int nitems, int nblocks, const CgItem &one, hipStream_t stream)
{
    if (!items) {
        nitems = 1;
        nblocks = one.nblk;
    }
    if (nitems < 1 || nblocks < 1) return hipErrorInvalidValue;
    const dim3 blocks(nblocks), probs(nitems), th(256);
    switch (step) {
    case CG_START: hipLaunchKernelGGL(cg_block_kernel<CG_START>, blocks, th, 0, stream, items, nitems, one); break;
    case CG_PQ: hipLaunchKernelGGL(cg_block_kernel<CG_PQ>, blocks, th, 0, stream, items, nitems, one); break;
    case CG_XR: hipLaunchKernelGGL(cg_block_kernel<CG_XR>, blocks, th, 0, stream, items, nitems, one); break;
    case CG_P: hipLaunchKernelGGL(cg_block_kernel<CG_P>, blocks, th, 0, stream, items, nitems, one); break;
    case CG_RES: hipLaunchKernelGGL(cg_block_kernel<CG_RES>, blocks, th, 0, stream, items, nitems, one); break;
    case CG_ADD: hipLaunchKernelGGL(cg_block_kernel<CG_ADD>, blocks, th, 0, stream, items, nitems, one); break;
    case CG_SUB: hipLaunchKernelGGL(cg_block_kernel<CG_SUB>, blocks, th, 0, stream, items, nitems, one); break;
    case CG_START_SUM: hipLaunchKernelGGL(cg_item_kernel<CG_START_SUM>, probs, th, 0, stream, items, one); break;
    case CG_ALPHA: hipLaunchKernelGGL(cg_item_kernel<CG_ALPHA>, probs, th, 0, stream, items, one); break;
    case CG_BETA: hipLaunchKernelGGL(cg_item_kernel<CG_BETA>, probs, th, 0, stream, items, one); break;
    case CG_RES_SUM: hipLaunchKernelGGL(cg_item_kernel<CG_RES_SUM>, probs, th, 0, stream, items, one); break;
    case CG_MIRROR: hipLaunchKernelGGL(cg_item_kernel<CG_MIRROR>, probs, th, 0, stream, items, one); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

#endif

}  // namespace dwfmm
