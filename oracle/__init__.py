"""FP64 CPU oracle for the dimension weighted FMM -- TEST INFRASTRUCTURE ONLY.

This package wraps ``dwfmm_oracle.c`` (plain C, FP64, OpenMP) through ctypes.
It is the independent reference the GPU library is checked against.  Only the
test suite, the smoke entry point and the benchmark's CPU-baseline leg may use
it; the GPU library never imports, links or calls anything in here, and this
package never imports the GPU library.

Each function cites the part of the paper (arXiv 2402.09531) it follows; the
C file header lists the readings taken where the paper is silent.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dwfmm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MATERN32, GAUSSIAN, EXPONENTIAL, POLY = 0, 1, 2, 3
KERNELS = {"matern32": MATERN32, "gaussian": GAUSSIAN, "exponential": EXPONENTIAL, "poly": POLY}
W_R1, W_R2, W_R3, W_EXPLICIT, W_THM = 0, 1, 2, 3, 4


def compile_source(src: str, out: str) -> None:
    """gcc with the oracle's flags (FP64, no fast-math): C source -> shared library."""
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", out, src, "-lm"])


def build(force: bool = False) -> str:
    """Compile the oracle in place (when its source is newer than the library)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        compile_source(_SRC, tmp)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        # a test that plants a mistake in a copy of the C source names that copy's library here
        path = os.environ.get("DWFMM_ORACLE_LIB") or build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        lp = C.POINTER(C.c_long)
        up = C.POINTER(C.c_ubyte)
        L.orc_kernel.restype = C.c_double
        L.orc_kernel.argtypes = [C.c_int, C.c_double, C.c_int, dp, dp]
        L.orc_weights.restype = C.c_int
        L.orc_weights.argtypes = [C.c_int, C.c_int, dp, C.c_double, dp, dp]
        L.orc_index_set.restype = C.c_long
        L.orc_index_set.argtypes = [C.c_int, dp, C.c_double, C.c_int, up, C.c_long]
        L.orc_axis_nodes.restype = None
        L.orc_axis_nodes.argtypes = [C.c_int, dp]
        L.orc_legendre.restype = C.c_double
        L.orc_legendre.argtypes = [C.c_int, C.c_double]
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [dp, C.c_long, C.c_int, dp, C.c_int, C.c_double, C.c_int, C.c_double,
                                 C.c_double, C.c_int, dp]
        L.orc_create_ex.restype = C.c_void_p
        L.orc_create_ex.argtypes = [dp, C.c_long, C.c_int, dp, C.c_int, C.c_double, C.c_int, C.c_double,
                                    C.c_double, C.c_int, dp, C.c_int, C.c_long, C.c_int, C.c_int]
        L.orc_lebesgue.restype = C.c_double
        L.orc_lebesgue.argtypes = [C.c_void_p, C.c_long]
        L.orc_radical_inverse.restype = C.c_double
        L.orc_radical_inverse.argtypes = [C.c_long, C.c_int]
        L.orc_halton_candidates.restype = None
        L.orc_halton_candidates.argtypes = [C.c_int, C.POINTER(C.c_int), C.c_long, dp]
        L.orc_afp_select.restype = C.c_int
        L.orc_afp_select.argtypes = [C.c_int, C.c_long, up, C.c_long, dp, lp]
        L.orc_afp_candidates.restype = C.c_long
        L.orc_afp_candidates.argtypes = [C.c_long]
        L.orc_eval_create.restype = C.c_void_p
        L.orc_eval_create.argtypes = [C.c_void_p, dp, C.c_long]
        L.orc_eval_destroy.restype = None
        L.orc_eval_destroy.argtypes = [C.c_void_p]
        L.orc_eval_apply.restype = None
        L.orc_eval_apply.argtypes = [C.c_void_p, dp, dp, C.c_int]
        L.orc_eval_sizes.restype = None
        L.orc_eval_sizes.argtypes = [C.c_void_p, lp]
        L.orc_eval_get.restype = None
        L.orc_eval_get.argtypes = [C.c_void_p, lp, lp, lp, dp, dp, lp, lp, lp, lp]
        L.orc_destroy.restype = None
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_matvec_ex.restype = None
        L.orc_matvec_ex.argtypes = [C.c_void_p, dp, dp, C.c_int, C.c_int, C.c_long, C.c_long, dp, dp]
        L.orc_cg.restype = C.c_int
        L.orc_cg.argtypes = [C.c_void_p, C.c_double, dp, dp, C.c_int, C.c_double, C.c_int, dp]
        L.orc_sizes.restype = None
        L.orc_sizes.argtypes = [C.c_void_p, lp]
        L.orc_get_tree.restype = None
        L.orc_get_tree.argtypes = [C.c_void_p, lp, lp, lp, dp, dp]
        L.orc_get_lists.restype = None
        L.orc_get_lists.argtypes = [C.c_void_p, lp, lp, lp, lp]
        L.orc_get_basis.restype = None
        L.orc_get_basis.argtypes = [C.c_void_p, up, dp, dp, dp, dp]
        L.orc_near_entries.restype = C.c_double
        L.orc_near_entries.argtypes = [C.c_void_p]
        L.orc_num_threads.restype = C.c_int
        L.orc_num_threads.argtypes = []
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _lp(a):
    return a.ctypes.data_as(C.POINTER(C.c_long)) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def kernel(kind: str, ell: float, x, y) -> float:
    """Kernel value K(x, y) as the oracle evaluates it."""
    x = _f64(x); y = _f64(y)
    return lib().orc_kernel(KERNELS[kind], float(ell), int(x.size), _dp(x), _dp(y))


def weights(rule: int, b=None, eta: float = 0.8, aux=None, d: int | None = None) -> np.ndarray:
    """Dimension weights omega_k (Thm 4.6; Sec 6.2; readings R1/R2)."""
    b = None if b is None else _f64(b)
    aux = None if aux is None else _f64(aux)
    dd = d if d is not None else (b.size if b is not None else aux.size)
    out = np.zeros(dd)
    rc = lib().orc_weights(rule, dd, _dp(b), float(eta), _dp(aux), _dp(out))
    if rc != 0:
        raise ValueError("bad weight rule")
    return out


def index_set(omega, q: float, box_rule: bool = False, count_only: bool = False):
    """Weighted total degree index set Lambda_{omega,q,d} (Sec 4), canonical order."""
    omega = _f64(omega)
    d = omega.size
    n = lib().orc_index_set(d, _dp(omega), float(q), int(box_rule), None, 0)
    if count_only:
        return n
    out = np.zeros((n, d), dtype=np.uint8)
    lib().orc_index_set(d, _dp(omega), float(q), int(box_rule),
                        out.ctypes.data_as(C.POINTER(C.c_ubyte)), n)
    return out


def axis_nodes(m: int) -> np.ndarray:
    """Leja-ordered Chebyshev (first kind) nodes on [0,1], m+1 of them."""
    z = np.zeros(m + 1)
    lib().orc_axis_nodes(int(m), _dp(z))
    return z


def legendre(j: int, t: float) -> float:
    """Orthonormal Legendre polynomial on [0,1] (Sec 5.2)."""
    return lib().orc_legendre(int(j), float(t))


def radical_inverse(i: int, p: int) -> float:
    """Halton coordinate: the radical inverse of i in base p."""
    return lib().orc_radical_inverse(int(i), int(p))


def halton_candidates(mk, count: int) -> np.ndarray:
    """AFP candidates (Sec 5.4): Halton points 1..count over the axes with m_k > 0, else 1/2."""
    mk = np.ascontiguousarray(mk, dtype=np.int32)
    Y = np.zeros((count, mk.size))
    lib().orc_halton_candidates(mk.size, mk.ctypes.data_as(C.POINTER(C.c_int)), int(count), _dp(Y))
    return Y


def afp_select(alpha, Y) -> np.ndarray:
    """Indices of the candidates Y chosen by the pivoted QR of the Vandermonde matrix (Sec 5.4)."""
    alpha = np.ascontiguousarray(alpha, dtype=np.uint8)
    Y = _f64(Y)
    nx, d = alpha.shape
    out = np.zeros(nx, dtype=np.int64)
    rc = lib().orc_afp_select(d, nx, alpha.ctypes.data_as(C.POINTER(C.c_ubyte)), Y.shape[0], _dp(Y), _lp(out))
    if rc != 0:
        raise ValueError("oracle: candidates do not span the polynomial space")
    return out


def afp_candidates(nx: int) -> int:
    return int(lib().orc_afp_candidates(int(nx)))


NODES_CHEB_LEJA = 0
NODES_AFP = 1


class Plan:
    """Tree, partition, index set, nodes and transfer matrices (Secs 4, 5.1, 5.2, 5.4)."""

    def __init__(self, points, dim_weights, leaf_size: int, eta: float, kernel: str, ell: float,
                 q: float, weight_rule: int = W_R1, weight_aux=None, node_rule: int = NODES_CHEB_LEJA,
                 n_candidates: int = 0, tensor_set: bool = False, half_diagonal: bool = False):
        pts = _f64(points)
        self.n, self.d = pts.shape
        b = _f64(dim_weights)
        aux = None if weight_aux is None else _f64(weight_aux)
        h = lib().orc_create_ex(_dp(pts), self.n, self.d, _dp(b), int(leaf_size), float(eta),
                                KERNELS[kernel], float(ell), float(q), int(weight_rule), _dp(aux),
                                int(node_rule), int(n_candidates), int(bool(tensor_set)),
                                int(bool(half_diagonal)))
        if not h:
            raise ValueError("oracle: invalid arguments")
        self._h = h
        s = np.zeros(7, dtype=np.int64)
        lib().orc_sizes(h, _lp(s))
        _, _, self.J, self.ncl, self.nx, self.nF, self.nN = (int(v) for v in s)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    # --- matvec -------------------------------------------------------
    def matvec(self, x, parts: int = 3, leaf_range=(0, 0), want_moments: bool = False):
        """y = K~ x; parts bit0 nearfield, bit1 farfield (eq. (LowRankBlock))."""
        x = _f64(x)
        squeeze = x.ndim == 1
        if squeeze:
            x = x[:, None]
        nrhs = x.shape[1]
        y = np.zeros((self.n, nrhs))
        mom = loc = None
        if want_moments:
            mom = np.zeros((self.ncl, self.nx, nrhs))
            loc = np.zeros((self.ncl, self.nx, nrhs))
        lib().orc_matvec_ex(self._h, _dp(x), _dp(y), nrhs, int(parts), int(leaf_range[0]),
                            int(leaf_range[1]), _dp(mom), _dp(loc))
        y = y[:, 0] if squeeze else y
        if want_moments:
            return y, mom, loc
        return y

    def cg(self, lam: float, f, rtol: float, max_iter: int = 10000, x0=None):
        """CG on (K~ + lambda I) alpha = f (eq. (LGS)); returns alpha, info rows."""
        f = _f64(f)
        squeeze = f.ndim == 1
        if squeeze:
            f = f[:, None]
        nrhs = f.shape[1]
        alpha = np.zeros_like(f) if x0 is None else _f64(x0).reshape(f.shape).copy()
        info = np.zeros((nrhs, 5))
        lib().orc_cg(self._h, float(lam), _dp(f), _dp(alpha), nrhs, float(rtol), int(max_iter), _dp(info))
        infos = [dict(iters=int(r[0]), neg_curvature_steps=int(r[1]), rel_res_recursive=float(r[2]),
                      rel_res_true=float(r[3]), status=int(r[4])) for r in info]
        return (alpha[:, 0] if squeeze else alpha), infos

    # --- structure ----------------------------------------------------
    def tree(self):
        perm = np.zeros(self.n, dtype=np.int64)
        cb = np.zeros(self.ncl, dtype=np.int64)
        ce = np.zeros(self.ncl, dtype=np.int64)
        lo = np.zeros((self.ncl, self.d))
        hi = np.zeros((self.ncl, self.d))
        lib().orc_get_tree(self._h, _lp(perm), _lp(cb), _lp(ce), _dp(lo), _dp(hi))
        return dict(perm=perm, begin=cb, end=ce, lo=lo, hi=hi)

    def lebesgue(self, n_samples: int = 20000) -> float:
        """Sampled Lebesgue constant (corners and Halton points 1..n_samples)."""
        return float(lib().orc_lebesgue(self._h, int(n_samples)))

    def lists(self):
        Fp = np.zeros(self.ncl + 1, dtype=np.int64)
        Fs = np.zeros(max(self.nF, 1), dtype=np.int64)
        Np = np.zeros(self.ncl + 1, dtype=np.int64)
        Ns = np.zeros(max(self.nN, 1), dtype=np.int64)
        lib().orc_get_lists(self._h, _lp(Fp), _lp(Fs), _lp(Np), _lp(Ns))
        return dict(Fptr=Fp, Fsrc=Fs[:self.nF], Nptr=Np, Nsrc=Ns[:self.nN])

    def basis(self):
        alpha = np.zeros((self.nx, self.d), dtype=np.uint8)
        xi = np.zeros((self.nx, self.d))
        V = np.zeros((self.nx, self.nx))
        Vi = np.zeros((self.nx, self.nx))
        om = np.zeros(self.d)
        lib().orc_get_basis(self._h, alpha.ctypes.data_as(C.POINTER(C.c_ubyte)), _dp(xi), _dp(V),
                            _dp(Vi), _dp(om))
        return dict(alpha=alpha, xi=xi, V=V, Vinv=Vi, omega=om)

    def near_entries(self) -> float:
        """E_N = sum over nearfield blocks of |nu| |nu'|."""
        return lib().orc_near_entries(self._h)


def num_threads() -> int:
    return lib().orc_num_threads()


def set_threads(n: int) -> None:
    """OpenMP thread count of the following oracle calls (timing runs)."""
    lib().orc_set_threads(int(n))


class Eval:
    """Evaluation of K~(targets, sources) x at new points: a target tree of the source plan's depth
    and the level-wise (target, source) block partition with the same admissibility (Secs 5.1,
    5.2)."""

    def __init__(self, plan: Plan, targets):
        T = _f64(targets)
        assert T.ndim == 2 and T.shape[1] == plan.d
        self.plan = plan          # keeps the source plan alive
        h = lib().orc_eval_create(plan._h, _dp(T), T.shape[0])
        if not h:
            raise ValueError("oracle: invalid evaluation targets")
        self._h = h
        s = np.zeros(5, dtype=np.int64)
        lib().orc_eval_sizes(h, _lp(s))
        self.m, self.J, self.ncl, self.nF, self.nN = (int(v) for v in s)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and lib is not None:
            lib().orc_eval_destroy(h)
            self._h = None

    def apply(self, x):
        x = _f64(x)
        squeeze = x.ndim == 1
        if squeeze:
            x = x[:, None]
        y = np.zeros((self.m, x.shape[1]))
        lib().orc_eval_apply(self._h, _dp(x), _dp(y), x.shape[1])
        return y[:, 0] if squeeze else y

    def lists(self):
        d = self.plan.d
        perm = np.zeros(self.m, np.int64)
        cb = np.zeros(self.ncl, np.int64)
        ce = np.zeros(self.ncl, np.int64)
        lo = np.zeros((self.ncl, d))
        hi = np.zeros((self.ncl, d))
        Fp = np.zeros(self.ncl + 1, np.int64)
        Fs = np.zeros(max(self.nF, 1), np.int64)
        Np = np.zeros(self.ncl + 1, np.int64)
        Ns = np.zeros(max(self.nN, 1), np.int64)
        lib().orc_eval_get(self._h, _lp(perm), _lp(cb), _lp(ce), _dp(lo), _dp(hi), _lp(Fp), _lp(Fs), _lp(Np),
                           _lp(Ns))
        return dict(perm=perm, begin=cb, end=ce, lo=lo, hi=hi, Fptr=Fp, Fsrc=Fs[:self.nF], Nptr=Np,
                    Nsrc=Ns[:self.nN])
