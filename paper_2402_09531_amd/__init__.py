"""MI355X dimension weighted FMM (arXiv 2402.09531): Python binding of libdwfmm.so.

Thin ctypes marshalling over the C ABI in ``include/dwfmm.h``; every step of the
matvec and the solve runs in the library's HIP kernels.  Tensors passed in must
be contiguous float64 CUDA (HIP) tensors; streams come from
``torch.cuda.current_stream()``.  There is no CPU fallback: if the library is
not built, loading raises.

    tree = build_tree(points, dim_weights, leaf_size, eta)
    op   = fmm_create(tree, "matern32", ell, q)
    fmm_matvec(op, x, y)
    info = fmm_solve(op, lam, f, alpha, rtol, max_iter)
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdwfmm.so")

OK, E_INVALID, E_NONFINITE, E_NOMEM, E_HIP, E_NOT_CONVERGED, E_BREAKDOWN = range(7)
STATUS_NAMES = {0: "OK", 1: "E_INVALID", 2: "E_NONFINITE", 3: "E_NOMEM", 4: "E_HIP",
                5: "E_NOT_CONVERGED", 6: "E_BREAKDOWN"}
KERNELS = {"matern32": 0, "gaussian": 1, "exponential": 2, "poly": 3}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2}
WEIGHT_RULES = {"R1": 0, "R2": 1, "R3": 2, "explicit": 3}


class DwfmmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class _Kernel(C.Structure):
    _fields_ = [("kind", C.c_int32), ("ell", C.c_double)]


class _Opts(C.Structure):
    _fields_ = [("weight_rule", C.c_int32), ("omega", C.POINTER(C.c_double)), ("precision", C.c_int32),
                ("max_nrhs", C.c_int32), ("check_every", C.c_int32), ("ir_inner_rtol", C.c_double),
                ("ir_max_outer", C.c_int32), ("node_rule", C.c_int32), ("afp_candidates", C.c_int32),
                ("progress", C.c_void_p), ("progress_ctx", C.c_void_p), ("index_rule", C.c_int32),
                ("ir_max_inner", C.c_int32), ("cache_near", C.c_int32)]


# void (*)(void *ctx, int32_t iteration, int32_t nrhs, const double *rel_res)
_PROGRESS = C.CFUNCTYPE(None, C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_double))


NODE_RULES = {"cheb_leja": 0, "afp": 1}
INDEX_RULES = {"weighted_total_degree": 0, "tensor": 1}


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("neg_curvature_steps", C.c_int32), ("refine_steps", C.c_int32),
                ("status", C.c_int32), ("rel_res_recursive", C.c_double), ("rel_res_true", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None

EXPORTS = ["dwfmm_build_tree", "dwfmm_build_tree_ex", "dwfmm_fmm_create", "dwfmm_fmm_matvec", "dwfmm_fmm_matvec_parts",
           "dwfmm_fmm_solve", "dwfmm_fmm_matvec_static", "dwfmm_estimate_bytes", "dwfmm_op_bytes", "dwfmm_op_destroy",
           "dwfmm_tree_destroy", "dwfmm_last_error", "dwfmm_tree_info", "dwfmm_tree_stats", "dwfmm_tree_get", "dwfmm_op_info",
           "dwfmm_op_basis", "dwfmm_op_lebesgue", "dwfmm_op_moments", "dwfmm_op_timing", "dwfmm_batch_create", "dwfmm_batch_matvec",
           "dwfmm_batch_m2l_shapes", "dwfmm_batch_m2l_layout", "dwfmm_batch_destroy", "dwfmm_eval_create", "dwfmm_eval_apply",
           "dwfmm_eval_info", "dwfmm_eval_tree_get", "dwfmm_eval_destroy", "dwfmm_server_create", "dwfmm_server_submit", "dwfmm_server_tick",
           "dwfmm_server_result", "dwfmm_server_bytes", "dwfmm_server_destroy", "dwfmm_batch_solve", "dwfmm_op_bytes_for",
           "dwfmm_server_finished", "dwfmm_server_stats", "dwfmm_tree_leaf_order"]


def lib():
    """Load libdwfmm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2402_09531_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, dp, i64p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)
        L.dwfmm_build_tree.argtypes = [vp, C.c_int64, C.c_int32, dp, C.c_int32, C.c_double, vp, C.POINTER(vp)]
        L.dwfmm_build_tree_ex.argtypes = [vp, C.c_int64, C.c_int32, dp, C.c_int32, C.c_double, C.c_int,
                                          vp, C.POINTER(vp)]
        L.dwfmm_fmm_create.argtypes = [vp, _Kernel, C.c_double, C.POINTER(_Opts), vp, C.POINTER(vp)]
        L.dwfmm_fmm_matvec.argtypes = [vp, vp, vp, C.c_int32, vp]
        L.dwfmm_fmm_matvec_static.argtypes = [vp, vp, vp, C.c_int32, vp]
        L.dwfmm_fmm_matvec_parts.argtypes = [vp, vp, vp, C.c_int32, C.c_int32, C.c_int32, vp]
        L.dwfmm_fmm_solve.argtypes = [vp, C.c_double, vp, vp, C.c_int32, C.c_double, C.c_int32, vp,
                                      C.POINTER(SolveInfo)]
        L.dwfmm_estimate_bytes.argtypes = [C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int32]
        L.dwfmm_estimate_bytes.restype = C.c_size_t
        L.dwfmm_op_bytes.argtypes = [vp]
        L.dwfmm_op_bytes.restype = C.c_size_t
        L.dwfmm_op_bytes_for.argtypes = [vp, C.c_double, C.POINTER(_Opts)]
        L.dwfmm_op_bytes_for.restype = C.c_size_t
        L.dwfmm_op_destroy.argtypes = [vp]
        L.dwfmm_op_destroy.restype = None
        L.dwfmm_tree_destroy.argtypes = [vp]
        L.dwfmm_tree_destroy.restype = None
        L.dwfmm_last_error.restype = C.c_char_p
        L.dwfmm_tree_info.argtypes = [vp, i64p]
        L.dwfmm_tree_stats.argtypes = [vp, i64p]
        L.dwfmm_tree_leaf_order.argtypes = [vp, C.POINTER(C.c_int32), dp, C.c_int32, C.POINTER(C.c_int32)]
        L.dwfmm_tree_leaf_order.restype = C.c_int
        L.dwfmm_tree_get.argtypes = [vp, i64p, i64p, i64p, dp, dp, i64p, i64p, i64p, i64p]
        L.dwfmm_op_info.argtypes = [vp, i64p]
        L.dwfmm_op_basis.argtypes = [vp, C.POINTER(C.c_uint8), dp, dp, dp]
        L.dwfmm_op_lebesgue.argtypes = [vp, C.c_int64, dp]
        L.dwfmm_op_moments.argtypes = [vp, dp, dp, C.c_int32]
        L.dwfmm_op_timing.argtypes = [vp, C.c_int32, dp]
        L.dwfmm_batch_create.argtypes = [C.POINTER(vp), C.c_int32, C.c_int32, vp, C.POINTER(vp)]
        L.dwfmm_batch_create.restype = C.c_int
        L.dwfmm_batch_matvec.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), vp]
        L.dwfmm_batch_matvec.restype = C.c_int
        L.dwfmm_batch_m2l_shapes.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_double), C.c_int32,
                                             C.POINTER(C.c_int32)]
        L.dwfmm_batch_m2l_shapes.restype = C.c_int
        L.dwfmm_batch_m2l_layout.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_double), C.c_int32,
                                             C.POINTER(C.c_int32)]
        L.dwfmm_batch_m2l_layout.restype = C.c_int
        L.dwfmm_batch_solve.argtypes = [vp, C.c_double, C.POINTER(vp), C.POINTER(vp), C.c_double, C.c_int32,
                                        C.c_int32, vp, C.POINTER(SolveInfo)]
        L.dwfmm_batch_solve.restype = C.c_int
        L.dwfmm_eval_create.argtypes = [vp, vp, C.c_int64, vp, C.POINTER(vp)]
        L.dwfmm_eval_create.restype = C.c_int
        L.dwfmm_eval_apply.argtypes = [vp, vp, vp, C.c_int32, vp]
        L.dwfmm_eval_apply.restype = C.c_int
        L.dwfmm_eval_info.argtypes = [vp, C.POINTER(C.c_int64)]
        L.dwfmm_eval_info.restype = C.c_int
        i64p = C.POINTER(C.c_int64)
        f64p = C.POINTER(C.c_double)
        L.dwfmm_eval_tree_get.argtypes = [vp, i64p, i64p, i64p, f64p, f64p, i64p, i64p, i64p, i64p]
        L.dwfmm_eval_tree_get.restype = C.c_int
        L.dwfmm_eval_destroy.argtypes = [vp]
        L.dwfmm_eval_destroy.restype = None
        L.dwfmm_batch_destroy.argtypes = [vp]
        L.dwfmm_batch_destroy.restype = None
        L.dwfmm_server_create.argtypes = [C.c_size_t, C.c_int32, C.c_int32, vp, C.POINTER(vp)]
        L.dwfmm_server_submit.argtypes = [vp, vp, C.POINTER(C.c_int64)]
        L.dwfmm_server_tick.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.dwfmm_server_result.argtypes = [vp, C.c_int64, dp, C.POINTER(SolveInfo), dp, C.POINTER(C.c_int32)]
        for name in ("dwfmm_server_create", "dwfmm_server_submit", "dwfmm_server_tick", "dwfmm_server_result"):
            getattr(L, name).restype = C.c_int
        L.dwfmm_server_finished.argtypes = [vp, C.POINTER(C.c_int64), C.c_int32, C.POINTER(C.c_int32)]
        L.dwfmm_server_finished.restype = C.c_int
        L.dwfmm_server_stats.argtypes = [vp, dp]
        L.dwfmm_server_stats.restype = C.c_int
        L.dwfmm_server_bytes.argtypes = [vp]
        L.dwfmm_server_bytes.restype = C.c_size_t
        L.dwfmm_server_destroy.argtypes = [vp]
        L.dwfmm_server_destroy.restype = None
        for name in ["dwfmm_build_tree", "dwfmm_build_tree_ex", "dwfmm_fmm_create", "dwfmm_fmm_matvec",
                     "dwfmm_fmm_matvec_static",
                     "dwfmm_fmm_matvec_parts",
                     "dwfmm_fmm_solve", "dwfmm_tree_info", "dwfmm_tree_stats", "dwfmm_tree_get", "dwfmm_op_info", "dwfmm_op_basis",
                     "dwfmm_op_lebesgue", "dwfmm_op_moments", "dwfmm_op_timing"]:
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(status: int):
    if status != OK:
        raise DwfmmError(status, lib().dwfmm_last_error().decode())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dev_f64(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 GPU tensor")
    return C.c_void_p(t.data_ptr())


def _i64(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64)) if a is not None else None


def _f64p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


class Tree:
    """Handle of a dwfmm_tree (cluster tree and block partition)."""

    def __init__(self, handle):
        self._h = handle
        info = np.zeros(8, dtype=np.int64)
        _check(lib().dwfmm_tree_info(self._h, _i64(info)))
        self.n, self.d, self.J, self.ncl, self.nF, self.nN, self.nleaf, self.leaf = (int(v) for v in info)

    def host(self):
        """Tree order, boxes and block lists as NumPy arrays."""
        perm = np.zeros(self.n, np.int64)
        b = np.zeros(self.ncl, np.int64)
        e = np.zeros(self.ncl, np.int64)
        lo = np.zeros((self.ncl, self.d))
        hi = np.zeros((self.ncl, self.d))
        Fp = np.zeros(self.ncl + 1, np.int64)
        Fs = np.zeros(max(self.nF, 1), np.int64)
        Np = np.zeros(self.ncl + 1, np.int64)
        Ns = np.zeros(max(self.nN, 1), np.int64)
        _check(lib().dwfmm_tree_get(self._h, _i64(perm), _i64(b), _i64(e), _f64p(lo), _f64p(hi), _i64(Fp),
                                    _i64(Fs), _i64(Np), _i64(Ns)))
        return dict(perm=perm, begin=b, end=e, lo=lo, hi=hi, Fptr=Fp, Fsrc=Fs[:self.nF], Nptr=Np,
                    Nsrc=Ns[:self.nN])

    def stats(self):
        """dwfmm_tree_stats: (most blocks one leaf owns in the symmetric nearfield, longest nearfield
        list of a leaf, owned blocks in total)."""
        out = np.zeros(3, dtype=np.int64)
        _check(lib().dwfmm_tree_stats(self._h, _i64(out)))
        return int(out[0]), int(out[1]), int(out[2])

    def leaf_order(self):
        """(order of the owner leaves in the symmetric nearfield launches, -1 = padding; nearfield
        work per leaf)."""
        cnt = C.c_int32()
        _check(lib().dwfmm_tree_leaf_order(self._h, None, None, 0, C.byref(cnt)))
        order = np.zeros(max(cnt.value, 1), dtype=np.int32)
        work = np.zeros(self.nleaf)
        _check(lib().dwfmm_tree_leaf_order(self._h, order.ctypes.data_as(C.POINTER(C.c_int32)), _f64p(work),
                                           cnt.value, C.byref(cnt)))
        return order[:cnt.value], work

    def near_entries(self) -> float:
        """E_N = sum over nearfield blocks |nu||nu'|."""
        h = self.host()
        sz = h["end"] - h["begin"]
        tgt = np.repeat(np.arange(self.ncl), np.diff(h["Nptr"]))
        return float((sz[tgt] * sz[h["Nsrc"]]).sum())

    def close(self):
        if self._h:
            lib().dwfmm_tree_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Op:
    """Handle of a dwfmm_op (FMM operator)."""

    def __init__(self, handle, tree: Tree):
        self._h = handle
        self.tree = tree
        info = np.zeros(7, dtype=np.int64)
        _check(lib().dwfmm_op_info(self._h, _i64(info)))
        self.nx, self.max_nrhs, self.precision, self.bytes, self.gauss_split, self.gauss_split32 = (int(v) for v in info[:6])

    @property
    def near_tiles_state(self) -> int:
        """dwfmm_op_info's tile-cache state: 0 none, 1 allocated and unwritten, 2 written."""
        info = np.zeros(7, dtype=np.int64)
        _check(lib().dwfmm_op_info(self._h, _i64(info)))
        return int(info[6])

    def basis(self):
        d = self.tree.d
        alpha = np.zeros((self.nx, d), np.uint8)
        xi = np.zeros((self.nx, d))
        Vinv = np.zeros((self.nx, self.nx))
        om = np.zeros(d)
        _check(lib().dwfmm_op_basis(self._h, alpha.ctypes.data_as(C.POINTER(C.c_uint8)), _f64p(xi), _f64p(Vinv),
                                    _f64p(om)))
        return dict(alpha=alpha, xi=xi, Vinv=Vinv, omega=om)

    def lebesgue(self, n_samples: int = 20000) -> float:
        """dwfmm_op_lebesgue: sampled Lebesgue constant of the nodes (corners + Halton points)."""
        out = C.c_double()
        _check(lib().dwfmm_op_lebesgue(self._h, int(n_samples), C.byref(out)))
        return out.value

    def moments(self, nrhs: int = 1):
        m = np.zeros((self.tree.ncl, self.nx, nrhs))
        l = np.zeros_like(m)
        _check(lib().dwfmm_op_moments(self._h, _f64p(m), _f64p(l), nrhs))
        return m, l

    def timing(self, enable: bool):
        """Read (p2p_ms_total, m2l_ms_total, n_timed) since the last call, then set timing on/off."""
        out = np.zeros(3)
        _check(lib().dwfmm_op_timing(self._h, int(enable), _f64p(out)))
        return float(out[0]), float(out[1]), int(out[2])

    def close(self):
        if self._h:
            lib().dwfmm_op_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


ADMISSIBILITY = {"full": 0, "half": 1}


def build_tree(points, dim_weights, leaf_size: int, eta: float, stream=None, admissibility: str = "full") -> Tree:
    """dwfmm_build_tree (dwfmm_build_tree_ex for admissibility="half"): points is an N x d float64
    GPU tensor, dim_weights host values b_k; admissibility compares eta times the box gap with the
    full ("full") or half ("half") box diagonal."""
    n, d = points.shape
    b = np.ascontiguousarray(dim_weights, dtype=np.float64)
    h = C.c_void_p()
    if admissibility == "full":
        _check(lib().dwfmm_build_tree(_dev_f64(points, "points"), n, d, _f64p(b), int(leaf_size), float(eta),
                                      _stream(stream), C.byref(h)))
    else:
        _check(lib().dwfmm_build_tree_ex(_dev_f64(points, "points"), n, d, _f64p(b), int(leaf_size), float(eta),
                                         ADMISSIBILITY[admissibility], _stream(stream), C.byref(h)))
    return Tree(h)


def fmm_create(tree: Tree, kernel: str, ell: float, q: float, precision: str = "fp64", max_nrhs: int = 1,
               weight_rule: str = "R1", omega=None, check_every: int = 1, ir_inner_rtol: float = 0.0,
               ir_max_outer: int = 30, nodes: str = "cheb_leja", afp_candidates: int = 0, progress=None,
               index_set: str = "weighted_total_degree", ir_max_inner: int = 0, cache_near: bool = False,
               stream=None) -> Op:
    """dwfmm_fmm_create (nodes: "cheb_leja" or "afp", the approximate Fekete points; index_set:
    "weighted_total_degree" or "tensor"; progress: optional callable(iteration, rel_res list) run at
    the solver's host convergence checks; cache_near: keep the BF16 several-rhs nearfield tiles)."""
    om = None if omega is None else np.ascontiguousarray(omega, dtype=np.float64)
    cb = None
    if progress is not None:
        cb = _PROGRESS(lambda _ctx, it, n, rr: progress(int(it), [rr[i] for i in range(n)]))
    opts = _Opts(WEIGHT_RULES[weight_rule], _f64p(om), PRECISIONS[precision], int(max_nrhs), int(check_every),
                 float(ir_inner_rtol), int(ir_max_outer), NODE_RULES[nodes], int(afp_candidates),
                 C.cast(cb, C.c_void_p) if cb is not None else None, None, INDEX_RULES[index_set],
                 int(ir_max_inner), int(bool(cache_near)))
    h = C.c_void_p()
    _check(lib().dwfmm_fmm_create(tree._h, _Kernel(KERNELS[kernel], float(ell)), float(q), C.byref(opts),
                                  _stream(stream), C.byref(h)))
    op = Op(h, tree)
    op._progress_cb = cb   # the C side keeps the pointer: keep the trampoline alive with the operator
    return op


def fmm_matvec(op: Op, x, y, stream=None, parts: int | None = None, precision: str | None = None):
    """dwfmm_fmm_matvec (or dwfmm_fmm_matvec_parts when parts/precision are given): y = K~ x."""
    nrhs = 1 if x.dim() == 1 else x.shape[1]
    if parts is None and precision is None:
        _check(lib().dwfmm_fmm_matvec(op._h, _dev_f64(x, "x"), _dev_f64(y, "y"), nrhs, _stream(stream)))
    else:
        prec = op.precision if precision is None else PRECISIONS[precision]
        _check(lib().dwfmm_fmm_matvec_parts(op._h, _dev_f64(x, "x"), _dev_f64(y, "y"), nrhs,
                                            3 if parts is None else int(parts), prec, _stream(stream)))


STATIC_SCRATCH_BYTES = 64 << 20


def fmm_matvec_static(op: Op, x, y, stream=None):
    """dwfmm_fmm_matvec_static: y = K~ x with the library's static per-GPU workspace (allocates
    nothing; calls on one GPU must not overlap)."""
    nrhs = 1 if x.dim() == 1 else x.shape[1]
    _check(lib().dwfmm_fmm_matvec_static(op._h, _dev_f64(x, "x"), _dev_f64(y, "y"), nrhs, _stream(stream)))


def static_scratch_bytes(op: Op, nrhs: int) -> int:
    """Workspace bytes of dwfmm_fmm_matvec_static (the header's formula; each part rounded to 256)."""
    a = lambda b: (b + 255) // 256 * 256  # noqa: E731
    t = op.tree
    need = a(8 * t.n * nrhs) + 2 * a(8 * t.ncl * op.nx * nrhs)
    if nrhs == 1:
        need += a(1024 * t.nleaf) + a(1024 * t.stats()[2])
    else:
        need += a(2 * t.n * nrhs)  # the charges in BF16
    return need


def fmm_solve(op: Op, lam: float, f, alpha, rtol: float, max_iter: int = 10000, stream=None,
              raise_on_error: bool = False):
    """dwfmm_fmm_solve: (K~ + lam I) alpha = f; alpha holds the start vector.  Returns per-column info dicts."""
    nrhs = 1 if f.dim() == 1 else f.shape[1]
    infos = (SolveInfo * nrhs)()
    st = lib().dwfmm_fmm_solve(op._h, float(lam), _dev_f64(f, "f"), _dev_f64(alpha, "alpha"), nrhs, float(rtol),
                               int(max_iter), _stream(stream), infos)
    if st not in (OK, E_NOT_CONVERGED, E_BREAKDOWN) or (raise_on_error and st != OK):
        _check(st)
    return [i.as_dict() for i in infos]


class Eval:
    """Handle of a dwfmm_eval: K~(targets, sources) x at new points."""

    def __init__(self, handle, op):
        self._h = handle
        self.op = op            # the source operator must outlive the plan
        info = np.zeros(5, dtype=np.int64)
        _check(lib().dwfmm_eval_info(self._h, _i64(info)))
        self.m, self.J, self.ncl, self.nF, self.nN = (int(v) for v in info)

    def tree(self):
        d = self.op.tree.d
        out = dict(perm=np.zeros(self.m, np.int64), begin=np.zeros(self.ncl, np.int64),
                   end=np.zeros(self.ncl, np.int64), lo=np.zeros((self.ncl, d)), hi=np.zeros((self.ncl, d)),
                   Fptr=np.zeros(self.ncl + 1, np.int64), Fsrc=np.zeros(max(self.nF, 1), np.int64),
                   Nptr=np.zeros(self.ncl + 1, np.int64), Nsrc=np.zeros(max(self.nN, 1), np.int64))
        _check(lib().dwfmm_eval_tree_get(self._h, *[_i64(out[k]) if out[k].dtype == np.int64 else _f64p(out[k])
                                                    for k in ("perm", "begin", "end", "lo", "hi", "Fptr", "Fsrc",
                                                              "Nptr", "Nsrc")]))
        out["Fsrc"] = out["Fsrc"][:self.nF]
        out["Nsrc"] = out["Nsrc"][:self.nN]
        return out

    def close(self):
        if self._h:
            lib().dwfmm_eval_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def eval_create(op: Op, targets, stream=None) -> Eval:
    """dwfmm_eval_create: a plan to evaluate K~(targets, sources) x at the m x d device targets."""
    h = C.c_void_p()
    _check(lib().dwfmm_eval_create(op._h, _dev_f64(targets, "targets"), targets.shape[0], _stream(stream),
                                   C.byref(h)))
    return Eval(h, op)


def eval_apply(ev: Eval, x, y, stream=None):
    """dwfmm_eval_apply: y (m x nrhs) = K~(targets, sources) x (N x nrhs), device tensors."""
    nrhs = 1 if x.dim() == 1 else x.shape[1]
    _check(lib().dwfmm_eval_apply(ev._h, _dev_f64(x, "x"), _dev_f64(y, "y"), nrhs, _stream(stream)))


BATCH_GRAPH = 1
BATCH_TUNE = 2
BATCH_M2L_PERSISTENT = 4


def BATCH_M2L_WAVES(w: int) -> int:
    return w << 4


class Batch:
    """Handle of a dwfmm_batch: one matvec over many operators per call."""

    def __init__(self, handle, ops):
        self._h = handle
        self.ops = list(ops)   # keeps the operators alive

    def m2l_shapes(self):
        """(waves per cluster of each M2L launch, tuned ms [launch][4, 2, 1 waves] or -1)."""
        cnt = C.c_int32()
        _check(lib().dwfmm_batch_m2l_shapes(self._h, None, None, 0, C.byref(cnt)))
        n = cnt.value
        wpc = (C.c_int32 * max(n, 1))()
        ms = (C.c_double * max(3 * n, 1))()
        _check(lib().dwfmm_batch_m2l_shapes(self._h, wpc, ms, n, C.byref(cnt)))
        return [wpc[i] for i in range(n)], np.array([ms[i] for i in range(3 * n)]).reshape(n, 3)

    def m2l_layout(self):
        """(persistent grid of each M2L launch, 0 = one workgroup per 4 / waves clusters; tuned ms
        of the persistent layout [launch][4, 2, 1 waves] or -1)."""
        cnt = C.c_int32()
        _check(lib().dwfmm_batch_m2l_layout(self._h, None, None, 0, C.byref(cnt)))
        n = cnt.value
        grid = (C.c_int32 * max(n, 1))()
        ms = (C.c_double * max(3 * n, 1))()
        _check(lib().dwfmm_batch_m2l_layout(self._h, grid, ms, n, C.byref(cnt)))
        return [grid[i] for i in range(n)], np.array([ms[i] for i in range(3 * n)]).reshape(n, 3)

    def close(self):
        if self._h:
            lib().dwfmm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_create(ops, graph: bool = False, tune: bool = False, m2l_waves: int | None = None,
                 persistent: bool = False, stream=None) -> Batch:
    """dwfmm_batch_create over a list of Op (graph capture, M2L shape tuning, a forced shape, the
    persistent M2L layout)."""
    arr = (C.c_void_p * len(ops))(*[o._h for o in ops])
    h = C.c_void_p()
    flags = (BATCH_GRAPH if graph else 0) | (BATCH_TUNE if tune else 0) | \
        (BATCH_M2L_WAVES(m2l_waves) if m2l_waves else 0) | (BATCH_M2L_PERSISTENT if persistent else 0)
    _check(lib().dwfmm_batch_create(arr, len(ops), flags, _stream(stream), C.byref(h)))
    return Batch(h, ops)


def batch_matvec(batch: Batch, xs, ys, stream=None):
    """dwfmm_batch_matvec: ys[i] = K~_i xs[i] for every operator of the batch."""
    n = len(batch.ops)
    if len(xs) != n or len(ys) != n:
        raise ValueError("xs and ys must have one tensor per operator")
    xa = (C.c_void_p * n)(*[_dev_f64(x, "x").value for x in xs])
    ya = (C.c_void_p * n)(*[_dev_f64(y, "y").value for y in ys])
    _check(lib().dwfmm_batch_matvec(batch._h, xa, ya, _stream(stream)))


def batch_solve(batch: Batch, lam: float, fs, alphas, rtol: float, max_iter: int = 10000, check_every: int = 8,
                stream=None, raise_on_status: bool = False):
    """dwfmm_batch_solve: (K~_i + lam I) alphas[i] = fs[i] for every operator of the batch (alphas hold
    the start vectors and receive the solutions).  Returns one info dict per problem; a
    not-converged or breakdown status is reported in the infos (raised only with raise_on_status)."""
    n = len(batch.ops)
    if len(fs) != n or len(alphas) != n:
        raise ValueError("fs and alphas must have one tensor per operator")
    fa = (C.c_void_p * n)(*[_dev_f64(f, "f").value for f in fs])
    aa = (C.c_void_p * n)(*[_dev_f64(a, "alpha").value for a in alphas])
    infos = (SolveInfo * n)()
    st = lib().dwfmm_batch_solve(batch._h, float(lam), fa, aa, float(rtol), int(max_iter), int(check_every),
                                 _stream(stream), infos)
    if st not in (OK, E_NOT_CONVERGED, E_BREAKDOWN) or (raise_on_status and st != OK):
        _check(st)
    return [infos[i].as_dict() for i in range(n)]


class _Request(C.Structure):
    _fields_ = [("n", C.c_int64), ("d", C.c_int32), ("points", C.POINTER(C.c_double)),
                ("dim_weights", C.POINTER(C.c_double)), ("f", C.POINTER(C.c_double)), ("leaf_size", C.c_int32),
                ("eta", C.c_double), ("kernel", _Kernel), ("q", C.c_double), ("lam", C.c_double),
                ("rtol", C.c_double), ("max_iter", C.c_int32), ("precision", C.c_int32)]


class Server:
    """dwfmm_server: continuous-batching CG solve server (requests carry host arrays)."""

    def __init__(self, budget_bytes: int, max_active: int = 64, check_every: int = 1, stream=None):
        h = C.c_void_p()
        self._stream = _stream(stream)
        _check(lib().dwfmm_server_create(C.c_size_t(int(budget_bytes)), int(max_active), int(check_every),
                                         self._stream, C.byref(h)))
        self._h = h
        self._n = {}

    def submit(self, points, dim_weights, f, leaf_size, eta, kernel, ell, q, lam, rtol, max_iter,
               precision="fp64") -> int:
        pts = np.ascontiguousarray(points, dtype=np.float64)
        b = np.ascontiguousarray(dim_weights, dtype=np.float64)
        fv = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        n, d = pts.shape
        req = _Request(n, d, _f64p(pts), _f64p(b), _f64p(fv), int(leaf_size), float(eta),
                       _Kernel(KERNELS[kernel], float(ell)), float(q), float(lam), float(rtol), int(max_iter),
                       PRECISIONS[precision])
        rid = C.c_int64()
        _check(lib().dwfmm_server_submit(self._h, C.byref(req), C.byref(rid)))
        self._n[rid.value] = n
        return rid.value

    def tick(self):
        """One scheduling step; returns (active, queued)."""
        a, q = C.c_int32(), C.c_int32()
        _check(lib().dwfmm_server_tick(self._h, C.byref(a), C.byref(q)))
        return a.value, q.value

    def result(self, rid: int, with_times: bool = False):
        """(alpha, info) -- with with_times, (alpha, info, times) with times = seconds since the server's
        creation at submit, hand-off, activation and retirement -- if request rid finished, else None."""
        alpha = np.zeros(self._n[rid])
        info = SolveInfo()
        done = C.c_int32()
        times = np.zeros(4)
        _check(lib().dwfmm_server_result(self._h, int(rid), _f64p(alpha), C.byref(info), _f64p(times),
                                         C.byref(done)))
        if not done.value:
            return None
        del self._n[rid]
        return (alpha, info.as_dict(), times) if with_times else (alpha, info.as_dict())

    def finished(self):
        """Ids of the requests finished and not yet collected by result()."""
        cnt = C.c_int32()
        _check(lib().dwfmm_server_finished(self._h, None, 0, C.byref(cnt)))
        ids = (C.c_int64 * max(cnt.value, 1))()
        _check(lib().dwfmm_server_finished(self._h, ids, cnt.value, C.byref(cnt)))
        return [ids[i] for i in range(cnt.value)]

    def stats(self) -> dict:
        """Host-side accounting of the ticks (dwfmm_server_stats)."""
        out = np.zeros(6)
        _check(lib().dwfmm_server_stats(self._h, _f64p(out)))
        return {"ticks": int(out[0]), "plan_rebuilds": int(out[1]), "rebuild_s": float(out[2]),
                "launch_s": float(out[3]), "wait_s": float(out[4]), "retire_s": float(out[5])}

    def bytes_held(self) -> int:
        return int(lib().dwfmm_server_bytes(self._h))

    def close(self):
        if self._h:
            lib().dwfmm_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def op_bytes(op: Op) -> int:
    """dwfmm_op_bytes: device bytes held by the operator and its tree."""
    return int(lib().dwfmm_op_bytes(op._h))


def op_bytes_for(tree: Tree, q: float, precision: str = "fp64", max_nrhs: int = 1, weight_rule: str = "R1",
                 omega=None, nodes: str = "cheb_leja", index_set: str = "weighted_total_degree",
                 cache_near: bool = False) -> int:
    """dwfmm_op_bytes_for: the device bytes an operator with these options would hold on this tree."""
    om = None if omega is None else np.ascontiguousarray(omega, dtype=np.float64)
    opts = _Opts(WEIGHT_RULES[weight_rule], _f64p(om), PRECISIONS[precision], int(max_nrhs), 1, 0.0, 30,
                 NODE_RULES[nodes], 0, None, None, INDEX_RULES[index_set], 0, int(bool(cache_near)))
    return int(lib().dwfmm_op_bytes_for(tree._h, float(q), C.byref(opts)))


def estimate_bytes(n: int, d: int, leaf_size: int, n_x: int, nrhs: int) -> int:
    return int(lib().dwfmm_estimate_bytes(n, d, leaf_size, n_x, nrhs))
