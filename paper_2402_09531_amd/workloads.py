"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers and names workloads; it holds none of the
method's arithmetic, so both the GPU library and the CPU oracle can be fed the
same FP64 arrays from it without sharing any computation.

Points follow the anisotropic setting of the paper (Sec 2, the axis-parallel box
[0,b_1] x ... x [0,b_d]; Sec 6.2 rescales uniform samples by b_k = k^-r):
``X = rng.random((N, d)) * b`` with ``b_k = k^-r``, then right-hand sides
``rng.standard_normal((N, nrhs))`` from the same generator.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    d: int
    r: float               # dimension weights b_k = k^-r
    kernel: str            # matern32 | gaussian | exponential | poly
    ell: float
    q: float
    leaf: int
    eta: float
    nrhs: int
    seed: int
    lam: float = 1e-6
    rtol: float = 1e-8
    rhs_fn: str = "sin_sum"  # CG right-hand side f(x)
    extra: dict = field(default_factory=dict)


# Workloads.  Sizes, kernels and parameters of the matvec/solve configurations:
#   small:  N=4096,  d=4,  b_k=k^-2, Matern-3/2 l=1, q=4, leaf 64,  eta 0.8
#   d10:    N=1e6,   d=10, b_k=k^-2, Matern-3/2 l=1, q=6, leaf 128, eta 0.8
#   d20:    N=1e6,   d=20, b_k=k^-3, Gaussian exp(-r^2/0.5), q=6, leaf 128, eta 0.8
WORKLOADS = {
    "small_d4": Workload("small_d4", 4096, 4, 2.0, "matern32", 1.0, 4, 64, 0.8, 1, 0,
                         rhs_fn="sin_sum"),
    "n1m_d10": Workload("n1m_d10", 1_000_000, 10, 2.0, "matern32", 1.0, 6, 128, 0.8, 1, 2,
                        rhs_fn="exp_norm2"),
    "n1m_d20": Workload("n1m_d20", 1_000_000, 20, 3.0, "gaussian", 0.5, 6, 128, 0.8, 1, 3,
                        rhs_fn="sin_sum"),
    "n1m_d20_r32": Workload("n1m_d20_r32", 1_000_000, 20, 3.0, "gaussian", 0.5, 6, 128, 0.8, 32, 3,
                            rhs_fn="sin_sum"),
}


def dim_weights(d: int, r: float) -> np.ndarray:
    """b_k = k^-r, k = 1..d."""
    return np.arange(1, d + 1, dtype=np.float64) ** (-float(r))


def points(n: int, d: int, r: float, seed: int, rng: np.random.Generator | None = None) -> np.ndarray:
    """N uniform samples in [0, b_1] x ... x [0, b_d], row-major N x d FP64."""
    rng = np.random.default_rng(seed) if rng is None else rng
    return rng.random((n, d)) * dim_weights(d, r)[None, :]


def make(w: Workload, n: int | None = None, nrhs: int | None = None):
    """Points, dimension weights and N(0,1) right-hand sides for a workload.

    ``n``/``nrhs`` override the sizes (smaller parity cases of the same shape).
    Returns (X [N,d], b [d], x [N,nrhs]).
    """
    n = w.n if n is None else n
    nrhs = w.nrhs if nrhs is None else nrhs
    rng = np.random.default_rng(w.seed)
    X = points(n, w.d, w.r, w.seed, rng)
    x = rng.standard_normal((n, nrhs))
    return X, dim_weights(w.d, w.r), x


def rhs(w: Workload, X: np.ndarray) -> np.ndarray:
    """Data values f(x_i) for the CG solve: sin(sum_k x_k) or exp(-|x|^2)."""
    if w.rhs_fn == "sin_sum":
        return np.sin(X.sum(axis=1))
    if w.rhs_fn == "exp_norm2":
        return np.exp(-(X * X).sum(axis=1))
    raise ValueError(w.rhs_fn)
