"""Independent NumPy restatements of the paper's definitions, used only to pin
the oracle (never the other way round).  Each helper is written from the
mathematical definition with library primitives (numpy.polynomial, numpy.linalg),
not from the oracle's C code.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from numpy.polynomial import chebyshev as npcheb
from numpy.polynomial import legendre as npleg


def kernel_matrix(kind: str, ell: float, A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Dense [K(a_i, b_j)] for the kernels used by the workloads."""
    D2 = ((A[:, None, :] - B[None, :, :]) ** 2).sum(-1)
    if kind == "matern32":
        s = math.sqrt(3.0) * np.sqrt(D2) / ell
        return (1.0 + s) * np.exp(-s)
    if kind == "gaussian":
        return np.exp(-D2 / ell)
    if kind == "exponential":
        return np.exp(-np.sqrt(D2) / ell)
    if kind == "poly":
        p = int(ell)
        v = 1.0 + A[:, :p] @ B[:, :p].T
        return v + np.outer(A[:, 0] ** 2, B[:, 0] ** 2)
    raise ValueError(kind)


def index_set_bruteforce(omega, q, box=False):
    """All alpha in N^d with sum omega_k alpha_k <= q (or max alpha_k <= q), by exhaustive search."""
    d = len(omega)
    bounds = [int(q) if box else (int(math.floor(q / w + 1e-9)) if w > 0 else 0) for w in omega]
    out = []
    for a in itertools.product(*[range(b + 1) for b in bounds]):
        if box or sum(w * ai for w, ai in zip(omega, a)) <= q + 1e-9:
            out.append(a)
    return out


def legendre01(j: int, t):
    """sqrt(2j+1) P_j(2t-1) through numpy's Legendre series evaluation."""
    c = np.zeros(j + 1)
    c[j] = 1.0
    return math.sqrt(2 * j + 1) * npleg.legval(2.0 * np.asarray(t) - 1.0, c)


def leg_tensor_matrix(alpha: np.ndarray, T: np.ndarray) -> np.ndarray:
    """[p_alpha(t_i)]_{i, alpha} for points T (n x d)."""
    n, d = T.shape
    out = np.ones((n, alpha.shape[0]))
    for a, al in enumerate(alpha):
        for k in range(d):
            if al[k]:
                out[:, a] *= legendre01(int(al[k]), T[:, k])
    return out


def cheb_leja(m: int) -> np.ndarray:
    """m+1 first-kind Chebyshev points on [0,1] (numpy chebpts1), Leja ordered from 1/2."""
    if m == 0:
        return np.array([0.5])
    t = np.sort((npcheb.chebpts1(m + 1) + 1.0) / 2.0)
    rest = list(t)
    dist = [abs(v - 0.5) for v in rest]
    dm = min(dist)
    first = min(v for v, dv in zip(rest, dist) if dv <= dm + 1e-9 * max(dm, 1.0))
    z = [first]
    rest.remove(first)
    while rest:
        prods = [np.prod([abs(v - zz) for zz in z]) for v in rest]
        pm = max(prods)
        pick = min(v for v, p in zip(rest, prods) if p >= pm * (1 - 1e-9))
        z.append(pick)
        rest.remove(pick)
    return np.array(z)


def lagrange_on_box(alpha, xi, lo, hi, X):
    """L[i, a] = l_a(a_box^-1 x_i) with l = V^-T p (V from numpy), degenerate axes -> 1/2."""
    w = hi - lo
    T = np.where(w > 0, (X - lo) / np.where(w > 0, w, 1.0), 0.5)
    V = leg_tensor_matrix(alpha, xi)
    P = leg_tensor_matrix(alpha, T)
    return np.linalg.solve(V.T, P.T).T  # rows: V^-T p(t_i)


def box_nodes(xi, lo, hi):
    w = hi - lo
    return np.where(w > 0, lo + xi * w, lo)


def dense_ktilde(plan, X, kind, ell, alpha, xi):
    """Dense K~ written straight from the block definition: nearfield blocks are
    kernel entries, farfield blocks are L_nu S L_nu'^T with the Lagrange bases of
    each box evaluated directly (no nesting)."""
    tr = plan.tree()
    ls = plan.lists()
    n = X.shape[0]
    K = np.zeros((n, n))
    perm = tr["perm"]

    def idx(c):
        return perm[tr["begin"][c]:tr["end"][c]]

    for c in range(plan.ncl):
        for f in range(ls["Fptr"][c], ls["Fptr"][c + 1]):
            s = ls["Fsrc"][f]
            I, Jn = idx(c), idx(s)
            La = lagrange_on_box(alpha, xi, tr["lo"][c], tr["hi"][c], X[I])
            Lb = lagrange_on_box(alpha, xi, tr["lo"][s], tr["hi"][s], X[Jn])
            S = kernel_matrix(kind, ell, box_nodes(xi, tr["lo"][c], tr["hi"][c]),
                              box_nodes(xi, tr["lo"][s], tr["hi"][s]))
            K[np.ix_(I, Jn)] = La @ S @ Lb.T
        for f in range(ls["Nptr"][c], ls["Nptr"][c + 1]):
            s = ls["Nsrc"][f]
            I, Jn = idx(c), idx(s)
            K[np.ix_(I, Jn)] = kernel_matrix(kind, ell, X[I], X[Jn])
    return K
