"""Pins of the oracle's evaluation at new points, y = K~(targets, sources) x.

Checked without the oracle's own arithmetic where possible: with the sources as targets the
evaluation is the square matvec; every (target, source) pair lies in exactly one farfield or
nearfield block and the blocks obey the admissibility rule; a kernel in P_Lambda (x) P_Lambda is
reproduced exactly at arbitrary targets; the error against direct kernel sums falls with q; fewer
targets than leaves (empty target clusters) and a single target work.
"""
import numpy as np
import pytest

import pinlib as PL
from paper_2402_09531_amd import workloads as W


def setup(orc, n=2000, m=900, d=4, kind="matern32", ell=1.0, q=5, leaf=32, seed=0, scale=1.05):
    X = W.points(n, d, 2.0, 100 + seed)
    b = W.dim_weights(d, 2.0)
    T = W.points(m, d, 2.0, 200 + seed) * scale
    P = orc.Plan(X, b, leaf, 0.8, kind, ell, q)
    return X, T, P, orc.Eval(P, T)


def test_sources_as_targets_is_the_matvec(orc):
    X = W.points(2500, 5, 2.0, 3)
    P = orc.Plan(X, W.dim_weights(5, 2.0), 40, 0.8, "gaussian", 0.5, 5)
    E = orc.Eval(P, X)
    x = np.random.default_rng(4).standard_normal((2500, 2))
    assert E.nF == P.nF and E.nN == P.nN
    assert np.array_equal(E.apply(x), P.matvec(x))


@pytest.mark.parametrize("m", [900, 37, 1])
def test_blocks_cover_every_pair_once_and_are_admissible(orc, m):
    X, T, P, E = setup(orc, m=m)
    L = E.lists()
    S = P.tree()
    cover = np.zeros((m, X.shape[0]), dtype=np.int32)
    eta = 0.8

    def idx(tree, c):
        return tree["perm"][tree["begin"][c]:tree["end"][c]]

    def admissible(lo1, hi1, lo2, hi2):
        gap = np.maximum(np.maximum(lo2 - hi1, lo1 - hi2), 0.0)
        return (gap ** 2).sum() >= eta ** 2 * max(((hi1 - lo1) ** 2).sum(), ((hi2 - lo2) ** 2).sum())

    leaf0 = 2 ** E.J - 1
    for c in range(E.ncl):
        for f in range(L["Fptr"][c], L["Fptr"][c + 1]):
            s = L["Fsrc"][f]
            assert admissible(L["lo"][c], L["hi"][c], S["lo"][s], S["hi"][s])
            if c > 0:
                pc, ps = (c - 1) // 2, (s - 1) // 2
                assert not admissible(L["lo"][pc], L["hi"][pc], S["lo"][ps], S["hi"][ps])
            cover[np.ix_(idx(L, c), idx(S, s))] += 1
        for f in range(L["Nptr"][c], L["Nptr"][c + 1]):
            s = L["Nsrc"][f]
            assert c >= leaf0 and s >= leaf0
            assert not admissible(L["lo"][c], L["hi"][c], S["lo"][s], S["hi"][s])
            cover[np.ix_(idx(L, c), idx(S, s))] += 1
    assert np.all(cover == 1)
    # target boxes are tight around their points
    for c in range(E.ncl):
        pts = T[idx(L, c)]
        if len(pts):
            assert np.array_equal(L["lo"][c], pts.min(0)) and np.array_equal(L["hi"][c], pts.max(0))


def test_polynomial_kernel_is_exact_at_new_points(orc):
    X, T, P, E = setup(orc, kind="poly", ell=4.0, q=4, scale=1.3)
    assert E.nF > 0
    x = np.random.default_rng(5).standard_normal(X.shape[0])
    y = E.apply(x)
    yd = PL.kernel_matrix("poly", 4.0, T, X) @ x
    assert np.linalg.norm(y - yd) <= 1e-12 * np.linalg.norm(yd)


def test_error_against_direct_sums_falls_with_q(orc):
    X = W.points(3000, 4, 2.0, 8)
    T = W.points(700, 4, 2.0, 9)
    b = W.dim_weights(4, 2.0)
    x = np.random.default_rng(10).standard_normal(3000)
    yd = PL.kernel_matrix("matern32", 1.0, T, X) @ x
    errs = []
    for q in (1, 4, 7, 10):
        P = orc.Plan(X, b, 32, 0.8, "matern32", 1.0, q)
        E = orc.Eval(P, T)
        errs.append(np.linalg.norm(E.apply(x) - yd) / np.linalg.norm(yd))
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1)), errs
    assert errs[-1] < 1e-2 * errs[0]
