"""Pins of the oracle's approximate Fekete points (Sec 5.4).

The paper takes the nodes as the pivots of a column-pivoted QR of the Vandermonde matrix
over Halton candidates.  Pinned here without the oracle's own arithmetic: the Halton
coordinates against exact fractions; the greedy rule against a brute-force search that
maximises the Gram determinant of the chosen Vandermonde columns at every step; the
resulting interpolation (unisolvent, cardinal, the polynomial kernel reproduced exactly)
and the whole matvec against numpy's block-by-block K~ on the AFP node set.
"""
from fractions import Fraction

import numpy as np
import pytest

import pinlib as PL
from paper_2402_09531_amd import workloads as W


def radical_inverse_exact(i: int, p: int) -> Fraction:
    out, scale = Fraction(0), Fraction(1, p)
    while i > 0:
        out += (i % p) * scale
        i //= p
        scale /= p
    return out


@pytest.mark.parametrize("p", [2, 3, 5, 7, 71])
def test_radical_inverse_is_exact(orc, p):
    for i in list(range(1, 200)) + [12345, 99991]:
        assert orc.radical_inverse(i, p) == float(radical_inverse_exact(i, p))


def test_candidates_use_consecutive_primes_on_active_axes(orc):
    mk = [3, 0, 2, 0, 1]
    Y = orc.halton_candidates(mk, 50)
    primes = {0: 2, 2: 3, 4: 5}
    for j in range(50):
        for k in range(5):
            want = float(radical_inverse_exact(j + 1, primes[k])) if k in primes else 0.5
            assert Y[j, k] == want


def greedy_by_gram_determinant(Vt, steps):
    """Brute force: step k takes the column maximising det(G) of the chosen columns plus it,
    G the Gram matrix of the full Vandermonde columns (volume of the parallelotope)."""
    chosen, best_vals = [], []
    for _ in range(steps):
        vals = np.full(Vt.shape[1], -1.0)
        for j in range(Vt.shape[1]):
            if j in chosen:
                continue
            C = Vt[:, chosen + [j]]
            vals[j] = np.linalg.det(C.T @ C)
        chosen.append(int(np.argmax(vals)))
        best_vals.append(vals)
    return chosen, best_vals


@pytest.mark.parametrize("d,r,q,M", [(1, 2.0, 5, 40), (2, 2.0, 4, 60), (3, 2.0, 3, 80)])
def test_pivots_maximise_the_volume_greedily(orc, d, r, q, M):
    omega = orc.weights(orc.W_R1, W.dim_weights(d, r))
    alpha = orc.index_set(omega, q)
    mk = alpha.max(axis=0)
    Y = orc.halton_candidates(mk, M)
    sel = orc.afp_select(alpha, Y)
    Vt = PL.leg_tensor_matrix(alpha.astype(int), Y).T       # basis by row, candidate by column
    brute, vals = greedy_by_gram_determinant(Vt, len(sel))
    for k in range(len(sel)):
        v = vals[k]
        # the oracle's pick attains the greedy maximum (ties within rounding allowed)
        assert v[sel[k]] >= v.max() * (1 - 1e-9), (k, sel[k], brute[k])
        if sel[k] != brute[k]:
            assert abs(v[sel[k]] - v[brute[k]]) <= 1e-9 * v.max()
        if k < len(sel) - 1 and sel[k] != brute[k]:
            break   # a tie broke differently: later steps are no longer comparable
    assert len(set(sel.tolist())) == len(sel)


def test_first_pivots_sit_at_the_ends_in_one_dimension(orc):
    """d = 1: the Legendre column norm sum_j p_j(t)^2 peaks at t = 0 and t = 1, so the first two
    pivots are the candidates nearest the two ends."""
    alpha = np.arange(7, dtype=np.uint8)[:, None]
    Y = orc.halton_candidates([6], 255)
    sel = orc.afp_select(alpha, Y)
    ends = {int(np.argmin(Y[:, 0])), int(np.argmax(Y[:, 0]))}
    assert set(sel[:2].tolist()) == ends


def afp_plan(orc, X, b, leaf, eta, kind, ell, q):
    return orc.Plan(X, b, leaf, eta, kind, ell, q, node_rule=orc.NODES_AFP)


def test_afp_nodes_interpolate(orc):
    X = W.points(600, 4, 2.0, 21)
    b = W.dim_weights(4, 2.0)
    P = afp_plan(orc, X, b, 20, 0.8, "matern32", 1.0, 4)
    B = P.basis()
    alpha, xi = B["alpha"].astype(int), B["xi"]
    # the nodes are the candidates the selection names, in pivot order
    Y = orc.halton_candidates(alpha.max(axis=0), orc.afp_candidates(P.nx))
    sel = orc.afp_select(B["alpha"], Y)
    assert np.array_equal(xi, Y[sel])
    V = PL.leg_tensor_matrix(alpha, xi)
    L = V @ np.linalg.inv(V)
    assert np.allclose(L, np.eye(P.nx), atol=1e-11)
    assert np.linalg.cond(V) < 1e4


@pytest.mark.parametrize("kind,ell,q", [("matern32", 1.0, 4), ("exponential", 0.7, 3)])
def test_afp_matvec_equals_block_definition(orc, kind, ell, q):
    X = W.points(600, 4, 2.0, 21)
    P = afp_plan(orc, X, W.dim_weights(4, 2.0), 20, 0.8, kind, ell, q)
    assert P.nF > 0
    B = P.basis()
    Kt = PL.dense_ktilde(P, X, kind, ell, B["alpha"].astype(int), B["xi"])
    Y = P.matvec(np.eye(600))
    assert np.abs(Y - Kt).max() <= 1e-12 * np.abs(Kt).max()


def test_afp_polynomial_kernel_is_exact(orc):
    X = W.points(800, 4, 2.0, 2)
    x = np.random.default_rng(1).standard_normal(800)
    P = afp_plan(orc, X, W.dim_weights(4, 2.0), 32, 0.8, "poly", 4.0, 4)
    assert P.nF > 0
    y = P.matvec(x)
    yd = PL.kernel_matrix("poly", 4.0, X, X) @ x
    assert np.linalg.norm(y - yd) <= 1e-12 * np.linalg.norm(yd)
