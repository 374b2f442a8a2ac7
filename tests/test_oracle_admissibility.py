"""Pins of the oracle's two admissibility readings (Sec 5.2, eq. (admissibility)).

Full diagonal: dist(B, B') >= eta max diag; half diagonal: eta dist(B, B') >= max diag / 2.
Checked from the boxes alone (plain numpy, unsquared): farfield blocks are admissible and
their parent blocks are not, nearfield leaf blocks are not admissible, every (target, source)
pair lies in exactly one block, and the half rule at eta equals the full rule at 1/(2 eta)
where both thresholds are exact (eta = 0.5 and 1).
"""
import numpy as np
import pytest

from paper_2402_09531_amd import workloads as W


def gap_and_diag(lo, hi, u, v):
    gap = np.maximum(np.maximum(lo[v] - hi[u], lo[u] - hi[v]), 0.0)
    return np.sqrt((gap ** 2).sum()), max(np.sqrt(((hi[u] - lo[u]) ** 2).sum()),
                                          np.sqrt(((hi[v] - lo[v]) ** 2).sum()))


def admissible(lo, hi, u, v, eta, half):
    dist, diag = gap_and_diag(lo, hi, u, v)
    return eta * dist >= 0.5 * diag if half else dist >= eta * diag


@pytest.mark.parametrize("half,eta", [(False, 0.8), (True, 0.8), (True, 0.5), (True, 1.3)])
def test_partition_obeys_its_rule_and_covers_every_pair_once(orc, half, eta):
    n, d = 1500, 4
    X = W.points(n, d, 2.0, 31)
    P = orc.Plan(X, W.dim_weights(d, 2.0), 24, eta, "matern32", 1.0, 3, half_diagonal=half)
    T, L = P.tree(), P.lists()
    lo, hi = T["lo"], T["hi"]
    leaf0 = 2 ** P.J - 1
    cover = np.zeros((n, n), dtype=np.int32)

    def idx(c):
        return T["perm"][T["begin"][c]:T["end"][c]]

    for c in range(P.ncl):
        for f in range(L["Fptr"][c], L["Fptr"][c + 1]):
            s = L["Fsrc"][f]
            assert admissible(lo, hi, c, s, eta, half)
            if c > 0:
                assert not admissible(lo, hi, (c - 1) // 2, (s - 1) // 2, eta, half)
            cover[np.ix_(idx(c), idx(s))] += 1
        for f in range(L["Nptr"][c], L["Nptr"][c + 1]):
            s = L["Nsrc"][f]
            assert c >= leaf0 and s >= leaf0
            assert not admissible(lo, hi, c, s, eta, half)
            cover[np.ix_(idx(c), idx(s))] += 1
    assert np.all(cover == 1)


def test_half_rule_changes_the_partition(orc):
    """At eta = 0.8 the half rule admits blocks the full rule does not (dist >= 0.625 diag)."""
    X = W.points(3000, 4, 2.0, 32)
    b = W.dim_weights(4, 2.0)
    full = orc.Plan(X, b, 32, 0.8, "matern32", 1.0, 3)
    half = orc.Plan(X, b, 32, 0.8, "matern32", 1.0, 3, half_diagonal=True)
    assert half.nN < full.nN


@pytest.mark.parametrize("eta_half,eta_full", [(0.5, 1.0), (1.0, 0.5)])
def test_half_rule_equals_full_rule_at_the_reciprocal_of_twice_eta(orc, eta_half, eta_full):
    X = W.points(4000, 5, 2.0, 33)
    b = W.dim_weights(5, 2.0)
    h = orc.Plan(X, b, 40, eta_half, "gaussian", 0.5, 4, half_diagonal=True)
    f = orc.Plan(X, b, 40, eta_full, "gaussian", 0.5, 4)
    Lh, Lf = h.lists(), f.lists()
    for key in ("Fptr", "Fsrc", "Nptr", "Nsrc"):
        assert np.array_equal(Lh[key], Lf[key]), key
    x = np.random.default_rng(34).standard_normal(4000)
    # the weights (and hence the index set) depend on eta only through rule R3; R1 is used here
    assert np.array_equal(h.matvec(x), f.matvec(x))
