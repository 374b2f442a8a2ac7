"""The oracle's kernel functions pinned by library routines and special values.

The Matern covariance of smoothness nu and length scale ell in the sqrt(2 nu) r / ell form,
    k_nu(r) = 2^(1 - nu) / Gamma(nu) * z^nu * K_nu(z),   z = sqrt(2 nu) r / ell,
with K_nu the modified Bessel function of the second kind (scipy.special.kv), is the
Matern-3/2 kernel of the workloads at nu = 3/2 and the exponential kernel of Sec 6.2 at
nu = 1/2.  The Gaussian exp(-r^2 / ell) is the normal density of variance ell / 2 relative
to its peak (scipy.stats.norm).  None of these routines is the oracle's formula retyped.
"""
import math

import numpy as np
import pytest
from scipy import special, stats


def matern_bessel(nu, ell, r):
    z = math.sqrt(2.0 * nu) * r / ell
    if z == 0.0:
        return 1.0
    return 2.0 ** (1.0 - nu) / special.gamma(nu) * z ** nu * special.kv(nu, z)


def pairs(d, count, scale, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((count, d))
    Y = X + rng.standard_normal((count, d)) * scale * rng.random((count, 1))
    return X, Y


@pytest.mark.parametrize("kind,nu", [("matern32", 1.5), ("exponential", 0.5)])
@pytest.mark.parametrize("ell", [0.3, 1.0, 2.5])
def test_matern_family_against_bessel(orc, kind, nu, ell):
    for d in (1, 3, 10):
        X, Y = pairs(d, 200, 2.0 * ell, 17 + d)
        for x, y in zip(X, Y):
            r = float(np.sqrt(((x - y) ** 2).sum()))
            want = matern_bessel(nu, ell, r)
            got = orc.kernel(kind, ell, x, y)
            assert abs(got - want) <= 1e-13 * max(want, 1e-300) + 1e-300, (d, r, got, want)


@pytest.mark.parametrize("ell", [2e-4, 0.5, 3.0])
def test_gaussian_against_normal_density(orc, ell):
    sd = math.sqrt(ell / 2.0)
    for d in (1, 4, 20):
        X, Y = pairs(d, 200, 2.0 * sd, 5 + d)
        for x, y in zip(X, Y):
            r = float(np.sqrt(((x - y) ** 2).sum()))
            want = stats.norm.pdf(r, scale=sd) / stats.norm.pdf(0.0, scale=sd)
            got = orc.kernel("gaussian", ell, x, y)
            assert abs(got - want) <= 1e-13 * want + 1e-300, (d, r, got, want)


def test_special_values_fix_the_length_scale(orc):
    e = math.e
    for ell in (0.25, 1.0, 4.0):
        # Matern-3/2 at sqrt(3) r / ell = 1: 2 / e; the exponential at r = ell and the Gaussian at
        # r^2 = ell: 1 / e; every kernel is 1 at r = 0
        x = np.zeros(3)
        assert math.isclose(orc.kernel("matern32", ell, x, np.array([ell / math.sqrt(3.0), 0, 0])), 2 / e,
                            rel_tol=1e-15)
        assert math.isclose(orc.kernel("exponential", ell, x, np.array([0, ell, 0])), 1 / e, rel_tol=1e-15)
        assert math.isclose(orc.kernel("gaussian", ell, x, np.array([0, 0, math.sqrt(ell)])), 1 / e,
                            rel_tol=1e-15)
        for kind in ("matern32", "exponential", "gaussian"):
            v = np.array([0.3, -1.0, 2.0])
            assert orc.kernel(kind, ell, v, v) == 1.0


def test_radial_and_symmetric(orc):
    """Each kernel depends on |x - y| only: symmetric, translation invariant, and the same for
    every direction of the difference (a rotation of it)."""
    rng = np.random.default_rng(9)
    Q, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    for kind, ell in (("matern32", 0.7), ("exponential", 0.4), ("gaussian", 0.9)):
        for _ in range(50):
            x, y, t = rng.standard_normal((3, 6))
            k = orc.kernel(kind, ell, x, y)
            assert math.isclose(k, orc.kernel(kind, ell, y, x), rel_tol=1e-15)
            assert math.isclose(k, orc.kernel(kind, ell, x + t, y + t), rel_tol=1e-12)
            assert math.isclose(k, orc.kernel(kind, ell, np.zeros(6), Q @ (y - x)), rel_tol=1e-12)


def test_poly_test_kernel_values(orc):
    """The polynomial test kernel 1 + sum_{k < p} x_k y_k + (x_0 y_0)^2 (p = ell axes), at
    points where the sum is exact in binary."""
    x = np.array([0.5, 2.0, -1.0, 3.0])
    y = np.array([4.0, 0.25, 8.0, 1.0])
    # p = 2: 1 + (2 + 0.5) + (2)^2; p = 4: 1 + (2 + 0.5 - 8 + 3) + 4
    assert orc.kernel("poly", 2.0, x, y) == 7.5
    assert orc.kernel("poly", 4.0, x, y) == 2.5
