"""Pins of the oracle's sampled Lebesgue constant (Sec 5.4).

For m + 1 first-kind Chebyshev points the Lebesgue function is largest at the interval ends,
where it has the closed form (1/(m+1)) sum_{k=0}^{m} cot((2k+1) pi / (4(m+1))); on a tensor
index set with per-axis Chebyshev nodes the Lebesgue function is the product of the 1-D ones,
so its maximum is the product of the closed forms.  A single node (q = 0) gives exactly 1.
"""
import math

import numpy as np
import pytest

from paper_2402_09531_amd import workloads as W


def cheb_lebesgue(m):
    return sum(1.0 / math.tan((2 * k + 1) * math.pi / (4 * (m + 1))) for k in range(m + 1)) / (m + 1)


def test_closed_form_small_cases():
    # two points: sqrt(2); three points: 5/3 (textbook values)
    assert abs(cheb_lebesgue(1) - math.sqrt(2.0)) < 1e-15
    assert abs(cheb_lebesgue(2) - 5.0 / 3.0) < 1e-15


@pytest.mark.parametrize("m", range(0, 10))
def test_one_dimension_matches_closed_form(orc, m):
    X = W.points(200, 1, 0.0, 1)
    P = orc.Plan(X, [1.0], 32, 0.8, "matern32", 1.0, m)
    assert P.nx == m + 1
    assert abs(P.lebesgue(500) - cheb_lebesgue(m)) <= 1e-13 * cheb_lebesgue(m)


@pytest.mark.parametrize("d,q", [(2, 3), (3, 2), (3, 4)])
def test_tensor_set_is_the_product(orc, d, q):
    X = W.points(300, d, 2.0, 2)
    P = orc.Plan(X, W.dim_weights(d, 2.0), 32, 0.8, "matern32", 1.0, q, tensor_set=True)
    assert P.nx == (q + 1) ** d
    want = cheb_lebesgue(q) ** d
    assert abs(P.lebesgue(2000) - want) <= 1e-12 * want


def test_single_node_and_monotone_in_samples(orc):
    X = W.points(300, 4, 2.0, 3)
    b = W.dim_weights(4, 2.0)
    assert orc.Plan(X, b, 32, 0.8, "matern32", 1.0, 0).lebesgue(100) == 1.0
    P = orc.Plan(X, b, 32, 0.8, "matern32", 1.0, 5)
    vals = [P.lebesgue(s) for s in (0, 100, 1000, 5000)]
    assert vals[0] >= 1.0 and all(vals[i] <= vals[i + 1] for i in range(3))
