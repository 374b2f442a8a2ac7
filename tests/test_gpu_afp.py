"""Approximate Fekete points (Sec 5.4) in the library against the oracle.

The library selects its nodes with its own greedy (Gram-Schmidt) pivoting; the oracle with
Householder QR.  The selected node sets must be identical, and the matvec built on them must
match the oracle to 1e-12 in FP64, also at the paper's Sec 6.2 settings (exponential kernel,
eta = 0.5, q = 8, d = 20).
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2402_09531_amd as dw  # noqa: E402
from paper_2402_09531_amd import workloads as W  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = [
    # name, n, d, r, kernel, ell, q, leaf, eta, nrhs
    ("d4_matern", 4096, 4, 2.0, "matern32", 1.0, 4, 64, 0.8, 1),
    ("d10_matern_q6", 20000, 10, 2.0, "matern32", 1.0, 6, 128, 0.8, 1),
    ("d20_gauss_q6_3rhs", 15000, 20, 3.0, "gaussian", 0.5, 6, 128, 0.8, 3),
    ("d20_exp_eta05_q8", 20000, 20, 2.0, "exponential", 0.3, 8, 128, 0.5, 1),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_afp_nodes_and_matvec_match_oracle(orc, case):
    name, n, d, r, kind, ell, q, leaf, eta, nrhs = case
    say(f"[afp] {name}")
    rng = np.random.default_rng(31 + n)
    X = W.points(n, d, r, 40 + n)
    b = W.dim_weights(d, r)
    x = rng.standard_normal((n, nrhs))
    P = orc.Plan(X, b, leaf, eta, kind, ell, q, node_rule=orc.NODES_AFP)
    tree = dw.build_tree(torch.from_numpy(X).cuda(), b, leaf, eta)
    op = dw.fmm_create(tree, kind, ell, q, max_nrhs=nrhs, nodes="afp")
    Bo, Bg = P.basis(), op.basis()
    assert np.array_equal(Bo["alpha"], Bg["alpha"])
    assert np.array_equal(Bo["xi"], Bg["xi"]), "node sets differ"
    xd = torch.from_numpy(x).cuda()
    yd = torch.empty_like(xd)
    dw.fmm_matvec(op, xd, yd)
    torch.cuda.synchronize()
    yr = P.matvec(x)
    e = np.linalg.norm(yd.cpu().numpy() - yr) / np.linalg.norm(yr)
    say(f"   n_x {P.nx}, far blocks {P.nF}, relative error vs oracle {e:.2e}")
    assert e <= 1e-12


def test_large_index_set_on_the_general_coupling(orc):
    """n_x above 64 (here 95: d = 20, b_k = k^-2, q = 8, the Sec 6.2 weights) runs the coupling
    on the general kernel; two right-hand sides, Chebyshev-Leja nodes."""
    n, d, r, kind, ell, q, leaf, eta = 12000, 20, 2.0, "exponential", 0.3, 8, 128, 0.5
    X = W.points(n, d, r, 77)
    b = W.dim_weights(d, r)
    x = np.random.default_rng(78).standard_normal((n, 2))
    P = orc.Plan(X, b, leaf, eta, kind, ell, q, weight_rule=orc.W_R3)
    assert P.nx > 64
    tree = dw.build_tree(torch.from_numpy(X).cuda(), b, leaf, eta)
    op = dw.fmm_create(tree, kind, ell, q, max_nrhs=2, weight_rule="R3")
    assert op.nx == P.nx
    xd = torch.from_numpy(x).cuda()
    yd = torch.empty_like(xd)
    dw.fmm_matvec(op, xd, yd)
    torch.cuda.synchronize()
    yr = P.matvec(x)
    e = np.linalg.norm(yd.cpu().numpy() - yr) / np.linalg.norm(yr)
    say(f"[large n_x] n_x {P.nx}, far blocks {P.nF}, relative error vs oracle {e:.2e}")
    assert e <= 1e-12


@pytest.mark.parametrize("nodes", ["cheb_leja", "afp"])
@pytest.mark.parametrize("d,r,q,eta", [(4, 2.0, 4, 0.8), (10, 2.0, 6, 0.8), (20, 2.0, 8, 0.5)])
def test_sampled_lebesgue_constant_matches_oracle(orc, nodes, d, r, q, eta):
    """dwfmm_op_lebesgue against the oracle's sampled Lebesgue constant on the same samples."""
    X = W.points(3000, d, r, 50 + d)
    b = W.dim_weights(d, r)
    P = orc.Plan(X, b, 128, eta, "exponential", 0.3, q,
                 node_rule=orc.NODES_AFP if nodes == "afp" else orc.NODES_CHEB_LEJA)
    tree = dw.build_tree(torch.from_numpy(X).cuda(), b, 128, eta)
    op = dw.fmm_create(tree, "exponential", 0.3, q, nodes=nodes)
    lg, lo = op.lebesgue(3000), P.lebesgue(3000)
    say(f"[lebesgue] d={d} q={q} {nodes}: n_x {op.nx}, library {lg:.6f}, oracle {lo:.6f}")
    assert abs(lg - lo) <= 1e-12 * lo and lg >= 1.0


def test_sampled_lebesgue_constant_one_dimension():
    import math
    X = W.points(500, 1, 0.0, 5)
    tree = dw.build_tree(torch.from_numpy(X).cuda(), [1.0], 64, 0.8)
    for m in (1, 2, 5, 9):
        op = dw.fmm_create(tree, "matern32", 1.0, m)
        want = sum(1.0 / math.tan((2 * k + 1) * math.pi / (4 * (m + 1))) for k in range(m + 1)) / (m + 1)
        assert abs(op.lebesgue(200) - want) <= 1e-13 * want
