"""FMM evaluation at new points on the GPU against the oracle.

The target tree (leaves as point sets, boxes bitwise) and the (target, source) farfield and
nearfield lists must be identical to the oracle's; the evaluated values must match the oracle to
1e-12 (FP64), including fewer targets than leaves, a single target and several right-hand sides;
with the data sites as targets the evaluation is the operator's matvec.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2402_09531_amd as dw  # noqa: E402
from paper_2402_09531_amd import workloads as W  # noqa: E402

TOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


CASES = [
    # name, n, m, d, r, kernel, ell, q, leaf, eta, nrhs, target scale
    ("d4_matern", 6000, 2500, 4, 2.0, "matern32", 1.0, 5, 64, 0.8, 1, 1.1),
    ("d20_gauss_3rhs", 20000, 7000, 20, 3.0, "gaussian", 0.5, 6, 128, 0.8, 3, 1.05),
    # one rhs on the MFMA cross nearfield: the Gaussian in split form (every exponent within range),
    # and with a length scale so short that the split form is refused and the direct form runs
    ("d20_gauss_1rhs", 20000, 7000, 20, 3.0, "gaussian", 0.5, 6, 128, 0.8, 1, 1.05),
    ("d6_gauss_short", 6000, 2000, 6, 1.0, "gaussian", 2e-4, 4, 64, 0.8, 1, 1.1),
    ("d7_exp", 9000, 3000, 7, 2.0, "exponential", 0.3, 5, 100, 0.5, 1, 1.2),
    ("few_targets", 6000, 37, 4, 2.0, "matern32", 1.0, 4, 64, 0.8, 1, 1.0),
    ("one_target", 6000, 1, 4, 2.0, "matern32", 1.0, 4, 64, 0.8, 2, 1.0),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_eval_matches_oracle(orc, case):
    name, n, m, d, r, kind, ell, q, leaf, eta, nrhs, scale = case
    say(f"[eval] {name}: n={n} m={m} d={d} nrhs={nrhs}")
    rng = np.random.default_rng(500 + n + m)
    X = W.points(n, d, r, 600 + n)
    T = W.points(m, d, r, 700 + m) * scale
    b = W.dim_weights(d, r)
    x = rng.standard_normal((n, nrhs))
    P = orc.Plan(X, b, leaf, eta, kind, ell, q)
    E = orc.Eval(P, T)
    tree = dw.build_tree(torch.from_numpy(X).cuda(), b, leaf, eta)
    op = dw.fmm_create(tree, kind, ell, q, max_nrhs=nrhs)
    ev = dw.eval_create(op, torch.from_numpy(T).cuda())
    assert (ev.m, ev.J, ev.ncl, ev.nF, ev.nN) == (E.m, E.J, E.ncl, E.nF, E.nN)
    Lo, Lg = E.lists(), ev.tree()
    for key in ("begin", "end", "Fptr", "Fsrc", "Nptr", "Nsrc"):
        assert np.array_equal(Lo[key], Lg[key]), key
    ne = Lo["end"] > Lo["begin"]
    assert np.array_equal(Lo["lo"][ne], Lg["lo"][ne]) and np.array_equal(Lo["hi"][ne], Lg["hi"][ne])
    for c in np.nonzero(ne)[0]:
        a, z = Lo["begin"][c], Lo["end"][c]
        assert set(Lo["perm"][a:z].tolist()) == set(Lg["perm"][a:z].tolist())
    xd = torch.from_numpy(x).cuda()
    yd = torch.empty((m, nrhs), dtype=torch.float64, device="cuda")
    dw.eval_apply(ev, xd, yd)
    torch.cuda.synchronize()
    yr = E.apply(x)
    e = rel(yd.cpu().numpy(), yr)
    say(f"   far blocks {E.nF}, near blocks {E.nN}, relative error vs oracle {e:.2e}")
    assert e <= TOL


def test_eval_at_the_data_sites_is_the_matvec():
    n, d = 8000, 6
    X = W.points(n, d, 2.0, 11)
    b = W.dim_weights(d, 2.0)
    x = np.random.default_rng(12).standard_normal((n, 1))
    Xd = torch.from_numpy(X).cuda()
    tree = dw.build_tree(Xd, b, 64, 0.8)
    op = dw.fmm_create(tree, "matern32", 1.0, 5)
    ev = dw.eval_create(op, Xd)
    assert ev.nF == tree.nF and ev.nN == tree.nN
    xd = torch.from_numpy(x).cuda()
    y1, y2 = torch.empty_like(xd), torch.empty_like(xd)
    dw.eval_apply(ev, xd, y1)
    dw.fmm_matvec(op, xd, y2)
    torch.cuda.synchronize()
    assert rel(y1.cpu().numpy(), y2.cpu().numpy()) <= 1e-13


def test_eval_rejects_bad_arguments():
    X = W.points(500, 3, 2.0, 1)
    tree = dw.build_tree(torch.from_numpy(X).cuda(), W.dim_weights(3, 2.0), 32, 0.8)
    op = dw.fmm_create(tree, "matern32", 1.0, 4)
    bad = torch.from_numpy(X[:10].copy()).cuda()
    bad[3, 1] = float("nan")
    with pytest.raises(dw.DwfmmError):
        dw.eval_create(op, bad)
    ev = dw.eval_create(op, torch.from_numpy(X[:10].copy()).cuda())
    x = torch.zeros((500, 2), dtype=torch.float64, device="cuda")
    y = torch.empty((10, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(dw.DwfmmError):
        dw.eval_apply(ev, x, y)   # 2 rhs on an operator created for 1
