"""Batches of independent problems: each problem's result in the batch equals its own matvec.

The batched launches run the same kernel bodies in the same reduction order as the
single-problem launches, so results must be bitwise equal (FP64 and FP32 modes), also
when the batch is replayed from a captured HIP graph several times with other work in
between, for problems that fall back to single launches, for every M2L tile shape
(1, 2 or 4 waves per cluster), in the persistent M2L layout (a fixed grid striding over the
work list) and for the shapes and layouts the tuner picks.  One problem per
batch is also checked against the CPU oracle.
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


def make_problems(seed=11):
    rng = np.random.default_rng(seed)
    specs = []
    # (n, d, r, kernel, ell, q, leaf, eta, precision)
    for i in range(10):
        n = int(round(np.exp(rng.uniform(np.log(500), np.log(20000)))))
        d = int(rng.integers(4, 17))
        kind = ["matern32", "gaussian", "exponential"][i % 3]
        prec = "fp32" if i % 4 == 1 else "fp64"
        specs.append((n, d, 2.0 + (i % 2), kind, 0.7, 4 + (i % 3), 128 if i % 5 else 64, 0.8, prec))
    # fall back to single launches: polynomial kernel, leaves above 128 points
    specs.append((3000, 4, 2.0, "poly", 4.0, 4, 64, 0.8, "fp64"))
    specs.append((5000, 3, 2.0, "matern32", 1.0, 4, 200, 0.8, "fp64"))
    probs = []
    for k, (n, d, r, kind, ell, q, leaf, eta, prec) in enumerate(specs):
        X = W.points(n, d, r, 100 + k)
        b = W.dim_weights(d, r)
        tree = dw.build_tree(torch.from_numpy(X).cuda(), b, leaf, eta)
        op = dw.fmm_create(tree, kind, ell, q, precision=prec)
        probs.append(dict(X=X, b=b, tree=tree, op=op, spec=(n, d, r, kind, ell, q, leaf, eta, prec)))
    return probs


@pytest.mark.parametrize("graph,shape", [(False, None), (True, None), (False, 1), (False, 2), (True, "tune"),
                                         (True, "persistent"), (False, "persistent-2")])
def test_batch_equals_single(orc, graph, shape):
    probs = make_problems()
    ops = [p["op"] for p in probs]
    tune = shape == "tune"
    persistent = isinstance(shape, str) and shape.startswith("persistent")
    waves = 2 if shape == "persistent-2" else (None if tune or persistent else shape)
    batch = dw.batch_create(ops, graph=graph, tune=tune, m2l_waves=waves, persistent=persistent)
    wpc, ms = batch.m2l_shapes()
    grid, ms_p = batch.m2l_layout()
    say(f"[batch graph={graph} shape={shape}] M2L launches {len(wpc)}: waves {wpc}, persistent grid {grid}")
    assert len(wpc) >= 2 and len(grid) == len(wpc)
    if tune:
        say(f"   tuned ms [4, 2, 1 waves]: {ms.round(4).tolist()}, persistent: {ms_p.round(4).tolist()}")
        for k, (w, g) in enumerate(zip(wpc, grid)):
            col = {4: 0, 2: 1, 1: 2}[w]
            chosen = (ms_p if g else ms)[k, col]
            times = [t for t in np.concatenate([ms[k], ms_p[k]]) if t > 0]
            assert ms[k, 0] > 0 and ms_p[k, 0] > 0 and chosen == min(times)
    elif persistent:
        assert all(g == 1024 for g in grid) and np.all(ms_p == -1)
        assert all(w == (2 if waves == 2 else 4) for w in wpc)
    elif shape == 2:
        assert all(w == 2 for w in wpc) and all(g == 0 for g in grid)
    elif shape == 1:
        assert 1 in wpc and all(w in (1, 4) for w in wpc)
    else:
        assert all(w == 4 for w in wpc) and np.all(ms == -1) and all(g == 0 for g in grid)
    rng = np.random.default_rng(5)
    for rep in range(3):
        xs = [torch.from_numpy(rng.standard_normal((p["X"].shape[0], 1))).cuda() for p in probs]
        ys = [torch.full_like(x, float("nan")) for x in xs]
        dw.batch_matvec(batch, xs, ys)
        torch.cuda.synchronize()
        # eager single-problem matvecs in between replays
        for p, x, y in zip(probs, xs, ys):
            y1 = torch.empty_like(x)
            dw.fmm_matvec(p["op"], x, y1)
            torch.cuda.synchronize()
            assert torch.equal(y, y1), p["spec"]
        say(f"[batch graph={graph} shape={shape}] replay {rep}: {len(probs)} problems bitwise equal to single matvecs")
    # one FP64 problem of the batch against the oracle
    p = probs[0]
    n, d, r, kind, ell, q, leaf, eta, prec = p["spec"]
    P = orc.Plan(p["X"], p["b"], leaf, eta, kind, ell, q)
    yr = P.matvec(xs[0].cpu().numpy())
    e = np.linalg.norm(ys[0].cpu().numpy() - yr) / np.linalg.norm(yr)
    assert e <= 1e-12


def test_batch_with_coincident_points(orc):
    """Problems whose leaves hold coincident points (zero-size boxes, self block in the farfield)
    next to ordinary ones, FP64 and FP32 (split and direct Gaussian, Matern): batched results
    bitwise equal to single matvecs, FP64 within 1e-12 of the oracle."""
    probs = []
    for k, (kind, prec) in enumerate([("gaussian", "fp64"), ("matern32", "fp64"), ("gaussian", "fp32"),
                                      ("matern32", "fp32")]):
        X = W.points(3000 + 500 * k, 6, 2.0, 70 + k)
        X[:300] = X[0]
        X[1000:1040] = X[1001]
        b = W.dim_weights(6, 2.0)
        tree = dw.build_tree(torch.from_numpy(X).cuda(), b, 32, 0.8)
        op = dw.fmm_create(tree, kind, 0.7, 4, precision=prec)
        probs.append((X, b, kind, prec, op))
    batch = dw.batch_create([p[-1] for p in probs], graph=True)
    rng = np.random.default_rng(75)
    xs = [torch.from_numpy(rng.standard_normal((p[0].shape[0], 1))).cuda() for p in probs]
    ys = [torch.full_like(x, float("nan")) for x in xs]
    dw.batch_matvec(batch, xs, ys)
    torch.cuda.synchronize()
    for (X, b, kind, prec, op), x, y in zip(probs, xs, ys):
        y1 = torch.empty_like(x)
        dw.fmm_matvec(op, x, y1)
        torch.cuda.synchronize()
        assert torch.equal(y, y1), (kind, prec)
        if prec == "fp64":
            P = orc.Plan(X, b, 32, 0.8, kind, 0.7, 4)
            yr = P.matvec(x.cpu().numpy())
            assert np.linalg.norm(y.cpu().numpy() - yr) <= 1e-12 * np.linalg.norm(yr), kind
    say("[batch] coincident points: 4 problems bitwise equal to single matvecs")
