"""Reduced-precision modes against the FP64 oracle, and FP64 iterative refinement.

FP32 mode: nearfield and coupling in FP32 (Gram tiles on FP32 MFMA, hardware exp2);
BF16 mode: as FP32, and with several right-hand sides the nearfield product K Q and the
coupling product S m run on BF16 MFMA with FP32 accumulation (with one rhs there is no
product for a BF16 MFMA to carry, and BF16 runs the FP32 nearfield and coupling).  The error
bounds below are the stated accuracy of each mode against the FP64 oracle, about three times
the largest error measured over these cases: the relative 2-norm over the output, and the
largest entry error against its row scale (K~|x|)_i (all kernels here are positive, so K~|x|
is the FMM value of the sum of absolute terms).  The solve refines in FP64 and must reach the
FP64 tolerance.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2402_09531_amd as dw  # noqa: E402
from paper_2402_09531_amd import workloads as W  # noqa: E402

NORM_BOUND = {("fp32", False): 5e-6, ("fp32", True): 6e-6, ("bf16", False): 5e-6, ("bf16", True): 6e-3}
ROW_BOUND = {("fp32", False): 1.5e-7, ("fp32", True): 5e-7, ("bf16", False): 1.5e-7, ("bf16", True): 4e-4}
# The direct form's FP32 squared distance |x-c|^2 + |y-c|^2 - 2 (x-c).(y-c) carries an absolute error of
# about 2^-24 (|x-c|^2 + |y-c|^2), i.e. a relative error of that over ell in the kernel value: with
# the short length scale (nearfield reach^2 / ell in the thousands) a row's error reaches 1.2e-5 of
# its scale in FP32 (measured), so that case states its own row bound, three times that.  In BF16 its
# rows are sums of a few terms, so the rounding of each product's operands to BF16 (2^-9 relative
# each) is not averaged out: 3.9e-3 of the row scale measured, bound 1.2e-2.
ROW_BOUND_CASE = {("d6_gauss_short_5rhs", "fp32"): 4e-5, ("d6_gauss_short_5rhs", "bf16"): 1.2e-2}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


CASES = [
    # name, n, d, r, kernel, ell, q, leaf, eta, nrhs
    ("d20_gauss_1rhs", 30000, 20, 3.0, "gaussian", 0.5, 6, 128, 0.8, 1),
    ("d10_matern_1rhs", 20000, 10, 2.0, "matern32", 1.0, 6, 128, 0.8, 1),
    ("d20_gauss_32rhs", 12000, 20, 3.0, "gaussian", 0.5, 6, 128, 0.8, 32),
    ("d7_exp_5rhs", 6000, 7, 2.0, "exponential", 0.3, 5, 100, 0.5, 5),
    # Gaussian whose nearfield exponents pass the split form's bound: the direct form
    ("d6_gauss_short_5rhs", 6000, 6, 1.0, "gaussian", 2e-4, 4, 64, 0.8, 5),
]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_reduced_precision_matvec_error(orc, case, prec):
    name, n, d, r, kind, ell, q, leaf, eta, nrhs = case
    rng = np.random.default_rng(7 + n)
    X = W.points(n, d, r, n, rng)
    b = W.dim_weights(d, r)
    x = rng.standard_normal((n, nrhs))
    P = orc.Plan(X, b, leaf, eta, kind, ell, q)
    tree = dw.build_tree(torch.from_numpy(X).cuda(), b, leaf, eta)
    op = dw.fmm_create(tree, kind, ell, q, max_nrhs=nrhs)
    # the FP32 nearfield's split Gaussian (exponents within 80) for the d = 20 cases, the direct form
    # for the short length scale
    assert op.gauss_split32 == (kind == "gaussian" and ell > 1e-3)
    xd = torch.from_numpy(x).cuda()
    yd = torch.empty_like(xd)
    dw.fmm_matvec(op, xd, yd, precision=prec)
    torch.cuda.synchronize()
    y_ref = P.matvec(x)
    y = yd.cpu().numpy()
    e = rel(y, y_ref)
    # element-wise: each entry's error against its row scale (K~|x|)_i (all three kernels are positive)
    ya = P.matvec(np.abs(x))
    er = float(np.max(np.abs(y - y_ref) / ya))
    say(f"[{prec}] {name}: relative error vs FP64 oracle {e:.3e}, largest entry error / row scale {er:.3e}")
    assert e <= NORM_BOUND[(prec, nrhs > 1)]
    assert er <= ROW_BOUND_CASE.get((name, prec), ROW_BOUND[(prec, nrhs > 1)])
    assert e > 1e-13  # the reduced path really ran


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("nrhs", [1, 3, 20])
def test_reduced_precision_coincident_points(orc, prec, nrhs):
    """Zero-size leaf boxes (all points equal) put the self block in the farfield; the reduced
    nearfield kernels must skip it as the FP64 ones do."""
    X = W.points(700, 5, 2.0, 21)
    X[:160] = X[0]
    X[400:430] = X[401]
    b = W.dim_weights(5, 2.0)
    x = np.random.default_rng(23).standard_normal((700, nrhs))
    P = orc.Plan(X, b, 32, 0.8, "gaussian", 1.0, 5)
    tree = dw.build_tree(torch.from_numpy(X).cuda(), b, 32, 0.8)
    op = dw.fmm_create(tree, "gaussian", 1.0, 5, max_nrhs=nrhs)
    xd = torch.from_numpy(x).cuda()
    yd = torch.empty_like(xd)
    dw.fmm_matvec(op, xd, yd, precision=prec)
    torch.cuda.synchronize()
    y, y_ref = yd.cpu().numpy(), P.matvec(x)
    e = rel(y, y_ref)
    er = float(np.max(np.abs(y - y_ref) / P.matvec(np.abs(x))))
    say(f"[{prec} coincident x{nrhs}] relative error vs FP64 oracle {e:.3e}, largest entry error / row scale {er:.3e}")
    assert e <= NORM_BOUND[(prec, nrhs > 1)]
    assert er <= ROW_BOUND[(prec, nrhs > 1)]


@pytest.mark.parametrize("prec,nrhs", [("fp32", 1), ("fp32", 4), ("bf16", 4)])
def test_iterative_refinement_reaches_fp64_tolerance(orc, prec, nrhs):
    """Inner CG in reduced precision, FP64 residuals: the oracle-measured residual of the
    refined alpha meets rtol = 1e-8 where K~ + lambda I is positive definite (the lowest
    eigenvalue of K~ at q = 4 is about -0.48, so lambda = 1)."""
    w = W.WORKLOADS["small_d4"]
    X, b, _ = W.make(w)
    lam, rtol = 1.0, 1e-8
    f = np.stack([np.sin((c + 1) * X.sum(1)) for c in range(nrhs)], 1)
    P = orc.Plan(X, b, w.leaf, w.eta, w.kernel, w.ell, w.q)
    tree = dw.build_tree(torch.from_numpy(X).cuda(), b, w.leaf, w.eta)
    op = dw.fmm_create(tree, w.kernel, w.ell, w.q, precision=prec, max_nrhs=nrhs)
    fd = torch.from_numpy(f).cuda()
    ad = torch.zeros_like(fd)
    infos = dw.fmm_solve(op, lam, fd, ad, rtol, 20000)
    say(f"[IR {prec} x{nrhs}] {infos[0]}")
    a = ad.cpu().numpy()
    res = np.linalg.norm(f - (P.matvec(a) + lam * a), axis=0) / np.linalg.norm(f, axis=0)
    for c in range(nrhs):
        assert infos[c]["status"] == 0
        assert infos[c]["refine_steps"] >= 1
        assert res[c] <= 1.05 * rtol
        assert abs(res[c] - infos[c]["rel_res_true"]) <= 1e-3 * rtol + 1e-12 * res[c]


# Farfield only, several rhs: FP32 and the BF16 coupling against the oracle's FP64 farfield.  The
# BF16 coupling evaluates S in FP32 and applies it on v_mfma_f32_16x16x16bf16_1k with FP32
# accumulation, S and the moments each carried as a pair of BF16 numbers (three products, each
# product good to about 2^-16); the bounds are about three times the measured errors.
FAR_NORM_BOUND = {"fp32": 6e-6, "bf16": 1.2e-4}
FAR_ROW_BOUND = {"fp32": 1.5e-6, "bf16": 1.1e-5}


@pytest.mark.parametrize("case", [
    # name, n, d, r, kernel, ell, q, leaf, eta, nrhs: one and two node tiles, one and two rhs tiles
    ("d20_gauss_32rhs", 12000, 20, 3.0, "gaussian", 0.5, 6, 128, 0.8, 32),
    ("d10_matern_17rhs", 15000, 10, 2.0, "matern32", 1.0, 6, 128, 0.8, 17),
    ("d7_exp_5rhs", 8000, 7, 2.0, "exponential", 0.3, 5, 100, 0.5, 5),
], ids=lambda c: c[0])
def test_reduced_precision_coupling_several_rhs(orc, case):
    name, n, d, r, kind, ell, q, leaf, eta, nrhs = case
    rng = np.random.default_rng(31 + n)
    X = W.points(n, d, r, n + 1, rng)
    b = W.dim_weights(d, r)
    x = rng.standard_normal((n, nrhs))
    P = orc.Plan(X, b, leaf, eta, kind, ell, q)
    assert P.nx <= 32  # the MFMA coupling for several rhs
    tree = dw.build_tree(torch.from_numpy(X).cuda(), b, leaf, eta)
    op = dw.fmm_create(tree, kind, ell, q, max_nrhs=nrhs)
    xd = torch.from_numpy(x).cuda()
    y_ref = P.matvec(x, parts=2)
    ya = P.matvec(np.abs(x), parts=2)
    ys = {}
    for prec in ("fp32", "bf16"):
        yd = torch.full_like(xd, float("nan"))
        dw.fmm_matvec(op, xd, yd, parts=2, precision=prec)
        torch.cuda.synchronize()
        y = ys[prec] = yd.cpu().numpy()
        e = rel(y, y_ref)
        er = float(np.max(np.abs(y - y_ref) / np.abs(ya)))
        say(f"[{prec} farfield] {name} n_x={P.nx}: relative error vs FP64 oracle {e:.3e}, "
            f"largest entry error / row scale {er:.3e}")
        assert e <= FAR_NORM_BOUND[prec] and er <= FAR_ROW_BOUND[prec]
    assert not np.array_equal(ys["bf16"], ys["fp32"])  # the BF16 products really ran


# kernel matrices unchanged when the points scale by s and the length scale with them
SCALED_ELL = {"gaussian": lambda ell, s: ell * s * s, "matern32": lambda ell, s: ell * s,
              "exponential": lambda ell, s: ell * s}
SCALE_CASES = [
    # name, n, d, r, kernel, ell, q, leaf, eta, nrhs
    ("d20_gauss_32rhs", 12000, 20, 3.0, "gaussian", 0.5, 6, 128, 0.8, 32),
    ("d10_matern_5rhs", 8000, 10, 2.0, "matern32", 1.0, 5, 128, 0.8, 5),
]


@pytest.mark.parametrize("s", [1e4, 1e-5])
@pytest.mark.parametrize("case", SCALE_CASES, ids=[c[0] for c in SCALE_CASES])
def test_bf16_several_rhs_point_scale(case, s):
    """The BF16 several-rhs nearfield forms its distances from FP16 parts of the centred coordinates
    after a power-of-two scale taken from the tree's reach: points scaled by 1e4 or 1e-5 (and the
    length scale with them, so that the kernel matrix is the same) keep the BF16 error of the
    unscaled problem against the FP64 result, and the FP64 results agree across the scales."""
    name, n, d, r, kind, ell, q, leaf, eta, nrhs = case
    rng = np.random.default_rng(11 + n)
    X = W.points(n, d, r, n, rng)
    b = W.dim_weights(d, r)
    x = torch.from_numpy(rng.standard_normal((n, nrhs))).cuda()
    out = {}
    for sc in (1.0, s):
        tree = dw.build_tree(torch.from_numpy(X * sc).cuda(), b * sc, leaf, eta)
        op = dw.fmm_create(tree, kind, SCALED_ELL[kind](ell, sc), q, max_nrhs=nrhs)
        for prec in ("fp64", "bf16"):
            y = torch.empty_like(x)
            dw.fmm_matvec(op, x, y, precision=prec)
            torch.cuda.synchronize()
            out[(sc, prec)] = y.cpu().numpy()
        ya = torch.empty_like(x)
        dw.fmm_matvec(op, x.abs(), ya, precision="fp64")
        torch.cuda.synchronize()
        out[(sc, "abs")] = ya.cpu().numpy()
    e64 = rel(out[(s, "fp64")], out[(1.0, "fp64")])
    errs = {}
    for sc in (1.0, s):
        y, y64, ya = out[(sc, "bf16")], out[(sc, "fp64")], out[(sc, "abs")]
        errs[sc] = (rel(y, y64), float(np.max(np.abs(y - y64) / ya)))
    say(f"[scale {s:g}] {name}: FP64 across scales {e64:.2e}; BF16 vs FP64 unscaled {errs[1.0][0]:.3e} "
        f"(rows {errs[1.0][1]:.3e}), scaled {errs[s][0]:.3e} (rows {errs[s][1]:.3e})")
    assert e64 <= 1e-10
    for sc in (1.0, s):
        assert errs[sc][0] <= NORM_BOUND[("bf16", True)]
        assert errs[sc][1] <= ROW_BOUND[("bf16", True)]
    # the scaled problem's BF16 error is that of the unscaled one, up to rounding differences
    assert errs[s][0] <= 1.5 * errs[1.0][0]
