"""GPU parity where leaves own or list more than 256 nearfield blocks.

The streaming nearfield kernels take a leaf's owned blocks (symmetric one-rhs kernels) or its
nearfield list (several-rhs and evaluation kernels) 256 at a time, each segment with its own size
prefix table.  With a large admissibility parameter eta most leaf pairs stay inadmissible, so the
lists grow past 256 (and past 512) on small inputs the oracle finishes in about a second; every
case asserts from the host lists that the long segments really occur, so the cases cannot drift
below the threshold.  This also covers the full-size N = 1e6, d = 10 Matern workload, where a leaf
lists about 530 blocks (Sec 5.2 nearfield; Sec 6.1 total degree set; the split Gaussian near the
bound of its exponents).
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2402_09531_amd as dw  # noqa: E402
from paper_2402_09531_amd import workloads as W  # noqa: E402

TOL = 1e-12
SEG = 256  # blocks per column-stream segment of the streaming kernels


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def row_err(y, yref, yabs):
    """Largest per-entry error against the entry's scale (K~|x|)_i, a positive-kernel row scale."""
    return float(np.max(np.abs(y - yref) / np.maximum(yabs, 1e-300)))


def build(X, b, leaf, eta, kind, ell, q, nrhs=1, **kw):
    tree = dw.build_tree(torch.from_numpy(np.ascontiguousarray(X)).cuda(), b, leaf, eta)
    op = dw.fmm_create(tree, kind, ell, q, max_nrhs=nrhs, **kw)
    return tree, op


def matvec(op, x, precision=None):
    xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    yd = torch.full_like(xd, float("nan"))
    dw.fmm_matvec(op, xd, yd, precision=precision)
    torch.cuda.synchronize()
    return yd.cpu().numpy()


def near_lengths(tree):
    h = tree.host()
    lf = tree.nleaf - 1
    return np.diff(h["Nptr"][lf:lf + tree.nleaf + 1])


# name, n, d, r, kernel, ell, q, leaf, eta: leaves of 19-30 points listing about 500 blocks each
GEOM = {
    "d6_matern": (20000, 6, 2.0, "matern32", 1.0, 4, 32, 3.0),
    "d4_gauss": (30000, 4, 2.0, "gaussian", 0.5, 4, 32, 4.0),
    "d4_gauss_short": (30000, 4, 2.0, "gaussian", 2e-4, 4, 32, 4.0),
    "d8_exp": (20000, 8, 2.0, "exponential", 0.3, 5, 32, 3.0),
    "d10_matern": (20000, 10, 2.0, "matern32", 1.0, 4, 32, 3.0),
}

FP64_CASES = [
    # (geometry, nrhs): one rhs runs the symmetric kernel over owned blocks, several rhs the
    # MFMA kernel over the whole list (one and two 16-wide rhs tiles)
    ("d6_matern", 1), ("d4_gauss", 1), ("d4_gauss_short", 1), ("d8_exp", 1), ("d10_matern", 1),
    ("d6_matern", 3), ("d4_gauss", 17), ("d8_exp", 32), ("d10_matern", 32),
]


@pytest.mark.parametrize("geom,nrhs", FP64_CASES, ids=[f"{g}_r{k}" for g, k in FP64_CASES])
def test_long_lists_fp64(orc, geom, nrhs):
    n, d, r, kind, ell, q, leaf, eta = GEOM[geom]
    rng = np.random.default_rng(900 + n + d)
    X = W.points(n, d, r, 901 + d, rng)
    b = W.dim_weights(d, r)
    x = rng.standard_normal((n, nrhs))
    P = orc.Plan(X, b, leaf, eta, kind, ell, q)
    tree, op = build(X, b, leaf, eta, kind, ell, q, nrhs)
    assert (tree.nF, tree.nN) == (P.nF, P.nN)
    own_max, near_max, _ = tree.stats()
    nl = near_lengths(tree)
    assert near_max == nl.max()
    say(f"[long {geom} x{nrhs}] leaves {tree.nleaf}, near list mean {nl.mean():.0f} max {near_max}, "
        f"owned max {own_max}, split Gaussian {op.gauss_split}")
    if nrhs == 1:
        assert own_max > SEG  # a second owned-block segment
    else:
        assert near_max > 2 * SEG and (nl > SEG).sum() > tree.nleaf // 2  # second and third list segments
    assert op.gauss_split == (kind == "gaussian" and ell > 1e-3)
    y = matvec(op, x)
    yr = P.matvec(x)
    e = rel(y, yr)
    ea = float(np.abs(y - yr).max() / np.abs(yr).max())
    say(f"   rel err {e:.3e}, max abs err / max |y| {ea:.3e}")
    assert e <= TOL and ea <= 10 * TOL


# Reduced precision, about three times the largest errors measured over these and the precision
# cases: the relative 2-norm error, and the largest entry error against its row scale (K~|x|)_i.
# BF16 with one rhs has no product for the BF16 MFMA and runs the FP32 nearfield.
NORM_BOUND = {("fp32", 1): 5e-6, ("fp32", 32): 6e-6, ("bf16", 1): 5e-6, ("bf16", 32): 6e-3}
ROW_BOUND = {("fp32", 1): 1.5e-7, ("fp32", 32): 5e-7, ("bf16", 1): 1.5e-7, ("bf16", 32): 4e-4}


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("geom,nrhs", [("d6_matern", 1), ("d4_gauss", 1), ("d6_matern", 32), ("d4_gauss", 32)])
def test_long_lists_reduced_precision(orc, geom, nrhs, prec):
    n, d, r, kind, ell, q, leaf, eta = GEOM[geom]
    rng = np.random.default_rng(910 + n + d)
    X = W.points(n, d, r, 911 + d, rng)
    b = W.dim_weights(d, r)
    x = rng.standard_normal((n, nrhs))
    P = orc.Plan(X, b, leaf, eta, kind, ell, q)
    tree, op = build(X, b, leaf, eta, kind, ell, q, nrhs)
    own_max, near_max, _ = tree.stats()
    assert (own_max if nrhs == 1 else near_max) > SEG
    y = matvec(op, x, precision=prec)
    yr = P.matvec(x)
    ya = P.matvec(np.abs(x))
    e, er = rel(y, yr), row_err(y, yr, ya)
    say(f"[long {prec} {geom} x{nrhs}] owned max {own_max}, near max {near_max}: rel err {e:.3e}, "
        f"largest entry error / row scale {er:.3e}")
    assert e <= NORM_BOUND[(prec, nrhs)] and er <= ROW_BOUND[(prec, nrhs)]
    assert e > 1e-13  # the reduced path really ran


@pytest.mark.parametrize("geom,nrhs", [("d6_matern", 1), ("d4_gauss", 1), ("d8_exp", 1), ("d6_matern", 3)])
def test_long_cross_lists_eval(orc, geom, nrhs):
    """Evaluation at new points: target leaves whose cross nearfield lists exceed 512 source leaves."""
    n, d, r, kind, ell, q, leaf, eta = GEOM[geom]
    m = n // 2
    rng = np.random.default_rng(920 + n)
    X = W.points(n, d, r, 921 + d)
    T = W.points(m, d, r, 922 + d)
    b = W.dim_weights(d, r)
    x = rng.standard_normal((n, nrhs))
    P = orc.Plan(X, b, leaf, eta, kind, ell, q)
    E = orc.Eval(P, T)
    tree, op = build(X, b, leaf, eta, kind, ell, q, nrhs)
    ev = dw.eval_create(op, torch.from_numpy(T).cuda())
    Lg = ev.tree()
    lf = (1 << ev.J) - 1
    nl = np.diff(Lg["Nptr"][lf:])
    say(f"[long eval {geom} x{nrhs}] target leaves {len(nl)}, cross list mean {nl.mean():.0f} max {nl.max()}")
    assert nl.max() > 2 * SEG and (nl > SEG).sum() > len(nl) // 4
    assert np.array_equal(E.lists()["Nptr"], Lg["Nptr"])
    xd = torch.from_numpy(x).cuda()
    yd = torch.full((m, nrhs), float("nan"), dtype=torch.float64, device="cuda")
    dw.eval_apply(ev, xd, yd)
    torch.cuda.synchronize()
    yr = E.apply(x)
    e = rel(yd.cpu().numpy(), yr)
    say(f"   rel err {e:.3e}")
    assert e <= TOL


def test_long_lists_batched(orc):
    """Batched launches over problems with long lists: bitwise equal to single matvecs, and the FP64
    problems within 1e-12 of the oracle."""
    specs = [("d6_matern", "fp64"), ("d4_gauss", "fp64"), ("d8_exp", "fp32"), ("d10_matern", "fp64")]
    probs = []
    for k, (g, prec) in enumerate(specs):
        n, d, r, kind, ell, q, leaf, eta = GEOM[g]
        n = n + 97 * k
        X = W.points(n, d, r, 930 + k)
        b = W.dim_weights(d, r)
        tree, op = build(X, b, leaf, eta, kind, ell, q, 1, precision=prec)
        assert tree.stats()[0] > SEG
        probs.append((X, b, tree, op, (n, d, r, kind, ell, q, leaf, eta, prec)))
    batch = dw.batch_create([p[3] for p in probs], graph=True)
    rng = np.random.default_rng(931)
    for rep in range(2):
        xs = [torch.from_numpy(rng.standard_normal((p[0].shape[0], 1))).cuda() for p in probs]
        ys = [torch.full_like(x, float("nan")) for x in xs]
        dw.batch_matvec(batch, xs, ys)
        torch.cuda.synchronize()
        for p, xd, yd in zip(probs, xs, ys):
            y1 = torch.empty_like(xd)
            dw.fmm_matvec(p[3], xd, y1)
            torch.cuda.synchronize()
            assert torch.equal(yd, y1), p[4]
        say(f"[long batch] replay {rep}: {len(probs)} problems bitwise equal to single matvecs")
    for p, xd, yd in zip(probs, xs, ys):
        n, d, r, kind, ell, q, leaf, eta, prec = p[4]
        if prec != "fp64":
            continue
        Pl = orc.Plan(p[0], p[1], leaf, eta, kind, ell, q)
        e = rel(yd.cpu().numpy(), Pl.matvec(xd.cpu().numpy()))
        say(f"   problem n={n} d={d} {kind}: rel err vs oracle {e:.3e}")
        assert e <= TOL


def test_full_size_d10_matern_sampled_rows(orc):
    """N = 1e6, d = 10 (Matern, q = 6, leaf 128, eta 0.8): a leaf lists about 530 nearfield blocks and
    owns about 265, so every streaming segment runs at the workload's own shape.  Rows of sampled
    target leaves (among them those with the longest lists), computed by the oracle one leaf at a
    time, against the GPU matvec with one and with 32 rhs."""
    w = W.WORKLOADS["n1m_d10"]
    say("[full-size d10] building inputs n=1e6 d=10")
    X, b, x = W.make(w)
    tree, op = build(X, b, w.leaf, w.eta, w.kernel, w.ell, w.q, 32)
    own_max, near_max, _ = tree.stats()
    nl = near_lengths(tree)
    say(f"   near list mean {nl.mean():.0f} max {near_max}, owned max {own_max}")
    assert own_max > SEG and near_max > 2 * SEG
    y1 = matvec(op, x)
    x32 = np.random.default_rng(12).standard_normal((w.n, 32))
    y32 = matvec(op, x32)
    P = orc.Plan(X, b, w.leaf, w.eta, w.kernel, w.ell, w.q)
    Tr = P.tree()
    rng = np.random.default_rng(13)
    nleaf = 2 ** P.J
    leaves = sorted(set(rng.choice(nleaf, size=3, replace=False).tolist() + [0, nleaf - 1, int(np.argmax(nl))]))
    for l in leaves:
        c = nleaf - 1 + l
        idx = Tr["perm"][Tr["begin"][c]:Tr["end"][c]]
        yr = P.matvec(x, leaf_range=(l, l + 1))
        e1 = np.linalg.norm(y1[idx] - yr[idx]) / np.linalg.norm(yr[idx])
        yr32 = P.matvec(x32, leaf_range=(l, l + 1))
        e32 = np.linalg.norm(y32[idx] - yr32[idx]) / np.linalg.norm(yr32[idx])
        say(f"   leaf {l} (list {nl[l]}): rel err 1 rhs {e1:.3e}, 32 rhs {e32:.3e}")
        assert e1 <= TOL and e32 <= TOL


@pytest.mark.parametrize("d,q,kind,nrhs", [(20, 1, "gaussian", 1), (6, 2, "matern32", 1), (6, 2, "exponential", 5),
                                            (6, 3, "matern32", 1)])
def test_total_degree_set_parity(orc, d, q, kind, nrhs):
    """Sec 6.1 TDI: the weighted set with omega = 1 (explicit weights) is the total degree set,
    C(q + d, d) points; matvec within 1e-12 of the oracle."""
    n = 12000
    rng = np.random.default_rng(940 + d + q)
    X = W.points(n, d, 2.0, 941 + d)
    b = W.dim_weights(d, 2.0)
    x = rng.standard_normal((n, nrhs))
    ones = np.ones(d)
    ell = 0.5 if kind == "gaussian" else 0.7
    P = orc.Plan(X, b, 128, 0.8, kind, ell, q, weight_rule=orc.W_EXPLICIT, weight_aux=ones)
    tree, op = build(X, b, 128, 0.8, kind, ell, q, nrhs, weight_rule="explicit", omega=ones)
    assert op.nx == P.nx == math.comb(q + d, d)
    Bo, Bg = P.basis(), op.basis()
    assert np.array_equal(Bo["alpha"], Bg["alpha"]) and np.array_equal(Bg["omega"], ones)
    x = x if nrhs > 1 else x[:, :1]
    e = rel(matvec(op, x), P.matvec(x))
    say(f"[TDI d={d} q={q} {kind} x{nrhs}] n_x {op.nx}, rel err {e:.3e}")
    assert e <= TOL


def test_weight_rule_R2_parity(orc):
    """Rule R2 (omega_k = 1 + log2(b_1/b_k)): the same weights, index set and matvec as the oracle."""
    n, d = 15000, 8
    X = W.points(n, d, 2.0, 951)
    b = W.dim_weights(d, 2.0)
    x = np.random.default_rng(952).standard_normal((n, 1))
    P = orc.Plan(X, b, 128, 0.8, "matern32", 1.0, 6, weight_rule=orc.W_R2)
    tree, op = build(X, b, 128, 0.8, "matern32", 1.0, 6, weight_rule="R2")
    Bo, Bg = P.basis(), op.basis()
    assert np.allclose(Bg["omega"], 1.0 + 2.0 * np.log2(np.arange(1, d + 1)), rtol=0, atol=1e-14)
    assert np.array_equal(Bo["alpha"], Bg["alpha"]) and op.nx == P.nx
    e = rel(matvec(op, x), P.matvec(x))
    say(f"[R2] n_x {op.nx}, rel err {e:.3e}")
    assert e <= TOL


def near_reach2(tree):
    """max over nearfield leaf pairs (t, s) of (R_t + |c_t - c_s| + R_s)^2 from the host boxes (R the
    half diagonal, c the midpoint): the bound the split Gaussian's exponents are checked against."""
    h = tree.host()
    lf = tree.nleaf - 1
    lo, hi = h["lo"][lf:], h["hi"][lf:]
    c, R = 0.5 * (lo + hi), 0.5 * np.linalg.norm(hi - lo, axis=1)
    tgt = np.repeat(np.arange(tree.nleaf), np.diff(h["Nptr"][lf:]))
    src = h["Nsrc"][h["Nptr"][lf]:] - lf
    reach = R[tgt] + np.linalg.norm(c[tgt] - c[src], axis=1) + R[src]
    return float((reach ** 2).max())


@pytest.mark.parametrize("nrhs", [1, 5])
@pytest.mark.parametrize("ratio,split", [(560.0, True), (598.0, True), (640.0, False)])
def test_split_gaussian_near_its_exponent_bound(orc, ratio, split, nrhs):
    """The split Gaussian multiplies three exponentials whose exponents reach |x-c|^2/ell + |y-c|^2/ell
    + 2(x-c).(y-c)/ell; up to the bound 600 on reach^2/ell the matvec must still meet 1e-12 (one rhs:
    the symmetric kernel with the row and column factors in the charges; several rhs: the exponent of
    the column factor starts the Gram chain, the row factor scales the sums); past it the direct
    form runs."""
    n, d = 20000, 6
    X = W.points(n, d, 2.0, 961)
    b = W.dim_weights(d, 2.0)
    x = np.random.default_rng(962).standard_normal((n, nrhs))
    tree0 = dw.build_tree(torch.from_numpy(X).cuda(), b, 64, 0.8)
    ell = near_reach2(tree0) / ratio
    del tree0
    P = orc.Plan(X, b, 64, 0.8, "gaussian", ell, 5)
    tree, op = build(X, b, 64, 0.8, "gaussian", ell, 5, nrhs)
    assert op.gauss_split == split
    y, yr = matvec(op, x), P.matvec(x)
    e = rel(y, yr)
    ea = float(np.abs(y - yr).max() / np.abs(yr).max())
    say(f"[split Gaussian reach^2/ell = {ratio}, {nrhs} rhs] ell {ell:.4g}, split {op.gauss_split}: rel err {e:.3e}, "
        f"max abs err / max |y| {ea:.3e}")
    assert e <= TOL and ea <= 10 * TOL


@pytest.mark.parametrize("geom", ["d6_matern", "d10_matern", "d4_gauss"])
def test_leaf_order_is_balanced_permutation(geom):
    """The symmetric nearfield takes the owner leaves in 8 contiguous segments of equal work (one
    per XCD, workgroup q on XCD q mod 8), costliest first within a segment: the order is a
    permutation of the leaves plus -1 padding, each XCD's leaves are one contiguous range, and no
    segment exceeds an eighth of the work by more than one leaf's work."""
    n, d, r, kind, ell, q, leaf, eta = GEOM[geom]
    X = W.points(n, d, r, 700 + d)
    tree, _ = build(X, W.dim_weights(d, r), leaf, eta, kind, ell, q)
    order, work = tree.leaf_order()
    nl = tree.nleaf
    assert len(order) % 8 == 0
    real = order[order >= 0]
    assert sorted(real.tolist()) == list(range(nl))
    total = work.sum()
    for k in range(8):
        seg = order[k::8]
        seg = seg[seg >= 0]
        if len(seg) == 0:
            continue
        assert sorted(seg.tolist()) == list(range(seg.min(), seg.max() + 1))  # contiguous range
        assert np.all(np.diff(work[seg]) <= 0)                                # costliest first
        assert work[seg].sum() <= total / 8 + work.max() + 1e-9 * total
    say(f"[leaf order] {geom}: {nl} leaves, segments of {[int(np.sum(order[k::8] >= 0)) for k in range(8)]} leaves")
