"""The BF16 several-rhs nearfield's tile cache (dwfmm_opts.cache_near).

The first BF16 matvec with several rhs writes the kernel tiles while computing them; later ones
read them instead of recomputing distances and kernel values.  The stored tiles are the BF16
values the computing kernel feeds its MFMAs, in the same order, so every result must be bitwise
the result without the cache: the writing call, the reading calls, a different rhs tile count, a
graph capture (which does not use the cache), the refinement solve, and trees whose leaves list
more than 256 blocks (several list segments per leaf).
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


GEOM = {
    # name: n, d, r, kernel, ell, q, leaf, eta
    "d20_gauss": (12000, 20, 3.0, "gaussian", 0.5, 6, 128, 0.8),
    "d10_matern": (15000, 10, 2.0, "matern32", 1.0, 6, 128, 0.8),
    "d6_gauss_short": (6000, 6, 1.0, "gaussian", 2e-4, 4, 64, 0.8),
    # leaves listing about 500 blocks: two or three list segments per leaf
    "d4_gauss_long": (30000, 4, 2.0, "gaussian", 0.5, 4, 32, 4.0),
}


def setup(name, cache, max_nrhs=32):
    n, d, r, kind, ell, q, leaf, eta = GEOM[name]
    X = W.points(n, d, r, 300 + n)
    tree = dw.build_tree(torch.from_numpy(X).cuda(), W.dim_weights(d, r), leaf, eta)
    op = dw.fmm_create(tree, kind, ell, q, precision="bf16", max_nrhs=max_nrhs, cache_near=cache)
    return tree, op, n


def mv(op, x):
    y = torch.empty_like(x)
    dw.fmm_matvec(op, x, y)
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.mark.parametrize("name", list(GEOM))
def test_cached_matvecs_bitwise_equal(name):
    tree, op0, n = setup(name, False)
    _, op1, _ = setup(name, True)
    assert op1.bytes > op0.bytes
    assert op1.bytes == dw.op_bytes_for(op1.tree, GEOM[name][5], precision="bf16", max_nrhs=32, cache_near=True)
    assert op0.near_tiles_state == 0 and op1.near_tiles_state == 1
    rng = np.random.default_rng(5)
    for nrhs in (32, 5, 17):
        x = torch.from_numpy(rng.standard_normal((n, nrhs))).cuda()
        y0 = mv(op0, x)
        for rep in range(2):   # the first 32-rhs call writes the tiles, every later one reads them
            y1 = mv(op1, x)
            assert op1.near_tiles_state == 2
            say(f"[tile cache] {name} nrhs {nrhs} call {rep}: max |diff| {np.abs(y1 - y0).max():.3e}")
            assert np.array_equal(y1, y0)


def test_graph_capture_and_solve_with_cache():
    tree, op0, n = setup("d20_gauss", False, 8)
    _, op1, _ = setup("d20_gauss", True, 8)
    rng = np.random.default_rng(6)
    x = torch.from_numpy(rng.standard_normal((n, 8))).cuda()
    y0 = mv(op0, x)
    # captured before any eager call: the graph computes its tiles (the cache stays unwritten)
    y = torch.empty_like(x)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, capture_error_mode="thread_local"):
        dw.fmm_matvec(op1, x, y)
    for _ in range(2):
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy(), y0)
    assert op1.near_tiles_state == 1        # the captured launches did not write the tiles
    assert np.array_equal(mv(op1, x), y0)   # eager: writes the tiles
    assert op1.near_tiles_state == 2
    assert np.array_equal(mv(op1, x), y0)   # reads them
    f = torch.from_numpy(np.sin(rng.random((n, 8)).sum(1, keepdims=True) + np.arange(8))).cuda().contiguous()
    a0, a1 = torch.zeros_like(f), torch.zeros_like(f)
    i0 = dw.fmm_solve(op0, 100.0, f, a0, 1e-8, 400)
    i1 = dw.fmm_solve(op1, 100.0, f, a1, 1e-8, 400)
    assert [i["iters"] for i in i0] == [i["iters"] for i in i1]
    assert torch.equal(a0, a1)
    assert all(i["status"] == 0 for i in i1)


def test_cache_option_checks():
    n, d, r, kind, ell, q, leaf, eta = GEOM["d10_matern"]
    X = W.points(2000, d, r, 3)
    tree = dw.build_tree(torch.from_numpy(X).cuda(), W.dim_weights(d, r), leaf, eta)
    for prec, m in (("fp64", 32), ("fp32", 32), ("bf16", 1)):
        with pytest.raises(dw.DwfmmError) as ei:
            dw.fmm_create(tree, kind, ell, q, precision=prec, max_nrhs=m, cache_near=True)
        assert ei.value.status == dw.E_INVALID
