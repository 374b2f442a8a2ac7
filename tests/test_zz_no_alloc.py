"""The allocation-free matvec (dwfmm_fmm_matvec_static) against the ordinary matvec.

Same kernels with the workspace in the library's static per-GPU array: the results must equal
dwfmm_fmm_matvec bitwise (and so meet the 1e-12 FP64 parity bar), on consecutive calls whose second
input is smaller than the first (the array keeps the first call's contents), with one and with
several rhs, in reduced precision, and a workspace above the array's size is refused.
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


def make(n, d, r, kind, ell, q, leaf, eta, seed, **kw):
    X = W.points(n, d, r, seed)
    b = W.dim_weights(d, r)
    tree = dw.build_tree(torch.from_numpy(X).cuda(), b, leaf, eta)
    return dw.fmm_create(tree, kind, ell, q, **kw)


def both(op, x):
    xd = torch.from_numpy(x).cuda()
    y0 = torch.full_like(xd, float("nan"))
    y1 = torch.full_like(xd, float("nan"))
    dw.fmm_matvec(op, xd, y0)
    dw.fmm_matvec_static(op, xd, y1)
    torch.cuda.synchronize()
    return y0.cpu().numpy(), y1.cpu().numpy()


@pytest.mark.parametrize("first,second", [
    # (n, d, r, kernel, ell, q, leaf, eta, nrhs, precision): a larger call, then a smaller one
    ((30000, 10, 2.0, "matern32", 1.0, 6, 128, 0.8, 1, "fp64"), (5001, 4, 2.0, "gaussian", 0.5, 4, 64, 0.8, 1, "fp64")),
    ((20000, 20, 3.0, "gaussian", 0.5, 6, 128, 0.8, 8, "fp64"), (3000, 6, 2.0, "exponential", 0.4, 4, 64, 0.8, 3, "fp64")),
    ((8000, 6, 2.0, "matern32", 1.0, 4, 32, 3.0, 1, "fp64"), (9000, 7, 2.0, "matern32", 1.0, 5, 100, 0.5, 2, "fp64")),
    ((16000, 10, 2.0, "matern32", 1.0, 6, 128, 0.8, 16, "bf16"), (4000, 8, 2.0, "gaussian", 0.5, 5, 128, 0.8, 1, "fp32")),
])
def test_static_matvec_equals_matvec(first, second):
    rng = np.random.default_rng(77)
    for k, (n, d, r, kind, ell, q, leaf, eta, nrhs, prec) in enumerate((first, second)):
        op = make(n, d, r, kind, ell, q, leaf, eta, 780 + k, max_nrhs=nrhs, precision=prec)
        need = dw.static_scratch_bytes(op, nrhs)
        assert need <= dw.STATIC_SCRATCH_BYTES
        x = rng.standard_normal((n, nrhs))
        y0, y1 = both(op, x)
        e = np.linalg.norm(y1 - y0) / np.linalg.norm(y0)
        say(f"[static {k}] n={n} d={d} {kind} nrhs={nrhs} {prec}: workspace {need / 2**20:.1f} MiB, "
            f"rel diff {e:.1e}, bitwise {np.array_equal(y0, y1)}")
        assert np.all(np.isfinite(y1))
        assert e <= 1e-12
        assert np.array_equal(y0, y1)


def test_static_matvec_nrhs_beyond_max_nrhs():
    """The static workspace is sized per call: an operator created for one rhs serves 5."""
    op = make(6000, 5, 2.0, "gaussian", 0.5, 4, 64, 0.8, 790)
    x = np.random.default_rng(791).standard_normal((6000, 5))
    xd = torch.from_numpy(x).cuda()
    y = torch.empty_like(xd)
    dw.fmm_matvec_static(op, xd, y)
    torch.cuda.synchronize()
    yc = np.empty_like(x)
    for c in range(5):  # one rhs at a time through the ordinary matvec
        xc = torch.from_numpy(np.ascontiguousarray(x[:, c:c + 1])).cuda()
        yd = torch.empty_like(xc)
        dw.fmm_matvec(op, xc, yd)
        torch.cuda.synchronize()
        yc[:, c] = yd.cpu().numpy()[:, 0]
    e = np.linalg.norm(y.cpu().numpy() - yc) / np.linalg.norm(yc)
    say(f"[static nrhs 5 on a one-rhs operator] rel diff {e:.1e}")
    assert e <= 1e-12


def test_static_matvec_rejects_large_workspace():
    op = make(120000, 10, 2.0, "matern32", 1.0, 6, 128, 0.8, 795)
    need = dw.static_scratch_bytes(op, 1)
    assert need > dw.STATIC_SCRATCH_BYTES
    xd = torch.zeros((120000, 1), dtype=torch.float64, device="cuda")
    yd = torch.empty_like(xd)
    with pytest.raises(dw.DwfmmError) as ei:
        dw.fmm_matvec_static(op, xd, yd)
    assert ei.value.status == dw.E_INVALID and "exceeds the static scratch" in str(ei.value)
    say(f"[static] refused a workspace of {need / 2**20:.0f} MiB: {ei.value}")
    # the ordinary matvec still works on the same operator
    dw.fmm_matvec(op, xd, yd)
    torch.cuda.synchronize()
    assert torch.all(yd == 0)
