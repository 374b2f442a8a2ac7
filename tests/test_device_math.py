"""The FP64 exponential and square root of the nearfield kernels, checked on the CPU.

The device code evaluates e^x (x <= 0) by Cody-Waite reduction and a degree-10 polynomial,
and 2^t by splitting off the nearest integer and a degree-10 polynomial.
Here its constants are read from the kernel source, compared with what the coefficient
generator derives, and the same operation sequence is replayed in numpy (each fused
multiply-add formed in extended precision and rounded once to double) against numpy's exp.
The square root (hardware reciprocal-square-root seed, then a two-term series correction
g (1 + e/2 + 3e^2/8)) is replayed the same way from seeds carrying a relative error up to 2^-20.
The Matern nearfield's 2^(-s log2(e)) splits off the nearest integer with the constant 1.5 2^52
instead of a rounding instruction; that split is replayed bit for bit, including the integer
read from the low 32 bits of the rounded sum.
"""
import importlib.util
import io
import pathlib
import re
from contextlib import redirect_stdout
from fractions import Fraction

import numpy as np

CSRC = pathlib.Path(__file__).resolve().parents[1] / "paper_2402_09531_amd" / "csrc"


def device_constants():
    src = (CSRC / "kernels.hip").read_text()
    # the kernels call 2^t behind an underflow clamp
    assert "double exp2_nonpos(double t) { return exp2_bounded(fmax(t, -1075.0)); }" in src
    body = src[src.index("double exp_bounded(double x)"):]
    body = body[:body.index("return ldexp")]
    log2e = float(re.search(r"rint\(x \* ([0-9.e+-]+)\)", body).group(1))
    ln2 = [float(v) for v in re.findall(r"fma\(-n, ([0-9.e+-]+), ", body)]
    top = float(re.search(r"double p = ([0-9.e+-]+);", body).group(1))
    rest = [float(v) for v in re.findall(r"fma\(p, r, ([0-9.e+-]+)\)", body)]
    return log2e, ln2, [top] + rest   # polynomial coefficients, highest degree first


def fma(a, b, c):
    L = np.longdouble
    return (L(a) * L(b) + L(c)).astype(np.float64)


def exp_device(x, log2e, ln2, coef):
    n = np.rint(x * log2e)
    r = fma(-n, ln2[0], x)
    r = fma(-n, ln2[1], r)
    p = np.full_like(x, coef[0])
    for c in coef[1:]:
        p = fma(p, r, c)
    return np.ldexp(p, n.astype(np.int64))


def test_constants_match_generator():
    spec = importlib.util.spec_from_file_location("gen_exp_coeffs", CSRC / "gen_exp_coeffs.py")
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    buf = io.StringIO()
    with redirect_stdout(buf):
        mod.main()
    out = buf.getvalue()
    gen = [float(v) for v in re.findall(r"c\d+ = np\.float64\(([0-9.e+-]+)\)", out)]
    log2e, ln2, coef = device_constants()
    assert len(coef) == len(gen) == 11                     # degree 10
    assert coef[::-1] == gen                               # printed to full double precision
    assert ln2[0] + ln2[1] == np.log(2.0) and ln2[0] == np.float64(np.log(np.longdouble(2)))
    assert log2e == 1.0 / np.log(2.0) or abs(log2e * np.log(2.0) - 1) < 2e-16


def test_relative_error_few_ulp():
    log2e, ln2, coef = device_constants()
    rng = np.random.default_rng(0)
    x = np.concatenate([-rng.random(200_000) * 2.0, -rng.random(200_000) * 50.0,
                        -rng.random(100_000) * 700.0, -np.linspace(0.0, 1e-3, 10_001)])
    got = exp_device(x, log2e, ln2, coef)
    ref = np.exp(x.astype(np.longdouble))
    rel = np.abs((got - ref) / ref).astype(np.float64)
    assert rel.max() <= 5e-16, rel.max()          # a few units in the last place
    assert exp_device(np.array([0.0]), log2e, ln2, coef)[0] == 1.0


def test_underflow_and_clamp():
    coef = device_constants2()
    t = np.array([-1075.0, -1100.0, -1e6, -1e300])
    got = exp2_device(t, coef, clamp=True)
    assert np.all(got >= 0.0) and np.all(got <= 5e-324)
    # e^x for the row and column factors stays accurate down to the arguments they take
    log2e, ln2, coef_e = device_constants()
    x = -np.linspace(0.0, 700.0, 70_001)
    rel = np.abs(exp_device(x, log2e, ln2, coef_e) / np.exp(x.astype(np.longdouble)) - 1).astype(np.float64)
    assert rel.max() <= 5e-16


def device_constants2():
    src = (CSRC / "kernels.hip").read_text()
    body = src[src.index("double exp2_bounded(double t)"):]
    body = body[:body.index("}")]
    assert "const double n = rint(t);" in body and "return ldexp(exp2_frac(t - n), (int)n);" in body
    poly = src[src.index("double exp2_frac(double f)"):]
    poly = poly[:poly.index("}")]
    top = float(re.search(r"double p = ([0-9.e+-]+);", poly).group(1))
    rest = [float(v) for v in re.findall(r"fma\(p, f, ([0-9.e+-]+)\)", poly)]
    return [top] + rest


def exp2_device(t, coef, clamp=False):
    if clamp:
        t = np.maximum(t, -1075.0)
    n = np.rint(t)
    f = t - n
    p = np.full_like(t, coef[0])
    for c in coef[1:]:
        p = fma(p, f, c)
    return np.ldexp(p, n.astype(np.int64))


def test_exp2_constants_match_generator():
    spec = importlib.util.spec_from_file_location("gen_exp_coeffs", CSRC / "gen_exp_coeffs.py")
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    buf = io.StringIO()
    with redirect_stdout(buf):
        mod.main()
    gen = [float(v) for v in re.findall(r"b\d+ = np\.float64\(([0-9.e+-]+)\)", buf.getvalue())]
    coef = device_constants2()
    assert len(coef) == len(gen) == 11
    assert coef[::-1] == gen
    # 2^f = e^(f ln 2) and both interpolate at the mapped Chebyshev points: the two
    # polynomials agree on [-1/2, 1/2] (up to the rounding of their coefficients)
    _, _, ce = device_constants()
    f = np.linspace(-0.5, 0.5, 4001, dtype=np.longdouble)
    r = f * np.log(np.longdouble(2))
    p2 = np.zeros_like(f)
    pe = np.zeros_like(f)
    for b, c in zip(coef, ce):
        p2 = p2 * f + np.longdouble(b)
        pe = pe * r + np.longdouble(c)
    assert np.max(np.abs(p2 / pe - 1)) <= 1e-16


def test_exp2_relative_error_few_ulp():
    coef = device_constants2()
    rng = np.random.default_rng(3)
    t = np.concatenate([rng.uniform(-2.0, 2.0, 200_000), rng.uniform(-80.0, 80.0, 200_000),
                        rng.uniform(-1000.0, 1000.0, 100_000), np.linspace(-1e-3, 1e-3, 10_001),
                        np.arange(-20.0, 21.0), np.arange(-20.0, 21.0) + 0.5])
    got = exp2_device(t, coef)
    ref = np.exp2(t.astype(np.longdouble))
    rel = np.abs((got - ref) / ref).astype(np.float64)
    assert rel.max() <= 5e-16, rel.max()
    assert np.array_equal(exp2_device(np.arange(-30.0, 31.0), coef), np.exp2(np.arange(-30.0, 31.0)))


def sqrt_device(x, seed):
    g = x * seed
    e = fma(-g, seed, 1.0)
    w = g * e
    return fma(w, fma(e, 0.375, 0.5), g)


def test_sqrt_iteration_few_ulp():
    src = (CSRC / "kernels.hip").read_text()
    body = src[src.index("double sqrt_pos(double x)"):]
    body = body[:body.index("}")]
    # the sequence replayed here is the one in the source
    for frag in ("__builtin_amdgcn_rsq(x)", "g = x * y;", "e = fma(-g, y, 1.0);", "w = g * e;",
                 "return fma(w, fma(e, 0.375, 0.5), g);"):
        assert frag in body, frag
    assert body.count("fma(") == 3
    rng = np.random.default_rng(1)
    x = np.concatenate([10.0 ** rng.uniform(-300, 300, 200_000), rng.random(200_000) * 50.0, [1e-300, 1.0, 4.0]])
    seed = (1.0 / np.sqrt(x.astype(np.longdouble))).astype(np.float64)
    seed *= 1.0 + rng.uniform(-2.0 ** -20, 2.0 ** -20, x.size)
    got = sqrt_device(x, seed)
    ref = np.sqrt(x.astype(np.longdouble))
    rel = np.abs((got - ref) / ref).astype(np.float64)
    assert rel.max() <= 3e-16, rel.max()


def fma_exact(a, b, c):
    """a b + c rounded once to double (exact rational arithmetic, correctly rounded)."""
    return np.array([float(Fraction(x) * Fraction(y) + Fraction(z)) for x, y, z in
                     np.broadcast(a, b, c)], dtype=np.float64)


def test_matern_round_to_integer_split():
    src = (CSRC / "kernels.hip").read_text()
    body = src[src.index("__device__ __forceinline__ double matern_s2(double s2)"):]
    body = body[:body.index("\n}\n")]
    for frag in ("kRound = 6755399441055744.0", "const double m = fma(s, -kLog2e, kRound);",
                 "const double n = m - kRound;",
                 "ldexp(exp2_frac(fma(s, -kLog2e, -n)), __double2loint(m))", "return fma(s, e, e);"):
        assert frag in body, frag
    big = 6755399441055744.0
    assert big == 1.5 * 2.0 ** 52
    coef = device_constants2()
    log2e = 1.4426950408889634
    rng = np.random.default_rng(7)
    # s log2(e) <= 1000 is the range the caller guarantees; the half-integer points are ties
    s = np.concatenate([rng.random(12_000) * (1000.0 / log2e), rng.random(4_000) * 4.0,
                        np.arange(0.0, 1000.0) / log2e, (np.arange(0.0, 1000.0) + 0.5) / log2e, [0.0, 1e-150]])
    m = fma_exact(s, -log2e, big)
    n = m - big
    # n is an integer nearest the exact product -s log2(e), and the low word of m holds it
    t_exact = [-Fraction(x) * Fraction(log2e) for x in s]
    assert all(abs(t - Fraction(v)) <= Fraction(1, 2) for t, v in zip(t_exact, n))
    assert np.array_equal(n, np.rint(n))
    low = (m.view(np.int64) & 0xFFFFFFFF).astype(np.uint32).view(np.int32)
    assert np.array_equal(low.astype(np.float64), n)
    f = fma_exact(s, -log2e, -n)
    assert np.all(np.abs(f) <= 0.5)
    p = np.full_like(f, coef[0])
    for c in coef[1:]:
        p = fma(p, f, c)
    e = np.ldexp(p, low.astype(np.int64))
    ref = np.exp2(-(s.astype(np.longdouble) * np.longdouble(log2e)))
    nz = ref > 1e-300
    rel = np.abs((e[nz] - ref[nz]) / ref[nz]).astype(np.float64)
    assert rel.max() <= 5e-16, rel.max()
    # the kernel value (1 + s) 2^(-s log2(e)) with log2(e) rounded to double as in the source
    # (that rounding, 2.0e-17, moves e^-s by at most s ln2 2.1e-17 relative), in extended precision
    k = fma(s, e, e)
    sl = s.astype(np.longdouble)
    kref = (1 + sl) * ref
    rk = np.abs((k[nz] - kref[nz]) / kref[nz]).astype(np.float64)
    assert rk.max() <= 1e-15, rk.max()
    kexp = (1 + sl) * np.exp(-sl)
    rx = np.abs((k[nz] - kexp[nz]) / kexp[nz]).astype(np.float64)
    assert np.all(rx <= 1e-15 + s[nz] * np.log(2.0) * 2.1e-17), rx.max()
