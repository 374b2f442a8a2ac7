"""Coefficients of the FP64 exponentials used by the nearfield kernels.

exp(x) = 2^n * p(r),  n = rint(x / ln 2),  r = x - n ln 2 in [-ln2/2, ln2/2]
(Cody-Waite range reduction with a two-part ln 2).  p is the degree-10 polynomial
that interpolates e^r at the 11 Chebyshev points of the first kind on
[-ln2/2, ln2/2] (near-minimax; interpolation error 2.9e-16 relative, about one
unit in the last place), turned into monomial coefficients.
2^t = 2^n * p2(f),  n = rint(t),  f = t - n in [-1/2, 1/2] (exact in FP64), where p2 is
the degree-10 interpolant of 2^f at the 11 first-kind Chebyshev points of [-1/2, 1/2]
(the same function as p, since 2^f = e^(f ln 2)).
Everything is done in numpy's extended precision and the results are printed rounded to
double.  Run: python gen_exp_coeffs.py
"""
import numpy as np

L = np.longdouble


def interpolant(h, fun, deg=10):
    """Monomial coefficients (lowest first) of the interpolant of fun at the deg + 1
    first-kind Chebyshev points of [-h, h], and its largest relative error there."""
    k = np.arange(deg + 1, dtype=L)
    nodes = h * np.cos((2 * k + 1) * L(np.pi) / (2 * (deg + 1)))
    V = np.vander(nodes, deg + 1, increasing=True)
    vals = fun(nodes)
    # solve the Vandermonde system in extended precision by Gaussian elimination
    A = np.concatenate([V, vals[:, None]], axis=1).astype(L)
    n = deg + 1
    for c in range(n):
        p = c + int(np.argmax(np.abs(A[c:, c])))
        A[[c, p]] = A[[p, c]]
        A[c] = A[c] / A[c, c]
        for r in range(n):
            if r != c:
                A[r] = A[r] - A[r, c] * A[c]
    coef = A[:, -1]
    x = np.linspace(-h, h, 20001, dtype=L)
    approx = np.zeros_like(x)
    for c in coef[::-1]:
        approx = approx * x + c
    return coef, np.max(np.abs(approx / fun(x) - 1))


def main():
    ln2 = L(np.log(L(2)))
    coef, err = interpolant(ln2 / 2, np.exp)
    coef2, err2 = interpolant(L(0.5), lambda f: np.exp(f * ln2))
    ln2_hi = np.float64(ln2)
    ln2_lo = np.float64(ln2 - L(ln2_hi))
    print(f"// max relative interpolation error on [-ln2/2, ln2/2]: {float(err):.3e}")
    print(f"ln2_hi = {ln2_hi!r}, ln2_lo = {ln2_lo!r}, log2e = {np.float64(1 / ln2)!r}")
    for i, c in enumerate(coef):
        print(f"c{i} = {np.float64(c)!r}")
    print(f"// base 2: max relative interpolation error on [-1/2, 1/2]: {float(err2):.3e}")
    for i, c in enumerate(coef2):
        print(f"b{i} = {np.float64(c)!r}")


if __name__ == "__main__":
    main()
