"""Coefficients of the FP64 exponential used by the nearfield kernels.

exp(x) = 2^n * p(r),  n = rint(x / ln 2),  r = x - n ln 2 in [-ln2/2, ln2/2]
(Cody-Waite range reduction with a two-part ln 2).  p is the degree-10 polynomial
that interpolates e^r at the 11 Chebyshev points of the first kind on
[-ln2/2, ln2/2] (near-minimax; interpolation error 2.9e-16 relative, about one
unit in the last place), turned into monomial coefficients.  Everything is done in numpy's extended precision and
the results are printed rounded to double.  Run: python gen_exp_coeffs.py
"""
import numpy as np

L = np.longdouble


def main():
    h = L(np.log(L(2))) / 2
    deg = 10
    k = np.arange(deg + 1, dtype=L)
    nodes = h * np.cos((2 * k + 1) * L(np.pi) / (2 * (deg + 1)))
    V = np.vander(nodes, deg + 1, increasing=True)
    vals = np.exp(nodes)
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
    err = np.max(np.abs(approx / np.exp(x) - 1))
    ln2 = L(np.log(L(2)))
    ln2_hi = np.float64(ln2)
    ln2_lo = np.float64(ln2 - L(ln2_hi))
    print(f"// max relative interpolation error on [-ln2/2, ln2/2]: {float(err):.3e}")
    print(f"ln2_hi = {ln2_hi!r}, ln2_lo = {ln2_lo!r}, log2e = {np.float64(1 / ln2)!r}")
    for i, c in enumerate(coef):
        print(f"c{i} = {np.float64(c)!r}")


if __name__ == "__main__":
    main()
