"""Exact rational helpers for the pin tests (Fractions only).

Cell averages of monomials over unit cells, exact polynomial integrals and a
small exact linear solver.  They let the tests derive reconstruction weights
and smoothness-indicator values from first principles, by routes independent
of the oracle's floating-point derivation.
"""
from fractions import Fraction as Fr
from math import factorial


def cell_avg_monomial(l, m):
    """Average of xi^l over the unit cell [m - 1/2, m + 1/2]."""
    a, b = Fr(2 * m - 1, 2), Fr(2 * m + 1, 2)
    return (b ** (l + 1) - a ** (l + 1)) / (l + 1)


def cell_avg_poly(coefs, m):
    """Average of sum_l coefs[l] xi^l over [m - 1/2, m + 1/2]."""
    return sum(Fr(c) * cell_avg_monomial(l, m) for l, c in enumerate(coefs))


def poly_eval(coefs, x):
    return sum(Fr(c) * Fr(x) ** l for l, c in enumerate(coefs))


def poly_deriv(coefs, j=1):
    out = list(coefs)
    for _ in range(j):
        out = [l * out[l] for l in range(1, len(out))]
    return out


def integral_sq(coefs, a=Fr(-1, 2), b=Fr(1, 2)):
    """Exact integral of (sum c_l xi^l)^2 over [a, b]."""
    sq = [Fr(0)] * max(1, 2 * len(coefs) - 1)
    for i, ci in enumerate(coefs):
        for j, cj in enumerate(coefs):
            sq[i + j] += Fr(ci) * Fr(cj)
    return sum(c * (b ** (e + 1) - a ** (e + 1)) / (e + 1) for e, c in enumerate(sq))


def js_beta_of_poly(coefs, r):
    """Jiang-Shu measure sum_{j=1}^{r-1} int_{-1/2}^{1/2} (p^(j))^2 of a known
    polynomial p (exact)."""
    return sum(integral_sq(poly_deriv(coefs, j)) for j in range(1, r))


def solve(A, b):
    """Exact Gauss-Jordan solve of a square system."""
    n = len(A)
    M = [list(map(Fr, row)) + [Fr(bb)] for row, bb in zip(A, b)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [x - f * y for x, y in zip(M[r], M[c])]
    return [M[i][n] / M[i][i] for i in range(n)]


def face_weights(lo, hi):
    """Weights c_m (m = lo..hi) of the face value at xi = 1/2 that is exact for
    every polynomial of degree <= hi - lo, found from the exactness conditions
    sum_m c_m avg_m(xi^l) = (1/2)^l."""
    r = hi - lo + 1
    A = [[cell_avg_monomial(l, m) for m in range(lo, hi + 1)] for l in range(r)]
    b = [Fr(1, 2) ** l for l in range(r)]
    return solve(A, b)


def falling(n, k):
    return factorial(n) // factorial(n - k)
