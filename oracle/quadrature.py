"""Pixel integration rules for the oracle -- TEST INFRASTRUCTURE ONLY.

Sec. 3.1 (Eq. 14) integrates each pixel by a weighted sum over abscissae; Sec.
4.5 compares the N x N midpoint rules ("subN") with the Cartesian squares of
Gauss-Kronrod rules g3k7, g5k11 and g7k15 (Patterson 1968), whose embedded
Gauss rule gives a per-pixel error estimate. This module builds the 1-D rules
from their definitions, in float64, on the pixel interval [-1/2, 1/2] with
weights summing to 1:

* Gauss-Legendre with n nodes: the roots of the Legendre polynomial P_n, found
  by Newton's method on the three-term recurrence, weights 2 / ((1 - x^2) P_n'(x)^2).
* Kronrod extension to 2n + 1 nodes: the n Gauss nodes plus the n + 1 roots of
  the Stieltjes polynomial E_{n+1}, the monic polynomial orthogonal to every
  polynomial of degree <= n with respect to the weight P_n on [-1, 1]. Its
  coefficients solve an exact rational linear system (fractions); its roots are
  polished by Newton's method. The 2n + 1 weights make the rule exact for
  Legendre polynomials of degree <= 2n (a linear system in that basis).

Only the tests (pins: exactness for monomials up to degree 3n + 1, Gauss nodes
against numpy's leggauss, interlacing, positivity, symmetry) and the parity
tests use it.
"""
from fractions import Fraction

import numpy as np


def _legendre(n, x):
    """P_n(x) and P_n'(x) by the three-term recurrence."""
    p0, p1 = np.ones_like(x), x.copy()
    if n == 0:
        return p0, np.zeros_like(x)
    for k in range(2, n + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    dp = n * (x * p1 - p0) / (x * x - 1.0)
    return p1, dp


def gauss_legendre(n):
    """Nodes and weights of the n-point Gauss-Legendre rule on [-1, 1]."""
    i = np.arange(1, n + 1)
    x = np.cos(np.pi * (i - 0.25) / (n + 0.5))
    for _ in range(100):
        p, dp = _legendre(n, x)
        dx = p / dp
        x = x - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    p, dp = _legendre(n, x)
    w = 2.0 / ((1.0 - x * x) * dp * dp)
    order = np.argsort(x)
    return x[order], w[order]


def _legendre_coeffs(n):
    """Exact monomial coefficients of P_n (lowest degree first)."""
    a, b = [Fraction(1)], [Fraction(0), Fraction(1)]
    if n == 0:
        return a
    for k in range(2, n + 1):
        c = [Fraction(0)] * (k + 1)
        for j, v in enumerate(b):
            c[j + 1] += Fraction(2 * k - 1, k) * v
        for j, v in enumerate(a):
            c[j] -= Fraction(k - 1, k) * v
        a, b = b, c
    return b


def _moment(m):
    """Integral of x^m over [-1, 1]."""
    return Fraction(0) if m % 2 else Fraction(2, m + 1)


def stieltjes(n):
    """Exact coefficients (lowest first, monic) of E_{n+1} for the Legendre weight."""
    pn = _legendre_coeffs(n)
    # int P_n(x) x^k E(x) dx = 0, k = 0..n; E(x) = x^{n+1} + sum_j c_j x^j
    def ip(k, j):
        return sum(cf * _moment(i + k + j) for i, cf in enumerate(pn))
    A = [[ip(k, j) for j in range(n + 1)] for k in range(n + 1)]
    rhs = [-ip(k, n + 1) for k in range(n + 1)]
    # Gaussian elimination over the rationals; E has the parity of n + 1, so
    # half of its coefficients vanish and the matrix is singular in those: drop them.
    keep = [j for j in range(n + 1) if (n + 1 - j) % 2 == 0]
    rows = [k for k in range(n + 1) if any(A[k][j] != 0 for j in keep)]
    M = [[A[k][j] for j in keep] + [rhs[k]] for k in rows]
    m = len(keep)
    M = _row_reduce(M, m)
    c = [Fraction(0)] * (n + 2)
    for t, j in enumerate(keep):
        c[j] = M[t][m]
    c[n + 1] = Fraction(1)
    return c


def _row_reduce(M, m):
    M = [row[:] for row in M]
    r = 0
    for col in range(m):
        piv = next(i for i in range(r, len(M)) if M[i][col] != 0)
        M[r], M[piv] = M[piv], M[r]
        M[r] = [v / M[r][col] for v in M[r]]
        for i in range(len(M)):
            if i != r and M[i][col] != 0:
                f = M[i][col]
                M[i] = [a - f * b for a, b in zip(M[i], M[r])]
        r += 1
    return M[:m]


def gauss_kronrod(n):
    """(nodes, Kronrod weights, embedded Gauss weights) on [-1, 1]: 2n + 1 nodes,
    Gauss weights zero at the Stieltjes nodes."""
    xg, wg = gauss_legendre(n)
    c = stieltjes(n)
    cf = np.array([float(v) for v in c])
    r = np.roots(cf[::-1]).real
    dc = [v * i for i, v in enumerate(c)][1:]
    polished = []
    for x0 in r:                                         # Newton polish, evaluated exactly in rationals
        x = Fraction(float(x0))
        for _ in range(8):
            f = sum(cv * x ** i for i, cv in enumerate(c))
            d = sum(dv * x ** i for i, dv in enumerate(dc))
            x = Fraction(float(x - f / d))
        polished.append(float(x))
    r = np.array(polished)
    x = np.sort(np.concatenate([xg, r]))
    # weights: exact for P_0..P_{2n}
    V = np.stack([_legendre(k, x)[0] if k else np.ones_like(x) for k in range(2 * n + 1)])
    rhs = np.zeros(2 * n + 1)
    rhs[0] = 2.0
    wk = np.linalg.solve(V, rhs)
    gw = np.zeros_like(x)
    for xi, wi in zip(xg, wg):
        gw[np.argmin(np.abs(x - xi))] = wi
    return x, wk, gw


def pixel_rule(name):
    """(offsets in pixel units on [-1/2, 1/2], weights summing to 1, embedded
    Gauss weights or None) for 'pointN'... names: 'subN' (N x N midpoint),
    'g3k7', 'g5k11', 'g7k15'."""
    if name.startswith("sub") or name == "point":
        N = 1 if name == "point" else int(name[3:])
        x = (np.arange(N) + 0.5) / N - 0.5
        return x, np.full(N, 1.0 / N), None
    n = {"g3k7": 3, "g5k11": 5, "g7k15": 7}[name]
    x, wk, gw = gauss_kronrod(n)
    return 0.5 * x, 0.5 * wk, 0.5 * gw
