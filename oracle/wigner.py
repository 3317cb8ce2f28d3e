"""Wigner coupling coefficients in exact rational arithmetic (oracle).

Pinned: every function here is checked in tests/test_oracle_wigner.py
against sympy.physics.wigner (a library routine), closed forms and
orthogonality relations.

All spins are passed doubled (2j as an integer) so half-integers are exact.

* ``w6j`` follows the paper's Appendix A, Eq. (A3): the Racah single sum over
  n between n_min = max(n~1..n~5) and n_max = min(n~6..n~8) with the
  triangle coefficient g~ of Eq. (A4), zero if a triangle or integrality
  condition fails.
* ``w9j`` follows Eq. (A2): sum over x of (-1)^(2x) (2x+1) times three 6j;
  x runs in integer steps over the range printed there, with x < 0 skipped
  (the triangle conditions inside the 6j zero all other terms).
* ``ctilde`` is Eq. (4): sqrt((2j1'+1)(2j2'+1)(2j+1)(2k+1)) W9j.
"""
from fractions import Fraction
from math import factorial, isqrt
import math


def _tri(a, b, c):
    """Triangle and integrality condition for doubled spins a, b, c."""
    return (abs(a - b) <= c <= a + b) and ((a + b + c) % 2 == 0)


def _gt2(a, b, c):
    """Square of the triangle coefficient g~(a,b,c) of Eq. (A4), as a Fraction."""
    return Fraction(factorial((a + b - c) // 2) * factorial((a - b + c) // 2)
                    * factorial((-a + b + c) // 2), factorial((a + b + c) // 2 + 1))


def _sqrt_frac(f):
    """Float square root of a non-negative Fraction (one rounding)."""
    return math.sqrt(f.numerator) / math.sqrt(f.denominator) if f.numerator < 2 ** 52 \
        else math.exp(0.5 * (math.log(f.numerator) - math.log(f.denominator)))


def w6j_exact(a, b, c, d, e, f):
    """Return (sign*sqrt_part, sum_part) with 6j = sqrt(sqrt_part) * sum_part exactly."""
    if not (_tri(a, b, c) and _tri(c, d, e) and _tri(a, e, f) and _tri(b, d, f)):
        return Fraction(0), Fraction(0)
    n2 = (a + b + c) // 2
    n3 = (c + d + e) // 2
    n4 = (a + e + f) // 2
    n5 = (b + d + f) // 2
    n6 = (a + b + d + e) // 2
    n7 = (a + c + d + f) // 2
    n8 = (b + c + e + f) // 2
    nmin = max(0, n2, n3, n4, n5)
    nmax = min(n6, n7, n8)
    s = Fraction(0)
    for n in range(nmin, nmax + 1):
        den = (factorial(n - n2) * factorial(n - n3) * factorial(n - n4) * factorial(n - n5)
               * factorial(n6 - n) * factorial(n7 - n) * factorial(n8 - n))
        s += Fraction((-1) ** n * factorial(n + 1), den)
    return _gt2(a, b, c) * _gt2(c, d, e) * _gt2(a, e, f) * _gt2(b, d, f), s


def w6j(a, b, c, d, e, f):
    """Wigner 6j {a b c; d e f} (doubled spins) as float."""
    sq, s = w6j_exact(a, b, c, d, e, f)
    if s == 0:
        return 0.0
    return float(s) * _sqrt_frac(sq)


def w9j(j1, j2, j, k1, k2, k, j1p, j2p, jp):
    """Wigner 9j {j1 j2 j; k1 k2 k; j1' j2' j'} by Eq. (A2) (doubled spins)."""
    xmin = max(j1 - jp, j2 - k, k1 - j2p)
    xmax = min(j1 + jp, j2 + k, k1 + j2p)
    tot = 0.0
    x = xmin
    while x <= xmax:
        if x >= 0:
            t = (w6j(j1, j2, j, k, jp, x) * w6j(k1, k2, k, j2, x, j2p)
                 * w6j(j1p, j2p, jp, x, j1, k1))
            tot += (-1) ** x * (x + 1) * t
        x += 2
    return tot


def ctilde(j1, j2, j, k1, k2, k, j1p, j2p, jp):
    """Scalar factor C~ of Eq. (4) (doubled spins)."""
    w = w9j(j1, j2, j, k1, k2, k, j1p, j2p, jp)
    if w == 0.0:
        return 0.0
    return math.sqrt((j1p + 1) * (j2p + 1) * (j + 1) * (k + 1)) * w


def cg(j1, m1, j2, m2, J, M):
    """Clebsch-Gordan <j1 m1; j2 m2 | J M> (doubled arguments), Racah formula."""
    if m1 + m2 != M or abs(m1) > j1 or abs(m2) > j2 or abs(M) > J:
        return 0.0
    if not _tri(j1, j2, J) or (j1 + m1) % 2 or (j2 + m2) % 2 or (J + M) % 2:
        return 0.0
    F = factorial
    pre = Fraction((J + 1) * F((j1 + j2 - J) // 2) * F((j1 - j2 + J) // 2)
                   * F((-j1 + j2 + J) // 2), F((j1 + j2 + J) // 2 + 1))
    pre *= (F((j1 + m1) // 2) * F((j1 - m1) // 2) * F((j2 + m2) // 2)
            * F((j2 - m2) // 2) * F((J + M) // 2) * F((J - M) // 2))
    s = Fraction(0)
    for kk in range(0, (j1 + j2 - J) // 2 + 1):
        d = [kk, (j1 + j2 - J) // 2 - kk, (j1 - m1) // 2 - kk, (j2 + m2) // 2 - kk,
             (J - j2 + m1) // 2 + kk, (J - j1 - m2) // 2 + kk]
        if min(d) < 0:
            continue
        den = 1
        for x in d:
            den *= F(x)
        s += Fraction((-1) ** kk, den)
    return float(s) * _sqrt_frac(pre)
