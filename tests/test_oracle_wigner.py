"""Pins of oracle/wigner.py: library routine (sympy), closed forms, identities."""
import itertools
import math
import random

import pytest
from sympy import Rational, sqrt as ssqrt
from sympy.physics.wigner import wigner_6j, wigner_9j, clebsch_gordan

from oracle.wigner import w6j, w9j, cg, ctilde

pytestmark = pytest.mark.filterwarnings("ignore")


def R(x2):
    return Rational(x2, 2)


def _tri(a, b, c):
    return abs(a - b) <= c <= a + b and (a + b + c) % 2 == 0


def test_w6j_against_sympy():
    rng = random.Random(1)
    n = 0
    while n < 120:
        a, b, d, e = (rng.randint(0, 6) for _ in range(4))
        c = rng.randint(0, 6)
        f = rng.randint(0, 6)
        if not (_tri(a, b, c) and _tri(c, d, e) and _tri(a, e, f) and _tri(b, d, f)):
            continue
        ref = float(wigner_6j(R(a), R(b), R(c), R(d), R(e), R(f)))
        assert abs(w6j(a, b, c, d, e, f) - ref) < 1e-14
        n += 1


def test_w6j_zero_outside_triangles():
    assert w6j(1, 1, 4, 1, 1, 0) == 0.0
    assert w6j(2, 2, 1, 2, 2, 0) == 0.0


def test_w6j_closed_form_with_zero():
    # {a b c; 0 c b} = (-1)^(a+b+c) / sqrt((2b+1)(2c+1))
    for a, b, c in itertools.product(range(0, 7), repeat=3):
        if not _tri(a, b, c):
            continue
        ref = (-1) ** ((a + b + c) // 2) / math.sqrt((b + 1) * (c + 1))
        assert abs(w6j(a, b, c, 0, c, b) - ref) < 1e-14


def test_w6j_orthogonality():
    # sum_x (2x+1)(2f+1) {a b x; c d f}{a b x; c d f'} = delta_ff'
    for a, b, c, d in itertools.product(range(0, 4), repeat=4):
        fs = [f for f in range(0, 8) if _tri(a, d, f) and _tri(c, b, f)]
        for f in fs:
            for fp in fs:
                s = sum((x + 1) * (f + 1) * w6j(a, b, x, c, d, f) * w6j(a, b, x, c, d, fp)
                        for x in range(0, 8))
                if not any(_tri(a, b, x) and _tri(c, d, x) for x in range(8)):
                    continue
                assert abs(s - (1.0 if f == fp else 0.0)) < 1e-13


def test_w9j_against_sympy():
    rng = random.Random(2)
    n = 0
    while n < 60:
        j1, j2, k1, k2 = (rng.randint(0, 4) for _ in range(4))
        j = rng.randint(0, 8)
        k = rng.randint(0, 4)
        j1p, j2p, jp = rng.randint(0, 5), rng.randint(0, 5), rng.randint(0, 8)
        rows = [(j1, j2, j), (k1, k2, k), (j1p, j2p, jp)]
        cols = [(j1, k1, j1p), (j2, k2, j2p), (j, k, jp)]
        if not all(_tri(*t) for t in rows + cols):
            continue
        ref = float(wigner_9j(R(j1), R(j2), R(j), R(k1), R(k2), R(k), R(j1p), R(j2p), R(jp),
                              prec=64))
        assert abs(w9j(j1, j2, j, k1, k2, k, j1p, j2p, jp) - ref) < 1e-13
        n += 1


def test_w9j_zero_reduces_to_6j():
    # {a b e; c d e; f f 0} = (-1)^(b+c+e+f) / sqrt((2e+1)(2f+1)) {a b e; d c f}
    for a, b, c, d, e, f in itertools.product(range(0, 4), repeat=6):
        if not (_tri(a, b, e) and _tri(c, d, e) and _tri(a, c, f) and _tri(b, d, f)):
            continue
        ref = (-1) ** ((b + c + e + f) // 2) / math.sqrt((e + 1) * (f + 1)) * w6j(a, b, e, d, c, f)
        assert abs(w9j(a, b, e, c, d, e, f, f, 0) - ref) < 1e-13


def test_cg_against_sympy():
    for j1, j2 in itertools.product(range(0, 5), repeat=2):
        for J in range(abs(j1 - j2), j1 + j2 + 1, 2):
            for m1 in range(-j1, j1 + 1, 2):
                for m2 in range(-j2, j2 + 1, 2):
                    M = m1 + m2
                    if abs(M) > J:
                        continue
                    ref = float(clebsch_gordan(R(j1), R(j2), R(J), R(m1), R(m2), R(M)))
                    assert abs(cg(j1, m1, j2, m2, J, M) - ref) < 1e-14


def test_ctilde_is_coupled_product_element():
    """Eq. (4) under <J'M'|T^k_q|JM> = <JM;kq|J'M'><J'||T||J>, primed = bra.

    Builds <(j1'j2')j'M'| [T^k1 x U^k2]^k_q |(j1 j2) j M> from Clebsch-Gordan
    sums with unit reduced elements and compares it with C~ <jM;kq|j'M'>.
    """
    rng = random.Random(3)
    done = 0
    while done < 40:
        j1, j2, k1, k2 = rng.randint(0, 3), rng.randint(0, 2), rng.randint(0, 2), rng.randint(0, 2)
        j = rng.randint(0, 5)
        k = rng.randint(0, 4)
        j1p, j2p, jp = rng.randint(0, 4), rng.randint(0, 3), rng.randint(0, 6)
        if not all(_tri(*t) for t in [(j1, j2, j), (k1, k2, k), (j1p, j2p, jp),
                                       (j1, k1, j1p), (j2, k2, j2p), (j, k, jp)]):
            continue
        # pick M, q with a non-zero <jM;kq|j'M'>
        best = None
        for M in range(-j, j + 1, 2):
            for q in range(-k, k + 1, 2):
                c = cg(j, M, k, q, jp, M + q)
                if abs(c) > 1e-3:
                    best = (M, q, c)
                    break
            if best:
                break
        if best is None:
            continue
        M, q, cgv = best
        Mp = M + q
        val = 0.0
        for m1 in range(-j1, j1 + 1, 2):
            m2 = M - m1
            if abs(m2) > j2:
                continue
            a = cg(j1, m1, j2, m2, j, M)
            if a == 0.0:
                continue
            for q1 in range(-k1, k1 + 1, 2):
                q2 = q - q1
                if abs(q2) > k2:
                    continue
                b = cg(k1, q1, k2, q2, k, q)
                m1p, m2p = m1 + q1, m2 + q2
                if abs(m1p) > j1p or abs(m2p) > j2p:
                    continue
                val += (a * b * cg(j1p, m1p, j2p, m2p, jp, Mp)
                        * cg(j1, m1, k1, q1, j1p, m1p) * cg(j2, m2, k2, q2, j2p, m2p))
        assert abs(val - ctilde(j1, j2, j, k1, k2, k, j1p, j2p, jp) * cgv) < 1e-13
        done += 1
