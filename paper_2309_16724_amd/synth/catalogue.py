"""Operator catalogue shared by the input format: family ids and label lists.

Every reduced block operator handed to the library belongs to one family.
A family has a spin rank k (stored doubled), a fermion parity, a change of
particle number and a position axis (its labels).  Labels are orbital
indices (0-based) of the full problem.  The block of a family is either the
left block L = [0, p) or the right block R = [p+2, L); sites are p and p+1.

    id  name  2k  dN  labels (in canonical order)
    0   H     0   0   one position
    1   C     1  +1   i in block                          a+_i
    2   A0    0  +2   (i<=j) in block            (L only) [a+_i a+_j]^0
    3   A1    2  +2   (i<j)  in block            (L only) [a+_i a+_j]^1
    4   B0    0   0   (i<=j) in block            (L only) [a+_i a~_j]^0
    5   B1    2   0   (i<=j) in block            (L only) [a+_i a~_j]^1
    6   S     1  -1   x outside the block        sum (xj|kl) [[a+_k a~_l]^0 a~_j]^1/2
    7   P0    0  -2   outside pairs (x<=y)       sum (xj|yl) [a~_l a~_j]^0
    8   P1    2  -2   outside pairs (x<y)        sum (xj|yl) [a~_l a~_j]^1
    9   Q0    0   0   outside pairs (x<=y)       sum W0_ij [a+_i a~_j]^0
    10  Q1    2   0   outside pairs (x<=y)       sum W1_ij [a+_i a~_j]^1

with W0_ij = 2 (ij|xy) - (iy|xj) and W1_ij = sqrt(3) (iy|xj); the internal
indices j, k, l, i run over the block.  Outside labels: for L they are the
orbitals [p, L) and, for pairs, only pairs with at least one site orbital
(p or p+1); for R they are [0, p+2) and all pairs of them.
"""

H, C, A0, A1, B0, B1, S, P0, P1, Q0, Q1 = range(11)
NAMES = ["H", "C", "A0", "A1", "B0", "B1", "S", "P0", "P1", "Q0", "Q1"]
TWO_K = [0, 1, 0, 2, 0, 2, 1, 0, 2, 0, 2]
DN = [0, 1, 2, 2, 0, 0, -1, -2, -2, 0, 0]
LEFT_FAMILIES = [H, C, A0, A1, B0, B1, S, P0, P1, Q0, Q1]
RIGHT_FAMILIES = [H, C, S, P0, P1, Q0, Q1]


def block_range(role: str, n_orb: int, p: int):
    return (0, p) if role == "L" else (p + 2, n_orb)


def outside(role: str, n_orb: int, p: int):
    return list(range(p, n_orb)) if role == "L" else list(range(0, p + 2))


def labels(fam: int, role: str, n_orb: int, p: int):
    """Canonical label list of a family on block ``role``."""
    lo, hi = block_range(role, n_orb, p)
    inside = list(range(lo, hi))
    if fam == H:
        return [()]
    if fam == C:
        return [(i,) for i in inside]
    if fam in (A0, B0, B1):
        return [(i, j) for i in inside for j in inside if i <= j]
    if fam == A1:
        return [(i, j) for i in inside for j in inside if i < j]
    out = outside(role, n_orb, p)
    if fam == S:
        return [(x,) for x in out]
    strict = fam == P1
    res = []
    for x in out:
        for y in out:
            if (x < y) if strict else (x <= y):
                if role == "L" and x >= p + 2 and y >= p + 2:
                    continue
                res.append((x, y))
    return res
