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

Label order (fixes the position index of every family member):
  single labels: ascending.
  pairs inside L (A, B) and right-block pairs (P, Q on R), in groups:
    1. x < y, both in L, lexicographic      2. (x, x), x in L, ascending
    3. (x, p), x in L, ascending            4. (x, p+1), x in L, ascending
    5. pairs of the two site orbitals: (p, p), (p, p+1), (p+1, p+1)
  (groups 3-5 exist only for R; families with x < y drop the diagonal ones).
  left-block pairs (P, Q on L): lexicographic (x outer, y inner).
This grouping keeps the positions of the partner operators of one
operator-table row consecutive, so their products form long stripes.
A left block may instead hold P and Q for every pair of its outside orbitals
(``all_pairs``: x <= y, x < y for P1, both in [p, L), lexicographic), the
form a renormalization needs to produce P and Q of the next block.
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


def labels(fam: int, role: str, n_orb: int, p: int, all_pairs: bool = False):
    """Canonical label list of a family on block ``role`` (``all_pairs``: a
    left block's P and Q over every outside pair)."""
    lo, hi = block_range(role, n_orb, p)
    inside = list(range(lo, hi))
    if fam == H:
        return [()]
    if fam == C:
        return [(i,) for i in inside]
    if fam in (A0, B0, B1):
        return grouped_pairs(inside, p, False, with_sites=False)
    if fam == A1:
        return grouped_pairs(inside, p, True, with_sites=False)
    out = outside(role, n_orb, p)
    if fam == S:
        return [(x,) for x in out]
    strict = fam == P1
    if role == "R":
        return grouped_pairs(list(range(0, p)), p, strict, with_sites=True)
    res = []
    for x in out:
        for y in out:
            if (x < y) if strict else (x <= y):
                if x >= p + 2 and y >= p + 2 and not all_pairs:
                    continue
                res.append((x, y))
    return res


def grouped_pairs(inner, p, strict, with_sites):
    """Pairs of ``inner`` orbitals (and, for the right block, sites) in group order."""
    res = [(x, y) for x in inner for y in inner if x < y]
    if not strict:
        res += [(x, x) for x in inner]
    if with_sites:
        res += [(x, p) for x in inner]
        res += [(x, p + 1) for x in inner]
        res += [(p, p + 1)] if strict else [(p, p), (p, p + 1), (p + 1, p + 1)]
    return res
