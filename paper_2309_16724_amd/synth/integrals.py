"""Seeded one- and two-electron integrals of the synthetic Hamiltonian.

The Hamiltonian is the spin-free two-body operator of Eq. (1) of the paper
with real orbitals, written in chemist notation:

    H = sum_ij h_ij E_ij + 1/2 sum_ijkl (ij|kl) sum_{s,t} a+_is a+_kt a_lt a_js

Draw order (numpy PCG64 generator ``default_rng(seed)``):
  1. h: the upper triangle i <= j in row-major order, standard normals,
     scaled by exp(-|i-j|/2), then mirrored.
  2. (ij|kl): canonical quadruples i>=j, k>=l, (ij)>=(kl) by compound index,
     in lexicographic order; |N(0, sd=0.5)| scaled by
     exp(-(|i-j|+|k-l|)/3), expanded to all 8 index permutations.
"""
import numpy as np


def make_integrals(n_orb: int, seed: int):
    """Return (h, eri) with h of shape (L, L) and eri of shape (L, L, L, L)."""
    L = int(n_orb)
    rng = np.random.default_rng(seed)
    iu = [(i, j) for i in range(L) for j in range(i, L)]
    z = rng.standard_normal(len(iu))
    h = np.zeros((L, L))
    for (i, j), zz in zip(iu, z):
        val = zz * np.exp(-abs(i - j) / 2.0)
        h[i, j] = val
        h[j, i] = val
    quads = []
    for i in range(L):
        for j in range(i + 1):
            ij = i * (i + 1) // 2 + j
            for k in range(i + 1):
                for l in range(k + 1):
                    kl = k * (k + 1) // 2 + l
                    if kl <= ij:
                        quads.append((i, j, k, l))
    v = np.abs(rng.normal(0.0, 0.5, size=len(quads)))
    eri = np.zeros((L, L, L, L))
    for (i, j, k, l), vv in zip(quads, v):
        val = vv * np.exp(-(abs(i - j) + abs(k - l)) / 3.0)
        for (a, b, c, d) in ((i, j, k, l), (j, i, k, l), (i, j, l, k), (j, i, l, k),
                             (k, l, i, j), (l, k, i, j), (k, l, j, i), (l, k, j, i)):
            eri[a, b, c, d] = val
    return h, eri


def middle_bond(n_orb: int) -> int:
    """0-based index p of the left site of the middle two-site bond.

    For even L the two sites are orbitals L/2-1 and L/2 (0-based); for odd L
    they are floor(L/2)-1 and floor(L/2).
    """
    return n_orb // 2 - 1
