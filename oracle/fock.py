"""Determinant-space Hamiltonian, full CI and <S^2> (oracle).

Spin-orbital order: orbital j has bit 2j (spin up) and bit 2j+1 (spin
down); a determinant is a+_{b1} a+_{b2} ... |0> with b1 < b2 < ... .  The
Hamiltonian is Eq. (1) of the paper in its spin-free form,

    H = sum_ij h_ij E_ij + 1/2 sum_ijkl (ij|kl) (E_ij E_kl - delta_jk E_il),
    E_ij = sum_s a+_is a_js,

(E_ij E_kl - delta_jk E_il equals sum_st a+_is a+_kt a_lt a_js), assembled from
single-excitation matrices in one (N, M_S) sector.

Pinned in tests/test_oracle_fock.py: Hubbard dimer closed form, the
non-interacting limit (orbital energies of h), S^2 eigenvalues S(S+1),
hermiticity, and a direct string-by-string check of the identity above
on random determinants.
"""
import itertools
import numpy as np
import scipy.sparse as sp


def popcount(x):
    x = np.asarray(x, dtype=np.int64)
    c = np.zeros_like(x)
    y = x.copy()
    while np.any(y):
        c += y & 1
        y >>= 1
    return c


def sector_states(n_orb, n_elec, two_m):
    """Sorted determinants (int64) with n_elec electrons and 2*M_S = two_m."""
    nup = (n_elec + two_m) // 2
    ndn = (n_elec - two_m) // 2
    if nup < 0 or ndn < 0 or nup > n_orb or ndn > n_orb or nup + ndn != n_elec:
        return np.zeros(0, dtype=np.int64)
    out = []
    for ups in itertools.combinations(range(n_orb), nup):
        u = sum(1 << (2 * j) for j in ups)
        for dns in itertools.combinations(range(n_orb), ndn):
            out.append(u + sum(1 << (2 * j + 1) for j in dns))
    return np.array(sorted(out), dtype=np.int64)


def excitation(states_from, states_to, a, b):
    """Sparse matrix of a+_a a_b (spin-orbital bits) from one list to another."""
    det = states_from
    has_b = ((det >> b) & 1) == 1
    mid = det ^ (1 << b)
    ok = has_b & ((((mid >> a) & 1) == 0))
    src = np.nonzero(ok)[0]
    d0 = det[src]
    m0 = mid[src]
    new = m0 | (1 << a)
    sgn = popcount(d0 & ((1 << b) - 1)) + popcount(m0 & ((1 << a) - 1))
    pos = np.searchsorted(states_to, new)
    pos = np.minimum(pos, len(states_to) - 1)
    hit = states_to[pos] == new
    vals = np.where(sgn[hit] % 2 == 1, -1.0, 1.0)
    return sp.csr_matrix((vals, (pos[hit], src[hit])),
                         shape=(len(states_to), len(states_from)))


def hamiltonian(h, eri, states):
    """Sparse H restricted to one (N, M_S) determinant list."""
    L = h.shape[0]
    n = len(states)
    E = {}
    for i in range(L):
        for j in range(L):
            E[(i, j)] = (excitation(states, states, 2 * i, 2 * j)
                         + excitation(states, states, 2 * i + 1, 2 * j + 1)).tocoo()
    rows = np.concatenate([E[k].row for k in E])
    cols = np.concatenate([E[k].col for k in E])
    vals = np.concatenate([E[k].data for k in E])
    which = np.concatenate([np.full(E[k].nnz, k[0] * L + k[1]) for k in E])

    def combo(coef):
        """sum_kl coef[k, l] E_kl as one CSR matrix."""
        c = coef.reshape(-1)[which]
        return sp.csr_matrix((vals * c, (rows, cols)), shape=(n, n))

    one = h.copy()
    for i in range(L):
        for l in range(L):
            # - 1/2 sum_j (ij|jl) E_il  (the delta_jk part of E_ij E_kl)
            one[i, l] -= 0.5 * sum(eri[i, j, j, l] for j in range(L))
    H = combo(one)
    parts = [H]
    for i in range(L):
        for j in range(L):
            if not np.any(eri[i, j]):
                continue
            parts.append(0.5 * (E[(i, j)].tocsr() @ combo(eri[i, j])))
    out = parts[0]
    for m in parts[1:]:
        out = out + m
    return out.tocsr()


def s_squared(n_orb, states, two_m):
    """Sparse S^2 = S_- S_+ + S_z^2 + S_z on one (N, M_S) determinant list."""
    n_elec = int(popcount(states[:1])[0]) if len(states) else 0
    up = sector_states(n_orb, n_elec, two_m + 2)
    sz = two_m / 2.0
    n = len(states)
    S2 = sp.identity(n, format="csr") * (sz * sz + sz)
    if len(up):
        Sp = None
        for j in range(n_orb):
            t = excitation(states, up, 2 * j, 2 * j + 1)
            Sp = t if Sp is None else Sp + t
        S2 = S2 + (Sp.T @ Sp)
    return S2.tocsr()


def fci(h, eri, n_elec, two_s, n_roots=None):
    """Lowest energy of total spin S (two_s doubled) by dense diagonalisation.

    Diagonalises H in the M_S = S determinant space and returns the lowest
    root whose <S^2> equals S(S+1) within 1e-8, plus all roots and <S^2>.
    """
    L = h.shape[0]
    st = sector_states(L, n_elec, two_s)
    H = hamiltonian(h, eri, st).toarray()
    S2 = s_squared(L, st, two_s)
    w, v = np.linalg.eigh(H)
    s2 = np.sum(v * (S2 @ v), axis=0)
    S = two_s / 2.0
    for i in range(len(w)):
        if abs(s2[i] - S * (S + 1)) < 1e-8:
            return w[i], v[:, i], st, w, s2
    raise RuntimeError("no root of the requested spin")


def product_basis_matrix(prob, he, states):
    """Columns: determinant-space vectors of the product states used by ``he``.

    A product state |a>_L |d>_sites |b>_R is the Jordan-Wigner product of the
    exact block states (Fock vectors supplied by the input generator) and
    the two site states; with orbital-major bit order it is the determinant
    whose bits are the concatenation of the parts.  Returns a dense matrix
    [len(states), n_product] and the list of product keys (gL, d, iL, iR)
    in the order used by ``flatten``.
    """
    p = prob.p
    bl, br = prob.left, prob.right
    nL = p
    cols = []
    keys = []
    index = {int(s): i for i, s in enumerate(states)}

    def group_vectors(blk, mb, g):
        vecs = [None] * mb.gdim[g]
        for (s, M2), (gg, o) in mb.gidx.items():
            if gg != g:
                continue
            S2 = blk.sectors[s][1]
            V = blk.basis[s][(S2 - M2) // 2]
            for a in range(V.shape[1]):
                vecs[o + a] = V[:, a]
        return vecs

    for gL in sorted(he.mL.gdim):
        vL = group_vectors(bl, he.mL, gL)
        for d in range(16):
            gR = he._gR(gL, d)
            if gR not in he.mR.gdim:
                continue
            vR = group_vectors(br, he.mR, gR)
            dbits = (d // 4) | ((d % 4) << 2)
            for ia, va in enumerate(vL):
                for ib, vb in enumerate(vR):
                    col = np.zeros(len(states))
                    for xa in np.nonzero(va)[0]:
                        for xb in np.nonzero(vb)[0]:
                            det = int(xa) | (dbits << (2 * nL)) | (int(xb) << (2 * (nL + 2)))
                            if det in index:
                                col[index[det]] += va[xa] * vb[xb]
                    cols.append(col)
                    keys.append((gL, d, ia, ib))
    return np.stack(cols, axis=1), keys


def u1_to_flat(u1, keys):
    """Product-basis dict (values [1, dimL, dimR]) -> flat vector in ``keys`` order."""
    out = np.zeros(len(keys))
    for n, (gL, d, ia, ib) in enumerate(keys):
        m = u1.get((gL, d))
        if m is not None:
            out[n] = m[0, ia, ib]
    return out


def flat_to_u1(flat, keys, he):
    out = {}
    for n, (gL, d, ia, ib) in enumerate(keys):
        key = (gL, d)
        if key not in out:
            gR = he._gR(gL, d)
            out[key] = np.zeros((1, he.mL.gdim[gL], he.mR.gdim[gR]))
        out[key][0, ia, ib] = flat[n]
    return out


def heff_fock(prob, he, psi):
    """y = P^T H P psi with P built in the determinant space (exact blocks)."""
    st = sector_states(prob.n_orb, prob.n_elec, prob.two_s)
    B, keys = product_basis_matrix(prob, he, st)
    H = hamiltonian(prob.h, prob.eri, st)
    x = B @ u1_to_flat(he.expand(psi), keys)
    y = B.T @ (H @ x)
    return he.project(flat_to_u1(y, keys, he))[:, 0]
