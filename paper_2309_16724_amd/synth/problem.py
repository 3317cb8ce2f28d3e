"""Two-site problems: sector tables, reduced block operators, integrals.

Two builders:

* ``exact_problem``: block operators of small blocks computed exactly from
  the block's Fock space.  Multiplets are the highest-weight eigenstates of
  the block Hamiltonian in every (N, S) sector; the M < S members follow by
  the spin-lowering operator (Condon-Shortley phases).  Reduced elements use
  the convention <J'M'|T^k_q|JM> = <JM; kq|J'M'> <J'||T||J>.  Optional
  truncation keeps the ``max_mult`` lowest-energy multiplets.
* ``random_problem``: synthetic sector tables shaped like the paper's
  workloads and random reduced blocks obeying the selection rules; the
  diagonal-label members of the self-adjoint families are made
  self-adjoint so that the effective Hamiltonian is symmetric.

Layout of every operator family on a block: one record per
(family, row sector, column sector) holding all positions of the family,
stored as [npos][rows][cols] with each matrix column-major.
"""
from dataclasses import dataclass, field
import os
from math import factorial, sqrt
import numpy as np
import scipy.sparse as sp

from . import catalogue as cat
from .integrals import make_integrals, middle_bond


# ---------------------------------------------------------------- containers
@dataclass
class BlockData:
    role: str                       # "L" or "R"
    n_orb: int
    p: int                          # left site of the bond
    sectors: list                   # [(N, two_s, dim)]
    records: list = field(default_factory=list)   # [(fam, row_sec, col_sec, off, npos)]
    data: np.ndarray = None         # float64, concatenated records
    # exact blocks only: per sector a list (over M = S, S-1, ..., -S) of
    # Fock-space matrices (4^n x dim); plus the block's orbital range
    basis: list = None
    # left blocks: P and Q over every outside pair (catalogue.labels)
    all_pairs: bool = False

    def labels(self, fam):
        return cat.labels(fam, self.role, self.n_orb, self.p, self.all_pairs)

    @property
    def dim(self):
        return sum(s[2] for s in self.sectors)

    def rec_array(self):
        """Records as an int64 array [n, 5]: fam, row_sec, col_sec, off, npos."""
        return np.array(self.records, dtype=np.int64).reshape(-1, 5)

    def block(self, fam, row_sec, col_sec):
        """All positions of one record as an array [npos, rows, cols] (or None)."""
        for (f, r, c, off, npos) in self.records:
            if f == fam and r == row_sec and c == col_sec:
                dr, dc = self.sectors[r][2], self.sectors[c][2]
                a = self.data[off:off + npos * dr * dc]
                return a.reshape(npos, dc, dr).transpose(0, 2, 1)
        return None

    def families(self):
        return sorted({r[0] for r in self.records})


@dataclass
class Problem:
    n_orb: int
    n_elec: int
    two_s: int
    p: int
    h: np.ndarray
    eri: np.ndarray
    left: BlockData
    right: BlockData
    kind: str = "exact"


# ------------------------------------------------------------ small helpers
def _cg(j1, m1, j2, m2, J, M):
    """Clebsch-Gordan <j1 m1; j2 m2 | J M>, all arguments doubled integers."""
    if m1 + m2 != M or abs(m1) > j1 or abs(m2) > j2 or abs(M) > J:
        return 0.0
    if J < abs(j1 - j2) or J > j1 + j2 or (j1 + j2 + J) % 2:
        return 0.0
    if (j1 + m1) % 2 or (j2 + m2) % 2 or (J + M) % 2:
        return 0.0
    f = factorial
    a = (j1 + j2 - J) // 2
    b = (j1 - j2 + J) // 2
    c = (-j1 + j2 + J) // 2
    pre = sqrt((J + 1) * f(a) * f(b) * f(c) / f((j1 + j2 + J) // 2 + 1))
    pre *= sqrt(f((j1 + m1) // 2) * f((j1 - m1) // 2) * f((j2 + m2) // 2)
                * f((j2 - m2) // 2) * f((J + M) // 2) * f((J - M) // 2))
    s = 0.0
    for k in range(0, (j1 + j2 - J) // 2 + 1):
        d = [k, (j1 + j2 - J) // 2 - k, (j1 - m1) // 2 - k, (j2 + m2) // 2 - k,
             (J - j2 + m1) // 2 + k, (J - j1 - m2) // 2 + k]
        if min(d) < 0:
            continue
        den = 1
        for x in d:
            den *= f(x)
        s += (-1) ** k / den
    return pre * s


def _valid_spins(n, N):
    """Doubled total spins available to N electrons in n spatial orbitals."""
    if N < 0 or N > 2 * n:
        return []
    smax = min(N, 2 * n - N)
    return list(range(smax % 2, smax + 1, 2))


def weyl_dim(n, N, two_s):
    """Number of spin multiplets (N, S) in n orbitals (Weyl-Paldus)."""
    S2 = two_s
    if (N + S2) % 2 or S2 < 0:
        return 0
    a = (N - S2) // 2
    b = n - (N + S2) // 2
    if a < 0 or b < 0 or N > 2 * n:
        return 0
    from math import comb
    return (S2 + 1) * comb(n + 1, a) * comb(n + 1, b) // (n + 1)


# ------------------------------------------------------ Fock-space operators
class _Fock:
    """Fock space of n spatial orbitals; spin-orbital bit 2j (up), 2j+1 (down)."""

    def __init__(self, n):
        self.n = n
        self.dim = 4 ** n
        st = np.arange(self.dim, dtype=np.int64)
        self.nel = np.array([bin(x).count("1") for x in st])
        up = np.zeros(self.dim, dtype=np.int64)
        dn = np.zeros(self.dim, dtype=np.int64)
        for j in range(n):
            up += (st >> (2 * j)) & 1
            dn += (st >> (2 * j + 1)) & 1
        self.two_m = (up - dn).astype(np.int64)
        self._cre = {}
        for j in range(n):
            for s in (0, 1):
                self._cre[(j, s)] = self._make_cre(2 * j + s)

    def _make_cre(self, b):
        st = np.arange(self.dim, dtype=np.int64)
        free = ((st >> b) & 1) == 0
        src = st[free]
        dst = src | (1 << b)
        below = src & ((1 << b) - 1)
        sign = np.array([(-1) ** bin(x).count("1") for x in below], dtype=float)
        return sp.csr_matrix((sign, (dst, src)), shape=(self.dim, self.dim))

    def cre(self, j, s):          # a+_{j,s}; s = 0 up, 1 down
        return self._cre[(j, s)]

    def ann(self, j, s):
        return self._cre[(j, s)].T.tocsr()

    # rank-1/2 tensor components, q doubled (+1 / -1)
    def t_cre(self, j, q):
        return self.cre(j, 0 if q > 0 else 1)

    def t_ann(self, j, q):        # a~_q = (-1)^(1/2-q) a_{-q}
        return self.ann(j, 1) if q > 0 else -self.ann(j, 0)


def _couple(T, kT, U, kU, K):
    """Components {Q: matrix} of [T (x) U]^K; T, U dicts {q: matrix}, doubled ranks."""
    out = {}
    for Q in range(-K, K + 1, 2):
        acc = None
        for qt, mt in T.items():
            qu = Q - qt
            if qu not in U:
                continue
            c = _cg(kT, qt, kU, qu, K, Q)
            if c == 0.0:
                continue
            term = c * (mt @ U[qu])
            acc = term if acc is None else acc + term
        if acc is not None:
            out[Q] = acc
    return out


def _sz(F):
    return sp.diags(F.two_m / 2.0)


def _s_plus(F):
    acc = sp.csr_matrix((F.dim, F.dim))
    for j in range(F.n):
        acc = acc + F.cre(j, 0) @ F.ann(j, 1)
    return acc.tocsr()


# ---------------------------------------------------------- exact builder
def _block_hamiltonian(F, h, eri, orbs):
    n = F.n
    E = {}
    for a in range(n):
        for b in range(n):
            E[(a, b)] = F.cre(a, 0) @ F.ann(b, 0) + F.cre(a, 1) @ F.ann(b, 1)
    H = sp.csr_matrix((F.dim, F.dim))
    for a in range(n):
        for b in range(n):
            ia, ib = orbs[a], orbs[b]
            if h[ia, ib] != 0.0:
                H = H + h[ia, ib] * E[(a, b)]
    for a in range(n):
        for b in range(n):
            for c in range(n):
                for d in range(n):
                    v = eri[orbs[a], orbs[b], orbs[c], orbs[d]]
                    if v == 0.0:
                        continue
                    t = E[(a, b)] @ E[(c, d)]
                    if b == c:
                        t = t - E[(a, d)]
                    H = H + 0.5 * v * t
    return H.tocsr()


def _multiplets(F, H):
    """Highest-weight multiplet vectors per (N, 2S), sorted by energy."""
    Sp = _s_plus(F)
    Sm = Sp.T.tocsr()
    Sz = _sz(F)
    S2 = (Sm @ Sp + Sz @ Sz + Sz).tocsr()
    res = []
    for N in range(0, 2 * F.n + 1):
        for two_s in _valid_spins(F.n, N):
            idx = np.where((F.nel == N) & (F.two_m == two_s))[0]
            if len(idx) == 0:
                continue
            s2 = S2[idx][:, idx].toarray()
            w, v = np.linalg.eigh(s2)
            S = two_s / 2.0
            keep = np.abs(w - S * (S + 1)) < 1e-8
            V = v[:, keep]
            if V.shape[1] == 0:
                continue
            Hs = H[idx][:, idx].toarray()
            e, u = np.linalg.eigh(V.T @ Hs @ V)
            W = V @ u
            for c in range(W.shape[1]):
                k = int(np.argmax(np.abs(W[:, c]) > np.abs(W[:, c]).max() - 1e-10))
                if W[k, c] < 0:
                    W[:, c] = -W[:, c]
            full = np.zeros((F.dim, W.shape[1]))
            full[idx] = W
            for c in range(W.shape[1]):
                res.append((float(e[c]), N, two_s, full[:, c]))
    return res, Sm


def _m_ladder(vec_hw, two_s, Sm):
    """Columns for M = S, S-1, ..., -S (doubled), Condon-Shortley lowering."""
    out = [vec_hw]
    cur = vec_hw
    two_m = two_s
    while two_m > -two_s:
        S, M = two_s / 2.0, two_m / 2.0
        cur = (Sm @ cur) / sqrt((S + M) * (S - M + 1))
        out.append(cur)
        two_m -= 2
    return out


def _reduce(T, k2, basis, sectors):
    """Reduced blocks {(b, a): matrix} of tensor T (dict q -> Fock matrix)."""
    blocks = {}
    for a, (Na, sa, da) in enumerate(sectors):
        for b, (Nb, sb, db) in enumerate(sectors):
            if sb < abs(sa - k2) or sb > sa + k2:
                continue
            best = None
            for q in range(-k2, k2 + 1, 2):
                ma = sb - q
                if abs(ma) > sa or q not in T:
                    continue
                c = _cg(sa, ma, k2, q, sb, sb)
                if c != 0.0 and (best is None or abs(c) > abs(best[0])):
                    best = (c, q, ma)
            if best is None:
                continue
            c, q, ma = best
            Vb = basis[b][0]
            Va = basis[a][(sa - ma) // 2]
            m = (Vb.T @ (T[q] @ Va)) / c
            if np.abs(m).max() > 1e-13:
                blocks[(b, a)] = m
    return blocks


def _family_tensors(F, fam, lab, orbs, eri):
    """Fock-matrix components of one family member (dict q -> matrix)."""
    loc = {o: i for i, o in enumerate(orbs)}
    cre = lambda j: {1: F.t_cre(j, 1), -1: F.t_cre(j, -1)}
    ann = lambda j: {1: F.t_ann(j, 1), -1: F.t_ann(j, -1)}
    n = F.n
    if fam == cat.C:
        return {q: m for q, m in cre(loc[lab[0]]).items()}
    if fam in (cat.A0, cat.A1):
        K = 0 if fam == cat.A0 else 2
        return _couple(cre(loc[lab[0]]), 1, cre(loc[lab[1]]), 1, K)
    if fam in (cat.B0, cat.B1):
        K = 0 if fam == cat.B0 else 2
        return _couple(cre(loc[lab[0]]), 1, ann(loc[lab[1]]), 1, K)
    if fam == cat.S:
        x = lab[0]
        out = {}
        for j in range(n):
            W = None
            for k in range(n):
                for l in range(n):
                    v = eri[x, orbs[j], orbs[k], orbs[l]]
                    if v == 0.0:
                        continue
                    e0 = _couple(cre(k), 1, ann(l), 1, 0)[0]
                    W = v * e0 if W is None else W + v * e0
            if W is None:
                continue
            for q, m in ann(j).items():
                out[q] = W @ m if q not in out else out[q] + W @ m
        return out
    if fam in (cat.P0, cat.P1):
        K = 0 if fam == cat.P0 else 2
        x, y = lab
        out = {}
        for j in range(n):
            for l in range(n):
                v = eri[x, orbs[j], y, orbs[l]]
                if v == 0.0:
                    continue
                for q, m in _couple(ann(l), 1, ann(j), 1, K).items():
                    out[q] = v * m if q not in out else out[q] + v * m
        return out
    if fam in (cat.Q0, cat.Q1):
        K = 0 if fam == cat.Q0 else 2
        x, y = lab
        out = {}
        for i in range(n):
            for j in range(n):
                if K == 0:
                    w = 2.0 * eri[orbs[i], orbs[j], x, y] - eri[orbs[i], y, x, orbs[j]]
                else:
                    w = sqrt(3.0) * eri[orbs[i], y, x, orbs[j]]
                if w == 0.0:
                    continue
                for q, m in _couple(cre(i), 1, ann(j), 1, K).items():
                    out[q] = w * m if q not in out else out[q] + w * m
        return out
    raise ValueError(fam)


def _pack(block: BlockData, fam_blocks):
    """fam_blocks: {fam: {(row, col): array [npos, rows, cols]}} -> records/data."""
    recs, chunks, off = [], [], 0
    for fam in sorted(fam_blocks):
        for (r, c) in sorted(fam_blocks[fam]):
            arr = fam_blocks[fam][(r, c)]
            npos = arr.shape[0]
            flat = np.ascontiguousarray(arr.transpose(0, 2, 1)).reshape(-1)
            recs.append((fam, r, c, off, npos))
            chunks.append(flat)
            off += flat.size
    block.records = recs
    block.data = np.concatenate(chunks) if chunks else np.zeros(0)


def build_exact_block(role, n_orb, p, h, eri, max_mult=None, all_pairs=False):
    lo, hi = cat.block_range(role, n_orb, p)
    orbs = list(range(lo, hi))
    n = len(orbs)
    F = _Fock(n)
    H = _block_hamiltonian(F, h, eri, orbs)
    mults, Sm = _multiplets(F, H)
    if max_mult is not None and len(mults) > max_mult:
        order = sorted(range(len(mults)),
                       key=lambda i: (mults[i][0], mults[i][1], mults[i][2], i))
        keep = set(order[:max_mult])
        mults = [m for i, m in enumerate(mults) if i in keep]
    # group into sectors in (N, 2S) order, energy order inside
    groups = {}
    for e, N, s2, v in mults:
        groups.setdefault((N, s2), []).append((e, v))
    sectors, basis = [], []
    for key in sorted(groups):
        items = sorted(groups[key], key=lambda t: t[0])
        hw = np.stack([v for _, v in items], axis=1)
        sectors.append((key[0], key[1], hw.shape[1]))
        ladder = _m_ladder(hw, key[1], Sm)
        basis.append(ladder)
    blk = BlockData(role, n_orb, p, sectors, basis=basis, all_pairs=all_pairs and role == "L")
    fams = cat.LEFT_FAMILIES if role == "L" else cat.RIGHT_FAMILIES
    fam_blocks = {}
    for fam in fams:
        labs = blk.labels(fam)
        if fam == cat.H:
            per = [_reduce({0: H}, 0, basis, sectors)]
        else:
            per = [_reduce(_family_tensors(F, fam, lab, orbs, eri), cat.TWO_K[fam],
                           basis, sectors) for lab in labs]
        keys = sorted({k for d in per for k in d})
        if not keys:
            continue
        fb = {}
        for (b, a) in keys:
            db, da = sectors[b][2], sectors[a][2]
            arr = np.zeros((len(per), db, da))
            for i, d in enumerate(per):
                if (b, a) in d:
                    arr[i] = d[(b, a)]
            fb[(b, a)] = arr
        fam_blocks[fam] = fb
    _pack(blk, fam_blocks)
    return blk


def exact_problem(n_orb, n_elec, two_s, seed, p=None, max_mult=None, all_pairs=False):
    """Problem with blocks built exactly from their Fock spaces (all_pairs:
    the left block's P and Q over every outside pair)."""
    h, eri = make_integrals(n_orb, seed)
    if p is None:
        p = middle_bond(n_orb)
    left = build_exact_block("L", n_orb, p, h, eri, max_mult, all_pairs)
    right = build_exact_block("R", n_orb, p, h, eri, max_mult)
    return Problem(n_orb, n_elec, two_s, p, h, eri, left, right, "exact")


# ---------------------------------------------------------- random builder
def synthetic_sectors(n, n_share, D, rng, spin_ratio=0.6, sigma_frac=0.15, cap=True):
    """Sector table of a synthetic block of n orbitals with about D multiplets.

    d(N, S) ~ exp(-(N - n_share)^2 / (2 sigma^2)) * spin_ratio^(2S), capped by
    the number of multiplets the block can hold (``cap``), rounded, kept if
    at least 1.  Without the cap a block of few orbitals can carry large
    sectors (abstract blocks for kernel tests with few labels).
    """
    cand = []
    sigma = max(1.0, sigma_frac * n)
    for N in range(0, 2 * n + 1):
        for s2 in _valid_spins(n, N):
            cmax = weyl_dim(n, N, s2)
            if cmax <= 0:
                continue
            if not cap:
                cmax = 1 << 30
            w = np.exp(-(N - n_share) ** 2 / (2 * sigma ** 2)) * spin_ratio ** s2
            cand.append([N, s2, w, cmax])
    tot = sum(c[2] for c in cand)
    secs = []
    for N, s2, w, cmax in cand:
        d = int(round(D * w / tot))
        d = min(d, cmax)
        if d >= 1:
            secs.append((N, s2, d))
    return secs


def _rand_records(role, n_orb, p, sectors, fams, all_pairs=False):
    """Record list [(fam, row_sec, col_sec, npos)] of a synthetic block: every
    (row, column) sector pair the family's electron change and spin rank
    allow (block Hamiltonian: diagonal pairs only), families in order, pairs
    sorted (the packing order of ``_pack``)."""
    recs = []
    for fam in sorted(fams):
        npos = len(cat.labels(fam, role, n_orb, p, all_pairs))
        if npos == 0:
            continue
        k2, dn = cat.TWO_K[fam], cat.DN[fam]
        pairs = []
        for a, (Na, sa, da) in enumerate(sectors):
            for b, (Nb, sb, db) in enumerate(sectors):
                if Nb != Na + dn or sb < abs(sa - k2) or sb > sa + k2:
                    continue
                if fam == cat.H and a != b:
                    continue
                pairs.append((b, a))
        for (b, a) in sorted(pairs):
            recs.append((fam, b, a, npos))
    return recs


def _fill_record(data, off, npos, db, da, seed, key, scale):
    """Random reduced blocks of one record, written straight into its packed
    place ([npos][cols][rows], i.e. each db x da matrix column-major): entries
    N(0, 1) * scale / sqrt(da) from the record's own stream (seeded by the
    problem seed and the record key, so records can be drawn in any order)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed] + list(key)))
    v = data[off:off + npos * db * da]
    rng.standard_normal(out=v)
    v *= scale / sqrt(max(da, 1))
    return rng


def _rand_block(role, n_orb, p, sectors, seed, op_scale, share, n, all_pairs=False):
    """Synthetic block: records, packed data, self-adjoint constraints."""
    blk = BlockData(role, n_orb, p, sectors, all_pairs=all_pairs)
    fams = cat.LEFT_FAMILIES if role == "L" else cat.RIGHT_FAMILIES
    recs = _rand_records(role, n_orb, p, sectors, fams, all_pairs) if n > 0 else []
    offs, off = [], 0
    for (fam, b, a, npos) in recs:
        offs.append(off)
        off += npos * sectors[b][2] * sectors[a][2]
    data = np.empty(off)
    role_id = 0 if role == "L" else 1

    def job(i):
        fam, b, a, npos = recs[i]
        db, da = sectors[b][2], sectors[a][2]
        rng = _fill_record(data, offs[i], npos, db, da, seed, (role_id, fam, b, a),
                           1.0 if fam == cat.H else op_scale)
        if fam == cat.H:
            # spread block energies so the spectrum looks physical
            N = sectors[b][0]
            m = data[offs[i]:offs[i] + db * da].reshape(da, db)   # m[c, r] = H[r, c]
            m[np.arange(db), np.arange(db)] += np.sort(rng.uniform(0, 2.0 * n, db)) \
                + 0.5 * (N - share) ** 2

    from concurrent.futures import ThreadPoolExecutor
    order = sorted(range(len(recs)), key=lambda i: -(offs[i + 1] if i + 1 < len(offs) else off) + offs[i])
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        list(ex.map(job, order))
    # self-adjoint constraints: the block Hamiltonian and the diagonal-label
    # members of B0, B1, Q0, Q1 (T = T^dagger in the reduced convention)
    index = {(fam, b, a): i for i, (fam, b, a, npos) in enumerate(recs)}

    def mat(i, pos):
        fam, b, a, npos = recs[i]
        db, da = sectors[b][2], sectors[a][2]
        o = offs[i] + pos * db * da
        return data[o:o + db * da].reshape(da, db).T       # view of the db x da matrix

    for i, (fam, b, a, npos) in enumerate(recs):
        if fam == cat.H:
            diag = [0]
        elif fam in (cat.B0, cat.B1, cat.Q0, cat.Q1):
            diag = [k for k, lab in enumerate(blk.labels(fam)) if lab[0] == lab[1]]
        else:
            continue
        if b == a:
            for k in diag:
                m = mat(i, k)
                m[...] = 0.5 * (m + m.T)
        elif b < a and (fam, a, b) in index:
            # block (b, a) [rows b, cols a] from block (a, b):
            # T[b,a] = (-1)^((S_a - S_b)) sqrt((2S_a+1)/(2S_b+1)) T[a,b]^T
            sb, sa = sectors[b][1], sectors[a][1]
            ph = (-1) ** (((sa - sb) // 2) % 2) * sqrt((sa + 1) / (sb + 1))
            j = index[(fam, a, b)]
            for k in diag:
                mat(i, k)[...] = ph * mat(j, k).T
    blk.records = [(fam, b, a, offs[i], npos) for i, (fam, b, a, npos) in enumerate(recs)]
    blk.data = data
    return blk


def random_problem(n_orb, n_elec, two_s, seed, D, p=None, spin_ratio=0.6,
                   sigma_frac=0.15, op_scale=0.3, cap=True, D_right=None, all_pairs=False):
    """Problem with synthetic sector tables and random reduced operators.

    D multiplets per block (D_right for the right block when given).  Every
    record draws from its own stream, seeded by the problem seed and the
    record's (block, family, row sector, column sector), so the blocks are
    filled by parallel threads with the same result."""
    h, eri = make_integrals(n_orb, seed)
    if p is None:
        p = middle_bond(n_orb)
    blocks = []
    for role in ("L", "R"):
        lo, hi = cat.block_range(role, n_orb, p)
        n = hi - lo
        share = n_elec * n / n_orb
        Db = D if role == "L" or D_right is None else D_right
        secs = synthetic_sectors(n, share, Db, None, spin_ratio, sigma_frac, cap) if n > 0 \
            else [(0, 0, 1)]
        blocks.append(_rand_block(role, n_orb, p, secs, 10_000_000 + seed, op_scale, share, n,
                                  all_pairs and role == "L"))
    return Problem(n_orb, n_elec, two_s, p, h, eri, blocks[0], blocks[1], "random")


def random_vector(size, seed):
    """Seeded normalised starting vector (the Davidson initial guess)."""
    v = np.random.default_rng(seed).standard_normal(size)
    return v / np.linalg.norm(v)


def batch_specs(n, seed, L_range=(16, 32), D_range=(128, 768), spins=(0, 1), seed0=None):
    """(L, N, 2S, integral seed, D) of n independent solves: L and D uniform
    over the inclusive ranges, N = L electrons, S drawn from `spins` for even
    N and shifted by 1/2 for odd N (no state of odd N has integer spin);
    integral seeds seed0 + k (default seed * 1000 + k)."""
    rng = np.random.default_rng(seed)
    base = seed * 1000 if seed0 is None else seed0
    out = []
    for k in range(n):
        L = int(rng.integers(L_range[0], L_range[1] + 1))
        D = int(rng.integers(D_range[0], D_range[1] + 1))
        two_s = 2 * int(rng.choice(spins)) + (L % 2)
        out.append((L, L, two_s, base + k, D))
    return out


def batch_problems(n, seed, L_range=(16, 32), D_range=(128, 768), spins=(0, 1), seed0=None):
    """Seeded batch of random middle-bond problems from batch_specs."""
    return [random_problem(L, N, s2, sd, D=D)
            for L, N, s2, sd, D in batch_specs(n, seed, L_range, D_range, spins, seed0)]
