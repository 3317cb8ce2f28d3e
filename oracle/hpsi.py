"""H_eff psi from the plain definition, in the M-resolved product basis (oracle).

The effective Hamiltonian of the two-site step is H_eff = P^T H P, where P
maps the reduced coefficients of the coupled basis ((L l) S_Ll (r R) S_rR) S
(at M = S) onto product states |L S_L M_L>|l>|r>|R S_R M_R> (Jordan-Wigner
order L < l < r < R).  This module

1. expands the reduced wavefunction into that product basis with
   Clebsch-Gordan coefficients (``expand``), and every reduced block
   operator into its M-resolved matrices by the Wigner-Eckart theorem
   <J'M'|T^k_q|JM> = <JM; kq|J'M'> <J'||T||J>;
2. applies the second-quantised Hamiltonian of Eq. (1), split into groups
   of terms by how many of its orbital indices fall in L and in R.  Groups
   with two or more indices in a block use that block's pre-contracted
   (complementary) operators, whose definitions are in
   paper_2309_16724_amd.synth.catalogue; every other term is applied as an
   explicit product of single creation/annihilation operators with its
   integral as coefficient.  Spin sums are explicit, adjoints are matrix
   transposes, fermion signs come from reordering the factors into
   partition order and from the particle numbers of the ket;
3. projects back with the transpose of step 1 (``project``).

No 6j/9j recoupling, no sector-task table and no stripe grouping is used.
Grouping of Eq. (1) (n_X = number of indices in block X):
  n_L = 4 or n_R = 4   block Hamiltonians
  n_L = 3 / n_R = 3    1-index complementary S of that block
  n_L = 2, n_R = 2     normal pair operators of L with P, Q of R
  n_L = 2, n_R <= 1    P, Q of L;   n_R = 2, n_L <= 1   P, Q of R
  n_L <= 1, n_R <= 1   explicit products.
Pinned in tests/test_oracle_hpsi.py against P^T H P built in the full
determinant space from the exact block states, against full CI, and by
hermiticity.
"""
from math import sqrt
import numpy as np

from paper_2309_16724_amd.synth import catalogue as cat
from .wigner import cg
from .layout import psi_blocks, SITE

# site Fock states: 0 |0>, 1 |up>, 2 |dn>, 3 |up dn> = a+_up a+_dn |0>
SITE_N = [0, 1, 1, 2]
SITE_2M = [0, 1, -1, 0]
_CRE_UP = np.zeros((4, 4))
_CRE_UP[1, 0] = 1.0
_CRE_UP[3, 2] = 1.0
_CRE_DN = np.zeros((4, 4))
_CRE_DN[2, 0] = 1.0
_CRE_DN[3, 1] = -1.0


def site_cre(s2):
    return _CRE_UP if s2 > 0 else _CRE_DN


def site_ann(s2):
    return site_cre(s2).T


# multiplet -> {2m: Fock state}
SITE_MULT_STATES = [{0: 0}, {1: 1, -1: 2}, {0: 3}]


class MBlock:
    """M-resolved view of one block: groups (N, 2M) and expanded operators.

    ``sel`` (optional) restricts every expanded operator to a set of rows of
    each group ({group: sorted offsets}); groups missing from it take no
    rows.  ``tensor(..., side=0)`` returns an operator's selected rows (the
    rows an output needs); ``side=1`` its selected columns, which is what the
    selected rows of its transpose are made of."""

    def __init__(self, blk, sel=None):
        self.blk = blk
        self.sectors = blk.sectors
        self.gidx = {}      # (sector, 2M) -> (group, offset)
        self.gdim = {}
        for s, (N, S2, d) in enumerate(blk.sectors):
            for M2 in range(S2, -S2 - 1, -2):
                g = (N, M2)
                o = self.gdim.get(g, 0)
                self.gidx[(s, M2)] = (g, o)
                self.gdim[g] = o + d
        self.sel = sel
        self._cache = {}
        self._by_fam = {}
        for rec in blk.records:
            self._by_fam.setdefault(rec[0], []).append(rec)

    def rows(self, g):
        """Selected offsets of group g (all of them without a selection)."""
        if self.sel is None:
            return np.arange(self.gdim[g])
        return self.sel.get(g, np.zeros(0, dtype=np.int64))

    def _pick(self, g, o, d):
        """(positions in the selection of g, offsets within [o, o + d))."""
        r = self.rows(g)
        lo, hi = np.searchsorted(r, o), np.searchsorted(r, o + d)
        return np.arange(lo, hi), r[lo:hi] - o

    def identity(self):
        return {(g, g): np.eye(d)[self.rows(g)] for g, d in self.gdim.items()}

    def tensor(self, fam, pos, q, side=0):
        """M-resolved component q (doubled) of family member ``pos``: {(g', g): M}
        (selected rows for side 0, selected columns for side 1)."""
        if self.sel is None:
            side = 0
        key = (fam, pos, q, side)
        if key in self._cache:
            return self._cache[key]
        k2 = cat.TWO_K[fam]
        out = {}
        for (f, b, a, off, npos) in self._by_fam.get(fam, ()):
            Nb, Sb, db = self.sectors[b]
            Na, Sa, da = self.sectors[a]
            R = self.blk.data[off + pos * db * da: off + (pos + 1) * db * da]
            R = R.reshape(da, db).T
            for Ma in range(Sa, -Sa - 1, -2):
                Mb = Ma + q
                if abs(Mb) > Sb:
                    continue
                c = cg(Sa, Ma, k2, q, Sb, Mb)
                if c == 0.0:
                    continue
                ga, oa = self.gidx[(a, Ma)]
                gb, ob = self.gidx[(b, Mb)]
                if side == 0:
                    pi, ri = self._pick(gb, ob, db)
                    if len(pi) == 0:
                        continue
                    shape = (len(self.rows(gb)), self.gdim[ga])
                else:
                    pi, ci = self._pick(ga, oa, da)
                    if len(pi) == 0:
                        continue
                    shape = (self.gdim[gb], len(self.rows(ga)))
                m = out.get((gb, ga))
                if m is None:
                    m = np.zeros(shape)
                    out[(gb, ga)] = m
                if side == 0:
                    m[pi, oa:oa + da] += c * R[ri, :]
                else:
                    m[ob:ob + db, pi] += c * R[:, ci]
        self._cache[key] = out
        return out

    def labels(self, fam):
        return cat.labels(fam, self.blk.role, self.blk.n_orb, self.blk.p, getattr(self.blk, "all_pairs", False))

    def pos(self, fam, lab):
        return self.labels(fam).index(tuple(lab))


# ----------------------------------------------------------- op algebra
def op_T(a):
    return {(g, gp): m.T for (gp, g), m in a.items()}


def op_lin(*pairs):
    """Linear combination sum c_i * op_i of block operators."""
    out = {}
    for c, a in pairs:
        if c == 0.0:
            continue
        for k, m in a.items():
            if k in out:
                out[k] = out[k] + c * m
            else:
                out[k] = c * m
    return out


def _ph(x2):
    """(-1)^(x2/2) for an even doubled exponent x2."""
    assert x2 % 2 == 0
    return -1.0 if (x2 // 2) % 2 else 1.0


# ---------------------------------------------- spin-orbital block factors
def _memo(fn):
    def wrapped(self, *args):
        key = (fn.__name__,) + args
        hit = self._memo.get(key)
        if hit is None:
            hit = fn(self, *args)
            self._memo[key] = hit
        return hit
    wrapped.__name__ = fn.__name__
    return wrapped


class Factors:
    """Spin-orbital operators of one block, from its stored reduced families.

    Every method takes ``side`` last (see MBlock.tensor): side 0 gives the
    operator's selected rows, side 1 its selected columns; a transpose
    swaps the two."""

    def __init__(self, mb):
        self.mb = mb
        self._memo = {}

    @_memo
    def T(self, name, *args):
        """Transpose (adjoint) of the operator returned by method ``name``."""
        *a, side = args
        return op_T(getattr(self, name)(*a, 1 - side))

    @_memo
    def cre(self, x, s2, side):                # a+_{x s}
        return self.mb.tensor(cat.C, self.mb.pos(cat.C, (x,)), s2, side)

    @_memo
    def ann(self, x, s2, side):
        return op_T(self.cre(x, s2, 1 - side))

    @_memo
    def cc(self, x, y, s2, t2, side):         # a+_{x s} a+_{y t}
        if x > y:
            return op_lin((-1.0, self.cc(y, x, t2, s2, side)))
        terms = []
        for fam, K2 in ((cat.A0, 0), (cat.A1, 2)):
            if fam == cat.A1 and x == y:
                continue
            c = cg(1, s2, 1, t2, K2, s2 + t2)
            if c != 0.0:
                terms.append((c, self.mb.tensor(fam, self.mb.pos(fam, (x, y)), s2 + t2, side)))
        return op_lin(*terms)

    @_memo
    def ca(self, x, y, s2, t2, side):         # a+_{x s} a_{y t}
        if x > y:
            return op_T(self.ca(y, x, t2, s2, 1 - side))
        ph = _ph(1 + t2)                       # (-1)^(1/2 + t)
        terms = []
        for fam, K2 in ((cat.B0, 0), (cat.B1, 2)):
            c = cg(1, s2, 1, -t2, K2, s2 - t2)
            if c != 0.0:
                terms.append((ph * c, self.mb.tensor(fam, self.mb.pos(fam, (x, y)), s2 - t2, side)))
        return op_lin(*terms)

    @_memo
    def S(self, x, s2, side):                  # (S_x)_s = sum (xj|kl) E_kl a_{j s}
        t = self.mb.tensor(cat.S, self.mb.pos(cat.S, (x,)), -s2, side)
        return op_lin((-sqrt(2.0) * _ph(1 + s2), t))

    @_memo
    def P(self, x, y, t2, s2, side):           # (P_xy)_{ts} = sum (xj|yl) a_{l t} a_{j s}
        if x > y:
            return op_lin((-1.0, self.P(y, x, s2, t2, side)))
        ph = _ph(2 + t2 + s2)                  # (-1)^(1 + t + s)
        terms = []
        for fam, K2 in ((cat.P0, 0), (cat.P1, 2)):
            if fam == cat.P1 and x == y:
                continue
            c = cg(1, -t2, 1, -s2, K2, -t2 - s2)
            if c != 0.0:
                terms.append((ph * c, self.mb.tensor(fam, self.mb.pos(fam, (x, y)), -t2 - s2, side)))
        return op_lin(*terms)

    @_memo
    def Q(self, x, y, t2, s2, side):           # (Q_xy)_{ts}
        if x > y:
            return op_T(self.Q(y, x, s2, t2, 1 - side))
        terms = []
        if s2 == t2:
            terms.append((-1.0 / sqrt(2.0),
                          self.mb.tensor(cat.Q0, self.mb.pos(cat.Q0, (x, y)), 0, side)))
        c = cg(1, s2, 1, -t2, 2, s2 - t2)
        if c != 0.0:
            terms.append((-_ph(1 + t2) * c / sqrt(3.0),
                          self.mb.tensor(cat.Q1, self.mb.pos(cat.Q1, (x, y)), s2 - t2, side)))
        return op_lin(*terms)


# ----------------------------------------------------------- the problem
class HEff:
    """Oracle action of H_eff on reduced two-site wavefunctions."""

    def __init__(self, prob, sample=None):
        """sample: optional {block index: (rows, cols)} of reduced output
        elements; with it, ``apply_sample`` evaluates H_eff psi at exactly
        those elements (rows and columns of each listed output block) and
        every block operator is expanded only on the product-basis rows those
        elements project from.  The arithmetic per element is the same."""
        self.prob = prob
        self.L = prob.n_orb
        self.p = prob.p
        self.mL = MBlock(prob.left)
        self.mR = MBlock(prob.right)
        self.blocks, self.size = psi_blocks(prob.left.sectors, prob.right.sectors,
                                            prob.n_elec, prob.two_s)
        self.M2 = prob.two_s
        self.sample = None
        if sample is not None:
            self.sample = {int(b): (np.unique(np.asarray(r, dtype=np.int64)),
                                    np.unique(np.asarray(c, dtype=np.int64)))
                           for b, (r, c) in sample.items()}
            selL, selR = {}, {}
            for bi, (rows, cols) in self.sample.items():
                b = self.blocks[bi]
                SL, SR = prob.left.sectors[b["iL"]][1], prob.right.sectors[b["iR"]][1]
                for ML in range(SL, -SL - 1, -2):
                    g, o = self.mL.gidx[(b["iL"], ML)]
                    selL.setdefault(g, set()).update((o + rows).tolist())
                for MR in range(SR, -SR - 1, -2):
                    g, o = self.mR.gidx[(b["iR"], MR)]
                    selR.setdefault(g, set()).update((o + cols).tolist())
            self.mL.sel = {g: np.array(sorted(v), dtype=np.int64) for g, v in selL.items()}
            self.mR.sel = {g: np.array(sorted(v), dtype=np.int64) for g, v in selR.items()}
        self.fL = Factors(self.mL)
        self.fR = Factors(self.mR)
        self._terms = None

    # ------------------------------------------------------- partitions
    def part(self, x):
        if x < self.p:
            return 0
        if x == self.p:
            return 1
        if x == self.p + 1:
            return 2
        return 3

    def single(self, x, s2, dagger):
        """Factor (part, op, parity) for a+_{x s} (dagger) or a_{x s}."""
        pt = self.part(x)
        if pt in (1, 2):
            return (pt, site_cre(s2) if dagger else site_ann(s2), 1)
        f = self.fL if pt == 0 else self.fR
        return (pt, f.cre(x, s2, 0) if dagger else f.T("cre", x, s2, 0), 1)

    # ------------------------------------------------------- term list
    def terms(self):
        """List of (coefficient, factors, group); factors are (part, op, parity)."""
        if self._terms is None:
            self._terms = list(self._gen_terms())
        return self._terms

    def set_terms(self, terms):
        """Replace the term list (used by tests that plant mistakes)."""
        self._terms = list(terms)
        self._compiled = None

    def _gen_terms(self):
        L, p = self.L, self.p
        h, eri = self.prob.h, self.prob.eri
        spins = (1, -1)
        if p > 0:
            yield 1.0, [(0, self.mL.tensor(cat.H, 0, 0), 0)], "H_L"
        if p + 2 < L:
            yield 1.0, [(3, self.mR.tensor(cat.H, 0, 0), 0)], "H_R"
        # one-index complementary S (n_X = 3)
        for X, f, outs in ((0, self.fL, range(p, L) if p > 0 else []),
                           (3, self.fR, range(0, p + 2) if p + 2 < L else [])):
            for x in outs:
                for s in spins:
                    g = "S_L" if X == 0 else "S_R"
                    yield 1.0, [self.single(x, s, True), (X, f.S(x, s, 0), 1)], g
                    yield 1.0, [(X, f.T("S", x, s, 0), 1), self.single(x, s, False)], g + "+"
        # two-index complementary P, Q (n_X = 2)
        for X, f, outs in ((0, self.fL, list(range(p, L)) if p > 0 else []),
                           (3, self.fR, list(range(0, p + 2)) if p + 2 < L else [])):
            for x in outs:
                for y in outs:
                    if X == 0 and x >= p + 2 and y >= p + 2:
                        continue
                    same_block = X == 3 and x < p and y < p
                    for s in spins:
                        for t in spins:
                            Pm = f.P(x, y, t, s, 0)
                            PmT = f.T("P", x, y, t, s, 0)
                            Qm = f.Q(x, y, t, s, 0)
                            g = ("AB" if same_block else "PQ_L" if X == 0 else "PQ_R")
                            if same_block:
                                yield 0.5, [(0, self.fL.cc(x, y, s, t, 0), 0), (X, Pm, 0)], g + ":P"
                                yield 0.5, [(X, PmT, 0), (0, self.fL.T("cc", x, y, s, t, 0), 0)], \
                                    g + ":P+"
                                yield 1.0, [(X, Qm, 0), (0, self.fL.ca(x, y, t, s, 0), 0)], g + ":Q"
                            else:
                                yield 0.5, [self.single(x, s, True), self.single(y, t, True),
                                            (X, Pm, 0)], g + ":P"
                                yield 0.5, [(X, PmT, 0), self.single(y, t, False),
                                            self.single(x, s, False)], g + ":P+"
                                yield 1.0, [(X, Qm, 0), self.single(x, t, True),
                                            self.single(y, s, False)], g + ":Q"
        # explicit products (n_L <= 1 and n_R <= 1)
        nblk = lambda idx: (sum(1 for i in idx if i < p), sum(1 for i in idx if i >= p + 2))
        for i in range(L):
            for j in range(L):
                nl, nr = nblk((i, j))
                if nl > 1 or nr > 1 or h[i, j] == 0.0:
                    continue
                for s in spins:
                    yield h[i, j], [self.single(i, s, True), self.single(j, s, False)], "E1"
        for i in range(L):
            for j in range(L):
                for k in range(L):
                    for l in range(L):
                        nl, nr = nblk((i, j, k, l))
                        if nl > 1 or nr > 1:
                            continue
                        v = eri[i, j, k, l]
                        if v == 0.0:
                            continue
                        for s in spins:
                            for t in spins:
                                if i == k and s == t:
                                    continue
                                if j == l and s == t:
                                    continue
                                yield 0.5 * v, [self.single(i, s, True), self.single(k, t, True),
                                                self.single(l, t, False), self.single(j, s, False)], \
                                    "E2:%d%d" % nblk((i, j, k, l))

    # ------------------------------------------------------- expansion
    def expand(self, psi):
        """Reduced psi [size] or [size, nvec] -> {(gL, dot): [nvec, dimL, dimR]}."""
        psi = np.asarray(psi)
        if psi.ndim == 1:
            psi = psi[:, None]
        nv = psi.shape[1]
        out = {}
        S = self.M2
        for b in self.blocks:
            X = psi[b["off"]:b["off"] + b["dL"] * b["dR"]].reshape(b["dR"], b["dL"], nv)
            X = X.transpose(2, 1, 0)
            NL, SL, dL = self.prob.left.sectors[b["iL"]]
            NR, SR, dR = self.prob.right.sectors[b["iR"]]
            sl, sr = SITE[b["l"]][1], SITE[b["r"]][1]
            for ML in range(SL, -SL - 1, -2):
                for ml, stl in SITE_MULT_STATES[b["l"]].items():
                    c1 = cg(SL, ML, sl, ml, b["SLl"], ML + ml)
                    if c1 == 0.0:
                        continue
                    for mr, str_ in SITE_MULT_STATES[b["r"]].items():
                        MR = S - ML - ml - mr
                        if abs(MR) > SR or (SR - MR) % 2:
                            continue
                        c2 = cg(sr, mr, SR, MR, b["SrR"], mr + MR)
                        c3 = cg(b["SLl"], ML + ml, b["SrR"], mr + MR, S, S)
                        c = c1 * c2 * c3
                        if c == 0.0:
                            continue
                        gL, oL = self.mL.gidx[(b["iL"], ML)]
                        gR, oR = self.mR.gidx[(b["iR"], MR)]
                        key = (gL, 4 * stl + str_)
                        m = out.get(key)
                        if m is None:
                            m = np.zeros((nv, self.mL.gdim[gL], self.mR.gdim[gR]))
                            out[key] = m
                        m[:, oL:oL + dL, oR:oR + dR] += c * X
        return out

    def project(self, u1, nv=1):
        """Transpose of ``expand``: product-basis dict -> reduced [size, nvec]."""
        y = np.zeros((self.size, nv))
        S = self.M2
        for b in self.blocks:
            NL, SL, dL = self.prob.left.sectors[b["iL"]]
            NR, SR, dR = self.prob.right.sectors[b["iR"]]
            sl, sr = SITE[b["l"]][1], SITE[b["r"]][1]
            acc = np.zeros((nv, dL, dR))
            for ML in range(SL, -SL - 1, -2):
                for ml, stl in SITE_MULT_STATES[b["l"]].items():
                    c1 = cg(SL, ML, sl, ml, b["SLl"], ML + ml)
                    if c1 == 0.0:
                        continue
                    for mr, str_ in SITE_MULT_STATES[b["r"]].items():
                        MR = S - ML - ml - mr
                        if abs(MR) > SR or (SR - MR) % 2:
                            continue
                        c = c1 * cg(sr, mr, SR, MR, b["SrR"], mr + MR) \
                            * cg(b["SLl"], ML + ml, b["SrR"], mr + MR, S, S)
                        if c == 0.0:
                            continue
                        gL, oL = self.mL.gidx[(b["iL"], ML)]
                        gR, oR = self.mR.gidx[(b["iR"], MR)]
                        m = u1.get((gL, 4 * stl + str_))
                        if m is not None:
                            acc += c * m[:, oL:oL + dL, oR:oR + dR]
            y[b["off"]:b["off"] + dL * dR] = acc.transpose(2, 1, 0).reshape(dL * dR, nv)
        return y

    # ------------------------------------------------------- application
    def _gR(self, gL, d):
        NR = self.prob.n_elec - gL[0] - SITE_N[d // 4] - SITE_N[d % 4]
        MR = self.M2 - gL[1] - SITE_2M[d // 4] - SITE_2M[d % 4]
        return (NR, MR)

    def compiled(self):
        """Terms merged by their (L operator, R operator) pair.

        Each entry is (OL, OR, dot, pdot, pR): the block operators (None for
        the identity), the 16x16 two-site matrix (coefficient, reordering sign
        and the l-r Jordan-Wigner sign included) and the parities that fix the
        ket-dependent signs (-1)^(pdot N_L) and (-1)^(pR (N_L + N_dot)).
        """
        if getattr(self, "_compiled", None) is not None:
            return self._compiled
        merged = {}
        for coef, factors, _group in self.terms():
            sign = 1.0
            fs = list(factors)
            for i in range(len(fs)):
                for j in range(i + 1, len(fs)):
                    if fs[i][0] > fs[j][0] and fs[i][2] and fs[j][2]:
                        sign = -sign
            fs.sort(key=lambda f: f[0])
            OL = OR = None
            Ol = np.eye(4)
            Or = np.eye(4)
            par = [0, 0, 0, 0]
            for pt, op, pa in fs:
                par[pt] ^= pa
                if pt == 0:
                    assert OL is None
                    OL = op
                elif pt == 3:
                    assert OR is None
                    OR = op
                elif pt == 1:
                    Ol = Ol @ op
                else:
                    Or = Or @ op
            jw = np.array([-1.0 if (par[2] and SITE_N[l] % 2) else 1.0 for l in range(4)])
            dot = np.einsum("ab,cd->acbd", Ol, Or).reshape(16, 16)
            dot = dot * np.repeat(jw, 4)[None, :]
            key = (id(OL), id(OR), par[1] ^ par[2], par[3])
            if key in merged:
                merged[key][2] += sign * coef * dot
            else:
                merged[key] = [OL, OR, sign * coef * dot, par[1] ^ par[2], par[3]]
        self._compiled = [tuple(v) for v in merged.values() if np.any(v[2] != 0.0)]
        return self._compiled

    def apply_u1(self, u1):
        """Apply H to a product-basis dict whose values are [nvec, dimL, dimR].

        With a sample, outputs hold only the selected rows (left groups) and
        columns (right groups)."""
        out = {}
        restricted = self.sample is not None
        for OL, OR, dot, pdot, pR in self.compiled():
            colL = {}
            if OL is None:
                for g in self.mL.gdim:
                    if not restricted or len(self.mL.rows(g)):
                        colL[g] = [(g, None)]
            else:
                for (g2, g), m in OL.items():
                    colL.setdefault(g, []).append((g2, m))
            for (gL, d), X in u1.items():
                gR = self._gR(gL, d)
                NL = gL[0]
                nd = SITE_N[d // 4] + SITE_N[d % 4]
                s = 1.0
                if pdot and NL % 2:
                    s = -s
                if pR and (NL + nd) % 2:
                    s = -s
                rows = np.nonzero(dot[:, d])[0]
                if len(rows) == 0:
                    continue
                for gL2, mL in colL.get(gL, ()):
                    if mL is None:
                        Z = X[:, self.mL.rows(gL2), :] if restricted else X
                    else:
                        Z = np.matmul(mL, X)
                    cacheW = {}
                    for d2 in rows:
                        gR2 = self._gR(gL2, d2)
                        if gR2 in cacheW:
                            W = cacheW[gR2]
                        else:
                            if OR is None:
                                W = None if gR2 != gR else \
                                    (Z[:, :, self.mR.rows(gR2)] if restricted else Z)
                            else:
                                mR = OR.get((gR2, gR))
                                W = None if mR is None else np.matmul(Z, mR.T)
                            cacheW[gR2] = W
                        if W is None:
                            continue
                        key = (gL2, d2)
                        val = (s * dot[d2, d]) * W
                        if key in out:
                            out[key] += val
                        else:
                            out[key] = val.copy()
        return out

    def apply_sample(self, psi):
        """H_eff psi at the sample's elements: {block index: [rows, cols]}
        for psi of shape [size] (the projection of ``project`` restricted to
        those elements)."""
        assert self.sample is not None
        u1 = self.apply_u1(self.expand(np.asarray(psi, dtype=float)))
        S = self.M2
        out = {}
        for bi, (rows, cols) in self.sample.items():
            b = self.blocks[bi]
            NL, SL, dL = self.prob.left.sectors[b["iL"]]
            NR, SR, dR = self.prob.right.sectors[b["iR"]]
            sl, sr = SITE[b["l"]][1], SITE[b["r"]][1]
            acc = np.zeros((len(rows), len(cols)))
            for ML in range(SL, -SL - 1, -2):
                for ml, stl in SITE_MULT_STATES[b["l"]].items():
                    c1 = cg(SL, ML, sl, ml, b["SLl"], ML + ml)
                    if c1 == 0.0:
                        continue
                    for mr, str_ in SITE_MULT_STATES[b["r"]].items():
                        MR = S - ML - ml - mr
                        if abs(MR) > SR or (SR - MR) % 2:
                            continue
                        c = c1 * cg(sr, mr, SR, MR, b["SrR"], mr + MR) \
                            * cg(b["SLl"], ML + ml, b["SrR"], mr + MR, S, S)
                        if c == 0.0:
                            continue
                        gL, oL = self.mL.gidx[(b["iL"], ML)]
                        gR, oR = self.mR.gidx[(b["iR"], MR)]
                        m = u1.get((gL, 4 * stl + str_))
                        if m is None:
                            continue
                        pL = np.searchsorted(self.mL.rows(gL), oL + rows)
                        pR = np.searchsorted(self.mR.rows(gR), oR + cols)
                        acc += c * m[0][np.ix_(pL, pR)]
            out[bi] = acc
        return out

    def apply(self, psi):
        """H_eff psi for psi of shape [size] or [size, nvec]."""
        psi = np.asarray(psi, dtype=float)
        one = psi.ndim == 1
        nv = 1 if one else psi.shape[1]
        y = self.project(self.apply_u1(self.expand(psi)), nv)
        return y[:, 0] if one else y

    def dense(self, chunk=512):
        """Dense H_eff (small problems only)."""
        n = self.size
        H = np.zeros((n, n))
        for c0 in range(0, n, chunk):
            c1 = min(n, c0 + chunk)
            E = np.zeros((n, c1 - c0))
            E[np.arange(c0, c1), np.arange(c1 - c0)] = 1.0
            H[:, c0:c1] = self.apply(E)
        return H
