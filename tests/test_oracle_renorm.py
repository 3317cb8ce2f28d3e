"""Pins of the renormalization oracle (oracle/renorm.py).

Ground truth: the operators of the enlarged block [0, p + 1) built directly
in its Fock space (paper_2309_16724_amd.synth.problem.build_exact_block),
expressed in the basis that U maps the coupled product states onto.  With an
untruncated left block the product space of L x l is the whole Fock space of
the enlarged block, so every family must agree to rounding, truncated or not.
"""
import numpy as np
import pytest

from paper_2309_16724_amd.synth import catalogue as cat
from paper_2309_16724_amd.synth.problem import exact_problem, build_exact_block, random_problem
from oracle.renorm import renormalize, product_sectors, RENORM_FAMILIES
from oracle.layout import SITE
from oracle.hpsi import SITE_MULT_STATES
from oracle.wigner import cg


def exact_keep(left, big):
    """U of every product sector of left x site onto the states of the exact
    enlarged block ``big`` (same (N, 2S) order), from Fock-space overlaps."""
    p = left.p
    nf = 4 ** p
    bidx = {(N, S): b for b, (N, S, d) in enumerate(big.sectors)}
    keep = []
    for (N, S, rows, comps) in product_sectors(left.sectors):
        b = bidx.get((N, S))
        if b is None:
            continue
        V = big.basis[b][0]
        U = np.zeros((rows, V.shape[1]))
        for (iL, m, row0, d) in comps:
            SL = left.sectors[iL][1]
            s = SITE[m][1]
            for ms, f in SITE_MULT_STATES[m].items():
                ML = S - ms
                if abs(ML) > SL or (SL - ML) % 2:
                    continue
                c = cg(SL, ML, s, ms, S, S)
                if c == 0.0:
                    continue
                Lv = left.basis[iL][(SL - ML) // 2]
                U[row0:row0 + d, :] += c * (Lv.T @ V[f * nf + np.arange(nf), :])
        keep.append((N, S, U))
    return keep


def dense_records(blk, fam):
    return {(r, c): blk.block(fam, r, c) for (f, r, c, off, npos) in blk.records if f == fam}


def compare(got, want, fam, tol):
    g, w = dense_records(got, fam), dense_records(want, fam)
    scale = max([np.abs(a).max() for a in w.values()] + [1.0])
    worst = 0.0
    for key in set(g) | set(w):
        a = g.get(key)
        b = w.get(key)
        if a is None:
            a = np.zeros_like(b)
        if b is None:
            b = np.zeros_like(a)
        worst = max(worst, np.abs(a - b).max())
    assert worst <= tol * scale, (cat.NAMES[fam], worst, scale)


@pytest.mark.parametrize("n_orb,p,n_elec", [(6, 2, 6), (7, 3, 7)])
def test_untruncated_matches_fock_space(n_orb, p, n_elec):
    prob = exact_problem(n_orb, n_elec, n_elec % 2, 21, p=p)
    big = build_exact_block("L", n_orb, p + 1, prob.h, prob.eri)
    keep = exact_keep(prob.left, big)
    assert [(N, S, U.shape[1]) for N, S, U in keep] == big.sectors
    for N, S, U in keep:        # complete product space: U is orthogonal
        assert np.allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-12)
    got = renormalize(prob, keep)
    for fam in RENORM_FAMILIES:
        compare(got, big, fam, 1e-12)


def test_truncated_matches_fock_space():
    n_orb, p = 7, 3
    prob = exact_problem(n_orb, 7, 1, 22, p=p)
    big = build_exact_block("L", n_orb, p + 1, prob.h, prob.eri, max_mult=40)
    keep = exact_keep(prob.left, big)
    assert sum(U.shape[1] for _, _, U in keep) < sum(U.shape[0] for _, _, U in keep)
    got = renormalize(prob, keep)
    for fam in RENORM_FAMILIES:
        compare(got, big, fam, 1e-12)


def test_planted_mistakes_are_caught():
    """A wrong site sign or a dropped complementary term breaks the pins."""
    import oracle.renorm as R
    n_orb, p = 6, 2
    prob = exact_problem(n_orb, 6, 0, 23, p=p)
    big = build_exact_block("L", n_orb, p + 1, prob.h, prob.eri)
    keep = exact_keep(prob.left, big)
    orig_terms = R._h_terms

    def no_s(ps, p_, h, eri):
        for k, (coef, fs) in enumerate(orig_terms(ps, p_, h, eri)):
            if 1 <= k <= 4:      # the S_p terms
                continue
            yield coef, fs
    R._h_terms = no_s
    try:
        got = renormalize(prob, keep, families=(cat.H,))
        with pytest.raises(AssertionError):
            compare(got, big, cat.H, 1e-12)
    finally:
        R._h_terms = orig_terms
    orig_jw = R._ProductSpace.__init__

    def no_jw(self, blk):
        orig_jw(self, blk)
        self.jw = np.ones_like(self.jw)
    R._ProductSpace.__init__ = no_jw
    try:
        got = renormalize(prob, keep, families=(cat.B0,))
        with pytest.raises(AssertionError):
            compare(got, big, cat.B0, 1e-12)
    finally:
        R._ProductSpace.__init__ = orig_jw
    # S of the enlarged block without its Q_xp part
    orig_q = R.Factors.Q
    R.Factors.Q = lambda self, x, y, t, s, side: {} if x > y else orig_q(self, x, y, t, s, side)
    try:
        got = renormalize(prob, keep, families=(cat.S,))
        with pytest.raises(AssertionError):
            compare(got, big, cat.S, 1e-12)
    finally:
        R.Factors.Q = orig_q


def test_hamiltonian_is_symmetric_and_identity_keeps_l_members():
    """Random blocks: H of the enlarged block is symmetric in any orthogonal
    basis, and with U = identity the members living on L alone are the
    stored ones placed on the (L sector, site multiplet) diagonal blocks."""
    prob = random_problem(8, 8, 0, 5, 24, p=3)
    keep = [(N, S, np.eye(rows)) for (N, S, rows, comps) in product_sectors(prob.left.sectors)]
    got = renormalize(prob, keep, families=(cat.H, cat.C))
    for (f, r, c, off, npos) in got.records:
        if f == cat.H and r == c:
            m = got.block(cat.H, r, c)[0]
            assert np.allclose(m, m.T, atol=1e-12 * max(1.0, np.abs(m).max()))
    prods = product_sectors(prob.left.sectors)
    labs = cat.labels(cat.C, "L", prob.n_orb, prob.p)
    for ia, (Na, Sa, ra, ca) in enumerate(prods):
        for ib, (Nb, Sb, rb, cb) in enumerate(prods):
            blk = got.block(cat.C, ib, ia)
            if blk is None:
                continue
            for (iLa, ma, r0a, da) in ca:
                for (iLb, mb, r0b, db) in cb:
                    if ma != mb:
                        continue
                    src = prob.left.block(cat.C, iLb, iLa)
                    if src is None:
                        continue
                    # stored member times the recoupling of (S_L s) S with the site a spectator
                    sub = blk[:len(labs), r0b:r0b + db, r0a:r0a + da]
                    ratio = None
                    for pos in range(len(labs)):
                        a, b = sub[pos], src[pos]
                        if np.abs(b).max() > 1e-8:
                            rr = (a * b).sum() / (b * b).sum()
                            assert np.allclose(a, rr * b, atol=1e-10 * np.abs(b).max())
                            ratio = rr if ratio is None else ratio
                            assert abs(rr - ratio) < 1e-10


@pytest.mark.parametrize("n_orb,p,max_mult", [(6, 2, None), (7, 3, None), (7, 3, 40)])
def test_pair_families_match_fock_space(n_orb, p, max_mult):
    """P and Q of the enlarged block from a left block holding them for every
    outside pair, against the Fock-space block in the same form."""
    from oracle.renorm import PAIR_FAMILIES
    prob = exact_problem(n_orb, n_orb, n_orb % 2, 24, p=p, all_pairs=True)
    big = build_exact_block("L", n_orb, p + 1, prob.h, prob.eri, max_mult=max_mult, all_pairs=True)
    keep = exact_keep(prob.left, big)
    got = renormalize(prob, keep)
    assert got.all_pairs
    for fam in RENORM_FAMILIES + PAIR_FAMILIES:
        assert dense_records(big, fam), cat.NAMES[fam]
        compare(got, big, fam, 1e-12)


def exact_keep_right(right, big):
    """U of every product sector of site x right block onto the states of the
    exact enlarged right block ``big`` (Fock index site + 4 * block)."""
    from oracle.renorm import product_sectors_right
    nf = 4 ** (right.n_orb - right.p - 2)
    bidx = {(N, S): b for b, (N, S, d) in enumerate(big.sectors)}
    keep = []
    for (N, S, rows, comps) in product_sectors_right(right.sectors):
        b = bidx.get((N, S))
        if b is None:
            continue
        V = big.basis[b][0]
        U = np.zeros((rows, V.shape[1]))
        for (m, iR, row0, d) in comps:
            SR = right.sectors[iR][1]
            s = SITE[m][1]
            for ms, f in SITE_MULT_STATES[m].items():
                MR = S - ms
                if abs(MR) > SR or (SR - MR) % 2:
                    continue
                c = cg(s, ms, SR, MR, S, S)
                if c == 0.0:
                    continue
                Rv = right.basis[iR][(SR - MR) // 2]
                U[row0:row0 + d, :] += c * (Rv.T @ V[f + 4 * np.arange(nf), :])
        keep.append((N, S, U))
    return keep


@pytest.mark.parametrize("n_orb,p,max_mult", [(6, 2, None), (7, 2, None), (7, 2, 40)])
def test_right_block_matches_fock_space(n_orb, p, max_mult):
    """Site x right block: every family of the enlarged right block against
    the Fock-space block (untruncated and truncated)."""
    from oracle.renorm import renormalize_right, RIGHT_FAMILIES
    prob = exact_problem(n_orb, n_orb, n_orb % 2, 26, p=p)
    big = build_exact_block("R", n_orb, p - 1, prob.h, prob.eri, max_mult=max_mult)
    keep = exact_keep_right(prob.right, big)
    got = renormalize_right(prob, keep)
    for fam in RIGHT_FAMILIES:
        assert dense_records(big, fam), cat.NAMES[fam]
        compare(got, big, fam, 1e-12)
