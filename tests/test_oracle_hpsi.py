"""Pins of oracle/hpsi.py against the determinant space, full CI and symmetry."""
import json
import os

import numpy as np
import pytest

from paper_2309_16724_amd.synth.problem import exact_problem, random_problem
from oracle.hpsi import HEff
from oracle.fock import heff_fock, fci

GOLD = os.path.join(os.path.dirname(__file__), "golden", "fci_L8_seed0.json")

BONDS = [(6, 6, 0, p) for p in range(5)] + [(6, 6, 2, 2), (6, 5, 1, 1), (6, 5, 3, 3),
                                            (6, 7, 1, 2), (5, 4, 0, 2), (4, 4, 2, 1),
                                            (3, 3, 1, 0), (2, 2, 0, 0)]


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("L,N,two_s,p", BONDS)
def test_hpsi_equals_determinant_space(L, N, two_s, p):
    prob = exact_problem(L, N, two_s, 3, p=p)
    he = HEff(prob)
    x = np.random.default_rng(7).standard_normal(he.size)
    assert _rel(he.apply(x), heff_fock(prob, he, x)) < 1e-13


def test_hpsi_L8_middle_bond_and_truncation():
    for mm in (None, 32):
        prob = exact_problem(8, 8, 0, 0, max_mult=mm)
        he = HEff(prob)
        x = np.random.default_rng(8).standard_normal(he.size)
        assert _rel(he.apply(x), heff_fock(prob, he, x)) < 1e-13
        if mm is None:
            assert he.size == 1764 and len(he.blocks) == 102


def test_lowest_eigenvalue_is_full_ci():
    """Untruncated L=8 blocks: lowest eigenvalue of H_eff = FCI singlet energy."""
    gold = json.load(open(GOLD))
    prob = exact_problem(8, 8, 0, 0)
    w = np.linalg.eigvalsh(HEff(prob).dense())
    assert abs(w[0] - gold["E_fci_S0"]) < 1e-10
    # and the S=1/2, odd-N case at L=6 against a fresh FCI
    prob = exact_problem(6, 5, 1, 2)
    w = np.linalg.eigvalsh(HEff(prob).dense())
    assert abs(w[0] - fci(prob.h, prob.eri, 5, 1)[0]) < 1e-10


def test_truncated_is_variational():
    gold = json.load(open(GOLD))
    prob = exact_problem(8, 8, 0, 0, max_mult=32)
    w = np.linalg.eigvalsh(HEff(prob).dense())
    assert w[0] >= gold["E_fci_S0"] - 1e-10


@pytest.mark.parametrize("seed", [0, 1])
def test_random_blocks_hermitian(seed):
    prob = random_problem(6, 6, 0, seed, D=40)
    he = HEff(prob)
    rng = np.random.default_rng(seed)
    a, b = rng.standard_normal(he.size), rng.standard_normal(he.size)
    ha, hb = he.apply(a), he.apply(b)
    scale = np.linalg.norm(ha) * np.linalg.norm(b)
    assert abs(a @ hb - ha @ b) <= 1e-13 * scale


def test_planted_mistakes_are_caught():
    """Dropping any term group, or flipping its sign, breaks the determinant pin."""
    cases = [(6, 6, 0, p) for p in range(5)]
    probs = []
    for L, N, s, p in cases:
        prob = exact_problem(L, N, s, 3, p=p)
        he = HEff(prob)
        x = np.random.default_rng(9).standard_normal(he.size)
        probs.append((prob, he, x, heff_fock(prob, he, x)))
    groups = sorted({g.split(":")[0] for pr in probs for (_, _, g) in pr[1].terms()})
    assert len(groups) >= 8
    for g in groups:
        for mode in ("drop", "flip"):
            caught = False
            for prob, he, x, ref in probs:
                orig = he.terms()
                mod = []
                for c, f, gg in orig:
                    if gg.split(":")[0] == g:
                        if mode == "drop":
                            continue
                        c = -c
                    mod.append((c, f, gg))
                he2 = HEff(prob)
                he2.set_terms(mod)
                if _rel(he2.apply(x), ref) > 1e-6:
                    caught = True
                    break
            assert caught, (g, mode)


@pytest.mark.parametrize("kind,args,kw", [
    ("exact", (8, 8, 0, 0), dict()),
    ("exact", (6, 6, 0, 3), dict(p=0)),
    ("random", (24, 24, 0, 1), dict(D=64)),
    ("random", (7, 7, 1, 5), dict(D=200, cap=False)),
    ("random", (6, 6, 0, 7), dict(D=300, D_right=40, cap=False)),
])
def test_sampled_evaluation_equals_full_apply(kind, args, kw):
    """HEff with a sample (expanded operators restricted to the rows the
    sampled outputs project from) gives the full apply's values at those
    elements, at L = 24 too: the restriction the large-workload references
    are computed with (tests/golden/make_hpsi_samples.py)."""
    from paper_2309_16724_amd.synth.problem import random_problem
    prob = exact_problem(*args, **kw) if kind == "exact" else random_problem(*args, **kw)
    he = HEff(prob)
    x = np.random.default_rng(3).standard_normal(he.size)
    y = he.apply(x)
    rng = np.random.default_rng(4)
    nb = len(he.blocks)
    big = max(range(nb), key=lambda i: he.blocks[i]["dL"] * he.blocks[i]["dR"])
    pick = sorted({big} | set(rng.choice(nb, size=min(5, nb), replace=False).tolist()))
    sample = {bi: (rng.choice(he.blocks[bi]["dL"], size=min(3, he.blocks[bi]["dL"]), replace=False),
                   rng.choice(he.blocks[bi]["dR"], size=min(3, he.blocks[bi]["dR"]), replace=False))
              for bi in pick}
    hs = HEff(prob, sample)
    ys = hs.apply_sample(x)
    scale = np.abs(y).max()
    for bi, (r, c) in hs.sample.items():
        b = he.blocks[bi]
        Y = y[b["off"]:b["off"] + b["dL"] * b["dR"]].reshape(b["dR"], b["dL"]).T
        assert np.abs(Y[np.ix_(r, c)] - ys[bi]).max() <= 1e-13 * scale
