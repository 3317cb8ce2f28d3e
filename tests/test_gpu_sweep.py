"""A left-to-right two-site sweep through the library (Davidson, truncation,
renormalization at every bond) on an exact small system, against full CI."""
import numpy as np
import pytest

from paper_2309_16724_amd.synth.problem import exact_problem, build_exact_block
from oracle.fock import fci

pytestmark = pytest.mark.gpu
N_ORB, N_ELEC = 6, 6


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    return t


@pytest.fixture(scope="module")
def system():
    prob = exact_problem(N_ORB, N_ELEC, 0, 31, p=1)
    e_fci = fci(prob.h, prob.eri, N_ELEC, 0)[0]
    left = build_exact_block("L", N_ORB, 1, prob.h, prob.eri, all_pairs=True)
    rights = {p: build_exact_block("R", N_ORB, p, prob.h, prob.eri) for p in range(1, N_ORB - 1)}
    return prob, e_fci, left, rights


def _sweep(system, D):
    from paper_2309_16724_amd.hpsi import sweep_left_to_right
    prob, e_fci, left, rights = system
    print("sweep L=%d D=%d" % (N_ORB, D), flush=True)
    res = sweep_left_to_right(left, rights, prob.h, prob.eri, N_ELEC, 0, D)
    for bond, e, kept, w in res:
        print(bond, e - e_fci, kept, w, flush=True)
    assert [b for b, *_ in res] == list(range(1, N_ORB - 1))
    return res


def test_untruncated_sweep_is_full_ci(torch, system):
    """D above every sector's size: every bond's energy is the FCI energy."""
    e_fci = system[1]
    for bond, e, kept, w in _sweep(system, 4096):
        assert abs(e - e_fci) < 1e-8, (bond, e, e_fci)
        assert w is None or abs(w - 1.0) < 1e-12


def test_truncated_sweep_is_variational_and_nested(torch, system):
    """Truncated: exact until the first cut, above FCI after it, and a larger
    D (whose kept states contain the smaller D's, the same density matrices'
    leading eigenvectors) is never worse."""
    e_fci = system[1]
    small, large = _sweep(system, 12), _sweep(system, 20)
    for res in (small, large):
        cut = next(i for i, (_, _, kept, w) in enumerate(res) if w is not None and w < 1.0 - 1e-12)
        for i, (bond, e, kept, w) in enumerate(res):
            if i <= cut:
                assert abs(e - e_fci) < 1e-8, (bond, e)
            assert e > e_fci - 1e-9, (bond, e, e_fci)
    assert small[-1][1] - e_fci > 1e-6
    assert large[-1][1] <= small[-1][1] + 1e-10


def test_right_to_left_sweep(torch, system):
    """The mirror direction: exact left blocks, the right block grown from
    the last bond by right truncations and renormalizations; untruncated it
    is full CI at every bond, truncated it is variational."""
    from paper_2309_16724_amd.hpsi import sweep_right_to_left
    prob, e_fci = system[0], system[1]
    lefts = {p: build_exact_block("L", N_ORB, p, prob.h, prob.eri) for p in range(0, N_ORB - 1)}
    right = build_exact_block("R", N_ORB, N_ORB - 3, prob.h, prob.eri)
    for D in (4096, 12):
        print("sweep right to left D=%d" % D, flush=True)
        res = sweep_right_to_left(lefts, right, prob.h, prob.eri, N_ELEC, 0, D)
        assert [b for b, *_ in res] == list(range(N_ORB - 3, -1, -1))
        for bond, e, kept, w in res:
            print(bond, e - e_fci, kept, w, flush=True)
            if D == 4096:
                assert abs(e - e_fci) < 1e-8, (bond, e, e_fci)
            else:
                assert e > e_fci - 1e-9, (bond, e, e_fci)


def test_native_sweep_matches_the_composed_one(torch, system):
    """dmrg_sweep_left_to_right (blocks kept on the device) gives the energies
    of the sweep composed from the single entry points: full CI untruncated,
    the same truncated energies with D = 12."""
    from paper_2309_16724_amd.hpsi import sweep_native
    prob, e_fci, left, rights = system
    for D in (4096, 12):
        print("native sweep D=%d" % D, flush=True)
        res = sweep_native(rights, left, prob.h, prob.eri, N_ELEC, 0, D)
        ref = _sweep(system, D)
        assert [r[0] for r in res] == [r[0] for r in ref]
        for (bond, e, kept, w, it), (_, e2, kept2, w2) in zip(res, ref):
            print(bond, e - e_fci, kept, w, it, flush=True)
            assert abs(e - e2) < 1e-7, (bond, e, e2)
            if D == 4096:
                assert abs(e - e_fci) < 1e-8
            if kept2 is not None:
                assert kept == kept2 and abs(w - w2) < 1e-7


def test_native_right_to_left_sweep(torch, system):
    """dmrg_sweep_right_to_left against the composed mirror sweep: full CI
    untruncated, the same energies, kept counts and weights with D = 12."""
    from paper_2309_16724_amd.hpsi import sweep_native, sweep_right_to_left
    prob, e_fci = system[0], system[1]
    lefts = {p: build_exact_block("L", N_ORB, p, prob.h, prob.eri) for p in range(0, N_ORB - 2)}
    right = build_exact_block("R", N_ORB, N_ORB - 3, prob.h, prob.eri)
    for D in (4096, 12):
        print("native sweep right to left D=%d" % D, flush=True)
        res = sweep_native(lefts, right, prob.h, prob.eri, N_ELEC, 0, D, seed=200, right_to_left=True)
        ref = sweep_right_to_left(lefts, right, prob.h, prob.eri, N_ELEC, 0, D)
        assert [r[0] for r in res] == [r[0] for r in ref] == list(range(N_ORB - 3, -1, -1))
        for (bond, e, kept, w, it), (_, e2, kept2, w2) in zip(res, ref):
            print(bond, e - e_fci, kept, w, it, flush=True)
            assert abs(e - e2) < 1e-7, (bond, e, e2)
            if D == 4096:
                assert abs(e - e_fci) < 1e-8
            if kept2 is not None:
                assert kept == kept2 and abs(w - w2) < 1e-7


def test_chained_sweeps(torch, system):
    """A left-to-right sweep that returns its grown left blocks (all-pairs,
    on the device) feeding a right-to-left sweep: untruncated every bond of
    both is full CI; with D = 12 the second sweep's first bond is the first
    sweep's last problem (the same energy), and every energy stays above
    full CI."""
    from paper_2309_16724_amd.hpsi import sweep_native, release_blocks
    prob, e_fci, left, rights = system
    n = N_ORB
    for D in (4096, 12):
        print("chained sweeps D=%d" % D, flush=True)
        r1, grown = sweep_native(rights, left, prob.h, prob.eri, N_ELEC, 0, D, keep_blocks=True)
        assert [b.n_sec > 0 for b in grown] == [True] * (n - 3) + [False]
        lefts = {p: build_exact_block("L", n, p, prob.h, prob.eri) for p in range(0, 2)}
        lefts.update({p: grown[p - 2] for p in range(2, n - 2)})
        right = build_exact_block("R", n, n - 3, prob.h, prob.eri)
        r2, grown_r = sweep_native(lefts, right, prob.h, prob.eri, N_ELEC, 0, D, seed=300, right_to_left=True,
                                   keep_blocks=True)
        assert [b.n_sec > 0 for b in grown_r] == [True] * (n - 3) + [False]
        for bond, e, kept, w, it in r1 + r2:
            print(bond, e - e_fci, kept, w, it, flush=True)
            assert e > e_fci - 1e-9, (bond, e)
            if D == 4096:
                assert abs(e - e_fci) < 1e-8, (bond, e)
        e_last = dict((b, e) for b, e, *_ in r1)[n - 3]
        assert r2[0][0] == n - 3 and abs(r2[0][1] - e_last) < 1e-8
        release_blocks(grown)
        release_blocks(grown_r)
        assert all(b.n_sec == 0 and not b.data for b in grown)


def test_native_sweep_on_the_split_path(torch, system):
    """The left-to-right sweep with split-BF16 plans (5 slices) against the
    FP64 one: full CI untruncated, the FP64 sweep's energies with D = 12."""
    from paper_2309_16724_amd import binding as B
    from paper_2309_16724_amd.hpsi import sweep_native
    prob, e_fci, left, rights = system
    for D in (4096, 12):
        print("split sweep D=%d" % D, flush=True)
        ref = sweep_native(rights, left, prob.h, prob.eri, N_ELEC, 0, D)
        res = sweep_native(rights, left, prob.h, prob.eri, N_ELEC, 0, D, precision=B.DMRG_SPLIT_BF16, n_slices=5)
        for (bond, e, kept, w, it), (_, e2, kept2, w2, _) in zip(res, ref):
            print(bond, e - e_fci, e - e2, kept, w, it, flush=True)
            assert abs(e - e2) < 1e-8 and kept == kept2 and abs(w - w2) < 1e-7, bond
            if D == 4096:
                assert abs(e - e_fci) < 1e-8
