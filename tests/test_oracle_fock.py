"""Pins of oracle/fock.py: closed forms, S^2 spectrum and a string-level check."""
import itertools
import numpy as np
import pytest

from oracle.fock import fci, sector_states, hamiltonian, s_squared


def test_hubbard_dimer_closed_form():
    # two sites, hopping t, on-site U: E0(N=2, S=0) = (U - sqrt(U^2 + 16 t^2)) / 2
    for t, U in [(1.0, 4.0), (0.7, 1.3), (2.0, 0.0)]:
        h = np.array([[0.0, -t], [-t, 0.0]])
        eri = np.zeros((2, 2, 2, 2))
        eri[0, 0, 0, 0] = eri[1, 1, 1, 1] = U
        E0 = fci(h, eri, 2, 0)[0]
        assert abs(E0 - (U - np.sqrt(U * U + 16 * t * t)) / 2) < 1e-12


def test_noninteracting_limit():
    rng = np.random.default_rng(5)
    L = 5
    a = rng.standard_normal((L, L))
    h = a + a.T
    eri = np.zeros((L, L, L, L))
    eps = np.linalg.eigvalsh(h)
    for N in (2, 4, 6):
        E0 = fci(h, eri, N, 0)[0]
        assert abs(E0 - 2 * eps[: N // 2].sum()) < 1e-11
    # one unpaired electron: S = 1/2
    E0 = fci(h, eri, 3, 1)[0]
    assert abs(E0 - (2 * eps[0] + eps[1])) < 1e-11


def test_s2_spectrum():
    st = sector_states(4, 4, 0)
    S2 = s_squared(4, st, 0).toarray()
    w = np.linalg.eigvalsh(S2)
    allowed = [S * (S + 1) for S in (0, 1, 2)]
    assert all(min(abs(x - a) for a in allowed) < 1e-12 for x in w)
    # multiplicities: 4 orbitals, 4 electrons, M=0 -> 20 singlets, 15 triplets, 1 quintet
    counts = [int(np.sum(np.abs(w - a) < 1e-9)) for a in allowed]
    assert counts == [20, 15, 1]


def _apply_strings(h, eri, det):
    """Reference: sum over explicit strings a+ a+ a a, one determinant."""
    L = h.shape[0]

    def act(ops, x):
        sign = 1
        for b, cre in reversed(ops):
            occ = (x >> b) & 1
            if cre == bool(occ):
                return 0, None
            if bin(x & ((1 << b) - 1)).count("1") % 2:
                sign = -sign
            x ^= 1 << b
        return sign, x

    out = {}
    for i, j in itertools.product(range(L), repeat=2):
        for s in (0, 1):
            sg, y = act([(2 * i + s, True), (2 * j + s, False)], det)
            if sg:
                out[y] = out.get(y, 0.0) + sg * h[i, j]
    for i, j, k, l in itertools.product(range(L), repeat=4):
        for s in (0, 1):
            for t in (0, 1):
                sg, y = act([(2 * i + s, True), (2 * k + t, True), (2 * l + t, False),
                             (2 * j + s, False)], det)
                if sg:
                    out[y] = out.get(y, 0.0) + 0.5 * sg * eri[i, j, k, l]
    return out


def test_spin_free_form_equals_strings():
    from paper_2309_16724_amd.synth.integrals import make_integrals
    h, eri = make_integrals(3, 11)
    st = sector_states(3, 3, 1)
    H = hamiltonian(h, eri, st).toarray()
    idx = {int(s): n for n, s in enumerate(st)}
    for c, det in enumerate(st):
        ref = _apply_strings(h, eri, int(det))
        col = np.zeros(len(st))
        for y, v in ref.items():
            col[idx[y]] += v
        assert np.abs(H[:, c] - col).max() < 1e-13


def test_hamiltonian_symmetric():
    from paper_2309_16724_amd.synth.integrals import make_integrals
    h, eri = make_integrals(5, 4)
    st = sector_states(5, 5, 1)
    H = hamiltonian(h, eri, st)
    assert abs(H - H.T).max() < 1e-13
