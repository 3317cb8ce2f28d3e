"""Pins of the truncation oracle (oracle/truncate.py)."""
import numpy as np
import pytest

from paper_2309_16724_amd.synth.problem import exact_problem, random_problem, random_vector
from oracle.truncate import sector_matrices, truncate
from oracle.hpsi import HEff
from oracle.layout import psi_blocks


def _psi(prob, seed):
    _, size = psi_blocks(prob.left.sectors, prob.right.sectors, prob.n_elec, prob.two_s)
    return random_vector(size, seed)


def test_trace_is_the_norm():
    prob = random_problem(10, 10, 0, 3, 40, p=4)
    psi = _psi(prob, 5)
    tr = sum(float(np.sum(M * M)) for M, _ in sector_matrices(prob, psi).values())
    assert abs(tr - float(psi @ psi)) < 1e-12 * float(psi @ psi)


@pytest.mark.parametrize("n_orb,p", [(6, 2), (7, 3)])
def test_singlet_spectrum_matches_fock_space(n_orb, p):
    """A singlet's reduced density matrix of (L l) in the M-resolved product
    space has the eigenvalues w / (2S + 1) of every sector, 2S + 1 times."""
    n_elec = n_orb - (n_orb % 2)
    prob = exact_problem(n_orb, n_elec, 0, 27, p=p)
    psi = _psi(prob, 6)
    he = HEff(prob)
    u1 = he.expand(psi)
    rows, cols = {}, {}
    entries = []
    for (gL, d), m in u1.items():
        gR = he._gR(gL, d)
        l, r = d // 4, d % 4
        for i in range(m.shape[1]):
            ri = rows.setdefault((gL, l, i), len(rows))
            for j in range(m.shape[2]):
                cj = cols.setdefault((r, gR, j), len(cols))
                entries.append((ri, cj, m[0, i, j]))
    Psi = np.zeros((len(rows), len(cols)))
    for ri, cj, v in entries:
        Psi[ri, cj] += v
    fock = np.sort(np.linalg.eigvalsh(Psi @ Psi.T))[::-1]
    want = []
    for (N, S), (M, _) in sector_matrices(prob, psi).items():
        for w in np.linalg.eigvalsh(M @ M.T):
            want += [w / (S + 1)] * (S + 1)
    want = np.sort(np.array(want))[::-1]
    n = min(len(fock), len(want))
    assert np.abs(fock[:n] - want[:n]).max() < 1e-12 * fock[0]
    assert np.abs(fock[n:]).max(initial=0.0) < 1e-12 and np.abs(want[n:]).max(initial=0.0) < 1e-12


def test_selection_keeps_the_largest_and_all_reproduces_psi():
    prob = random_problem(10, 10, 0, 4, 40, p=4)
    psi = _psi(prob, 7)
    mats = sector_matrices(prob, psi)
    allw = np.sort(np.concatenate([np.linalg.eigvalsh(M @ M.T) for M, _ in mats.values()]))[::-1]
    for D in (5, 17, 40):
        keep, eig = truncate(prob, psi, D)
        kept = np.sort(np.concatenate([np.linalg.eigvalsh(mats[(N, S)][0] @ mats[(N, S)][0].T)[::-1][:U.shape[1]]
                                       for N, S, U in keep]))[::-1]
        assert sum(U.shape[1] for _, _, U in keep) == min(D, int(np.sum(allw > 0)))
        assert np.allclose(kept, allw[:len(kept)], rtol=0, atol=1e-14)
    total = sum(M.shape[0] for M, _ in mats.values())
    keep, _ = truncate(prob, psi, total, cutoff=-1.0)
    for N, S, U in keep:
        M = mats[(N, S)][0]
        assert np.allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-12)
        assert np.abs(U @ (U.T @ M) - M).max() < 1e-12


def test_right_trace_and_singlet_spectrum():
    """Right-growing mirror: the trace is |psi|^2, and for a singlet the two
    sides of the cut (L l) | (r R) share their nonzero reduced-density-matrix
    eigenvalues spin by spin (Schmidt decomposition in each S_Ll = S_rR)."""
    from oracle.truncate import sector_matrices_right
    prob = exact_problem(6, 6, 0, 28, p=2)
    psi = _psi(prob, 8)
    left = sector_matrices(prob, psi)
    right = sector_matrices_right(prob, psi)
    assert abs(sum(float(np.sum(M * M)) for M, _ in right.values()) - float(psi @ psi)) < 1e-12
    for S2 in sorted({S for (_, S) in left}):
        wl = np.sort(np.concatenate([np.linalg.eigvalsh(M @ M.T) for (N, S), (M, _) in left.items() if S == S2]))
        wr = np.sort(np.concatenate([np.linalg.eigvalsh(M @ M.T) for (N, S), (M, _) in right.items() if S == S2]
                                    or [np.zeros(0)]))
        wl, wr = wl[wl > 1e-13], wr[wr > 1e-13]
        assert len(wl) == len(wr) and np.abs(wl - wr).max(initial=0.0) < 1e-12, S2
