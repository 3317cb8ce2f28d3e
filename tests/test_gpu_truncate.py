"""GPU parity of the truncation (dmrg_truncate) against the oracle
(oracle/truncate.py), and the truncation -> renormalization chain."""
import sys

import numpy as np
import pytest

from paper_2309_16724_amd.synth import catalogue as cat
from paper_2309_16724_amd.synth.problem import random_problem, random_vector
from oracle.layout import psi_blocks
from oracle.truncate import truncate as o_truncate
from oracle.renorm import renormalize

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    return t


def _psi(prob, seed):
    _, size = psi_blocks(prob.left.sectors, prob.right.sectors, prob.n_elec, prob.two_s)
    return random_vector(size, seed)


@pytest.mark.parametrize("args,D", [
    (dict(n_orb=12, n_elec=12, two_s=0, seed=41, D=96, p=5, spin_ratio=0.3, sigma_frac=0.08), 60),
    (dict(n_orb=11, n_elec=11, two_s=1, seed=42, D=64, p=4), 200),
])
def test_truncation_matches_oracle(torch, args, D):
    from paper_2309_16724_amd.hpsi import truncate, keep_host
    _say("truncate parity %s D=%d" % (args, D))
    prob = random_problem(**args)
    psi = _psi(prob, 9)
    nrm = float(psi @ psi)
    cut = 1e-12 * nrm
    keep, u, (kw, tr) = truncate(prob, torch.from_numpy(psi).cuda(), D, cut)
    got = keep_host(prob, keep, u)
    want, eig = o_truncate(prob, psi, D, cut)
    assert [(n, s, U.shape[1]) for n, s, U in got] == [(n, s, U.shape[1]) for n, s, U in want]
    assert abs(tr - nrm) < 1e-12 * nrm
    wsum = sum(float(np.sum(eig[(n, s)][::-1][:U.shape[1]])) for n, s, U in want)
    assert abs(kw - wsum) < 1e-12 * nrm
    for (n, s, Ug), (_, _, Uw) in zip(got, want):
        assert np.abs(Ug.T @ Ug - np.eye(Ug.shape[1])).max() < 1e-12
        assert np.abs(Ug @ Ug.T - Uw @ Uw.T).max() < 1e-9, (n, s)


def test_truncation_then_renormalization(torch):
    """The GPU chain (truncate, then renormalize with its U) against the
    oracle chain: the renormalized block Hamiltonian has the same spectrum
    per sector (the eigenvector signs cancel in it)."""
    from paper_2309_16724_amd.hpsi import truncate, keep_host, Renorm
    prob = random_problem(12, 12, 0, 43, 80, p=5, spin_ratio=0.3, sigma_frac=0.08)
    psi = _psi(prob, 10)
    _say("truncate -> renormalize chain")
    keep, u, _ = truncate(prob, torch.from_numpy(psi).cuda(), 50, 1e-12 * float(psi @ psi))
    kh = keep_host(prob, keep, u)
    r = Renorm(prob, kh, fam_mask=1 << cat.H)
    r.apply()
    got = r.block()
    r.free()
    want = renormalize(prob, o_truncate(prob, psi, 50, 1e-12 * float(psi @ psi))[0], families=(cat.H,))
    for (f, row, col, off, npos) in want.records:
        a = np.linalg.eigvalsh(got.block(cat.H, row, col)[0])
        b = np.linalg.eigvalsh(want.block(cat.H, row, col)[0])
        assert np.abs(a - b).max() < 1e-9 * max(1.0, np.abs(b).max())


def test_right_truncation_matches_oracle_and_chains(torch):
    """Mirror: (right site) x (right block) against the oracle, then the
    right renormalization with its U against the oracle chain."""
    from paper_2309_16724_amd.hpsi import truncate, keep_host, Renorm
    from oracle.truncate import truncate_right
    from oracle.renorm import renormalize_right
    prob = random_problem(12, 12, 0, 44, 96, p=5, spin_ratio=0.3, sigma_frac=0.08)
    psi = _psi(prob, 11)
    cut = 1e-12 * float(psi @ psi)
    _say("truncate right")
    keep, u, (kw, tr) = truncate(prob, torch.from_numpy(psi).cuda(), 60, cut, right=True)
    got = keep_host(prob, keep, u, right=True)
    want, eig = truncate_right(prob, psi, 60, cut)
    assert [(n, s, U.shape[1]) for n, s, U in got] == [(n, s, U.shape[1]) for n, s, U in want]
    for (n, s, Ug), (_, _, Uw) in zip(got, want):
        assert np.abs(Ug @ Ug.T - Uw @ Uw.T).max() < 1e-9, (n, s)
    r = Renorm(prob, got, fam_mask=1 << cat.H, right=True)
    r.apply()
    blk = r.block()
    r.free()
    ref = renormalize_right(prob, want, families=(cat.H,))
    for (f, row, col, off, npos) in ref.records:
        a = np.linalg.eigvalsh(blk.block(cat.H, row, col)[0])
        b = np.linalg.eigvalsh(ref.block(cat.H, row, col)[0])
        assert np.abs(a - b).max() < 1e-9 * max(1.0, np.abs(b).max())
