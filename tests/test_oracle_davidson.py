"""Pins of oracle/davidson.py against dense eigh."""
import numpy as np

from paper_2309_16724_amd.synth.problem import exact_problem, random_problem, random_vector
from oracle.hpsi import HEff
from oracle.davidson import davidson


def test_davidson_matches_eigh_exact_blocks():
    prob = exact_problem(6, 6, 0, 3)
    H = HEff(prob).dense()
    w = np.linalg.eigvalsh(H)
    th, u, it, rn, nh = davidson(lambda v: H @ v, np.diag(H), random_vector(len(H), 100))
    assert rn <= 1e-8
    assert abs(th - w[0]) < 1e-10
    assert np.linalg.norm(H @ u - th * u) < 1e-8 * 1.0001


def test_davidson_restart_path():
    prob = random_problem(6, 6, 0, 5, D=60)
    H = HEff(prob).dense()
    w = np.linalg.eigvalsh(H)
    th, u, it, rn, nh = davidson(lambda v: H @ v, np.diag(H), random_vector(len(H), 101),
                                 m_max=6)
    assert it > 6          # restarts happened
    assert abs(th - w[0]) < 1e-10
