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


def test_relative_floor_by_hand():
    """The diagonal step's denominator floor is relative: |d - theta| is
    raised to floor * RMS(d - theta) (reading of the Davidson details)."""
    from oracle import mlp
    d = np.array([1.0, 2.0, 0.5 + 1e-9, 4.0])
    r = np.array([1.0, -2.0, 3.0, 0.5])
    th = 0.5
    den = d - th
    sigma = np.sqrt(np.mean(den * den))
    t = mlp.diagonal_step(d, r, th, floor=0.1)
    assert abs(t[2] - (-3.0 / (0.1 * sigma))) < 1e-12 * abs(t[2])
    assert np.allclose(t[[0, 1, 3]], -r[[0, 1, 3]] / den[[0, 1, 3]], rtol=1e-15)
    # a negative small denominator keeps its sign
    t = mlp.diagonal_step(d, r, 0.5 + 2e-9, floor=0.1)
    assert t[2] > 0


def test_relative_floor_is_scale_invariant():
    """Scaling H by a constant scales every Ritz value and residual and
    leaves the relative floor's iterates unchanged: same iteration count,
    energies in proportion."""
    rng = np.random.default_rng(7)
    n = 120
    g = rng.standard_normal((n, n))
    H = 0.3 * (g + g.T) + np.diag(np.linspace(-2.0, 6.0, n))
    x0 = random_vector(n, 103)
    a = davidson(lambda v: H @ v, np.diag(H), x0, tol=1e-9)
    H2 = 1000.0 * H
    b = davidson(lambda v: H2 @ v, np.diag(H2), x0, tol=1e-6)
    assert a[2] == b[2]
    assert abs(b[0] - 1000.0 * a[0]) < 1e-8 * abs(b[0])


def test_floor_active_near_convergence():
    """A diagonal element within the floor of the lowest eigenvalue (a
    weakly coupled basis state just above it), so the relative floor caps
    that element's denominator in every late iteration: the default solve
    converges to the dense eigh value."""
    rng = np.random.default_rng(11)
    n = 300
    g = rng.standard_normal((n, n))
    H = 0.8 * (g + g.T) / np.sqrt(n) + np.diag(rng.uniform(-3.0, 3.0, n))
    w0 = np.linalg.eigvalsh(H[1:, 1:])[0]
    c = 1e-3 * rng.standard_normal(n - 1)
    H[0, 1:] = c
    H[1:, 0] = c
    H[0, 0] = w0 + 1e-5
    w = np.linalg.eigvalsh(H)
    d = np.diag(H)
    sigma = np.sqrt(np.mean((d - w[0]) ** 2))
    assert d.min() - w[0] < 0.1 * 1e-2 * sigma     # the floor is active at the solution
    th, u, it, rn, nh = davidson(lambda v: H @ v, d, random_vector(n, 104))
    assert rn <= 1e-8
    assert abs(th - w[0]) < 1e-10
