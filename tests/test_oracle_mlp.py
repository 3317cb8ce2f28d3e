"""Pins of oracle/mlp.py: finite differences, brute-force loops, closed
forms of the loss gradient and of the first Adam step, training-row
normalisation, and the zero network reducing to the diagonal step."""
import numpy as np
import pytest

from oracle import mlp
from oracle.davidson import davidson
from oracle.hpsi import HEff
from paper_2309_16724_amd.synth.mlp_inputs import mlp_batch, mlp_params
from paper_2309_16724_amd.synth.problem import random_problem, random_vector


def test_forward_matches_explicit_loops():
    n_in, width = 2, 3
    p = mlp_params(n_in, width, 5).astype(np.float64)
    x, _, _ = mlp_batch(4, n_in, 6)
    g, _ = mlp.forward(p, x, width)
    # independent walk over the flat layout
    k = 0
    W1 = [[p[k + i * width + j] for j in range(width)] for i in range(n_in)]; k += n_in * width
    b1 = list(p[k:k + width]); k += width
    W2 = [[p[k + i * width + j] for j in range(width)] for i in range(width)]; k += width * width
    b2 = list(p[k:k + width]); k += width
    w3 = list(p[k:k + width]); k += width
    b3 = p[k]
    for row in range(4):
        h1 = [max(0.0, sum(float(x[row, i]) * W1[i][j] for i in range(n_in)) + b1[j]) for j in range(width)]
        h2 = [max(0.0, sum(h1[i] * W2[i][j] for i in range(width)) + b2[j]) for j in range(width)]
        ref = sum(h2[j] * w3[j] for j in range(width)) + b3
        assert abs(g[row] - ref) < 1e-14 * max(1.0, abs(ref))


@pytest.mark.parametrize("width", [4, 32])
def test_gradient_matches_central_differences(width):
    n_in = 2
    p = mlp_params(n_in, width, 11).astype(np.float64)
    x, a, b = mlp_batch(40, n_in, 12)
    _, gr = mlp.grad(p, x, a, b, width)
    rng = np.random.default_rng(0)
    idx = np.unique(np.concatenate([rng.integers(0, p.size, 60), [0, n_in * width, p.size - 1,
                                                                  p.size - 2]]))
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp.loss(pp, x, a, b, width) - mlp.loss(pm, x, a, b, width)) / (2 * h)
        assert abs(fd - gr[i]) <= 1e-6 * max(1e-3, abs(gr[i])) + 1e-9, (i, fd, gr[i])


def test_gradient_closed_form_constant_network():
    """W2 = 0, b2 > 0: g = w3 . b2 + b3 for every row, so d loss/d b3 and
    d loss/d w3 have closed forms and W1, b1 get no gradient."""
    n_in, width = 2, 8
    p = mlp_params(n_in, width, 3).astype(np.float64)
    w3 = mlp.unpack(p, n_in, width)[4].copy()
    b3 = mlp.unpack(p, n_in, width)[5]
    off = n_in * width + width
    p[off:off + width * width] = 0.0
    p[off + width * width:off + width * width + width] = np.linspace(0.1, 0.8, width)
    b2v = np.linspace(0.1, 0.8, width)
    x, a, b = (v.astype(np.float64) for v in mlp_batch(30, n_in, 4))
    g0 = w3 @ b2v + b3
    L, gr = mlp.grad(p, x, a, b, width)
    e = a * (1 + g0) - b
    assert abs(L - np.mean(e * e)) < 1e-14 * L
    assert abs(gr[-1] - np.mean(2 * e * a)) < 1e-13
    assert np.allclose(gr[-1 - width:-1], np.mean(2 * e * a) * b2v, rtol=1e-12, atol=1e-15)
    assert np.all(gr[:n_in * width + width] == 0.0)


def test_first_adam_step_closed_form():
    """At t = 1 bias correction gives m_hat = g, v_hat = g^2: the step is
    lr g / (|g| + eps)."""
    rng = np.random.default_rng(1)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p1, m1, v1 = mlp.adam_step(p, np.zeros(50), np.zeros(50), g, 1, 1e-3)
    assert np.allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)


def test_features_and_rows_by_hand():
    d = np.array([2.0, 0.0])
    f = mlp.features(d, np.array([3.0, 4.0]), 1.0)       # d - theta = +-1, sigma = 1, ||r|| = 5
    assert np.allclose(f[:, 0], np.arcsinh([1.0, -1.0]))
    assert np.allclose(f[:, 1], np.log10(5.0) / 8)
    # psi* = u + e with e orthogonal to u and <u|psi*> = 1: the exact correction is e
    u = np.array([1.0, 0.0, 0.0])
    e = np.array([0.0, 0.3, -0.4])
    x, a, b = mlp.training_rows(np.array([1.0, 2.0, 3.0]), np.array([0.0, 1.0, 1.0]), u, 0.5,
                                (u + e) / np.linalg.norm(u + e))
    assert np.allclose(b, e * np.sqrt(3) / 0.5)
    assert abs(np.sum(b * b) - 3) < 1e-12
    assert np.allclose(a, -np.array([0.0, 1.0, 1.0]) / np.array([0.5, 1.5, 2.5]) * np.sqrt(3) / 0.5)


def test_row_weight_cap():
    """A row with |a| > A_MAX is scaled to |a| = A_MAX, keeping b/a."""
    u = np.array([1.0, 0.0, 0.0, 0.0])
    e = np.array([0.0, 0.5, 0.5, 0.5])
    d = np.array([1.0, 2.0, 0.5 + 1e-6, 3.0])     # element 2: denominator 1e-6
    r = np.array([0.0, 1.0, 1.0, 1.0])
    # floor below the 1e-6 denominator, so the unfloored step is the raw row
    x, a, b = mlp.training_rows(d, r, u, 0.5, (u + e) / np.linalg.norm(u + e), floor=1e-8)
    s = np.sqrt(4) / np.linalg.norm(e)
    raw_a = -r / (d - 0.5) * s
    assert abs(abs(a[2]) - mlp.A_MAX) < 1e-12
    assert abs(b[2] / a[2] - (e[2] * s) / raw_a[2]) < 1e-12
    assert np.allclose(a[[1, 3]], raw_a[[1, 3]]) and np.allclose(b[[1, 3]], e[[1, 3]] * s)


def test_zero_network_is_diagonal_davidson():
    prob = random_problem(6, 6, 0, 5, D=60)
    H = HEff(prob).dense()
    d = np.diag(H).copy()
    x0 = random_vector(len(H), 100)
    width = 16
    p0 = np.zeros(mlp.n_params(2, width))
    ref = davidson(lambda v: H @ v, d, x0)
    got = davidson(lambda v: H @ v, d, x0, precond=lambda r, u, th: mlp.mlp_step(p0, width, d, r, th))
    assert got[2] == ref[2] and abs(got[0] - ref[0]) < 1e-14


def test_recorded_rows_label_the_converged_vector():
    """Rows built from the recorded iterations: the exact correction of the
    last recorded iteration points from u_k to psi*."""
    prob = random_problem(6, 6, 0, 5, D=60)
    H = HEff(prob).dense()
    d = np.diag(H).copy()
    rec = []
    th, psi, it, rn, _ = davidson(lambda v: H @ v, d, random_vector(len(H), 100), record=rec)
    assert len(rec) == it - 1
    r, u, t = rec[-1]
    x, a, b = mlp.training_rows(d, r, u, t, psi)
    ts = psi / (u @ psi) - u
    assert abs(u @ ts) < 1e-12
    assert np.allclose(b / np.linalg.norm(b), ts / np.linalg.norm(ts))
