"""Learned Davidson preconditioner, plain FP64 NumPy (oracle: test
infrastructure only, never called by the product path).

The paper says nothing about preconditioning (it names Lanczos or Davidson
for the effective-Hamiltonian diagonalisation, Sec. II).  The reading followed
here and by the HIP kernels:

* The network is a 3-layer perceptron g = w3 . relu(W2 relu(W1 x + b1) + b2)
  + b3 with n_in inputs and two hidden layers of width H (flat parameter
  vector laid out as W1[n_in][H], b1[H], W2[H][H], b2[H], w3[H], b3[1],
  row-major, W[k][j] multiplying input k into unit j).
* It corrects the diagonal Davidson step multiplicatively, per element:
  t_i = td_i (1 + g(x_i)), td_i = -r_i / (d_i - theta) (denominator magnitude
  floored at floor * sigma, the relative floor of the diagonal step).
* Per element features x_i = (asinh((d_i - theta) / sigma), log10(||r||) / 8),
  sigma = root mean square of d - theta over the problem's vector.
* Training pairs come from a converged solve psi*: at iteration k with Ritz
  pair (theta_k, u_k) the exact correction is t*_k = psi*/<u_k|psi*> - u_k
  (the step that would converge in one iteration).  One row per element with
  a_i = td_i s, b_i = t*_i s, s = sqrt(n) / ||t*_k||, and the loss is the mean
  over rows of (a_i (1 + g_i) - b_i)^2, so every record weighs the same.
  Rows whose |a_i| exceeds A_MAX (elements with a nearly vanishing
  denominator) are scaled by A_MAX / |a_i|: the row keeps its optimum
  g = b/a - 1 but cannot dominate the least-squares fit.
* Adam with bias correction.
"""
import numpy as np

N_IN = 2
A_MAX = 10.0


def n_params(n_in, width):
    return n_in * width + width + width * width + width + width + 1


def unpack(p, n_in, width):
    """Views (W1, b1, W2, b2, w3, b3) of the flat parameter vector."""
    p = np.asarray(p, dtype=np.float64)
    assert p.size == n_params(n_in, width)
    o = 0
    W1 = p[o:o + n_in * width].reshape(n_in, width); o += n_in * width
    b1 = p[o:o + width]; o += width
    W2 = p[o:o + width * width].reshape(width, width); o += width * width
    b2 = p[o:o + width]; o += width
    w3 = p[o:o + width]; o += width
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def forward(p, x, width):
    """g for every row of x (n x n_in); also returns the activations."""
    x = np.asarray(x, dtype=np.float64)
    W1, b1, W2, b2, w3, b3 = unpack(p, x.shape[1], width)
    z1 = x @ W1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0.0)
    g = h2 @ w3 + b3
    return g, (x, z1, h1, z2, h2)


def loss(p, x, a, b, width):
    g, _ = forward(p, x, width)
    e = np.asarray(a, float) * (1.0 + g) - np.asarray(b, float)
    return float(np.mean(e * e))


def grad(p, x, a, b, width):
    """(loss, d loss / d p) by back-propagation through the three layers."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    g, (x, z1, h1, z2, h2) = forward(p, x, width)
    n = x.shape[0]
    W1, b1, W2, b2, w3, b3 = unpack(p, x.shape[1], width)
    e = a * (1.0 + g) - b
    dg = 2.0 * e * a / n                      # d loss / d g_i
    gw3 = h2.T @ dg
    gb3 = dg.sum()
    dz2 = np.outer(dg, w3) * (z2 > 0)
    gW2 = h1.T @ dz2
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2.T) * (z1 > 0)
    gW1 = x.T @ dz1
    gb1 = dz1.sum(axis=0)
    flat = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gw3, [gb3]])
    return float(np.mean(e * e)), flat


def adam_step(p, m, v, gr, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t >= 1; returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * gr
    v = beta2 * v + (1.0 - beta2) * gr * gr
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


FLOOR = 1e-2


def floored(den, fl):
    """den with magnitudes below the absolute floor fl raised to fl."""
    return np.where(np.abs(den) < fl, np.where(den < 0, -fl, fl), den)


def sigma_of(diag, theta):
    """Root mean square of d - theta over one problem's vector."""
    den = np.asarray(diag, float) - theta
    return np.sqrt(np.mean(den * den))


def features(diag, r, theta):
    """Rows (asinh((d - theta)/sigma), log10 ||r|| / 8) for one problem."""
    den = np.asarray(diag, float) - theta
    sigma = sigma_of(diag, theta)
    rn = np.linalg.norm(r)
    return np.stack([np.arcsinh(den / sigma), np.full(den.size, np.log10(rn) / 8.0)], axis=1)


def diagonal_step(diag, r, theta, floor=FLOOR):
    """-r / (d - theta), |d - theta| floored at floor * sigma (relative floor)."""
    return -np.asarray(r, float) / floored(np.asarray(diag, float) - theta,
                                           floor * sigma_of(diag, theta))


def training_rows(diag, r, u, theta, psi_star, floor=FLOOR):
    """(x, a, b) of one Davidson iteration given the converged vector."""
    ts = psi_star / (u @ psi_star) - u
    s = np.sqrt(ts.size) / np.linalg.norm(ts)
    a = diagonal_step(diag, r, theta, floor) * s
    b = ts * s
    w = np.minimum(1.0, A_MAX / np.maximum(np.abs(a), 1e-300))
    return features(diag, r, theta), a * w, b * w


def mlp_step(p, width, diag, r, theta, floor=FLOOR):
    """Learned correction t = td (1 + g(x)) of one problem."""
    g, _ = forward(p, features(diag, r, theta), width)
    return diagonal_step(diag, r, theta, floor) * (1.0 + g)
