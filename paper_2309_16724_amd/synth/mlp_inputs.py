"""Seeded inputs for the learned-preconditioner network: parameter vectors
and synthetic training batches (float32, as the device stores them)."""
import numpy as np


def param_count(n_in, width):
    return n_in * width + width + width * width + width + width + 1


def mlp_params(n_in, width, seed, out_scale=0.1):
    """He-style random parameters in the flat layout W1, b1, W2, b2, w3, b3."""
    rng = np.random.default_rng(seed)
    parts = [rng.standard_normal(n_in * width) * np.sqrt(2.0 / n_in),
             rng.standard_normal(width) * 0.1,
             rng.standard_normal(width * width) * np.sqrt(2.0 / width),
             rng.standard_normal(width) * 0.1,
             rng.standard_normal(width) * np.sqrt(1.0 / width) * out_scale,
             rng.standard_normal(1) * 0.1]
    return np.concatenate(parts).astype(np.float32)


def mlp_batch(n, n_in, seed):
    """Rows x (n x n_in) and targets a, b shaped like preconditioner data."""
    rng = np.random.default_rng(seed)
    x = np.stack([np.arcsinh(rng.standard_normal(n) * 3.0)] +
                 [np.full(n, -rng.uniform(0.0, 1.0))] * (n_in - 1), axis=1)
    a = rng.standard_normal(n) * np.exp(rng.standard_normal(n))
    b = a * (1.0 + 0.5 * np.tanh(x[:, 0])) + 0.1 * rng.standard_normal(n)
    return x.astype(np.float32), a.astype(np.float32), b.astype(np.float32)
