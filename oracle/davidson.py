"""Plain Davidson eigensolver for the lowest eigenpair (oracle).

The paper names Lanczos or Davidson for the effective-Hamiltonian
diagonalisation (Sec. II) and fixes no details; the reading used here:
block size 1; subspace of at most m_max = 24 vectors, thick restart to the
current and previous Ritz vectors; two-pass classical Gram-Schmidt; the
correction t = -r / (diag - theta) with the denominator's magnitude floored
at floor * sigma, sigma the root mean square of diag - theta over the vector
(floor = 1e-2: a relative floor, so that the cap on the few elements with
diag ~ theta scales with the spread of the diagonal); convergence when
||r||_2 <= tol for the normalised Ritz vector.
Pinned in tests/test_oracle_davidson.py against dense eigh.
"""
import numpy as np


def _orth(V, t, passes=2):
    for _ in range(passes):
        t = t - V @ (V.T @ t)
    return t


FLOOR = 1e-2


def floor_abs(diag, theta, floor=FLOOR):
    """Absolute denominator floor: floor times the RMS of diag - theta."""
    den = np.asarray(diag, dtype=float) - theta
    return floor * np.sqrt(np.mean(den * den))


def davidson(hop, diag, x0, tol=1e-8, max_iter=1000, m_max=24, floor=FLOOR, precond=None,
             record=None):
    """Return (theta, u, n_iter, residual_norm, n_hop).

    precond(r, u, theta) -> t replaces the diagonal correction when given;
    record, a list, receives (r, u, theta) of every iteration that takes a
    correction step."""
    x = np.asarray(x0, dtype=float)
    x = x / np.linalg.norm(x)
    V = x[:, None]
    W = hop(x)[:, None]
    n_hop = 1
    u_prev = None
    theta = None
    for it in range(1, max_iter + 1):
        G = V.T @ W
        G = 0.5 * (G + G.T)
        w, s = np.linalg.eigh(G)
        theta = w[0]
        c = s[:, 0]
        u = V @ c
        hu = W @ c
        r = hu - theta * u
        rn = np.linalg.norm(r)
        if rn <= tol:
            return theta, u, it, rn, n_hop
        if record is not None:
            record.append((r.copy(), u.copy(), theta))
        if precond is None:
            den = diag - theta
            fl = floor_abs(diag, theta, floor)
            den = np.where(np.abs(den) < fl, np.where(den < 0, -fl, fl), den)
            t = -r / den
        else:
            t = precond(r, u, theta)
        if V.shape[1] >= m_max:
            # thick restart to span{u, u_prev}, orthonormalised in the
            # coefficient space of the orthonormal basis V
            cols = [c / np.linalg.norm(c)]
            if u_prev is not None:
                c2 = V.T @ u_prev
                for _ in range(2):
                    c2 = c2 - cols[0] * (cols[0] @ c2)
                n2 = np.linalg.norm(c2)
                if n2 > 1e-8:
                    cols.append(c2 / n2)
            Cm = np.stack(cols, axis=1)
            V = V @ Cm
            W = W @ Cm
        t = _orth(V, t)
        tn = np.linalg.norm(t)
        if tn < 1e-12:
            t = _orth(V, r)
            tn = np.linalg.norm(t)
        t = t / tn
        V = np.concatenate([V, t[:, None]], axis=1)
        W = np.concatenate([W, hop(t)[:, None]], axis=1)
        n_hop += 1
        u_prev = u
    return theta, u, max_iter, rn, n_hop
