"""Truncation of a two-site step (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

After the Davidson solve the two-site wavefunction is cut to at most D
multiplets of (left block x left site) before the renormalization (Sec. II:
the two-site DMRG step; the rule is left to the reviews the paper cites).
For every product sector (N, 2S) of the left block and the site -- rows
ordered as in oracle.renorm.product_sectors -- the reduced coefficients of
the wavefunction blocks whose (L l) part is that sector form a matrix M
(rows: the sector's components (L sector, site multiplet); columns: every
(r, R, S_rR) right part, concatenated in block order); the reduced density
matrix is rho = M M^T.  Its eigenvectors with the largest eigenvalues over
all sectors are kept (at most max_kept, eigenvalues <= cutoff dropped; ties
by sector order then eigenvalue index), as the columns of U in descending
eigenvalue order.

The mirror (``truncate_right``) cuts (right site x right block) for the
renormalization of the right block: sectors (N, 2S) of r x R with rows as in
oracle.renorm.product_sectors_right, M's columns the left parts
(L sector, l, S_Ll), rho = M M^T with M[(r, R), (left part)] = X^T.

Pinned in tests/test_oracle_truncate.py: the trace of rho over all sectors
is |psi|^2; for a singlet wavefunction the reduced density matrix of
(L l) in the M-resolved Fock space has the eigenvalues w / (2S + 1) of
every sector's rho, each 2S + 1 times; keeping every state reproduces psi.
"""
import numpy as np

from .layout import psi_blocks, SITE
from .renorm import product_sectors, product_sectors_right


def sector_matrices(prob, psi):
    """{(N, 2S): (M, comps)} of the left-growing truncation."""
    blocks, size = psi_blocks(prob.left.sectors, prob.right.sectors, prob.n_elec, prob.two_s)
    assert psi.size == size
    lsec = prob.left.sectors
    prods = {(N, S): comps for (N, S, rows, comps) in product_sectors(lsec)}
    rowpos = {}
    for key, comps in prods.items():
        for (iL, m, row0, d) in comps:
            rowpos[(key, iL, m)] = (row0, d)
    cols = {}
    for b in blocks:
        key = (lsec[b["iL"]][0] + SITE[b["l"]][0], b["SLl"])
        cols.setdefault(key, {}).setdefault((b["r"], b["iR"], b["SrR"]), b["dR"])
    out = {}
    for key, comps in prods.items():
        rows = sum(c[3] for c in comps)
        parts = cols.get(key, {})
        coff, n = {}, 0
        for c in sorted(parts, key=lambda c: (c[0], c[1], c[2])):
            coff[c] = n
            n += parts[c]
        out[key] = (np.zeros((rows, n)), comps, coff)
    for b in blocks:
        key = (lsec[b["iL"]][0] + SITE[b["l"]][0], b["SLl"])
        M, comps, coff = out[key]
        row0, d = rowpos[(key, b["iL"], b["l"])]
        X = psi[b["off"]:b["off"] + b["dL"] * b["dR"]].reshape(b["dR"], b["dL"]).T
        c0 = coff[(b["r"], b["iR"], b["SrR"])]
        M[row0:row0 + d, c0:c0 + b["dR"]] = X
    return {k: (M, comps) for k, (M, comps, coff) in out.items()}


def truncate(prob, psi, max_kept, cutoff=0.0):
    """(keep, eigenvalues): keep = [(N, 2S, U)] in product-sector order for
    the sectors that keep states; eigenvalues = {(N, 2S): ascending array}."""
    mats = sector_matrices(prob, np.asarray(psi, dtype=float))
    order = [(N, S) for (N, S, rows, comps) in product_sectors(prob.left.sectors)]
    eig, cand = {}, []
    for si, key in enumerate(order):
        M, comps = mats[key]
        rho = M @ M.T
        w, V = np.linalg.eigh(rho)
        eig[key] = (w, V)
        for i in range(len(w) - 1, -1, -1):
            if w[i] > cutoff:
                cand.append((-w[i], si, len(w) - 1 - i))
    cand.sort()
    take = {}
    for (_, si, rank) in cand[:max_kept]:
        take[si] = take.get(si, 0) + 1
    keep = []
    for si, key in enumerate(order):
        k = take.get(si, 0)
        if k == 0:
            continue
        w, V = eig[key]
        keep.append((key[0], key[1], V[:, ::-1][:, :k]))
    return keep, {k: v[0] for k, v in eig.items()}


def sector_matrices_right(prob, psi):
    """{(N, 2S): (M, comps)} of the right-growing truncation."""
    blocks, size = psi_blocks(prob.left.sectors, prob.right.sectors, prob.n_elec, prob.two_s)
    assert psi.size == size
    rsec = prob.right.sectors
    prods = {(N, S): comps for (N, S, rows, comps) in product_sectors_right(rsec)}
    rowpos = {}
    for key, comps in prods.items():
        for (m, iR, row0, d) in comps:
            rowpos[(key, m, iR)] = (row0, d)
    cols = {}
    for b in blocks:
        key = (rsec[b["iR"]][0] + SITE[b["r"]][0], b["SrR"])
        cols.setdefault(key, {}).setdefault((b["iL"], b["l"], b["SLl"]), b["dL"])
    out = {}
    for key, comps in prods.items():
        rows = sum(c[3] for c in comps)
        parts = cols.get(key, {})
        coff, n = {}, 0
        for c in sorted(parts):
            coff[c] = n
            n += parts[c]
        out[key] = (np.zeros((rows, n)), comps, coff)
    for b in blocks:
        key = (rsec[b["iR"]][0] + SITE[b["r"]][0], b["SrR"])
        M, comps, coff = out[key]
        row0, d = rowpos[(key, b["r"], b["iR"])]
        X = psi[b["off"]:b["off"] + b["dL"] * b["dR"]].reshape(b["dR"], b["dL"]).T
        c0 = coff[(b["iL"], b["l"], b["SLl"])]
        M[row0:row0 + d, c0:c0 + b["dL"]] = X.T
    return {k: (M, comps) for k, (M, comps, coff) in out.items()}


def truncate_right(prob, psi, max_kept, cutoff=0.0):
    """``truncate`` for (right site x right block): keep = [(N, 2S, U)] in the
    order of product_sectors_right."""
    mats = sector_matrices_right(prob, np.asarray(psi, dtype=float))
    order = [(N, S) for (N, S, rows, comps) in product_sectors_right(prob.right.sectors)]
    eig, cand = {}, []
    for si, key in enumerate(order):
        M, comps = mats[key]
        w, V = np.linalg.eigh(M @ M.T)
        eig[key] = (w, V)
        for i in range(len(w) - 1, -1, -1):
            if w[i] > cutoff:
                cand.append((-w[i], si, len(w) - 1 - i))
    cand.sort()
    take = {}
    for (_, si, rank) in cand[:max_kept]:
        take[si] = take.get(si, 0) + 1
    keep = []
    for si, key in enumerate(order):
        k = take.get(si, 0)
        if k:
            w, V = eig[key]
            keep.append((key[0], key[1], V[:, ::-1][:, :k]))
    return keep, {k: v[0] for k, v in eig.items()}
