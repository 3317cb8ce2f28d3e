"""Canonical list of SU(2) two-site wavefunction blocks (oracle's own copy).

A block is labelled (iL, l, 2S_Ll, r, iR, 2S_rR): left-block sector iL,
site multiplet l in {0: empty (s=0), 1: single (s=1/2), 2: double (s=0)},
intermediate spin S_Ll of (L x l), site multiplet r, right-block sector iR
and S_rR of (r x R).  The coupled state is ((L l) S_Ll (r R) S_rR) S with
the electron count of all four parts summing to N.  Canonical order: nested
loops in the order iL, l, 2S_Ll (ascending), r, iR, 2S_rR (ascending).
Each block is a column-major d_L x d_R matrix; blocks are concatenated.

Parity unpinned as a layout (it is a convention); its consequences are
pinned through the H.psi tests.
"""
SITE = [(0, 0), (1, 1), (2, 0)]   # (electrons, doubled spin) of site multiplets


def psi_blocks(lsec, rsec, n_elec, two_s):
    out = []
    off = 0
    for iL, (NL, SL, dL) in enumerate(lsec):
        for l, (nl, sl) in enumerate(SITE):
            for SLl in range(abs(SL - sl), SL + sl + 1, 2):
                for r, (nr, sr) in enumerate(SITE):
                    for iR, (NR, SR, dR) in enumerate(rsec):
                        if NL + nl + nr + NR != n_elec:
                            continue
                        for SrR in range(abs(sr - SR), sr + SR + 1, 2):
                            if not (abs(SLl - SrR) <= two_s <= SLl + SrR):
                                continue
                            out.append(dict(iL=iL, l=l, SLl=SLl, r=r, iR=iR, SrR=SrR,
                                            off=off, dL=dL, dR=dR))
                            off += dL * dR
    return out, off
