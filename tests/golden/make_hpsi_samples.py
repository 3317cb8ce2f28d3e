"""Writes tests/golden/hpsi_samples.json: H_eff psi at sampled elements of
the large workloads, evaluated by the oracle alone (oracle.hpsi.HEff with a
sample; calls nothing of the HIP library).

    python tests/golden/make_hpsi_samples.py [case ...]

Cases (generator arguments of paper_2309_16724_amd.synth.problem):
* L54_D2048: L=54 orbitals, N=54, S=0, integral seed 2, D=2048 multiplets per
  block with sector dims up to 894 (the metric's workload, the shape of the
  paper's CAS(54,54) runs, Sec. IV B).
* L6_sector2035: L=6, N=6, S=0, seed 7, uncapped 2-orbital blocks, left
  block D=4800 with one sector of 2035 multiplets, right D=160 (long K).
Per case: the largest wavefunction block plus seeded random blocks, four
seeded rows and columns of each (all of a smaller dimension), input psi the
normalised seeded vector of seed 100.  A checksum of the generated operator
data lets the test detect a drifted generator.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_2309_16724_amd.synth.problem import random_problem, random_vector  # noqa: E402
from oracle.hpsi import HEff  # noqa: E402

CASES = {
    "L54_D2048": dict(args=(54, 54, 0, 2), kw=dict(D=2048, spin_ratio=0.45, sigma_frac=0.03),
                      n_random_blocks=3, per_dim=4),
    "L6_sector2035": dict(args=(6, 6, 0, 7), kw=dict(D=4800, D_right=160, cap=False),
                          n_random_blocks=5, per_dim=4),
}
OUT = os.path.join(HERE, "hpsi_samples.json")


def checksum(prob):
    """Digest of the generated blocks (sector tables, records, a strided
    subsample of the data and the data sums)."""
    h = hashlib.sha256()
    for blk in (prob.left, prob.right):
        h.update(np.asarray(blk.sectors, dtype=np.int64).tobytes())
        h.update(blk.rec_array().tobytes())
        h.update(np.ascontiguousarray(blk.data[::9973]).tobytes())
    return h.hexdigest()[:32]


def make_case(name):
    spec = CASES[name]
    t0 = time.time()
    prob = random_problem(*spec["args"], **spec["kw"])
    he = HEff(prob)
    blocks = he.blocks
    rng = np.random.default_rng(12345)
    nb = len(blocks)
    big = max(range(nb), key=lambda i: blocks[i]["dL"] * blocks[i]["dR"])
    pick = sorted({big} | set(rng.choice(nb, size=spec["n_random_blocks"], replace=False).tolist()))
    k = spec["per_dim"]
    sample = {}
    for bi in pick:
        dL, dR = blocks[bi]["dL"], blocks[bi]["dR"]
        sample[bi] = (np.sort(rng.choice(dL, size=min(k, dL), replace=False)),
                      np.sort(rng.choice(dR, size=min(k, dR), replace=False)))
    hs = HEff(prob, sample)
    x = random_vector(hs.size, 100)
    ys = hs.apply_sample(x)
    out = {"generator": {"args": list(spec["args"]), "kw": spec["kw"]},
           "psi": "random_vector(size, 100)", "psi_len": int(hs.size), "n_blocks": nb,
           "checksum": checksum(prob),
           "samples": [{"block": int(bi), "dL": int(blocks[bi]["dL"]), "dR": int(blocks[bi]["dR"]),
                        "rows": [int(v) for v in sample[bi][0]],
                        "cols": [int(v) for v in sample[bi][1]],
                        "values": [[float(v) for v in row] for row in ys[bi]]} for bi in pick],
           "oracle_seconds": round(time.time() - t0, 1)}
    print(name, "done in %.1f s" % (time.time() - t0), flush=True)
    return out


def main():
    names = sys.argv[1:] or list(CASES)
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    data.setdefault("source", "oracle.hpsi.HEff(prob, sample).apply_sample (tests/golden/make_hpsi_samples.py)")
    data.setdefault("cases", {})
    for n in names:
        data["cases"][n] = make_case(n)
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1)


if __name__ == "__main__":
    main()
