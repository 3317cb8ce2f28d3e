"""GPU parity at the full large workloads against stored oracle values.

H_eff psi at sampled elements of (a) the L=54, D=2048 workload with sector
dims up to 894 (the metric's workload; the shape of the paper's CAS(54,54)
runs, Sec. IV B) and (b) an L=6 problem whose left block has one sector of
2035 multiplets (tiles with K and M near 2000).  The expected values were
written by tests/golden/make_hpsi_samples.py, which calls only the oracle
(oracle.hpsi.HEff with a sample).  Tolerances: FP64 1e-12 and split BF16
(s = 5) 1e-10, relative to the largest sampled magnitude, element by
element; both plans as bench.py builds them by default.
"""
import json
import os
import sys

import numpy as np
import pytest

from paper_2309_16724_amd.synth.problem import random_problem, random_vector

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hpsi_samples.json")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    return t


def _load(name):
    with open(GOLD) as f:
        return json.load(f)["cases"][name]


def _gather(y, blocks_off, s):
    dL, dR = s["dL"], s["dR"]
    off = blocks_off[s["block"]]
    Y = y[off:off + dL * dR].reshape(dR, dL).T
    return Y[np.ix_(s["rows"], s["cols"])]


@pytest.mark.parametrize("name", ["L6_sector2035", "L54_D2048"])
def test_large_workload_matches_oracle_samples(torch, name):
    from paper_2309_16724_amd.hpsi import Plan
    from oracle.layout import psi_blocks
    sys.path.insert(0, os.path.join(os.path.dirname(GOLD)))
    from make_hpsi_samples import checksum
    case = _load(name)
    g = case["generator"]
    _say("case %s: generating %s %s" % (name, g["args"], g["kw"]))
    prob = random_problem(*g["args"], **g["kw"])
    assert checksum(prob) == case["checksum"], "generator output differs from the stored case"
    blocks, size = psi_blocks(prob.left.sectors, prob.right.sectors, prob.n_elec, prob.two_s)
    assert size == case["psi_len"]
    offs = [b["off"] for b in blocks]
    x = torch.from_numpy(random_vector(size, 100)).cuda()
    ref = [np.array(s["values"]) for s in case["samples"]]
    scale = max(np.abs(r).max() for r in ref)
    for prec, ns, tol in ((0, 0, 1e-12), (1, 5, 1e-10)):
        _say("  precision %d s=%d: building plan" % (prec, ns))
        plan = Plan(prob, precision=prec, n_slices=ns)
        st = plan.stats()
        _say("  plan: %.2f TFLOP per H.psi, %d chunks" % (st["flops"] / 1e12, st["n_chunks"]))
        y = plan.apply(x)
        torch.cuda.synchronize()
        yh = y.cpu().numpy()
        plan.free()
        del y
        err = max(np.abs(_gather(yh, offs, s) - r).max() for s, r in zip(case["samples"], ref)) / scale
        _say("  precision %d: max sampled error %.3e (relative to %.3e)" % (prec, err, scale))
        assert err <= tol, (prec, err)
