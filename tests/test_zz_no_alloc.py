"""dmrg_apply_H_static (no device allocation; static scratch array) against
dmrg_apply_H on the same plans: two calls in a row, the second with a
smaller problem, FP64 and split plans, and the size check."""
import sys

import numpy as np
import pytest

from paper_2309_16724_amd.synth.problem import random_problem, exact_problem

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    return t


@pytest.mark.parametrize("prec,ns", [(0, 0), (1, 5)])
def test_static_entry_matches_apply(torch, prec, ns):
    from paper_2309_16724_amd.hpsi import Plan
    probs = [random_problem(16, 16, 0, 3, D=300), exact_problem(6, 6, 0, 3, p=2)]   # larger, then smaller
    for k, prob in enumerate(probs):
        # a workspace cap that fits the static array (the stripes are cut into chunks)
        plan = Plan(prob, precision=prec, n_slices=ns, workspace_bytes=32 << 20)
        st = plan.stats()
        _say("call %d: precision %d, psi_len %d, %d chunks" % (k, prec, st["psi_len"], st["n_chunks"]))
        x = torch.from_numpy(np.random.default_rng(10 + k).standard_normal(plan.size)).cuda()
        y_ref = plan.apply(x)
        y = torch.full_like(x, float("nan"))
        plan.apply_static(x, y)
        torch.cuda.synchronize()
        a, b = y_ref.cpu().numpy(), y.cpu().numpy()
        plan.free()
        assert np.all(np.isfinite(b))
        err = np.abs(a - b).max() / np.abs(a).max()
        _say("  static vs apply: %.3e" % err)
        assert err <= 1e-13


def test_static_entry_rejects_oversized_plans(torch):
    from paper_2309_16724_amd.hpsi import Plan
    prob = random_problem(16, 16, 0, 3, D=300)
    plan = Plan(prob, workspace_bytes=1 << 30)            # one chunk: stripes beyond the array
    x = torch.zeros(plan.size, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(RuntimeError, match="scratch"):
        plan.apply_static(x, y)
    plan.free()
