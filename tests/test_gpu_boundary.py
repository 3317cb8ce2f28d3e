"""The C ABI's ownership contract on the GPU: plan, autotuner and solver
memory through caller callbacks (PyTorch's caching allocator), and the
autotuner's on-disk cache across processes."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2309_16724_amd.synth.problem import random_problem, random_vector

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


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
def test_caller_allocator_gets_every_allocation(torch, prec, ns):
    """Every device allocation of the plan (build, autotuning, Davidson)
    goes through the callbacks and is returned; results are bitwise equal to
    a plan on hipMalloc memory."""
    from paper_2309_16724_amd.hpsi import Plan, TorchAllocator
    from paper_2309_16724_amd.binding import DMRG_PLAN_AUTOTUNE
    prob = random_problem(10, 10, 0, 21, D=120)
    alloc = TorchAllocator("cuda:0")
    p_ref = Plan(prob, precision=prec, n_slices=ns)
    p_cb = Plan(prob, precision=prec, n_slices=ns, allocator=alloc, flags=DMRG_PLAN_AUTOTUNE)
    st = p_cb.stats()
    _say("callbacks: %d allocations, %d bytes; plan holds %d bytes, tuned %d"
         % (alloc.calls, alloc.bytes, st["device_bytes"], st["tuned"]))
    assert alloc.calls > 0 and st["device_bytes"] > 0 and st["tuned"] > 0
    assert sum(alloc.live.values()) == st["device_bytes"]
    x = torch.from_numpy(random_vector(p_ref.size, 5)).cuda()
    # the tuned settings may differ from the defaults: compare with a plan of the same settings
    p_same = Plan(prob, precision=prec, n_slices=ns, kpart=st["kpart"], tile_policy=st["tile_policy"],
                  macro_min=st["macro_min"] if st["macro_min"] > 0 else -1,
                  wide_min=st["wide_min"] if st["wide_min"] > 0 else -1,
                  workspace_bytes=st["workspace_cap"])
    y_cb, y_same = p_cb.apply(x), p_same.apply(x)
    torch.cuda.synchronize()
    assert torch.equal(y_cb, y_same)
    n_before = alloc.calls
    e1, _, s1 = p_cb.davidson(x, check=False)
    e2, _, s2 = p_same.davidson(x, check=False)
    assert alloc.calls > n_before            # the solver's basis came from the callbacks too
    assert e1 == e2 and s1["iters"] == s2["iters"]
    assert sum(alloc.live.values()) == p_cb.stats()["device_bytes"]   # solver memory returned
    for p in (p_ref, p_cb, p_same):
        p.free()
    assert not alloc.live and alloc.frees == alloc.calls


CHILD = r"""
import json, sys
sys.path.insert(0, %r)
from paper_2309_16724_amd.hpsi import Plan
from paper_2309_16724_amd.binding import DMRG_PLAN_AUTOTUNE
from paper_2309_16724_amd.synth.problem import random_problem
plan = Plan(random_problem(10, 10, 0, 22, D=150), precision=1, n_slices=5, flags=DMRG_PLAN_AUTOTUNE,
            tune_cache=%r)
st = plan.stats()
plan.free()
print(json.dumps({k: st[k] for k in ("tuned", "kpart", "tile_policy", "macro_min", "wide_min", "workspace_cap")}))
"""


def test_tune_cache_survives_a_process_restart(torch, tmp_path):
    """A tuned choice written to the cache file by one process is read back
    by the next (no timing there: stats.tuned == -1) with the same settings."""
    path = tmp_path / "tune.txt"
    outs = []
    for k in range(2):
        r = subprocess.run([sys.executable, "-c", CHILD % (ROOT, str(path))], capture_output=True, text=True,
                           timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        outs.append(json.loads(r.stdout.strip().splitlines()[-1]))
        _say("process %d: %s" % (k, outs[-1]))
    assert outs[0]["tuned"] > 0 and outs[1]["tuned"] == -1
    for key in ("kpart", "tile_policy", "macro_min", "wide_min", "workspace_cap"):
        assert outs[0][key] == outs[1][key]
    assert len(path.read_text().strip().splitlines()) == 1
