"""Captured launch graphs, the autotuner and the XCD-aware tile mapping.

Every tile is computed by one wavefront in a fixed order, so a graph replay,
a different work-group-to-tile mapping or a Davidson run on a graph plan must
reproduce the eager results bit for bit; autotuned settings change the
split-K grouping (summation order) and are checked against the oracle."""
import sys

import numpy as np
import pytest

from paper_2309_16724_amd import binding as B
from paper_2309_16724_amd.synth.problem import exact_problem, random_problem, random_vector

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


def _apply(torch, plan, x):
    y = plan.apply(x)
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.mark.parametrize("precision,ns", [(0, 0), (1, 5)])
def test_graph_replays_match_eager(torch, precision, ns):
    from paper_2309_16724_amd.hpsi import Plan
    prob = random_problem(7, 7, 1, 8, D=150, cap=False)
    eager = Plan(prob, precision=precision, n_slices=ns)
    graph = Plan(prob, precision=precision, n_slices=ns, flags=B.DMRG_PLAN_GRAPH)
    xs = [torch.from_numpy(random_vector(eager.size, s)).cuda() for s in (1, 2)]
    refs = [_apply(torch, eager, x) for x in xs]
    ys = [torch.empty_like(x) for x in xs]
    for rep in range(4):
        for k in (0, 1):
            graph.apply(xs[k], ys[k])
            junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64).sum()   # eager work between
            eager.apply(xs[1 - k])
            torch.cuda.synchronize()
            assert np.array_equal(ys[k].cpu().numpy(), refs[k]), (rep, k)
            ys[k].fill_(float("nan"))
    del junk
    eager.free()
    graph.free()


def test_xcd_mapping_does_not_change_results(torch):
    from paper_2309_16724_amd.hpsi import Plan
    prob = random_problem(8, 8, 0, 4, D=120, cap=False)
    a = Plan(prob, flags=B.DMRG_PLAN_XCD)
    b = Plan(prob)
    x = torch.from_numpy(random_vector(a.size, 3)).cuda()
    assert a.stats()["xcd"] == 1 and b.stats()["xcd"] == 0
    assert np.array_equal(_apply(torch, a, x), _apply(torch, b, x))
    a.free()
    b.free()


def test_autotuned_plan_matches_oracle_and_is_cached(torch):
    from oracle.hpsi import HEff
    from paper_2309_16724_amd.hpsi import Plan
    prob = random_problem(7, 7, 1, 9, D=150, cap=False)
    he = HEff(prob)
    x = np.random.default_rng(4).standard_normal(he.size)
    ref = he.apply(x)
    for precision, ns, tol in ((0, 0, 1e-12), (1, 5, 1e-10)):
        p1 = Plan(prob, precision=precision, n_slices=ns, flags=B.DMRG_PLAN_AUTOTUNE)
        s1 = p1.stats()
        _say("autotune prec %d: tuned %d kpart %d policy %d cap %d (%.0f ms)"
             % (precision, s1["tuned"], s1["kpart"], s1["tile_policy"], s1["workspace_cap"], s1["tune_ms"]))
        assert s1["tuned"] >= 7
        y = _apply(torch, p1, torch.from_numpy(x).cuda())
        assert np.abs(y - ref).max() <= tol * np.abs(ref).max()
        p2 = Plan(prob, precision=precision, n_slices=ns, flags=B.DMRG_PLAN_AUTOTUNE)
        s2 = p2.stats()
        assert s2["tuned"] == 0
        assert (s2["kpart"], s2["tile_policy"], s2["workspace_cap"]) == \
            (s1["kpart"], s1["tile_policy"], s1["workspace_cap"])
        p1.free()
        p2.free()


def test_davidson_on_graph_plan_is_identical(torch):
    from paper_2309_16724_amd.hpsi import Plan
    prob = exact_problem(8, 8, 0, 0, max_mult=32)
    a = Plan(prob)
    b = Plan(prob, flags=B.DMRG_PLAN_GRAPH)
    x0 = torch.from_numpy(random_vector(a.size, 100)).cuda()
    ea, pa, sa = a.davidson(x0, m_max=8)
    eb, pb, sb = b.davidson(x0, m_max=8)
    assert sa["iters"] == sb["iters"] and ea == eb
    assert np.array_equal(pa.cpu().numpy(), pb.cpu().numpy())
    a.free()
    b.free()


def test_full_size_autotuned_matches_default(torch):
    """L=24, D=512 with every tuning flag against the default plan (which the
    FP64 parity tests check against the oracle)."""
    from paper_2309_16724_amd.hpsi import Plan
    prob = random_problem(24, 24, 0, 1, D=512)
    base = Plan(prob)
    x = torch.from_numpy(random_vector(base.size, 7)).cuda()
    y0 = _apply(torch, base, x)
    base.free()
    tuned = Plan(prob, flags=B.DMRG_PLAN_AUTOTUNE | B.DMRG_PLAN_GRAPH)
    st = tuned.stats()
    _say("L24 autotune: kpart %d policy %d cap %d, %d candidates in %.0f ms"
         % (st["kpart"], st["tile_policy"], st["workspace_cap"], st["tuned"], st["tune_ms"]))
    y1 = _apply(torch, tuned, x)
    y2 = _apply(torch, tuned, x)
    tuned.free()
    assert np.array_equal(y1, y2)
    assert np.abs(y1 - y0).max() <= 1e-13 * np.abs(y0).max()
