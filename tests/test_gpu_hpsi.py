"""GPU parity of dmrg_apply_H / dmrg_diag_H (FP64 path) against the oracle."""
import sys

import numpy as np
import pytest

from paper_2309_16724_amd.synth.problem import exact_problem, random_problem

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


def _gpu_apply(torch, prob, x, **kw):
    from paper_2309_16724_amd.hpsi import Plan
    plan = Plan(prob, **kw)
    y = plan.apply(torch.from_numpy(x).to("cuda:0"))
    torch.cuda.synchronize()
    out = y.cpu().numpy()
    plan.free()
    return out


CASES = [("exact", (6, 6, 0, 3), dict(p=p)) for p in (0, 2, 4)] + [
    ("exact", (2, 2, 0, 3), dict(p=0)),
    ("exact", (6, 5, 1, 3), dict(p=1)),
    ("exact", (8, 8, 0, 0), dict()),
    ("exact", (8, 8, 0, 0), dict(max_mult=32)),
    ("exact", (8, 8, 2, 0), dict()),
    ("random", (6, 6, 0, 7), dict(D=240, cap=False)),     # sectors up to ~70: ragged tiles
    ("random", (7, 7, 1, 8), dict(D=300, cap=False)),
]


@pytest.mark.parametrize("kind,args,kw", CASES)
def test_apply_matches_oracle(torch, kind, args, kw):
    from oracle.hpsi import HEff
    _say("case %s %s %s" % (kind, args, kw))
    prob = exact_problem(*args, **kw) if kind == "exact" else random_problem(*args, **kw)
    he = HEff(prob)
    x = np.random.default_rng(3).standard_normal(he.size)
    ref = he.apply(x)
    y = _gpu_apply(torch, prob, x)
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()


def test_diag_matches_oracle(torch):
    from oracle.hpsi import HEff
    from paper_2309_16724_amd.hpsi import Plan
    for prob in (exact_problem(6, 6, 0, 3), random_problem(6, 6, 0, 9, D=120, cap=False)):
        _say("diag %s" % (prob.left.sectors[:3],))
        he = HEff(prob)
        n = he.size
        idx = np.arange(n) if n <= 400 else np.random.default_rng(0).choice(n, 300, replace=False)
        E = np.zeros((n, len(idx)))
        E[idx, np.arange(len(idx))] = 1.0
        ref = np.einsum("ij,ij->j", E, he.apply(E))
        plan = Plan(prob)
        d = plan.diag().cpu().numpy()
        plan.free()
        assert np.abs(d[idx] - ref).max() <= 1e-12 * np.abs(ref).max()


def test_full_size_hermitian_and_deterministic(torch):
    """L=24, D=512 synthetic blocks: symmetric H_eff and bitwise reproducible H.psi."""
    from paper_2309_16724_amd.hpsi import Plan
    _say("full size L=24 D=512")
    prob = random_problem(24, 24, 0, 1, D=512)
    plan = Plan(prob)
    n = plan.size
    rng = np.random.default_rng(5)
    a = torch.from_numpy(rng.standard_normal(n)).cuda()
    b = torch.from_numpy(rng.standard_normal(n)).cuda()
    ha, hb = plan.apply(a), plan.apply(b)
    hb2 = plan.apply(b)
    torch.cuda.synchronize()
    lhs, rhs = float(a @ hb), float(ha @ b)
    scale = float(ha.norm() * b.norm())
    assert abs(lhs - rhs) <= 1e-12 * scale
    assert torch.equal(hb, hb2)
    plan.free()


def test_full_size_matches_host_task_loops(torch):
    """GPU grouping and kernels equal plain loops over the same task list."""
    from paper_2309_16724_amd import binding as B
    _say("full size vs host loops L=16 D=256")
    prob = random_problem(16, 16, 0, 2, D=256)
    x = np.random.default_rng(6).standard_normal(_psi_len(prob))
    y_host, _ = B.debug_host_apply(prob, x)
    y = _gpu_apply(torch, prob, x)
    assert np.abs(y - y_host).max() <= 1e-12 * np.abs(y_host).max()


def _psi_len(prob):
    from oracle.layout import psi_blocks
    return psi_blocks(prob.left.sectors, prob.right.sectors, prob.n_elec, prob.two_s)[1]


def test_workspace_chunking_same_result(torch):
    """A small workspace cap splits the stripes into several launches."""
    from paper_2309_16724_amd.hpsi import Plan
    prob = random_problem(8, 8, 0, 4, D=160, cap=False)
    x = np.random.default_rng(1).standard_normal(_psi_len(prob))
    p1 = Plan(prob)
    p2 = Plan(prob, workspace_bytes=1 << 18)
    assert p2.stats()["n_chunks"] > 1
    xt = torch.from_numpy(x).cuda()
    y1, y2 = p1.apply(xt), p2.apply(xt)
    torch.cuda.synchronize()
    assert float((y1 - y2).abs().max()) <= 1e-12 * float(y1.abs().max())
    p1.free()
    p2.free()


def test_full_size_matches_oracle(torch):
    """L=24, D=512 (the benchmark workload): every element against the oracle."""
    from oracle.hpsi import HEff
    _say("full size L=24 D=512 vs oracle (about 80 s of CPU)")
    prob = random_problem(24, 24, 0, 1, D=512)
    he = HEff(prob)
    x = np.random.default_rng(12).standard_normal(he.size)
    y = _gpu_apply(torch, prob, x)
    _say("gpu done; oracle running")
    ref = he.apply(x)
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()
