"""Batched plans: many independent two-site problems of uneven size in one
plan (one concatenated psi, one tile list).  Every segment is checked
against the oracle on its own problem, and batched Davidson against dense
diagonalisation and against single-problem solves."""
import sys

import numpy as np
import pytest

from paper_2309_16724_amd.synth.problem import (batch_problems, exact_problem, random_problem,
                                                random_vector)

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


def _mixed():
    return [exact_problem(6, 6, 0, 3, p=2),
            random_problem(6, 6, 0, 5, D=60),
            exact_problem(5, 5, 1, 1),
            random_problem(8, 8, 0, 9, D=40),
            random_problem(12, 12, 0, 11, D=64),
            random_problem(7, 7, 1, 8, D=100, cap=False)]


def _segments(plan, n):
    return [plan.layout(k) for k in range(n)]


@pytest.fixture(scope="module")
def mixed_ref():
    from oracle.hpsi import HEff
    probs = _mixed()
    hes = [HEff(p) for p in probs]
    xs = [np.random.default_rng(40 + k).standard_normal(h.size) for k, h in enumerate(hes)]
    refs = [h.apply(x) for h, x in zip(hes, xs)]
    return probs, xs, refs


def _batched_apply(torch, probs, xs, **kw):
    from paper_2309_16724_amd.hpsi import Plan
    plan = Plan(probs, **kw)
    segs = _segments(plan, len(probs))
    x = np.zeros(plan.size)
    for (off, ln), xk in zip(segs, xs):
        assert ln == xk.size
        x[off:off + ln] = xk
    y = plan.apply(torch.from_numpy(x).cuda()).cpu().numpy()
    plan.free()
    return [y[off:off + ln] for off, ln in segs]


def test_batch_layout_is_concatenation(torch):
    from paper_2309_16724_amd.hpsi import Plan
    probs = _mixed()
    plan = Plan(probs)
    segs = _segments(plan, len(probs))
    off = 0
    for s in segs:
        assert s[0] == off
        off += s[1]
    assert off == plan.size
    plan.free()


def test_batch_apply_matches_oracle(torch, mixed_ref):
    probs, xs, refs = mixed_ref
    _say("batched FP64 apply, %d problems" % len(probs))
    ys = _batched_apply(torch, probs, xs)
    for k, (y, ref) in enumerate(zip(ys, refs)):
        err = np.abs(y - ref).max() / np.abs(ref).max()
        _say("  problem %d size %d rel err %.2e" % (k, ref.size, err))
        assert err <= 1e-12


def test_batch_apply_equals_single_plans(torch, mixed_ref):
    probs, xs, _ = mixed_ref
    ys = _batched_apply(torch, probs, xs)
    for k in range(len(probs)):
        yk = _batched_apply(torch, [probs[k]], [xs[k]])[0]
        assert np.abs(ys[k] - yk).max() <= 1e-13 * np.abs(yk).max()


@pytest.mark.parametrize("ns", [4, 5])
def test_batch_split_matches_oracle(torch, mixed_ref, ns):
    from paper_2309_16724_amd.binding import DMRG_SPLIT_BF16
    probs, xs, refs = mixed_ref
    _say("batched split s=%d" % ns)
    bound = {4: 5e-9, 5: 1e-10}[ns]
    ys = _batched_apply(torch, probs, xs, precision=DMRG_SPLIT_BF16, n_slices=ns)
    for k, (y, ref) in enumerate(zip(ys, refs)):
        err = np.abs(y - ref).max() / np.abs(ref).max()
        _say("  problem %d rel err %.2e" % (k, err))
        assert err <= bound


def test_batch_davidson_matches_dense(torch):
    from oracle.hpsi import HEff
    from paper_2309_16724_amd.hpsi import Plan
    probs = _mixed()[:4]
    _say("batched Davidson vs dense, %d problems" % len(probs))
    plan = Plan(probs)
    x0 = torch.from_numpy(random_vector(plan.size, 100)).cuda()
    es, psi, st = plan.davidson(x0, m_max=12)
    psi = psi.cpu().numpy()
    segs = _segments(plan, len(probs))
    plan.free()
    assert st["converged"] == len(probs) and st["residual"] <= 1e-8
    for k, pr in enumerate(probs):
        w, v = np.linalg.eigh(HEff(pr).dense())
        off, ln = segs[k]
        assert abs(es[k] - w[0]) < 1e-8
        assert abs(abs(psi[off:off + ln] @ v[:, 0]) - 1.0) < 1e-8


def test_batch_davidson_uneven_matches_single(torch):
    from oracle.hpsi import HEff
    from paper_2309_16724_amd.hpsi import Plan
    probs = batch_problems(6, 7, L_range=(8, 12), D_range=(32, 96))
    _say("batched Davidson, uneven batch of %d" % len(probs))
    plan = Plan(probs)
    x0 = random_vector(plan.size, 100)
    es, psi, st = plan.davidson(torch.from_numpy(x0).cuda())
    psi = psi.cpu().numpy()
    segs = _segments(plan, len(probs))
    plan.free()
    assert st["converged"] == len(probs)
    for k, pr in enumerate(probs):
        off, ln = segs[k]
        single = Plan(pr)
        e1, _, st1 = single.davidson(torch.from_numpy(x0[off:off + ln].copy()).cuda())
        single.free()
        _say("  problem %d: batched %.12f single %.12f (%d its)" % (k, es[k], e1, st1["iters"]))
        assert abs(es[k] - e1) < 1e-8
        u = psi[off:off + ln]
        r = HEff(pr).apply(u) - es[k] * u
        assert np.linalg.norm(r) < 1e-7
