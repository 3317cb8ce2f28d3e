"""GPU kernels of the learned Davidson preconditioner against the FP64 oracle
(forward, loss gradient, Adam, training rows), the guard, and the gain of a
trained network over the diagonal preconditioner.

Tolerances: the device stores activations and parameters in FP32 and
accumulates layer 2 over 256 terms in FP32 (relative error up to about
256 * 2^-24 = 1.5e-5 per output in the worst case, ~1e-6 typically); the
backward reductions accumulate in FP64.  Outputs and learned steps are
compared norm-wise at 2e-5 / 1e-5 relative, loss and gradients at 1e-6
relative (measured 4e-8 to 3e-7)."""
import sys

import numpy as np
import pytest

from oracle import mlp as omlp
from paper_2309_16724_amd.synth.mlp_inputs import mlp_batch, mlp_params
from paper_2309_16724_amd.synth.problem import exact_problem, random_problem, random_vector

pytestmark = pytest.mark.gpu
W = 256


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    return t


def _net(p):
    from paper_2309_16724_amd.precond import MLP
    net = MLP(W, seed=0)
    net.set_params(p)
    return net


def _cuda(torch, *arrs):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


def test_forward_matches_oracle(torch):
    p = mlp_params(2, W, 1)
    x, _, _ = mlp_batch(3001, 2, 2)          # ragged: 3001 = 46 blocks of 64 + 57
    net = _net(p)
    g = net.forward(*_cuda(torch, x)).cpu().numpy()
    ref, _ = omlp.forward(p.astype(np.float64), x, W)
    err = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    _say("forward rel err %.2e" % err)
    assert err <= 2e-5
    net.free()


@pytest.mark.parametrize("n", [1, 4096, 5000])
def test_loss_gradient_matches_oracle(torch, n):
    p = mlp_params(2, W, 3)
    x, a, b = mlp_batch(n, 2, 4)
    net = _net(p)
    loss, gr = net.loss_grad(*_cuda(torch, x, a, b))
    gr = gr.cpu().numpy()
    lref, gref = omlp.grad(p.astype(np.float64), x, a, b, W)
    err = np.linalg.norm(gr - gref) / np.linalg.norm(gref)
    _say("n=%d loss %.6e (oracle %.6e) grad rel err %.2e" % (n, loss, lref, err))
    assert abs(loss - lref) <= 1e-6 * lref
    assert err <= 1e-6
    net.free()


def test_adam_steps_match_oracle(torch):
    p = mlp_params(2, W, 5)
    rng = np.random.default_rng(6)
    g1 = rng.standard_normal(p.size).astype(np.float32)
    g2 = rng.standard_normal(p.size).astype(np.float32)
    net = _net(p)
    for g in (g1, g2):
        net.adam_step(*_cuda(torch, g), lr=1e-3)
    got = net.get_params()
    q, m, v = p.astype(np.float64), np.zeros(p.size), np.zeros(p.size)
    for t, g in enumerate((g1, g2), start=1):
        q, m, v = omlp.adam_step(q, m, v, g.astype(np.float64), t, 1e-3)
    assert np.abs(got - q).max() <= 1e-6 * np.abs(q).max()
    net.free()


def test_training_lowers_loss_and_is_deterministic(torch):
    x, a, b = _cuda(torch, *mlp_batch(20000, 2, 7))
    p0 = mlp_params(2, W, 8)
    outs = []
    for _ in range(2):
        net = _net(p0)
        tr = net.train(x, a, b, steps=300, batch=1024, lr=1e-3, seed=9, trace=True)
        outs.append(net.get_params())
        net.free()
    _say("loss %.4f -> %.4f" % (tr[:20].mean(), tr[-20:].mean()))
    assert tr[-20:].mean() < 0.5 * tr[:20].mean()
    assert np.array_equal(outs[0], outs[1])


def _dav_gpu(torch, prob, mlp=None, **kw):
    from paper_2309_16724_amd.hpsi import Plan
    plan = Plan(prob)
    x0 = torch.from_numpy(random_vector(plan.size, 100)).cuda()
    e, psi, st = plan.davidson(x0, mlp=mlp, **kw)
    plan.free()
    return e, psi.cpu().numpy(), st


def test_collect_rows_match_oracle(torch):
    """First recorded iterations of the device capture against rows built
    by the oracle from its own Davidson run on the same start vector."""
    from oracle.davidson import davidson
    from oracle.hpsi import HEff
    from paper_2309_16724_amd.hpsi import Plan
    prob = random_problem(6, 6, 0, 5, D=60)
    H = HEff(prob).dense()
    d = np.diag(H).copy()
    x0 = random_vector(len(H), 100)
    rec = []
    th, psi, it, rn, _ = davidson(lambda v: H @ v, d, x0, record=rec)
    rows = [omlp.training_rows(d, r, u, t, psi) for r, u, t in rec if abs(u @ psi) >= 1e-3]
    plan = Plan(prob)
    x, a, b, nrec = plan.collect(torch.from_numpy(x0).cuda(), capacity=len(H) * 200)
    plan.free()
    x, a, b = x.cpu().numpy(), a.cpu().numpy(), b.cpu().numpy()
    n = len(H)
    _say("records: device %d oracle %d" % (nrec, len(rows)))
    assert x.shape[0] == nrec * n
    assert abs(nrec - len(rows)) <= 2
    for k in range(3):
        xr, ar, br = rows[k]
        sl = slice(k * n, (k + 1) * n)
        # a Ritz vector's sign is arbitrary: u -> -u flips r, td and t* together
        sg = np.sign(a[sl] @ ar)
        assert np.abs(x[sl] - xr).max() <= 1e-5 * max(1.0, np.abs(xr).max())
        assert np.linalg.norm(sg * a[sl] - ar) <= 1e-5 * np.linalg.norm(ar)
        assert np.linalg.norm(sg * b[sl] - br) <= 1e-5 * np.linalg.norm(br)


def test_zero_network_reproduces_diagonal_davidson(torch):
    from paper_2309_16724_amd.precond import MLP
    prob = random_problem(8, 8, 0, 9, D=40)
    net = MLP(W, seed=0)
    net.set_params(np.zeros(net.n_params, dtype=np.float32))
    e0, p0, s0 = _dav_gpu(torch, prob)
    e1, p1, s1 = _dav_gpu(torch, prob, mlp=net)
    assert s1["iters"] == s0["iters"] and s1["fallbacks"] == 0
    assert e1 == e0 and np.array_equal(p0, p1)
    net.free()


def test_guard_falls_back_on_corrupted_weights(torch):
    """Weights large enough to overflow FP32 make every learned step
    non-finite: each is rejected and the solve is the diagonal one."""
    from paper_2309_16724_amd.precond import MLP
    prob = random_problem(8, 8, 0, 9, D=40)
    net = MLP(W, seed=0)
    net.set_params(np.full(net.n_params, 3e38, dtype=np.float32))
    e0, p0, s0 = _dav_gpu(torch, prob)
    e1, p1, s1 = _dav_gpu(torch, prob, mlp=net)
    _say("iters %d fallbacks %d" % (s1["iters"], s1["fallbacks"]))
    assert s1["fallbacks"] == s1["iters"] - 1
    assert s1["iters"] == s0["iters"] and e1 == e0
    net.free()


def test_patience_switches_a_stalling_network_off(torch):
    """A network with large random weights gives finite steps that pass the
    guard yet need not help; with a short patience its learned steps are
    switched off and the solve still reaches the diagonal run's energy."""
    from paper_2309_16724_amd.precond import MLP
    prob = random_problem(8, 8, 0, 9, D=40)
    net = MLP(W, seed=0)
    net.set_params(mlp_params(2, W, 11, out_scale=10.0) * 3.0)
    e0, _, s0 = _dav_gpu(torch, prob)
    e1, _, s1 = _dav_gpu(torch, prob, mlp=net, mlp_patience=2)
    _say("diagonal %d its; stalling network %d its, switched %d, fallbacks %d"
         % (s0["iters"], s1["iters"], s1["switched"], s1["fallbacks"]))
    assert s0["switched"] == 0
    assert s1["converged"] == 1 and s1["switched"] == 1
    assert abs(e1 - e0) < 1e-8
    net.free()


TRAIN = [(8, 8, 0, s, 40, True) for s in (20, 21, 22, 23)] + [(7, 7, 1, s, 30, False) for s in (24, 25)]
HELD_OUT = [("random", (8, 8, 0, 9), dict(D=40)), ("random", (7, 7, 1, 6), dict(D=30, cap=False)),
            ("exact", (8, 8, 0, 0), {}), ("random", (8, 8, 0, 30), dict(D=40)),
            ("random", (9, 9, 1, 31), dict(D=40))]


def train_from_solves(torch, specs, steps=2000, batch=4096, seed=0):
    """Collect rows from the solves of `specs` and train a fresh network."""
    from paper_2309_16724_amd.hpsi import Plan
    from paper_2309_16724_amd.precond import MLP
    xs, as_, bs = [], [], []
    for L, N, s2, sd, D, cap in specs:
        plan = Plan(random_problem(L, N, s2, sd, D=D, cap=cap))
        x0 = torch.from_numpy(random_vector(plan.size, 100)).cuda()
        x, a, b, nrec = plan.collect(x0, capacity=plan.size * 400)
        plan.free()
        xs.append(x)
        as_.append(a)
        bs.append(b)
    x, a, b = torch.cat(xs), torch.cat(as_), torch.cat(bs)
    net = MLP(W, seed=seed)
    tr = net.train(x, a, b, steps=steps, batch=batch, lr=1e-3, seed=seed + 1, trace=True)
    return net, x.shape[0], tr


def test_trained_network_needs_fewer_iterations(torch):
    net, nrows, tr = train_from_solves(torch, TRAIN)
    _say("trained on %d rows, loss %.4f -> %.4f" % (nrows, tr[:50].mean(), tr[-50:].mean()))
    tot = [0, 0]
    for kind, args, kw in HELD_OUT:
        prob = exact_problem(*args, **kw) if kind == "exact" else random_problem(*args, **kw)
        e0, _, s0 = _dav_gpu(torch, prob)
        e1, _, s1 = _dav_gpu(torch, prob, mlp=net)
        _say("  %s %s: diagonal %d its, learned %d its (%d fallbacks), dE %.1e"
             % (args, kw, s0["iters"], s1["iters"], s1["fallbacks"], e1 - e0))
        assert s0["converged"] == 1 and s1["converged"] == 1
        assert abs(e1 - e0) < 1e-8
        tot[0] += s0["iters"]
        tot[1] += s1["iters"]
    _say("total iterations: diagonal %d, learned %d" % tuple(tot))
    assert tot[1] < tot[0]
    net.free()


def test_learned_step_matches_oracle(torch):
    """The fused learned correction dmrg_davidson applies (features from
    diag, theta, sigma and the residual norm; t = td (1 + g); relative floor)
    against oracle.mlp.mlp_step, per segment of a two-segment vector with
    ragged lengths and elements inside the floor."""
    p = mlp_params(2, W, 7)
    net = _net(p)
    rng = np.random.default_rng(8)
    lens = [3001, 1777]
    d, r, th, sg, rn, ref = [], [], [], [], [], []
    for k, n in enumerate(lens):
        dk = rng.uniform(-2.0, 6.0, n)
        tk = float(dk.min() + 0.3 * k)            # theta inside the diagonal's range for segment 1
        dk[:5] = tk + np.array([0.0, 1e-9, -1e-9, 1e-4, -1e-4])   # denominators below the floor
        rk = 1e-3 * rng.standard_normal(n)
        d.append(dk); r.append(rk); th.append(tk)
        sg.append(float(np.sqrt(np.mean((dk - tk) ** 2))))
        rn.append(float(np.linalg.norm(rk)))
        ref.append(omlp.mlp_step(p.astype(np.float64), W, dk, rk, tk))
    off = np.concatenate([[0], np.cumsum(lens)])
    t = net.step(*_cuda(torch, np.concatenate(d), np.concatenate(r)), off, th, sg, rn).cpu().numpy()
    for k in range(len(lens)):
        tk = t[off[k]:off[k + 1]]
        err = np.linalg.norm(tk - ref[k]) / np.linalg.norm(ref[k])
        _say("segment %d: learned step rel err %.2e" % (k, err))
        assert err <= 1e-5
    net.free()
