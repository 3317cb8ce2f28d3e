"""Benchmark of the SU(2) two-site H.psi hot path on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

One step = one H_eff psi over the whole wavefunction of the workload (all
operator-table rows, all sector tasks, both stripe stages).  Inputs are
seeded synthetic blocks already resident in HBM when timing starts.  Prints
one JSON line with the throughput in algorithmic TFLOP/s, the roofline of
the dominant kernel (per-launch HIP events on the library's stream) and the
CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # L orbitals, N electrons, 2S, integral seed, SU(2) bond dimension D per
    # block, and the sector allocation of the synthetic blocks (spin_ratio,
    # sigma_frac: see synth.problem.synthetic_sectors)
    "L24_D512": dict(n_orb=24, n_elec=24, two_s=0, seed=1, D=512),
    # sector dims 1..894 per block (R_D = 1.80), 30 TFLOP per H.psi: the
    # complexity of one middle-bond H.psi of the paper's CAS(54,54), D=2048 runs
    "L54_D2048": dict(n_orb=54, n_elec=54, two_s=0, seed=2, D=2048, spin_ratio=0.45, sigma_frac=0.03),
    "L64_D3072": dict(n_orb=64, n_elec=64, two_s=0, seed=4, D=3072),
}
# the learned preconditioner's evaluation workload (L=64, D=3072) keeps the
# flatter sector allocation (dims 1..206): its Davidson solves take hundreds
# of H.psi steps
GEN_KEYS = ("D", "spin_ratio", "sigma_frac")


def make_problem(w, all_pairs=False):
    """The workload's problem; all_pairs: its left block holds P and Q for
    every outside pair (the form a renormalization of every family needs;
    the other families are the same draws)."""
    from paper_2309_16724_amd.synth.problem import random_problem
    return random_problem(w["n_orb"], w["n_elec"], w["two_s"], w["seed"],
                          **{k: w[k] for k in GEN_KEYS if k in w}, all_pairs=all_pairs)


FP64_PEAK_TFLOPS = 78.6       # MI355X dense FP64 (matrix and vector)
BF16_PEAK_TFLOPS = 2516.6     # MI355X dense BF16 MFMA


def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "usable_cpus": usable}


def _oracle_rate(prob, flops_full, threads, budget_s):
    """Oracle H_eff psi on the whole wavefunction with `threads` BLAS threads:
    in full when a probe predicts at most budget_s, else on every k-th of its
    merged terms (scaled by the term count).  Returns (seconds for one full
    H.psi, description, process-time / wall-time)."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle.hpsi import HEff
    with threadpool_limits(limits=threads):
        he = HEff(prob)
        terms = he.compiled()
        x = np.random.default_rng(100).standard_normal(he.size)
        u1 = he.expand(x)
        probe = terms[::50]
        t0 = time.time()
        he._compiled = probe
        he.apply_u1(u1)
        est_full = max(time.time() - t0, 1e-3) * len(terms) / max(len(probe), 1)
        k = 1 if est_full <= budget_s else max(2, int(round(est_full / (0.5 * budget_s))))
        sample = terms[::k]
        he._compiled = sample
        t0, c0 = time.time(), time.process_time()
        he.apply_u1(u1)
        wall = time.time() - t0
        cpu = time.process_time() - c0
    t_full = wall * len(terms) / len(sample)
    if k == 1:
        desc = "full oracle H_eff psi (all %d merged terms, %.1f s wall)" % (len(terms), wall)
    else:
        desc = ("oracle H_eff psi over the full wavefunction restricted to every %d-th of its %d merged "
                "terms (%.1f s wall), scaled by %d/%d to one full H.psi (%.1f s)"
                % (k, len(terms), wall, len(terms), len(sample), t_full))
    return t_full, desc, cpu / max(wall, 1e-9)


def cpu_baseline(flops_bench, bench_workload):
    """The oracle timed on this host's cores (test infrastructure, never on
    the product path).  The M-resolved oracle cannot hold the metric's L=54
    workload (its expanded operators alone would need terabytes), so it is
    timed on the L=24, D=512 workload: in full with all usable cores, and on a
    term sample with one thread; value = that workload's algorithmic flops per
    oracle second."""
    from paper_2309_16724_amd import binding as B
    info = cpu_info()
    w = WORKLOADS["L24_D512"]
    prob = make_problem(w)
    _, st = B.debug_plan_host_apply(prob, None)
    flops = st["flops"]
    cores = info["usable_cpus"] or 1
    t_all, desc_all, par = _oracle_rate(prob, flops, cores, 60.0)
    t_one, desc_one, _ = _oracle_rate(prob, flops, 1, 12.0)
    return {
        "value": flops / t_all / 1e12,
        "unit": "TFLOP/s",
        "cores": cores,
        "kind": "oracle",
        "sample": "L24_D512 (L=24, D=512, %.1f GFLOP per H.psi): %s with %d BLAS threads "
                  "(process/wall time %.1f); the bench workload %s (%.1f TFLOP per H.psi) is beyond the "
                  "oracle's host memory" % (flops / 1e9, desc_all, cores, par, bench_workload,
                                            flops_bench / 1e12),
        "single_thread": {"value": flops / t_one / 1e12, "unit": "TFLOP/s", "sample": desc_one},
        **info,
    }


# HBM bytes per launch of the stage kernels at L54_D2048 from the FETCH_SIZE
# and WRITE_SIZE runs summarised in profiles/hpsi_L54_D2048_split5.md and
# profiles/hpsi_L54_D2048_fp64.md: FETCH scaled by 2.000 and WRITE by 1.000,
# what the same counters read for a plain 256 MiB device copy in the same
# runs.  A figure holds only while the sources that decide the kernel's memory
# traffic are the ones it was taken on (their hash); else null.
_SPLIT_SRC = ("kernels_split.hip", "plan.cpp", "plan.hpp", "model.cpp")
_F64_SRC = ("kernels_f64.hip", "plan.cpp", "plan.hpp", "model.cpp")
_REN_SRC = ("renorm.cpp", "kernels_f64.hip")
MEASURED_TRAFFIC = {
    ("L54_D2048", "stage1_wsplit5_kernel"): (1.6826e11, _SPLIT_SRC, "fd14f25f69d6d718"),
    ("L54_D2048", "stage2_wsplit5_kernel"): (2.2778e11, _SPLIT_SRC, "fd14f25f69d6d718"),
    ("L54_D2048", "stage_f64_kernel<1>"): (3.5086e11, _F64_SRC, "69c8d5cbc4f75ca9"),
    ("L54_D2048", "stage_f64_kernel<2>"): (1.0639e12, _F64_SRC, "69c8d5cbc4f75ca9"),
    # renormalization of the L54_D2048 left block (profiles/renorm_left_L54_D2048_fp64.md)
    ("L54_D2048", "renorm:stage_f64_kernel<1>"): (1.3855e11, _REN_SRC, "7150222daa7f2493"),
    ("L54_D2048", "renorm:stage_f64_kernel<2>"): (1.7818e11, _REN_SRC, "7150222daa7f2493"),
    # the right block through the right site (profiles/renorm_right_L54_D2048_fp64.md)
    ("L54_D2048", "renorm_right:stage_f64_kernel<1>"): (3.1297e11, _REN_SRC, "7150222daa7f2493"),
    ("L54_D2048", "renorm_right:stage_f64_kernel<2>"): (5.3775e11, _REN_SRC, "7150222daa7f2493"),
}


def measured_traffic(workload, kernel):
    entry = MEASURED_TRAFFIC.get((workload, kernel))
    if entry is None:
        return None
    nbytes, files, digest = entry
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2309_16724_amd", "csrc")
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return nbytes if h.hexdigest()[:16] == digest else None


def train_preconditioner(torch, specs, steps=2000, batch=4096, seed=0, width=256, floor=None):
    """Learned preconditioner: exact-correction rows of the given solves
    (device capture, with the relative floor the solves use), then minibatch
    Adam on the device."""
    import numpy as np
    from paper_2309_16724_amd.hpsi import Plan
    from paper_2309_16724_amd.precond import MLP
    from paper_2309_16724_amd.synth.problem import random_problem, random_vector
    t0 = time.time()
    xs, as_, bs, nrec = [], [], [], 0
    for L, N, s2, sd, D in specs:
        plan = Plan(random_problem(L, N, s2, sd, D=D))
        x0 = torch.from_numpy(random_vector(plan.size, 100)).cuda()
        x, a, b, nr = plan.collect(x0, capacity=plan.size * 500, **({} if floor is None else {"floor": floor}))
        plan.free()
        xs.append(x)
        as_.append(a)
        bs.append(b)
        nrec += nr
    x, a, b = torch.cat(xs), torch.cat(as_), torch.cat(bs)
    t1 = time.time()
    net = MLP(width, seed=seed)
    # the training objective on a fixed sample of 2^20 rows (minibatch losses
    # of heavy-tailed rows are too noisy to compare)
    g = torch.Generator(device="cpu").manual_seed(seed + 2)
    idx = torch.randint(0, x.shape[0], (1 << 20,), generator=g).to(x.device)
    xe, ae, be = x[idx].contiguous(), a[idx].contiguous(), b[idx].contiguous()
    loss0, _ = net.loss_grad(xe, ae, be)
    tr = net.train(x, a, b, steps=steps, batch=batch, lr=1e-3, seed=seed + 1, trace=True)
    loss1, _ = net.loss_grad(xe, ae, be)
    t2 = time.time()
    info = {"solves": len(specs), "records": nrec, "rows": int(x.shape[0]), "steps": steps,
            "batch": batch, "width": width, "collect_s": t1 - t0, "train_s": t2 - t1,
            "sample_loss_diagonal": float(((ae - be) ** 2).mean().item()),
            "sample_loss_before": float(loss0), "sample_loss_after": float(loss1),
            "minibatch_loss_deciles": [round(float(v.mean()), 4) for v in np.array_split(tr, 10)],
            "specs": [list(s_) for s_ in specs]}
    del xe, ae, be, idx
    del xs, as_, bs, x, a, b
    return net, info


def run_batch(args):
    """Batched uneven problems: one plan over many independent middle-bond
    problems, H.psi in FP64 and split-BF16 (s=5), autotuned."""
    import numpy as np
    import torch
    from paper_2309_16724_amd.binding import DMRG_PLAN_AUTOTUNE
    from paper_2309_16724_amd.hpsi import Plan
    from paper_2309_16724_amd.synth.problem import batch_specs, random_problem
    specs = batch_specs(args.batch, 3, seed0=1000)
    t0 = time.time()
    probs = [random_problem(L, N, s2, sd, D=D) for L, N, s2, sd, D in specs]
    print("# generated %d problems in %.1f s" % (len(probs), time.time() - t0), file=sys.stderr, flush=True)
    from paper_2309_16724_amd.binding import DMRG_PLAN_XCD
    res = {}
    ys = {}
    # the autotuner times candidates on a sample of four problems spread over
    # the batch's sizes (re-planning all 64 per candidate would cost minutes);
    # its choice of kpart, tile policy and XCD mapping is applied to the batch
    order = sorted(range(len(probs)), key=lambda k: specs[k][0] * specs[k][4] ** 2)
    sample = [order[int(round(q * (len(order) - 1)))] for q in (0.2, 0.45, 0.7, 0.95)]
    for name, prec, ns in (("fp64", 0, 0), ("split", 1, 5)):
        t1 = time.time()
        tuned = {"kpart": 0, "tile_policy": 0, "xcd": 0, "sample": None, "tune_ms": 0.0}
        if not args.no_autotune:
            tp = Plan([probs[k] for k in sample], precision=prec, n_slices=ns, flags=DMRG_PLAN_AUTOTUNE)
            ts = tp.stats()
            tp.free()
            tuned = {"kpart": ts["kpart"], "tile_policy": ts["tile_policy"], "xcd": ts["xcd"],
                     "sample": sample, "tune_ms": ts["tune_ms"]}
        plan = Plan(probs, precision=prec, n_slices=ns, kpart=tuned["kpart"], tile_policy=tuned["tile_policy"],
                    flags=DMRG_PLAN_XCD if tuned["xcd"] else 0)
        st = plan.stats()
        print("# batch plan %s built in %.1f s: %s" % (name, time.time() - t1, json.dumps(st)), file=sys.stderr,
              flush=True)
        x = torch.from_numpy(np.random.default_rng(100).standard_normal(plan.size)).cuda()
        y = torch.empty_like(x)
        for _ in range(args.warmup):
            plan.apply(x, y)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            plan.apply(x, y)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        segs = [plan.layout(k) for k in range(len(probs))]
        ys[name] = (y.cpu().numpy(), segs)
        res[name] = {"ms_per_step": ms, "tflops": st["flops"] / (ms * 1e-3) / 1e12, "flops": st["flops"],
                     "psi_len": st["psi_len"], "kpart": st["kpart"], "tile_policy": st["tile_policy"],
                     "xcd": st["xcd"], "workspace_cap": st["workspace_cap"], "autotune": tuned,
                     "n_chunks": st["n_chunks"]}
        plan.free()
    batch_dav = None
    if args.batch_davidson:
        # all problems solved together: one batched H.psi per iteration
        t1 = time.time()
        tn = res["fp64"]["autotune"]
        plan = Plan(probs, kpart=tn["kpart"], tile_policy=tn["tile_policy"], flags=DMRG_PLAN_XCD if tn["xcd"] else 0)
        from paper_2309_16724_amd.synth.problem import random_vector
        x0 = np.zeros(plan.size)
        for k in range(len(probs)):
            off, ln = plan.layout(k)
            x0[off:off + ln] = random_vector(ln, 100 + k)
        torch.cuda.synchronize()
        t2 = time.time()
        es, _, dst = plan.davidson(torch.from_numpy(x0).cuda(), tol=1e-8, check=False, verbose=1)
        t3 = time.time()
        plan.free()
        batch_dav = {"s_per_step": t3 - t2, "plan_build_s": t2 - t1, "iterations_max": dst["iters"],
                     "n_hpsi": dst["n_hpsi"], "converged": dst["converged"], "problems": len(probs),
                     "residual_max": dst["residual"], "t_hpsi_s": dst["t_hpsi_s"], "energies": es}
    yf, segs = ys["fp64"]
    yb, _ = ys["split"]
    errs = [float(np.abs(yb[o:o + n] - yf[o:o + n]).max() / np.abs(yf[o:o + n]).max()) for o, n in segs]
    out = {"metric": "batched H.psi TFLOP/s (split-BF16 s=5 and FP64)", "value": res["split"]["tflops"],
           "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": res["split"]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "bf16x5 slices, fp32 accumulate, fp64 fold", "data": "synthetic",
           "config": {"workload": "batch%d_L16-32_D128-768" % args.batch, "problems": len(probs),
                      "specs": [list(s_) for s_ in specs]},
           "fp64": res["fp64"], "split": res["split"],
           "split_rel_err_vs_fp64": {"max": max(errs), "median": float(np.median(errs))},
           "davidson": batch_dav}
    print(json.dumps(out), flush=True)


def time_hpsi(torch, plan, x, y, steps, warmup):
    """Graph-replayed H.psi: warm-up, then `steps` timed replays bracketed by
    synchronisation (ms per step); then the same number of eager launches
    with per-launch HIP events on the library's stream (per-stage kernel
    time and flops, the roofline's figures)."""
    for _ in range(warmup):
        plan.apply(x, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.apply(x, y)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    plan.set_profiling(True)
    for _ in range(steps):
        plan.apply(x, y)
    torch.cuda.synchronize()
    prof = {s_: plan.profile(s_) for s_ in (1, 2, 11, 12, 21, 22, 31, 32)}
    plan.set_profiling(False)
    return ms, prof


KERNEL_NAMES = {
    # profile code -> kernel (split s=5 plans, FP64 plans)
    31: ("stage1_wsplit5_kernel", None), 32: ("stage2_wsplit5_kernel", None),
    11: ("stage1_msplit5_kernel", None), 12: ("stage2_msplit5_kernel", None),
    21: ("stage1_split5_kernel", "stage_f64_kernel<1>"), 22: ("stage2_split5_kernel", "stage_f64_kernel<2>"),
}


def dominant(prof, split):
    """(kernel name, launches, ms, flops) of the tile kernel with the most time."""
    code = max((c for c in (11, 12, 21, 22, 31, 32) if prof[c][0] > 0), key=lambda c: prof[c][1])
    n, ms, fl = prof[code]
    return KERNEL_NAMES[code][0 if split else 1], n, ms, fl


# site multiplets (electrons, doubled spin): empty, one electron, doubly occupied
_SITE = ((0, 0), (1, 1), (2, 0))


def psi_layout(lsec, rsec, n_elec, two_s):
    """Wavefunction blocks in the order include/dmrg.h fixes (nested loops over
    left sector, l, 2S_Ll, r, right sector, 2S_rR; column-major dL x dR blocks
    concatenated): ([{iL, l, SLl, r, iR, SrR, off, dL, dR}], length)."""
    out, off = [], 0
    for iL, (NL, SL, dL) in enumerate(lsec):
        for l, (nl, sl) in enumerate(_SITE):
            for SLl in range(abs(SL - sl), SL + sl + 1, 2):
                for r, (nr, sr) in enumerate(_SITE):
                    for iR, (NR, SR, dR) in enumerate(rsec):
                        if NL + nl + nr + NR != n_elec:
                            continue
                        for SrR in range(abs(sr - SR), sr + SR + 1, 2):
                            if abs(SLl - SrR) <= two_s <= SLl + SrR:
                                out.append(dict(iL=iL, l=l, SLl=SLl, r=r, iR=iR, SrR=SrR, off=off, dL=dL, dR=dR))
                                off += dL * dR
    return out, off


def sampled_errors(yv, workload, prob):
    """Largest error of H.psi at the oracle's stored sample of this workload
    (tests/golden/hpsi_samples.json), relative to the largest sampled value."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "hpsi_samples.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        case = json.load(f).get("cases", {}).get(workload)
    if case is None:
        return None
    blocks, size = psi_layout(prob.left.sectors, prob.right.sectors, prob.n_elec, prob.two_s)
    if size != case["psi_len"]:
        return None
    err, scale, n = 0.0, 0.0, 0
    for smp in case["samples"]:
        b = blocks[smp["block"]]
        Y = yv[b["off"]:b["off"] + b["dL"] * b["dR"]].reshape(b["dR"], b["dL"]).T
        ref = np.array(smp["values"])
        err = max(err, float(np.abs(Y[np.ix_(smp["rows"], smp["cols"])] - ref).max()))
        scale = max(scale, float(np.abs(ref).max()))
        n += ref.size
    return {"max_rel": err / scale, "elements": n, "blocks": len(case["samples"])}


def davidson_runs(torch, args, plan_flags):
    """Davidson s/step: the diagonal-preconditioned solve with FP64 and with
    split H.psi on the --dav-workload, and the learned preconditioner against
    the diagonal one on the --mlp-workload (trained on L=24 solves).  Derived
    comparisons are reported only between converged solves; progress lines
    go to stderr every 25 iterations."""
    import numpy as np
    from paper_2309_16724_amd.hpsi import Plan
    fk = {} if args.dav_floor is None else {"floor": args.dav_floor}

    def start(plan):
        x_np = np.random.default_rng(100).standard_normal(plan.size)
        return torch.from_numpy(x_np / np.linalg.norm(x_np)).cuda()

    def solve(plan, x0, **kw):
        torch.cuda.synchronize()
        t0 = time.time()
        e, _, st = plan.davidson(x0, tol=1e-8, check=False, verbose=1, **fk, **kw)
        return e, st, time.time() - t0

    out = {"workload": args.dav_workload}
    prob = make_problem(WORKLOADS[args.dav_workload])
    plan = Plan(prob, flags=plan_flags)
    x0 = start(plan)
    e_dav, dst, t_dav = solve(plan, x0)
    print("# davidson fp64 %s: %d iterations, %.1f s" % (args.dav_workload, dst["iters"], t_dav),
          file=sys.stderr, flush=True)
    out["diagonal"] = {"s_per_step": t_dav, "iterations": dst["iters"], "n_hpsi": dst["n_hpsi"],
                       "converged": dst["converged"], "residual": dst["residual"], "energy": e_dav,
                       "sigma": dst["sigma"], "floor": args.dav_floor, "t_hpsi_s": dst["t_hpsi_s"]}
    plan.free()
    if not args.no_split_davidson:
        splan = Plan(prob, precision=1, n_slices=5, flags=plan_flags)
        e_sp, sst, t_sp = solve(splan, x0)
        print("# davidson split %s: %d iterations, %.1f s" % (args.dav_workload, sst["iters"], t_sp),
              file=sys.stderr, flush=True)
        both = dst["converged"] == 1 and sst["converged"] == 1
        out["split"] = {"s_per_step": t_sp, "iterations": sst["iters"], "converged": sst["converged"],
                        "residual": sst["residual"], "energy_minus_fp64": (e_sp - e_dav) if both else None}
    if not args.no_split_davidson and args.mixed_davidson:
        # mixed precision: split H.psi down to a residual the split error
        # (about 1e-8 in norm here) does not disturb, then an FP64 plan from
        # that vector to the tolerance; timed end to end, the FP64 plan's
        # construction included (the two plans do not fit in HBM together);
        # the split plan of the solve above is reused
        torch.cuda.synchronize()
        t0 = time.time()
        e_a, psi_a, st_a = splan.davidson(x0, tol=args.refine_tol, check=False, verbose=1, **fk)
        splan.free()
        rplan = Plan(prob, flags=plan_flags)
        e_b, psi_b, st_b = rplan.davidson(psi_a, tol=1e-8, check=False, verbose=1, **fk)
        torch.cuda.synchronize()
        t_mix = time.time() - t0
        rplan.free()
        ok = dst["converged"] == 1 and st_b["converged"] == 1
        print("# davidson split to %.0e then fp64: %d + %d iterations, %.1f s"
              % (args.refine_tol, st_a["iters"], st_b["iters"], t_mix), file=sys.stderr, flush=True)
        out["split_then_fp64"] = {"s_per_step": t_mix, "switch_residual": args.refine_tol,
                                  "split_iterations": st_a["iters"], "fp64_iterations": st_b["iters"],
                                  "converged": st_b["converged"], "residual": st_b["residual"],
                                  "energy_minus_fp64": (e_b - e_dav) if ok else None,
                                  "speedup_vs_fp64": (t_dav / t_mix) if ok else None}
    elif not args.no_split_davidson:
        splan.free()
    del prob
    if not args.no_mlp:
        net, info = train_preconditioner(torch, [(24, 24, 0, 10000 + k, 512) for k in range(4)], floor=args.dav_floor)
        print("# learned preconditioner: %s" % json.dumps(info), file=sys.stderr, flush=True)
        mprob = make_problem(WORKLOADS[args.mlp_workload])
        mplan = Plan(mprob, flags=plan_flags)
        x1 = start(mplan)
        e_d, d_st, t_d = solve(mplan, x1)
        e_m, m_st, t_m = solve(mplan, x1, mlp=net)
        net.free()
        mplan.free()
        both = d_st["converged"] == 1 and m_st["converged"] == 1
        out["learned"] = {"workload": args.mlp_workload,
                          "diagonal": {"s_per_step": t_d, "iterations": d_st["iters"],
                                       "converged": d_st["converged"], "energy": e_d},
                          "learned": {"s_per_step": t_m, "iterations": m_st["iters"],
                                      "converged": m_st["converged"], "residual": m_st["residual"],
                                      "fallbacks": m_st["fallbacks"], "switched": m_st["switched"]},
                          "energy_minus_diagonal": (e_m - e_d) if both else None,
                          "speedup_vs_diagonal": (t_d / t_m) if both else None,
                          "training": info}
    return out


def renorm_run(torch, workload, steps, warmup, prob=None, all_pairs=False, right=False):
    """Renormalization of the workload's left block through its left site,
    FP64: the families H, C, A0, A1, B0, B1, S of the enlarged block (with
    all_pairs the left block is drawn with P and Q over every outside pair and
    P0, P1, Q0, Q1 are produced too); every product sector keeps a quarter of
    its rows (about D states in all) through a U with orthonormal columns (QR
    of a seeded Gaussian matrix).  Timed like H.psi: warm-up, then `steps`
    applies bracketed by synchronisation.  right: the right block through
    the right site instead (site x block; H, C, S, P0, P1, Q0, Q1 of the
    enlarged right block)."""
    import numpy as np
    from paper_2309_16724_amd import binding as B
    from paper_2309_16724_amd.hpsi import Renorm
    if prob is None or (all_pairs and not right):
        t0 = time.time()
        prob = make_problem(WORKLOADS[workload], all_pairs=all_pairs)
        print("# left block of %s generated in %.1f s (%d elements)"
              % (workload, time.time() - t0, prob.left.data.size), file=sys.stderr, flush=True)
    secs, _ = B.renorm_product(prob, right=right)
    rng = np.random.default_rng(7)
    keep = [(n, s2, np.linalg.qr(rng.standard_normal((rows, max(1, rows // 4))))[0]) for (n, s2, rows) in secs]
    t0 = time.time()
    r = Renorm(prob, keep, right=right)
    st = r.stats()
    print("# renormalization lists built in %.1f s: %s" % (time.time() - t0, json.dumps(st)), file=sys.stderr,
          flush=True)
    for _ in range(warmup):
        r.apply()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        r.apply()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t1) * 1e3 / steps
    r.set_profiling(True)
    for _ in range(steps):
        r.apply()
    torch.cuda.synchronize()
    prof = {s_: r.profile(s_) for s_ in (1, 2)}
    r.set_profiling(False)
    first = r.out.clone()
    r.apply()
    torch.cuda.synchronize()
    repro = bool(torch.equal(first, r.out))
    del first
    # H of the new block is a scalar: diagonal sector blocks only, symmetric
    asym, nh = 0.0, 0
    for rec in r.recs[:r.n_rec]:
        if rec.fam != 0:
            continue
        n = keep[rec.row_sec][2].shape[1]
        m = r.out[rec.off:rec.off + n * n].view(n, n)
        asym = max(asym, float((m - m.T).abs().max() / max(float(m.abs().max()), 1e-300)))
        nh += 1
    flops = st["flops1"] + st["flops2"]
    tf = flops / (ms * 1e-3) / 1e12
    r.free()
    dom = max((1, 2), key=lambda s_: prof[s_][1])
    n_d, ms_d, fl_d = prof[dom]
    ach = (fl_d / n_d) / (ms_d / n_d * 1e-3) / 1e12
    kname = "stage_f64_kernel<%d>" % dom
    return {"ms": ms, "tflops": tf, "flops": flops, "flops_stage1": st["flops1"], "flops_stage2": st["flops2"],
            "kept_states": int(sum(u.shape[1] for _, _, u in keep)),
            "product_states": int(sum(u.shape[0] for _, _, u in keep)),
            "families": ("H C S P0 P1 Q0 Q1" if right else
                         "H C A0 A1 B0 B1 S" + (" P0 P1 Q0 Q1" if all_pairs else "")), "records": r.n_rec,
            "block_elems": int((prob.right if right else prob.left).data.size), "out_elems": st["out_elems"],
            "terms": st["n_terms"], "products": [st["n_products1"], st["n_products2"]],
            "tiles": [st["n_tiles1"], st["n_tiles2"]], "build_ms": st["build_ms"],
            "bitwise_repeat": repro, "h_blocks": nh, "h_asymmetry": asym,
            "stages_ms": {str(k): v[1] / max(v[0], 1) for k, v in prof.items()},
            "roofline": {"bound": "mfma", "kernel": kname, "achieved": ach, "peak": FP64_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": ach / FP64_PEAK_TFLOPS,
                         "traffic": measured_traffic(workload, ("renorm_right:" if right else "renorm:") + kname)}}


def truncation_run(torch, prob, D, reps=3):
    """Truncation of a two-site step on the workload (dmrg_truncate): the
    reduced density matrix of (left block x left site) per sector from a
    seeded normalized wavefunction, its eigenvectors, the D largest kept.
    Wall time of the whole call (lists, products, eigensolver, copies)."""
    import numpy as np
    from paper_2309_16724_amd.hpsi import truncate
    from paper_2309_16724_amd.binding import renorm_product
    _, size = psi_layout(prob.left.sectors, prob.right.sectors, prob.n_elec, prob.two_s)
    x = np.random.default_rng(100).standard_normal(size)
    psi = torch.from_numpy(x / np.linalg.norm(x)).cuda()
    secs, _ = renorm_product(prob)
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        keep, u, (kw, tr) = truncate(prob, psi, D, 1e-14)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    return {"ms": min(times), "ms_all": times, "max_kept": D, "kept": int(sum(k[2] for k in keep)),
            "kept_sectors": len(keep), "product_sectors": len(secs), "largest_sector_rows": max(r for _, _, r in secs),
            "kept_weight": kw, "trace": tr,
            "note": "random normalized wavefunction; rho per sector on the FP64 tile engine, rocSOLVER dsyevd"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="L54_D2048", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true", help="autotune the H.psi plans (DMRG_PLAN_AUTOTUNE)")
    ap.add_argument("--no-graph", action="store_true", help="time eager launches instead of graph replays")
    ap.add_argument("--no-mlp", action="store_true", help="skip the learned-preconditioner Davidson")
    ap.add_argument("--no-davidson", action="store_true", help="time H.psi only")
    ap.add_argument("--dav-workload", default="L54_D2048", choices=sorted(WORKLOADS),
                    help="workload of the Davidson solves (default: the H.psi workload's L=54, D=2048)")
    ap.add_argument("--mlp-workload", default="L24_D512", choices=sorted(WORKLOADS),
                    help="workload of the learned-versus-diagonal preconditioner comparison "
                         "(L64_D3072 for the learned preconditioner's evaluation configuration)")
    ap.add_argument("--no-split-davidson", action="store_true",
                    help="skip the Davidson solve with split-precision H.psi")
    ap.add_argument("--mixed-davidson", action="store_true",
                    help="also time the mixed-precision Davidson (split H.psi, then FP64 from --refine-tol)")
    ap.add_argument("--refine-tol", type=float, default=1e-6,
                    help="residual at which the mixed-precision Davidson leaves split H.psi for FP64")
    ap.add_argument("--dav-floor", type=float, default=None,
                    help="relative preconditioner floor of the Davidson solves (library default if omitted)")
    ap.add_argument("--hpsi-only", choices=("fp64", "split"),
                    help="time only H.psi of one precision (for profiler runs); also copies "
                         "256 MiB once with a plain device copy as a counter reference")
    ap.add_argument("--batch-davidson", action="store_true",
                    help="with --batch: also solve all problems with one batched Davidson (FP64)")
    ap.add_argument("--batch", type=int, default=0,
                    help="instead of the single workload, time H.psi of a batch of this many "
                         "uneven problems (L in [16, 32], D in [128, 768], S in {0, 1})")
    ap.add_argument("--no-autotune", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--no-renorm", action="store_true", help="skip the renormalization leg")
    ap.add_argument("--renorm-only", action="store_true",
                    help="time only the renormalization of the workload's left block (for profiler runs)")
    ap.add_argument("--renorm-right", action="store_true",
                    help="with --renorm-only: the right block through the right site instead")
    ap.add_argument("--renorm-all-pairs", action="store_true",
                    help="with --renorm-only: draw the left block with P and Q over every outside pair and "
                         "renormalize every family")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.batch:
        return run_batch(args)
    import numpy as np
    import torch
    from paper_2309_16724_amd.binding import DMRG_PLAN_AUTOTUNE, DMRG_PLAN_GRAPH
    from paper_2309_16724_amd.hpsi import Plan

    w = WORKLOADS[args.workload]
    t0 = time.time()
    prob = make_problem(w)
    secs = [s_[2] for s_ in prob.left.sectors] + [s_[2] for s_ in prob.right.sectors]
    rd = sum((s_[1] + 1) * s_[2] for s_ in prob.left.sectors) / sum(s_[2] for s_ in prob.left.sectors)
    print("# workload %s generated in %.1f s (sector dims %d..%d, R_D %.2f)"
          % (args.workload, time.time() - t0, min(secs), max(secs), rd), file=sys.stderr, flush=True)
    plan_flags = (0 if args.no_graph else DMRG_PLAN_GRAPH) | (DMRG_PLAN_AUTOTUNE if args.autotune else 0)

    def run(precision, ns, flags):
        t1 = time.time()
        plan = Plan(prob, precision=precision, n_slices=ns, flags=flags)
        st = plan.stats()
        print("# plan %s prec=%d s=%d built in %.1f s: %s" % (args.workload, precision, ns, time.time() - t1,
                                                              json.dumps(st)), file=sys.stderr, flush=True)
        x = torch.from_numpy(np.random.default_rng(100).standard_normal(plan.size)).cuda()
        x /= torch.linalg.norm(x)
        y = torch.empty_like(x)
        ms, prof = time_hpsi(torch, plan, x, y, args.steps, args.warmup)
        print("# per-stage (launches, ms, flops): %s" % json.dumps(prof), file=sys.stderr, flush=True)
        yv = y.cpu().numpy()
        plan.free()
        del x, y
        return st, ms, prof, yv

    if args.renorm_only:
        print(json.dumps({"renorm_only": True, "workload": args.workload,
                          **renorm_run(torch, args.workload, args.steps, args.warmup, prob,
                                                     args.renorm_all_pairs, args.renorm_right)}), flush=True)
        return
    if args.hpsi_only:
        ref = torch.empty(32 << 20, dtype=torch.float64, device="cuda")   # 256 MiB
        ref2 = torch.empty_like(ref)
        ref.fill_(1.0)
        ref2.copy_(ref)
        torch.cuda.synchronize()
        del ref, ref2
        prec, ns = (0, 0) if args.hpsi_only == "fp64" else (1, 5)
        st, ms, prof, _ = run(prec, ns, 0)
        print(json.dumps({"hpsi_only": args.hpsi_only, "workload": args.workload, "ms_per_step": ms,
                          "tflops": st["flops"] / (ms * 1e-3) / 1e12, "stages": prof,
                          "kpart": st["kpart"], "tile_policy": st["tile_policy"],
                          "workspace_cap": st["workspace_cap"]}), flush=True)
        return
    st64, ms64, prof64, y64 = run(0, 0, plan_flags)
    err64 = sampled_errors(y64, args.workload, prob)
    st5, ms5, prof5, y5 = run(1, 5, plan_flags)
    err5 = sampled_errors(y5, args.workload, prob)
    rel = float(np.abs(y5 - y64).max() / np.abs(y64).max())
    del y5, y64
    ren = None
    if not args.no_renorm:
        ren = renorm_run(torch, args.workload, args.steps, args.warmup, prob)
        ren["workload"] = "%s left block (orbitals 0..%d) x site %d" % (args.workload, prob.p - 1, prob.p)
        ren_r = renorm_run(torch, args.workload, args.steps, args.warmup, prob, right=True)
        ren_r["workload"] = "%s site %d x right block (orbitals %d..%d)" % (args.workload, prob.p + 1, prob.p + 2,
                                                                         prob.n_orb - 1)
        ren["right_block"] = ren_r
        ren["truncation"] = truncation_run(torch, prob, WORKLOADS[args.workload]["D"])
        print("# renormalization: %s" % json.dumps(ren), file=sys.stderr, flush=True)
    dav = None
    if not args.no_davidson:
        dav = davidson_runs(torch, args, plan_flags)
    kname5, n_l, ms_l, fl_l = dominant(prof5, True)
    achieved = (fl_l / n_l) / (ms_l / n_l * 1e-3) / 1e12
    split_peak = BF16_PEAK_TFLOPS / 15.0           # s = 5: 15 slice products per FP64 product
    kname64, n6, ms6, fl6 = dominant(prof64, False)
    tflops5 = st5["flops"] / (ms5 * 1e-3) / 1e12
    tflops64 = st64["flops"] / (ms64 * 1e-3) / 1e12
    ach64 = (fl6 / n6) / (ms6 / n6 * 1e-3) / 1e12
    gen = {k: w[k] for k in GEN_KEYS if k in w}
    out = {
        "metric": "H.psi TFLOP/s (split-BF16 s=5 at <=1e-10 rel err vs the FP64 oracle; algorithmic FP64-"
                  "equivalent flops); FP64 path and Davidson s/step alongside",
        "value": tflops5,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms5,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x5 slices, fp32 accumulate, fp64 fold",
        "data": "synthetic",
        "config": {"workload": args.workload, **{k: w[k] for k in ("n_orb", "n_elec", "two_s", "seed")},
                   **gen, "psi_len": int(st5["psi_len"]), "sector_dims": [min(secs), max(secs)],
                   "R_D": round(rd, 3), "flops_per_hpsi": st5["flops"], "n_slices": 5,
                   "timed": "eager launches" if args.no_graph else "graph replays (DMRG_PLAN_GRAPH)",
                   "split_plan": {k: st5[k] for k in ("kpart", "tile_policy", "workspace_cap", "n_chunks",
                                                      "launches", "tasks_ms", "plan_ms")},
                   "fp64_plan": {k: st64[k] for k in ("kpart", "tile_policy", "workspace_cap", "n_chunks",
                                                      "launches", "tasks_ms", "plan_ms")}},
        "split_rel_err_vs_oracle_samples": err5,
        "fp64_rel_err_vs_oracle_samples": err64,
        "split_rel_err_vs_fp64": rel,
        "fp64": {"value": tflops64, "ms_per_step": ms64,
                 "roofline": {"bound": "mfma", "kernel": kname64, "achieved": ach64,
                              "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ach64 / FP64_PEAK_TFLOPS,
                              "traffic": measured_traffic(args.workload, kname64)},
                 "stages_ms_per_step": {str(k): v[1] / args.steps for k, v in prof64.items()}},
        "speedup_split_vs_fp64": ms64 / ms5,
        "davidson": dav,
        "renormalization": ren,
        "split_stages_ms_per_step": {str(k): v[1] / args.steps for k, v in prof5.items()},
        "roofline": {"bound": "mfma", "kernel": kname5,
                     "achieved": achieved, "peak": split_peak, "unit": "TFLOP/s",
                     "frac": achieved / split_peak,
                     "traffic": measured_traffic(args.workload, kname5),
                     "peak_note": "BF16 dense 2516.6 TF/s divided by 15 slice products (s=5)"},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(st5["flops"], args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
