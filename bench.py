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
    # L orbitals, N electrons, 2S, integral seed, SU(2) bond dimension D per block
    "L24_D512": dict(n_orb=24, n_elec=24, two_s=0, seed=1, D=512),
    "L54_D2048": dict(n_orb=54, n_elec=54, two_s=0, seed=2, D=2048),
    "L64_D3072": dict(n_orb=64, n_elec=64, two_s=0, seed=4, D=3072),
}

FP64_PEAK_TFLOPS = 78.6       # MI355X dense FP64 (matrix and vector)
BF16_PEAK_TFLOPS = 2516.6     # MI355X dense BF16 MFMA


def cpu_baseline(prob, flops_full, target_s=15.0):
    """Time the oracle on every k-th of its merged terms over the whole wavefunction."""
    import numpy as np
    from oracle.hpsi import HEff
    he = HEff(prob)
    terms = he.compiled()
    x = np.random.default_rng(100).standard_normal(he.size)
    u1 = he.expand(x)
    # probe cost with a small stride, then pick the stride for ~target_s
    probe = terms[::50]
    t0, c0 = time.time(), time.process_time()
    he._compiled = probe
    he.apply_u1(u1)
    dt = max(time.time() - t0, 1e-3)
    est_full = dt * len(terms) / max(len(probe), 1)
    k = max(1, int(round(est_full / target_s)))
    sample = terms[::k]
    he._compiled = sample
    t0, c0 = time.time(), time.process_time()
    he.apply_u1(u1)
    wall = time.time() - t0
    cpu = time.process_time() - c0
    t_full = wall * len(terms) / len(sample)
    return {
        "value": flops_full / t_full / 1e12,
        "unit": "TFLOP/s",
        "cores": max(1, int(round(cpu / wall))),
        "kind": "oracle",
        "sample": "oracle H_eff psi over the full wavefunction restricted to every %d-th of its "
                  "%d merged terms (%.1f s wall), scaled by %d/%d to one full H.psi "
                  "(%.1f s); value = algorithmic flops of one H.psi / that time"
                  % (k, len(terms), wall, len(terms), len(sample), t_full),
    }


# HBM bytes per launch of the dominant stage kernels at L24_D512 from the
# FETCH_SIZE and WRITE_SIZE runs summarised in profiles/hpsi_L24_D512_split5.md
# and profiles/hpsi_L24_D512_fp64.md: FETCH scaled by 2.000 and WRITE by 1.000,
# what the same counters read for a plain 256 MiB device copy and fill in the
# same runs.  A figure holds only while the sources that decide the kernel's
# memory traffic are the ones it was taken on (their hash); else null.
MEASURED_TRAFFIC = {
    ("L24_D512", "stage2_split5_kernel"):
        (1.1229e10, ("kernels_split.hip", "plan.cpp", "plan.hpp", "model.cpp"), "f37f097fc51fca79"),
    ("L24_D512", "stage_f64_kernel<2>"):
        (9.7688e9, ("kernels_f64.hip", "plan.cpp", "plan.hpp", "model.cpp"), "6845b5fd10cebf51"),
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


def train_preconditioner(torch, specs, steps=2000, batch=4096, seed=0, width=256):
    """Learned preconditioner: exact-correction rows of the given solves
    (device capture), then minibatch Adam on the device."""
    import numpy as np
    from paper_2309_16724_amd.hpsi import Plan
    from paper_2309_16724_amd.precond import MLP
    from paper_2309_16724_amd.synth.problem import random_problem, random_vector
    t0 = time.time()
    xs, as_, bs, nrec = [], [], [], 0
    for L, N, s2, sd, D in specs:
        plan = Plan(random_problem(L, N, s2, sd, D=D))
        x0 = torch.from_numpy(random_vector(plan.size, 100)).cuda()
        x, a, b, nr = plan.collect(x0, capacity=plan.size * 500)
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="L24_D512", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the default tile settings instead of autotuning each plan")
    ap.add_argument("--no-mlp", action="store_true", help="skip the learned-preconditioner Davidson")
    ap.add_argument("--no-davidson", action="store_true", help="time H.psi only (large workloads)")
    ap.add_argument("--no-split-davidson", action="store_true",
                    help="skip the Davidson solve with split-precision H.psi")
    ap.add_argument("--dav-floor", type=float, default=None,
                    help="preconditioner denominator floor of the Davidson solves (library default if omitted)")
    ap.add_argument("--dav-verbose", action="store_true",
                    help="Davidson progress lines on stderr every 25 iterations (long solves)")
    ap.add_argument("--hpsi-only", choices=("fp64", "split"),
                    help="time only H.psi of one precision (for profiler runs); also copies "
                         "256 MiB once with a plain device copy as a counter reference")
    ap.add_argument("--batch-davidson", action="store_true",
                    help="with --batch: also solve all problems with one batched Davidson (FP64)")
    ap.add_argument("--batch", type=int, default=0,
                    help="instead of the single workload, time H.psi of a batch of this many "
                         "uneven problems (L in [16, 32], D in [128, 768], S in {0, 1})")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.batch:
        return run_batch(args)
    import numpy as np
    import torch
    from paper_2309_16724_amd.binding import DMRG_PLAN_AUTOTUNE
    from paper_2309_16724_amd.hpsi import Plan
    from paper_2309_16724_amd.synth.problem import random_problem

    w = WORKLOADS[args.workload]
    prob = random_problem(w["n_orb"], w["n_elec"], w["two_s"], w["seed"], D=w["D"])
    sizer = Plan(prob)
    x_np = np.random.default_rng(100).standard_normal(sizer.size)
    x_np /= np.linalg.norm(x_np)
    sizer.free()
    plan_flags = 0 if args.no_autotune else DMRG_PLAN_AUTOTUNE

    def run(precision, ns):
        plan = Plan(prob, precision=precision, n_slices=ns, flags=plan_flags)
        st = plan.stats()
        print("# plan %s prec=%d s=%d: %s" % (args.workload, precision, ns, json.dumps(st)),
              file=sys.stderr, flush=True)
        x = torch.from_numpy(x_np).cuda()
        y = torch.empty_like(x)
        for _ in range(args.warmup):
            plan.apply(x, y)
        torch.cuda.synchronize()
        # the timed region: per-launch HIP events on the library's stream
        plan.set_profiling(True)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(args.steps):
            plan.apply(x, y)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        prof = {s_: plan.profile(s_) for s_ in (1, 2)}
        plan.set_profiling(False)
        print("# per-stage (launches, ms, flops): %s" % json.dumps(prof), file=sys.stderr, flush=True)
        yv = y.cpu().numpy()
        plan.free()
        return st, ms, prof, yv

    if args.hpsi_only:
        ref = torch.empty(32 << 20, dtype=torch.float64, device="cuda")   # 256 MiB
        ref2 = torch.empty_like(ref)
        ref.fill_(1.0)
        ref2.copy_(ref)
        torch.cuda.synchronize()
        del ref, ref2
        prec, ns = (0, 0) if args.hpsi_only == "fp64" else (1, 5)
        st, ms, prof, _ = run(prec, ns)
        print(json.dumps({"hpsi_only": args.hpsi_only, "workload": args.workload, "ms_per_step": ms,
                          "tflops": st["flops"] / (ms * 1e-3) / 1e12, "stages": prof,
                          "kpart": st["kpart"], "tile_policy": st["tile_policy"],
                          "workspace_cap": st["workspace_cap"]}), flush=True)
        return
    st64, ms64, prof64, y64 = run(0, 0)
    st5, ms5, prof5, y5 = run(1, 5)
    rel = float(np.abs(y5 - y64).max() / np.abs(y64).max())
    davidson, learned, split_dav = None, None, None
    if not args.no_davidson:
        # Davidson s/step (FP64 path, diagonal preconditioner) on the same workload
        plan = Plan(prob, flags=plan_flags)
        x0 = torch.from_numpy(x_np).cuda()
        torch.cuda.synchronize()
        td = time.time()
        fk = {} if args.dav_floor is None else {"floor": args.dav_floor}
        e_dav, _, dst = plan.davidson(x0, tol=1e-8, check=False, verbose=int(args.dav_verbose), **fk)
        t_dav = time.time() - td
        davidson = {"s_per_step": t_dav, "iterations": dst["iters"], "n_hpsi": dst["n_hpsi"],
                    "converged": dst["converged"], "floor": args.dav_floor,
                    "residual": dst["residual"], "energy": e_dav, "precision": "fp64",
                    "preconditioner": "diagonal", "t_hpsi_s": dst["t_hpsi_s"]}
        if not args.no_mlp:
            net, info = train_preconditioner(torch, [(24, 24, 0, 10000 + k, 512) for k in range(4)])
            print("# learned preconditioner: %s" % json.dumps(info), file=sys.stderr, flush=True)
            torch.cuda.synchronize()
            tm = time.time()
            e_mlp, _, mst = plan.davidson(x0, tol=1e-8, mlp=net, check=False, verbose=int(args.dav_verbose), **fk)
            t_mlp = time.time() - tm
            net.free()
            learned = {"s_per_step": t_mlp, "iterations": mst["iters"], "n_hpsi": mst["n_hpsi"],
                       "converged": mst["converged"], "fallbacks": mst["fallbacks"],
                       "energy_minus_diagonal": e_mlp - e_dav, "t_hpsi_s": mst["t_hpsi_s"],
                       "speedup_vs_diagonal": t_dav / t_mlp, "training": info}
        plan.free()
        if not args.no_split_davidson:
            # the same solve with every H.psi in split precision
            splan = Plan(prob, precision=1, n_slices=5, flags=plan_flags)
            torch.cuda.synchronize()
            tsd = time.time()
            e_sp, _, sst = splan.davidson(x0, tol=1e-8, check=False, verbose=int(args.dav_verbose), **fk)
            split_dav = {"s_per_step": time.time() - tsd, "iterations": sst["iters"],
                         "converged": sst["converged"], "residual": sst["residual"],
                         "energy_minus_fp64": e_sp - e_dav}
            splan.free()
    dom = max((1, 2), key=lambda s_: prof5[s_][1])
    n_l, ms_l, fl_l = prof5[dom]
    achieved = (fl_l / n_l) / (ms_l / n_l * 1e-3) / 1e12
    split_peak = BF16_PEAK_TFLOPS / 15.0           # s = 5: 15 slice products per FP64 product
    dom64 = max((1, 2), key=lambda s_: prof64[s_][1])
    n6, ms6, fl6 = prof64[dom64]
    tflops5 = st5["flops"] / (ms5 * 1e-3) / 1e12
    tflops64 = st64["flops"] / (ms64 * 1e-3) / 1e12
    ach64 = (fl6 / n6) / (ms6 / n6 * 1e-3) / 1e12
    out = {
        "metric": "H.psi TFLOP/s (split-BF16 s=5 at <=1e-10 rel err vs FP64; algorithmic FP64-equivalent "
                  "flops); FP64 path and Davidson s/step alongside",
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
        "config": {"workload": args.workload, **w, "psi_len": int(x_np.size),
                   "flops_per_hpsi": st5["flops"], "n_slices": 5,
                   "split_plan": {k: st5[k] for k in ("kpart", "tile_policy", "workspace_cap")},
                   "fp64_plan": {k: st64[k] for k in ("kpart", "tile_policy", "workspace_cap")}},
        "split_rel_err_vs_fp64": rel,
        "fp64": {"value": tflops64, "ms_per_step": ms64,
                 "roofline": {"bound": "mfma", "kernel": "stage_f64_kernel<%d>" % dom64, "achieved": ach64,
                              "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ach64 / FP64_PEAK_TFLOPS,
                              "traffic": measured_traffic(args.workload, "stage_f64_kernel<%d>" % dom64)}},
        "speedup_split_vs_fp64": ms64 / ms5,
        "davidson": davidson,
        "davidson_learned": learned,
        "davidson_split": split_dav,
        "roofline": {"bound": "mfma", "kernel": "stage%d_split5_kernel" % dom,
                     "achieved": achieved, "peak": split_peak, "unit": "TFLOP/s",
                     "frac": achieved / split_peak,
                     "traffic": measured_traffic(args.workload, "stage%d_split5_kernel" % dom),
                     "peak_note": "BF16 dense 2516.6 TF/s divided by 15 slice products (s=5)"},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, st5["flops"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
