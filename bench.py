"""Benchmark of the SU(2) two-site H.psi hot path on one MI355X.

python bench.py --gpus 1 --steps K --warmup W [--workload L24_D512]

One step = one H_eff psi over the whole wavefunction of the workload (all
operator-table rows, all sector tasks, both stripe stages).  Inputs are
seeded synthetic blocks already resident in HBM.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # L orbitals, N electrons, 2S, integral seed, SU(2) bond dimension D
    "L24_D512": dict(n_orb=24, n_elec=24, two_s=0, seed=1, D=512),
    "L54_D2048": dict(n_orb=54, n_elec=54, two_s=0, seed=2, D=2048),
    "L64_D3072": dict(n_orb=64, n_elec=64, two_s=0, seed=4, D=3072),
}

FP64_PEAK_TFLOPS = 78.6


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="L24_D512", choices=sorted(WORKLOADS))
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2309_16724_amd.synth.problem import random_problem
    from paper_2309_16724_amd.hpsi import Plan

    w = WORKLOADS[args.workload]
    t0 = time.time()
    prob = random_problem(w["n_orb"], w["n_elec"], w["two_s"], w["seed"], D=w["D"])
    plan = Plan(prob)
    st = plan.stats()
    print("# plan: %s build %.1fs" % (json.dumps(st), time.time() - t0), file=sys.stderr, flush=True)
    x = torch.from_numpy(np.random.default_rng(100).standard_normal(plan.size)).cuda()
    x /= x.norm()
    y = torch.empty_like(x)
    for _ in range(args.warmup):
        plan.apply(x, y)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        plan.apply(x, y)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    tflops = st["flops"] / (ms * 1e-3) / 1e12
    out = {
        "metric": "H.psi TFLOP/s (FP64 path); split-BF16 and Davidson s/step reported separately",
        "value": tflops,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, **w, "psi_len": plan.size,
                   "flops_per_hpsi": st["flops"]},
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    plan.free()


if __name__ == "__main__":
    main()
