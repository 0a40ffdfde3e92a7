#!/usr/bin/env python3
"""Benchmark of the UniFrac hot path on one MI355X.

One step = one full distance matrix of the benchmark workload with inputs already resident
in HBM: embedding propagation, embedding transform, striped accumulation and
normalize/condense, ending with the condensed matrix in device memory.

Default workload: 4,096 samples on a 32,768-tip random coalescent tree (65,534 branches),
~800 features per sample with NegBin(10, 0.3) counts rarefied to 5,000, weighted normalized
UniFrac.  The headline value is the FP32 path; the FP64 path is timed on the same inputs
for the FP32-vs-FP64 comparison.  Max and mean absolute error of both against the FP64 CPU
oracle on a seeded sample of pairs are reported, and the same oracle run is timed on the
host cores as the CPU baseline.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# VALU issue rate of one MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (lane-ops/s).
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
# Algorithmic VALU operations per pair-branch update of the striped kernel:
#   num += L*|u - v|  (sub, fma with |.|)   den += L*(u + v)  (add, fma)
OPS_PER_UPDATE = {0: 4, 1: 2}   # den_mode 0: both stripes; 1: numerator only


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--method", default="weighted_normalized")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--compare", default="fp64", help="second precision timed for comparison ('' = none)")
    ap.add_argument("--emb-batch", type=int, default=0)
    ap.add_argument("--den-mode", type=int, default=0)
    ap.add_argument("--n", type=int, default=None, help="override the sample count")
    ap.add_argument("--tips", type=int, default=None, help="override the tip count")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target oracle CPU time")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy 3 times (HBM counter scale)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": src.numel() * 4, "dispatches": 3}))
        return
    import paper_2005_05826_amd as uf
    from synth import config_problem

    over = {}
    if args.n:
        over["n"] = args.n
    if args.tips:
        over["tips"] = args.tips
    t0 = time.time()
    prob = config_problem(2, **over)
    log(f"generated workload in {time.time() - t0:.1f}s: n={prob.n_samples} nodes={prob.n_nodes} "
        f"nnz={prob.indices.size}")
    n = prob.n_samples
    n_pairs = n * (n - 1) // 2
    B = prob.n_nodes - 1
    updates = n_pairs * B

    ctx = uf.Context(0)
    stream = torch.cuda.current_stream()
    plan = uf.Plan.from_problem(ctx, prob, stream=stream)
    info = plan.info
    tuning = dict(emb_batch=args.emb_batch, den_mode=args.den_mode)

    def run(prec, steps, warmup, profile):
        out = torch.empty(n_pairs, dtype=torch.float64, device="cuda:0")
        for _ in range(warmup):
            plan.distance(args.method, prec, out=out, tuning=tuning, stream=stream)
        plan.set_profiling(profile)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            plan.distance(args.method, prec, out=out, tuning=tuning, stream=stream)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / steps
        prof = plan.profile() if profile else {}
        plan.set_profiling(False)
        return dt, out, prof

    log(f"timing {args.precision}: {args.warmup} warmup + {args.steps} steps")
    dt, out, prof = run(args.precision, args.steps, args.warmup, True)
    log(f"{args.precision}: {dt * 1e3:.2f} ms/step; kernels {prof}")
    cmp = None
    if args.compare:
        log(f"timing {args.compare}")
        dt2, out2, prof2 = run(args.compare, max(1, args.steps // 2), 1, True)
        log(f"{args.compare}: {dt2 * 1e3:.2f} ms/step; kernels {prof2}")
        cmp = (dt2, out2, prof2)

    # roofline of the dominant kernel (the striped accumulation)
    launches, total_ms = prof.get("stripe", (0, 0.0))
    ops_per_step = OPS_PER_UPDATE[args.den_mode] * updates
    stripe_ms_per_step = total_ms / args.steps
    roofline = None
    if launches:
        achieved = ops_per_step / (stripe_ms_per_step * 1e-3) / 1e12
        roofline = {"kernel": "k_stripe", "bound": "alu", "achieved": round(achieved, 3),
                    "peak": round(VALU_PEAK_TOPS, 2), "unit": "Tops/s",
                    "frac": round(achieved / VALU_PEAK_TOPS, 4), "traffic": None,
                    "launches_per_step": launches // args.steps,
                    "avg_launch_ms": round(total_ms / launches, 4),
                    "ops_per_update": OPS_PER_UPDATE[args.den_mode]}

    # oracle: CPU baseline and error sample (same seeded pairs for both precisions)
    err = {}
    cpu = None
    if not args.no_cpu:
        from oracle import oracle
        rng = np.random.Generator(np.random.Philox(20050526 + 99))
        omethod = oracle.WEIGHTED_NORMALIZED if args.method == "weighted_normalized" else oracle.UNWEIGHTED

        def sample(m):
            i = rng.integers(0, n, size=m)
            j = rng.integers(0, n, size=m)
            keep = i != j
            return np.minimum(i[keep], j[keep]), np.maximum(i[keep], j[keep])

        pi, pj = sample(256)
        t = time.perf_counter()
        oracle.problem_pairs(prob, omethod, pi, pj)
        per_pair = (time.perf_counter() - t) / max(1, pi.size)
        m = int(min(max(args.cpu_seconds / max(per_pair, 1e-9), 500), 2_000_000))
        pi, pj = sample(m)
        threads = oracle.max_threads()
        log(f"oracle: {pi.size} sampled pairs on {threads} threads")
        t = time.perf_counter()
        want = oracle.problem_pairs(prob, omethod, pi, pj)
        cpu_s = time.perf_counter() - t
        cpu = {"value": round(pi.size * B / cpu_s, 1), "unit": "pair-branch updates/s",
               "cores": threads, "kind": "oracle",
               "sample": f"{pi.size} seeded random pairs of the workload (all {B} branches each), "
                         f"{cpu_s:.1f} s incl. walk-up counts of the touched samples",
               "seconds": round(cpu_s, 2)}
        idx = n * pi - pi * (pi + 1) // 2 + (pj - pi - 1)
        for prec, o in [(args.precision, out)] + ([(args.compare, cmp[1])] if cmp else []):
            got = o.cpu().numpy()[idx]
            e = np.abs(got - want)
            err[prec] = {"max_abs": float(e.max()), "mean_abs": float(e.mean()), "pairs": int(pi.size)}

    value = updates / dt
    res = {
        "metric": "sample-pair·branch updates/s + full-matrix wall time, FP32/MFMA vs FP64 plain",
        "value": round(value, 1),
        "unit": "pair-branch updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"weighted-normalized striped UniFrac, {n} samples, coalescent "
                               f"tree with {(prob.n_nodes + 1) // 2} tips ({B} branches)",
                   "n_samples": n, "branches": B, "levels": info.n_levels, "nnz": int(info.nnz),
                   "method": args.method, "precision": args.precision,
                   "emb_batch": args.emb_batch or "default", "den_mode": args.den_mode},
        "full_matrix_wall_ms": round(dt * 1e3, 3),
        "kernels_ms_per_step": {k: round(v[1] / args.steps, 3) for k, v in prof.items()},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "error_vs_oracle": err,
    }
    if cmp:
        dt2 = cmp[0]
        res["compare"] = {"precision": args.compare, "ms_per_step": round(dt2 * 1e3, 3),
                          "value": round(updates / dt2, 1),
                          "kernels_ms_per_step": {k: round(v[1] / max(1, args.steps // 2), 3)
                                                  for k, v in cmp[2].items()},
                          "speedup_of_headline": round(dt2 / dt, 3)}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
