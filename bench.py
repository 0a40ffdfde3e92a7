#!/usr/bin/env python3
"""Benchmark of the UniFrac hot path on one MI355X.  Prints one JSON line.

A step is one full distance matrix of the workload with the inputs already resident in HBM
(the plan was created before the timed region): embedding propagation, embedding
transform, accumulation (striped, or matrix-core for the unweighted form) and
normalize/condense, ending with the condensed matrix in device memory.

Workloads (--workload):
  striped (default)  4,096 samples, 32,768-tip random coalescent tree (65,534 branches),
                     ~800 features per sample, NegBin(10, 0.3) counts rarefied to 5,000;
                     weighted normalized.  Headline: the FP32 path with the denominator
                     from per-sample sums (den_mode 1) on tile shape 2; timed beside it on
                     the same inputs: plain FP64 (numerator and denominator stripes), FP32
                     in that same numerator-and-denominator form, and FP64 with the
                     per-sample denominator.
  binary_256         256 samples, 2,048-tip random binary tree, 95 % zeros, NegBin(20, 0.5)
                     counts rarefied to 1,000: plain FP64 unweighted and weighted normalized,
                     each timed on the GPU, and the oracle over the full matrix on all host
                     cores and on one thread.
  mfma               25,000 samples, 300,000-tip random binary tree, 1,500 Zipf(1.1)
                     presences per sample; unweighted on bf16 matrix cores (hi+lo split),
                     timed beside plain FP64 striped (about 28 s a step; --compare none
                     skips it).
  batch              64 jobs (samples uniform in 200..8,000, tips uniform in 1,000..64,000,
                     distributions of the 256-sample binary-tree case), each run weighted
                     normalized (FP32 striped)
                     and unweighted (matrix core): 128 jobs in one batch, replayed as a
                     captured HIP graph.
  large-uw           113,000 samples, 500,000-tip random binary tree: the full unweighted
                     matrix on the matrix cores.
  large-wn           the same inputs, weighted normalized FP32 striped: one GPU's share (a
                     contiguous 1/--share of the stripes) of a split of the full matrix, or
                     with --all-shares every share in turn (the full matrix).
  hbm                the striped kernel in its memory-bound regime: FP64 numerator and
                     denominator stripes, E = 8 branches per batch, on a 1 GB stripe state
                     (stripes [0, 2,560) of 25,000 samples; the distributions of the
                     striped workload on an 8,192-tip coalescent tree), so each batch streams 2 GB of state through
                     HBM; reported against the HBM roof.

The oracle (FP64 CPU) is timed on the host cores on a seeded sample of pairs as the CPU
baseline, and the same sample gives the max and mean absolute error of every GPU result.

The default run (the striped workload) also nests shorter records of the other targets in
its JSON line (--extras none leaves them out): the matrix-core workload against plain FP64
striped, the memory-bound regime against the HBM roof, the 256-sample FP64 workload with the
full-matrix oracle, the 64-job batch, the full unweighted matrix of the 113,000-sample
workload on the matrix cores, and the oracle over the full matrix of the striped workload
itself.
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

METRIC = "sample-pair·branch updates/s + full-matrix wall time, FP32/MFMA vs FP64 plain"
# Vector ALU peaks of one MI355X in lane-operations/s (one FMA, add or subtract on one lane
# is one operation): 256 CUs x 4 SIMDs x 2.4 GHz x lanes per clock, 32 lanes for FP32 and
# 16 for FP64, i.e. the datasheet's 157.3 and 78.6 TFLOP/s divided by 2 flops per FMA.
VALU_PEAK_TOPS = {"fp32": 256 * 4 * 32 * 2.4e9 / 1e12, "fp64": 256 * 4 * 16 * 2.4e9 / 1e12}
MFMA_BF16_PEAK_TFLOPS = 2500.0
HBM_PEAK_GBS = 8000.0
# Algorithmic VALU operations per pair-branch update of the striped kernel:
#   num += L*|u - v|  (sub, fma with |.|)   den += L*(u + v)  (add, fma)
OPS_PER_UPDATE = {0: 4, 1: 2}   # den_mode 0: both stripes; 1: numerator only

# HBM bytes per launch of the dominant kernel, from two rocprofv3 --pmc runs (FETCH_SIZE,
# then WRITE_SIZE, KiB per dispatch) of this script's default configuration of each
# workload, each scaled by what the same counter reads for a 1 GiB device copy
# (--copy-calibration: FETCH_SIZE reads 0.5 GiB, WRITE_SIZE 1 GiB, so x2.0 and x1.0).
# Keyed by workload and configuration; each entry records the SHA-256 of the sources it was
# measured on (the kernel file, and for the striped kernels also api.cpp, which sets their
# branch splits), and is reported as null once any of them has changed.
TRAFFIC = {
    "striped/4096x65534/fp32/den1/tile2/Edefault": {
        "src_sha256": "3689552ba0fdb464", "fetch": 40617685504, "write": 34360988416,
        "bytes": 74978673920, "profile": "profiles/k_stripe_fused_wn_fp32_4096x65534.md"},
    "mfma/25000x599998/k_chunk4096/variant0": {
        "src_sha256": "50b963d3b08070fc", "fetch": 214780838976, "write": 104080554176,
        "bytes": 318861393152, "profile": "profiles/k_mfma_gemm_uw_25000x599998.md"},
    "hbm/25000x16382/fp64/den0/tile2/E8": {
        "src_sha256": "3689552ba0fdb464", "fetch": 1723584764096, "write": 1990136533568,
        "bytes": 3713721297664, "profile": "profiles/k_stripe_fused_hbm_regime_fp64_25000x16382.md"},
}


def sources_sha(sources):
    """First 16 hex digits of the SHA-256 of the named csrc files, concatenated in order."""
    import hashlib
    h = hashlib.sha256()
    for source in sources:
        with open(os.path.join(ROOT, "paper_2005_05826_amd", "csrc", source), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def add_traffic(roofline, key, sources, launch_ms):
    """Sets roofline["traffic"] (HBM bytes per launch, or None) and, when known, the HBM
    bandwidth that traffic implies at the launch time measured here."""
    roofline["traffic"] = None
    ent = TRAFFIC.get(key)
    if not ent or sources_sha(sources) != ent["src_sha256"]:
        return
    roofline["traffic"] = ent["bytes"]
    gbs = ent["bytes"] / (launch_ms * 1e-3) / 1e9
    roofline["traffic_detail"] = {"fetch_bytes": ent["fetch"], "write_bytes": ent["write"],
                                  "hbm_GBs_at_measured_time": round(gbs, 1),
                                  "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                                  "profile": ent["profile"]}


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="striped",
                    choices=["striped", "binary_256", "mfma", "batch", "large-wn", "large-uw", "hbm"])
    ap.add_argument("--extras", default="all",
                    help="striped workload: nested records, comma-separated from "
                         "mfma,hbm,binary_256,full_oracle, or all / none")
    ap.add_argument("--share", type=int, default=8,
                    help="large-wn: compute 1/share of the stripes (one GPU's share)")
    ap.add_argument("--k-split", type=int, default=0,
                    help="striped: branch ranges over grid z (0 = automatic)")
    ap.add_argument("--count-width", type=int, default=2,
                    help="large-wn: bytes per embedding count (2 = 16-bit rows, resident; 4 = "
                         "int32 rows, 452 GB, generated batch by batch on the device)")
    ap.add_argument("--all-shares", action="store_true",
                    help="large-wn: compute every share in turn, i.e. the full matrix")
    ap.add_argument("--method", default=None)
    ap.add_argument("--precision", default=None)
    ap.add_argument("--compare", default=None,
                    help="precision timed for comparison ('' or none: no comparison runs)")
    ap.add_argument("--emb-batch", type=int, default=0)
    ap.add_argument("--den-mode", type=int, default=None,
                    help="striped headline: 1 = separable denominator (default), 0 = num+den stripes")
    ap.add_argument("--tile", type=int, default=None, help="striped headline tile shape (default 2)")
    ap.add_argument("--k-chunk", type=int, default=0)
    ap.add_argument("--variant", type=int, default=0,
                    help="matrix-core accumulation: 0 = chunk sums added into the output, 1 = FP64 registers")
    ap.add_argument("--n", type=int, default=None, help="override the sample count")
    ap.add_argument("--tips", type=int, default=None, help="override the tip count")
    ap.add_argument("--jobs", type=int, default=64, help="batch workload: number of jobs")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="target oracle CPU time")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy 3 times (HBM counter scale)")
    return ap.parse_args(argv)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def sample_pairs(rng, n, m):
    i = rng.integers(0, n, size=m)
    j = rng.integers(0, n, size=m)
    keep = i != j
    return np.minimum(i[keep], j[keep]), np.maximum(i[keep], j[keep])


def cond_index(n, i, j):
    return n * i - i * (i + 1) // 2 + (j - i - 1)


def oracle_sample(prob, method, seconds, seed, subset=None):
    """Time the oracle on a seeded pair sample sized for about `seconds` of CPU work.
    With `subset` the pairs are drawn among that many random samples (bounds the walk-up
    memory on very large workloads).  Returns (cpu_baseline dict, pi, pj, values)."""
    from oracle import oracle
    om = {"unweighted": oracle.UNWEIGHTED, "weighted_normalized": oracle.WEIGHTED_NORMALIZED,
          "weighted_unnormalized": oracle.WEIGHTED_UNNORMALIZED}[method]
    n = prob.n_samples
    B = prob.n_nodes - 1
    rng = np.random.Generator(np.random.Philox(seed))
    pool = np.sort(rng.choice(n, size=subset, replace=False)) if subset and subset < n else None

    def draw(m):
        if pool is None:
            return sample_pairs(rng, n, m)
        a, b = sample_pairs(rng, pool.size, m)
        return pool[a], pool[b]

    # Grow the sample until one run takes at least half the target: each next size is the
    # current one scaled by target / time, which cannot overshoot the target because the
    # fixed part of the cost (walking up the counts of the touched samples) stops growing.
    threads = oracle.max_threads()
    m = 64
    for _ in range(6):
        pi, pj = draw(m)
        t = time.perf_counter()
        want = oracle.problem_pairs(prob, om, pi, pj)
        cpu_s = time.perf_counter() - t
        if cpu_s >= 0.5 * seconds or m >= 2_000_000:
            break
        m = int(min(max(m * seconds / max(cpu_s, 1e-3), 2 * m), 2_000_000))
    log(f"oracle: {pi.size} sampled pairs on {threads} threads in {cpu_s:.1f} s")
    where = f" among {subset} random samples" if pool is not None else ""
    cpu = {"value": round(pi.size * B / cpu_s, 1), "unit": "pair-branch updates/s",
           "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
           "sample": f"{pi.size} seeded random pairs{where} ({method}, all {B} branches each), "
                     f"{cpu_s:.1f} s including walk-up counts of the touched samples",
           "seconds": round(cpu_s, 2)}
    # the per-core rate: one thread on the first pairs of the sample, about two seconds
    m1 = int(max(16, min(pi.size, pi.size * 2.0 / max(cpu_s * threads, 1e-3))))
    t = time.perf_counter()
    oracle.problem_pairs(prob, om, pi[:m1], pj[:m1], n_threads=1)
    t1 = time.perf_counter() - t
    cpu["one_thread"] = {"value": round(m1 * B / t1, 1), "pairs": m1, "seconds": round(t1, 2)}
    return cpu, pi, pj, want


def errors(out, n, pi, pj, want):
    import torch
    idx = torch.from_numpy(cond_index(n, pi, pj)).to(out.device)
    got = out[idx].double().cpu().numpy()
    e = np.abs(got - want)
    return {"max_abs": float(e.max()), "mean_abs": float(e.mean()), "pairs": int(pi.size)}


def timed_runs(plan, method, prec, tuning, out, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        plan.distance(method, prec, out=out, tuning=tuning, stream=stream)
    plan.set_profiling(True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        plan.distance(method, prec, out=out, tuning=tuning, stream=stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / steps
    prof = plan.profile()
    plan.set_profiling(False)
    return dt, prof


def end_to_end(uf, ctx, prob, method, prec, tuning, stream, runs):
    """Wall time from host inputs to host output: a new plan from the host tree and CSR table
    (validation, host preparation, uploads), the distances, and the condensed FP64 matrix
    copied back to host memory.  Best of `runs`."""
    import torch
    best = float("inf")
    for _ in range(runs):
        torch.cuda.synchronize()
        t = time.perf_counter()
        p2 = uf.Plan.from_problem(ctx, prob, stream=stream)
        host = p2.distance(method, prec, tuning=tuning, stream=stream)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t)
        p2.close()
        del host
    return {"ms": round(best * 1e3, 3), "runs": runs,
            "what": "host tree + CSR table -> new plan (validation, preparation, upload) -> "
                    "distances -> condensed FP64 matrix in host memory"}


def base_record(args, value, dt, dtype, config):
    return {"metric": METRIC, "value": round(value, 1), "unit": "pair-branch updates/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(dt * 1e3, 3), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config,
            "full_matrix_wall_ms": round(dt * 1e3, 3)}


def bench_striped(args):
    import torch
    import paper_2005_05826_amd as uf
    from synth import workload_problem
    method = args.method or "weighted_normalized"
    prec = args.precision or "fp32"
    compare = "fp64" if args.compare is None else args.compare
    if compare == "none":
        compare = ""
    over = {k: v for k, v in (("n", args.n), ("tips", args.tips)) if v}
    t0 = time.time()
    prob = workload_problem("coalescent_4096", **over)
    log(f"generated in {time.time() - t0:.1f}s: n={prob.n_samples} nodes={prob.n_nodes} nnz={prob.indices.size}")
    n, B = prob.n_samples, prob.n_nodes - 1
    n_pairs = n * (n - 1) // 2
    updates = n_pairs * B
    ctx = uf.Context(0)
    stream = torch.cuda.current_stream()
    plan = uf.Plan.from_problem(ctx, prob, stream=stream)
    den_mode = 1 if args.den_mode is None else args.den_mode
    tile = 2 if args.tile is None else args.tile
    tuning = dict(emb_batch=args.emb_batch, den_mode=den_mode, tile=tile, k_split=args.k_split)
    out = torch.empty(n_pairs, dtype=torch.float64, device="cuda:0")
    log(f"timing {prec} (den_mode {den_mode}, tile {tile}): {args.warmup} warmup + {args.steps} steps")
    dt, prof = timed_runs(plan, method, prec, tuning, out, args.steps, args.warmup, stream)
    log(f"{prec}: {dt * 1e3:.2f} ms/step; kernels {prof}")

    def stripe_roofline(p, tot_ms, steps, dm):
        ops = OPS_PER_UPDATE[dm] * updates
        achieved = ops / (tot_ms / steps * 1e-3) / 1e12
        return {"kernel": "k_stripe_fused", "bound": "alu", "achieved": round(achieved, 3),
                "peak": round(VALU_PEAK_TOPS[p], 2), "unit": "Tops/s",
                "frac": round(achieved / VALU_PEAK_TOPS[p], 4), "ops_per_update": OPS_PER_UPDATE[dm]}

    # the comparisons, each in its fastest measured tile shape: plain FP64 in the paper's
    # form (numerator and denominator stripes), the FP32 path in that same form, and FP64
    # with the per-sample denominator (the headline's form, so that the precision alone
    # differs)
    others = {}
    if compare:
        others["compare"] = (compare, dict(emb_batch=args.emb_batch, den_mode=0, tile=2))
    if compare and prec == "fp32" and (den_mode, tile) != (0, 2):
        others["fp32_num_den"] = ("fp32", dict(emb_batch=args.emb_batch, den_mode=0, tile=2))
    if compare == "fp64" and prec == "fp32" and den_mode == 1:
        others["fp64_per_sample_den"] = ("fp64", dict(emb_batch=args.emb_batch, den_mode=1, tile=0))
    outs = {}
    for name, (p2, tun2) in others.items():
        o2 = torch.empty_like(out)
        steps2 = max(1, args.steps // 2)
        d2, pr2 = timed_runs(plan, method, p2, tun2, o2, steps2, 1, stream)
        log(f"{name} {p2} {tun2}: {d2 * 1e3:.2f} ms/step; kernels {pr2}")
        rec = {"precision": p2, "den_mode": tun2["den_mode"], "tile": tun2["tile"],
               "ms_per_step": round(d2 * 1e3, 3), "value": round(updates / d2, 1),
               "kernels_ms_per_step": {k: round(v[1] / steps2, 3) for k, v in pr2.items()},
               "headline_speedup": round(d2 / dt, 3)}
        l2, t2 = pr2.get("stripe", (0, 0.0))
        if l2 and p2 in VALU_PEAK_TOPS:
            rec["roofline"] = stripe_roofline(p2, t2, steps2, tun2["den_mode"])
        if name == "compare":   # the paper's form, host to host
            rec["end_to_end"] = end_to_end(uf, ctx, prob, method, p2, tun2, stream, 1)
        outs[name] = (o2, rec)

    launches, total_ms = prof.get("stripe", (0, 0.0))
    roofline = None
    if launches:
        key = f"striped/{n}x{B}/{prec}/den{den_mode}/tile{tile}/E{args.emb_batch or 'default'}"
        roofline = stripe_roofline(prec, total_ms, args.steps, den_mode)
        roofline.update({"launches_per_step": launches // args.steps,
                         "avg_launch_ms": round(total_ms / launches, 4)})
        add_traffic(roofline, key, ("k_stripe.hip", "api.cpp"), total_ms / launches)
    res = base_record(args, updates / dt, dt, "f32" if prec == "fp32" else "f64",
                      {"workload": f"{method.replace('_', '-')} striped UniFrac, {n} samples, "
                                   f"coalescent tree with {(prob.n_nodes + 1) // 2} tips ({B} branches)",
                       "n_samples": n, "branches": B, "levels": plan.info.n_levels,
                       "nnz": int(plan.info.nnz), "method": method, "precision": prec,
                       "emb_batch": args.emb_batch or "default", "den_mode": den_mode,
                       "denominator": "per-sample sums" if den_mode else "stripes",
                       "tile": tile})
    res["kernels_ms_per_step"] = {k: round(v[1] / args.steps, 3) for k, v in prof.items()}
    res["roofline"] = roofline
    for name, (_, rec) in outs.items():
        res[name] = rec
    res["end_to_end"] = end_to_end(uf, ctx, prob, method, prec, tuning, stream, 3)
    log(f"end to end: {res['end_to_end']['ms']:.1f} ms")
    if not args.no_cpu:
        cpu, pi, pj, want = oracle_sample(prob, method, args.cpu_seconds, 20050526 + 99)
        res["cpu_baseline"] = cpu
        res["error_vs_oracle"] = {prec: errors(out, n, pi, pj, want)}
        for name, (o2, rec) in outs.items():
            res["error_vs_oracle"][name] = errors(o2, n, pi, pj, want)
    if "compare" in outs and n >= 3:
        r, _, _ = uf.mantel(ctx, out, outs["compare"][0], n)
        res["mantel_r2_vs_compare"] = round(r * r, 12)
    if getattr(args, "full_oracle", False):
        # every pair of the matrix against the oracle (about a minute and a half on 16 cores)
        from oracle import oracle
        om = {"unweighted": oracle.UNWEIGHTED, "weighted_normalized": oracle.WEIGHTED_NORMALIZED,
              "weighted_unnormalized": oracle.WEIGHTED_UNNORMALIZED}[method]
        log(f"oracle over the full matrix ({n_pairs} pairs x {B} branches)")
        t = time.perf_counter()
        want = oracle.problem_condensed(prob, om)
        cpu_s = time.perf_counter() - t
        log(f"full-matrix oracle: {cpu_s:.1f} s")

        def full_err(o):
            e = np.abs(o.double().cpu().numpy() - want)
            return {"max_abs": float(e.max()), "mean_abs": float(e.mean()), "pairs": int(e.size)}

        res["full_matrix_check"] = {
            "pairs": n_pairs, "oracle_seconds": round(cpu_s, 2), "oracle_threads": oracle.max_threads(),
            "oracle_rate": round(updates / cpu_s, 1), "unit": "pair-branch updates/s",
            "error_vs_oracle": dict({prec: full_err(out)}, **{k: full_err(o2) for k, (o2, _) in outs.items()})}
    return res


def bench_binary_256(args):
    """256 samples, 2,048-tip random binary tree: plain FP64 unweighted and weighted
    normalized (the default knobs) on the GPU, and the oracle over the full matrix on all
    host cores and on one thread."""
    import torch
    import paper_2005_05826_amd as uf
    from oracle import oracle
    from synth import workload_problem
    over = {k: v for k, v in (("n", args.n), ("tips", args.tips)) if v}
    prob = workload_problem("binary_256", **over)
    n, B = prob.n_samples, prob.n_nodes - 1
    n_pairs = n * (n - 1) // 2
    updates = n_pairs * B
    ctx = uf.Context(0)
    stream = torch.cuda.current_stream()
    plan = uf.Plan.from_problem(ctx, prob, stream=stream)
    om = {"unweighted": oracle.UNWEIGHTED, "weighted_normalized": oracle.WEIGHTED_NORMALIZED}
    per, outs = {}, {}
    for method in om:
        out = torch.empty(n_pairs, dtype=torch.float64, device="cuda:0")
        dt, prof = timed_runs(plan, method, "fp64", None, out, args.steps, args.warmup, stream)
        per[method] = {"ms_per_step": round(dt * 1e3, 4), "value": round(updates / dt, 1),
                       "kernels_ms_per_step": {k: round(v[1] / args.steps, 4) for k, v in prof.items()}}
        outs[method] = out
        log(f"binary_256 {method} fp64: {dt * 1e3:.3f} ms/step")
    # the step time from the same calls without the per-launch profiling events (HIP event
    # pairs around every launch class, which weigh on a call this short); the profiled run
    # above gives the kernel breakdown and the roofline
    for method in om:
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            plan.distance(method, "fp64", out=outs[method], stream=stream)
        torch.cuda.synchronize()
        dt_m = (time.perf_counter() - t) / args.steps
        per[method]["profiled_ms_per_step"] = per[method]["ms_per_step"]
        per[method]["ms_per_step"] = round(dt_m * 1e3, 4)
        per[method]["value"] = round(updates / dt_m, 1)
        log(f"binary_256 {method} fp64 without profiling events: {dt_m * 1e3:.3f} ms/step")
    dt = sum(v["ms_per_step"] for v in per.values()) * 1e-3
    res = base_record(args, 2 * updates / dt, dt, "f64",
                      {"workload": f"unweighted + weighted-normalized plain FP64 striped UniFrac, {n} "
                                   f"samples, random binary tree with {(prob.n_nodes + 1) // 2} tips "
                                   f"({B} branches)", "n_samples": n, "branches": B, "precision": "fp64"})
    res["methods"] = per
    stripe_ms = sum(v["kernels_ms_per_step"].get("stripe", 0.0) for v in per.values())
    if stripe_ms > 0:
        ach = OPS_PER_UPDATE[0] * 2 * updates / (stripe_ms * 1e-3) / 1e12
        res["roofline"] = {"kernel": "k_stripe_fused", "bound": "alu", "achieved": round(ach, 3),
                           "peak": round(VALU_PEAK_TOPS["fp64"], 2), "unit": "Tops/s",
                           "frac": round(ach / VALU_PEAK_TOPS["fp64"], 4), "traffic": None,
                           "note": "a 256-sample matrix fills a fraction of the device: launch "
                                   "and latency bound"}
    if not args.no_cpu:
        threads = oracle.max_threads()
        errs, t_all, t_one = {}, 0.0, 0.0
        for method, m in om.items():
            t = time.perf_counter()
            want = oracle.problem_condensed(prob, m)
            t_all += time.perf_counter() - t
            t = time.perf_counter()
            oracle.problem_condensed(prob, m, n_threads=1)
            t_one += time.perf_counter() - t
            e = np.abs(outs[method].cpu().numpy() - want)
            errs[method] = {"max_abs": float(e.max()), "mean_abs": float(e.mean()), "pairs": int(e.size)}
        res["cpu_baseline"] = {"value": round(2 * updates / t_all, 1), "unit": "pair-branch updates/s",
                               "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
                               "sample": f"the full matrix ({n_pairs} pairs x {B} branches), both methods",
                               "seconds": round(t_all, 3),
                               "one_thread": {"value": round(2 * updates / t_one, 1), "seconds": round(t_one, 3)}}
        res["error_vs_oracle"] = errs
    plan.close()
    return res


def bench_mfma(args):
    import torch
    import paper_2005_05826_amd as uf
    from synth import workload_problem
    # the matrix-core path against plain FP64 striped (numerator and denominator stripes)
    # on the same plan, unless --compare none
    compare = "fp64" if args.compare is None else ("" if args.compare == "none" else args.compare)
    over = {k: v for k, v in (("n", args.n), ("tips", args.tips)) if v}
    t0 = time.time()
    prob = workload_problem("zipf_25000", **over)
    log(f"generated in {time.time() - t0:.1f}s: n={prob.n_samples} nodes={prob.n_nodes}")
    n, B = prob.n_samples, prob.n_nodes - 1
    n_pairs = n * (n - 1) // 2
    updates = n_pairs * B
    ctx = uf.Context(0)
    stream = torch.cuda.current_stream()
    plan = uf.Plan.from_problem(ctx, prob, stream=stream)
    tuning = dict(k_chunk=args.k_chunk, variant=args.variant)
    out = torch.empty(n_pairs, dtype=torch.float64, device="cuda:0")
    dt, prof = timed_runs(plan, "unweighted", "mfma_bf16x2", tuning, out, args.steps, args.warmup, stream)
    log(f"mfma: {dt * 1e3:.2f} ms/step; kernels {prof}")
    launches, total_ms = prof.get("mfma", (0, 0.0))
    flops = 4.0 * B * n * (n + 1) / 2          # hi and lo, 2 flops each, upper triangle; padding not counted
    achieved = flops / (total_ms / args.steps * 1e-3) / 1e12 if launches else 0.0
    res = base_record(args, updates / dt, dt, "bf16",
                      {"workload": f"unweighted UniFrac on bf16 matrix cores, {n} samples, random "
                                   f"binary tree with {(prob.n_nodes + 1) // 2} tips ({B} branches)",
                       "n_samples": n, "branches": B, "method": "unweighted",
                       "precision": "mfma_bf16x2", "k_chunk": args.k_chunk or 4096,
                       "variant": args.variant})
    res["kernels_ms_per_step"] = {k: round(v[1] / args.steps, 3) for k, v in prof.items()}
    key = f"mfma/{n}x{B}/k_chunk{args.k_chunk or 4096}/variant{args.variant}"
    res["roofline"] = {"kernel": "k_mfma_gemm", "bound": "mfma", "achieved": round(achieved, 2),
                       "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": round(achieved / MFMA_BF16_PEAK_TFLOPS, 4),
                       "avg_launch_ms": round(total_ms / max(1, launches), 3)}
    if launches:
        add_traffic(res["roofline"], key, ("k_mfma.hip",), total_ms / launches)
    if compare:
        out2 = torch.empty_like(out)
        dt2, prof2 = timed_runs(plan, "unweighted", compare, dict(den_mode=0, tile=2), out2, 1, 0, stream)
        log(f"compare {compare}: {dt2 * 1e3:.1f} ms")
        res["compare"] = {"precision": compare, "den_mode": 0, "tile": 2, "ms_per_step": round(dt2 * 1e3, 3),
                          "value": round(updates / dt2, 1), "speedup_of_headline": round(dt2 / dt, 3),
                          "kernels_ms_per_step": {k: round(v[1], 3) for k, v in prof2.items()}}
    res["end_to_end"] = end_to_end(uf, ctx, prob, "unweighted", "mfma_bf16x2", tuning, stream, 1)
    log(f"end to end: {res['end_to_end']['ms']:.1f} ms")
    if not args.no_cpu:
        cpu, pi, pj, want = oracle_sample(prob, "unweighted", args.cpu_seconds, 20050526 + 98, subset=400)
        res["cpu_baseline"] = cpu
        res["error_vs_oracle"] = {"mfma_bf16x2": errors(out, n, pi, pj, want)}
        if compare:
            res["error_vs_oracle"][compare] = errors(out2, n, pi, pj, want)
    return res


def bench_batch(args):
    import torch
    import paper_2005_05826_amd as uf
    from synth import batch_job_specs, build_jobs
    t0 = time.time()
    specs = batch_job_specs(n_jobs=args.jobs)
    probs = build_jobs(specs)
    log(f"generated {len(probs)} jobs in {time.time() - t0:.1f}s")
    ctx = uf.Context(0)
    jobs, outs = [], []
    for p in probs:
        m = p.n_samples * (p.n_samples - 1) // 2
        for method, prec in (("weighted_normalized", "fp32"), ("unweighted", "mfma_bf16x2")):
            o = torch.empty(max(1, m), dtype=torch.float64, device="cuda:0")
            outs.append(o)
            jobs.append(dict(problem=p, method=method, precision=prec, out=o))
    # knobs: the autotuner times tile shape x batch depth (and the MFMA chunk) on the
    # largest job, unless they are given on the command line
    tuning = dict(emb_batch=args.emb_batch, tile=2 if args.tile is None else args.tile,
                  den_mode=1 if args.den_mode is None else args.den_mode, k_chunk=args.k_chunk,
                  variant=args.variant)
    tuned = {}
    if not args.emb_batch:
        big = int(np.argmax([p.n_samples * p.n_nodes for p in probs]))
        tplan = uf.Plan.from_problem(ctx, probs[big])
        best, ms = tplan.autotune("weighted_normalized", "fp32", base=dict(den_mode=tuning["den_mode"]), reps=1)
        bestm, msm = tplan.autotune("unweighted", "mfma_bf16x2", reps=1)
        tuning.update(emb_batch=best["emb_batch"], tile=best["tile"], k_chunk=bestm["k_chunk"],
                      variant=bestm["variant"])
        tuned = {"striped": best, "striped_ms": round(ms, 3), "mfma": bestm, "mfma_ms": round(msm, 3),
                 "on_job": {"n_samples": probs[big].n_samples, "branches": probs[big].n_nodes - 1}}
        tplan.close()
        log(f"autotuned: {tuned}")
    b = uf.Batch(ctx, jobs, tuning=tuning)
    for _ in range(max(1, args.warmup)):
        b.run()
    t = time.perf_counter()
    b.run()
    eager = time.perf_counter() - t
    b.capture()
    b.set_profiling(True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        b.run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / args.steps
    prof = b.profile()
    updates = sum(p.n_samples * (p.n_samples - 1) // 2 * (p.n_nodes - 1) for p in probs) * 2
    res = base_record(args, updates / dt, dt, "f32+bf16",
                      {"workload": f"{len(probs)} uneven jobs x (weighted normalized FP32 striped + "
                                   f"unweighted bf16 matrix core) in one captured HIP graph",
                       "jobs": len(jobs), "samples_range": [min(p.n_samples for p in probs),
                                                            max(p.n_samples for p in probs)],
                       "tips_range": [min((p.n_nodes + 1) // 2 for p in probs),
                                      max((p.n_nodes + 1) // 2 for p in probs)]})
    res["eager_run_ms"] = round(eager * 1e3, 3)
    # one graph holds both kernel families, so the roofline is the time the work would take
    # at the two peaks (FP32 VALU for the weighted updates, bf16 matrix cores for the
    # unweighted products) over the measured time
    wn_ops = OPS_PER_UPDATE[tuning["den_mode"]] * updates // 2
    uw_flops = sum(4 * (p.n_nodes - 1) * p.n_samples * (p.n_samples + 1) // 2 for p in probs)
    t_peak = wn_ops / (VALU_PEAK_TOPS["fp32"] * 1e12) + uw_flops / (MFMA_BF16_PEAK_TFLOPS * 1e12)
    res["roofline"] = {"kernel": "k_stripe_queue + k_mfma_queue (one graph)", "bound": "alu",
                       "achieved": round(t_peak * 1e3, 3), "peak": round(dt * 1e3, 3),
                       "unit": "ms at peak vs ms measured", "frac": round(t_peak / dt, 4),
                       "wn_fp32_ops": wn_ops, "uw_bf16_flops": uw_flops, "traffic": None}
    res["tuning"] = {"used": tuning, "autotune": tuned}
    res["kernels_ms_per_step"] = {k: round(v[1] / args.steps, 3) for k, v in prof.items()}
    if not args.no_cpu:
        # error sample on the largest job, both methods
        big = int(np.argmax([p.n_samples * p.n_nodes for p in probs]))
        p = probs[big]
        cpu, pi, pj, want = oracle_sample(p, "weighted_normalized", args.cpu_seconds / 2, 20050526 + 97)
        res["cpu_baseline"] = cpu
        res["error_vs_oracle"] = {"wn_fp32_largest_job": errors(outs[2 * big], p.n_samples, pi, pj, want)}
        _, pi, pj, want = oracle_sample(p, "unweighted", args.cpu_seconds / 4, 20050526 + 96)
        res["error_vs_oracle"]["uw_mfma_largest_job"] = errors(outs[2 * big + 1], p.n_samples, pi, pj, want)
    b.close()
    ctx.close()
    return res


def bench_large(args, part):
    """The 113,000-sample workload (500,000-tip random binary tree, ~1,000 features per
    sample, NegBin(8, 0.3) rarefied to 2,000).  large-uw: the full unweighted matrix on the
    matrix cores (presence bits 14 GB, FP64 shared lengths in the output).  large-wn: one
    GPU's share of an N-way split of the weighted normalized FP32 striped computation, a
    contiguous stripe range of 1/share of the stripes, with 16-bit count rows (226 GB);
    the condensed output (FP32, 25.5 GB) stays resident."""
    import torch
    import paper_2005_05826_amd as uf
    from synth import workload_problem
    over = {k: v for k, v in (("n", args.n), ("tips", args.tips)) if v}
    t0 = time.time()
    prob = workload_problem("binary_113000", **over)
    log(f"generated in {time.time() - t0:.1f}s: n={prob.n_samples} nodes={prob.n_nodes} nnz={prob.indices.size}")
    n, B = prob.n_samples, prob.n_nodes - 1
    n_pairs = n * (n - 1) // 2
    ctx = uf.Context(0)
    stream = torch.cuda.current_stream()
    plan = uf.Plan.from_problem(ctx, prob, stream=stream)
    S = n // 2
    if part == "uw":
        out = torch.empty(n_pairs, dtype=torch.float64, device="cuda:0")
        dt, prof = timed_runs(plan, "unweighted", "mfma_bf16x2", dict(k_chunk=args.k_chunk, variant=args.variant), out,
                              args.steps, args.warmup, stream)
        launches, total_ms = prof.get("mfma", (0, 0.0))
        flops = 4.0 * B * n * (n + 1) / 2
        achieved = flops / (total_ms / args.steps * 1e-3) / 1e12 if launches else 0.0
        res = base_record(args, n_pairs * B / dt, dt, "bf16",
                          {"workload": f"unweighted UniFrac on bf16 matrix cores, {n} samples, random "
                                       f"binary tree with {(prob.n_nodes + 1) // 2} tips ({B} branches)",
                           "n_samples": n, "branches": B, "precision": "mfma_bf16x2"})
        res["roofline"] = {"kernel": "k_mfma_gemm", "bound": "mfma", "achieved": round(achieved, 2),
                           "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "frac": round(achieved / MFMA_BF16_PEAK_TFLOPS, 4), "traffic": None}
        method = "unweighted"
    else:
        chunk = (S + args.share - 1) // args.share
        # the stripe ranges one step computes: one share, or all of them in turn (the full
        # matrix; the count rows stay resident and each range's state is freed after it)
        ranges = [(g * chunk, min(S, (g + 1) * chunk)) for g in range(args.share)] \
            if args.all_shares else [(0, chunk)]
        s0, s1 = ranges[0][0], ranges[-1][1]
        out = torch.empty(n_pairs, dtype=torch.float32, device="cuda:0")
        den_mode = 1 if args.den_mode is None else args.den_mode
        tuning = dict(emb_batch=args.emb_batch, den_mode=den_mode,
                      tile=2 if args.tile is None else args.tile, count_width=args.count_width)

        def step():
            for a, b in ranges:
                plan.distance_stripes(a, b, out, "weighted_normalized", "fp32", out_dtype="f32",
                                      tuning=tuning, stream=stream)
                if len(ranges) > 1:
                    torch.cuda.synchronize()
                    log(f"stripes [{a}, {b}) done")

        for _ in range(args.warmup):
            step()
        plan.set_profiling(True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / args.steps
        prof = plan.profile()
        plan.set_profiling(False)
        # pair-branch updates: every pair once for the full matrix (the last stripe of an
        # even n holds n/2 pairs), else n per stripe of the range
        updates = n_pairs * B if s1 == S else (s1 - s0) * n * B
        launches, total_ms = prof.get("stripe", (0, 0.0))
        achieved = OPS_PER_UPDATE[den_mode] * updates / (total_ms / args.steps * 1e-3) / 1e12 if launches else 0.0
        res = base_record(args, updates / dt, dt, "f32",
                          {"workload": f"weighted-normalized FP32 striped UniFrac, {n} samples, random "
                                       f"binary tree with {(prob.n_nodes + 1) // 2} tips ({B} branches), "
                                       + (f"full matrix, stripes in {len(ranges)} ranges of {chunk}"
                                          if len(ranges) > 1 else
                                          f"stripes [{s0}, {s1}) = 1/{args.share} of {S}"),
                           "n_samples": n, "branches": B, "stripes": [s0, s1],
                           "precision": "fp32", "count_width": args.count_width,
                           "count_rows": "generated per batch" if prof.get("generate") else "resident"})
        res["roofline"] = {"kernel": "k_stripe_fused", "bound": "alu", "achieved": round(achieved, 3),
                           "peak": round(VALU_PEAK_TOPS["fp32"], 2), "unit": "Tops/s",
                           "frac": round(achieved / VALU_PEAK_TOPS["fp32"], 4), "traffic": None}
        method = "weighted_normalized"
    res["kernels_ms_per_step"] = {k: round(v[1] / args.steps, 3) for k, v in prof.items()}
    if not args.no_cpu:
        cpu, pi, pj, want = oracle_sample(prob, method, args.cpu_seconds, 20050526 + 95, subset=300)
        res["cpu_baseline"] = cpu
        if part == "wn":   # only pairs held by the computed stripes
            d = pj - pi
            st = np.where(d <= S, d - 1, n - d - 1)
            keep = (st >= s0) & (st < s1)
            pi, pj, want = pi[keep], pj[keep], want[keep]
        if pi.size:
            res["error_vs_oracle"] = {method: errors(out, n, pi, pj, want)}
    plan.close()
    ctx.close()
    return res


def bench_hbm(args):
    import torch
    import paper_2005_05826_amd as uf
    from synth import workload_problem
    n = args.n or 25000
    prob = workload_problem("coalescent_4096", n=n, tips=args.tips or 8192, k=800, seed=20050526 + 7)
    n, B = prob.n_samples, prob.n_nodes - 1
    s0, s1 = 0, 2560
    E = args.emb_batch or 8
    ctx = uf.Context(0)
    stream = torch.cuda.current_stream()
    plan = uf.Plan.from_problem(ctx, prob, stream=stream)
    out = torch.empty(n * (n - 1) // 2, dtype=torch.float64, device="cuda:0")
    # shape 2 (three work-groups per CU) keeps more memory requests in flight than shape 0:
    # 83-84 % against 77 % of the HBM peak
    tile = 2 if args.tile is None else args.tile
    tuning = dict(emb_batch=E, den_mode=0, tile=tile, k_split=1)
    for _ in range(args.warmup):
        plan.distance_stripes(s0, s1, out, "weighted_normalized", "fp64", tuning=tuning, stream=stream)
    plan.set_profiling(True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        plan.distance_stripes(s0, s1, out, "weighted_normalized", "fp64", tuning=tuning, stream=stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / args.steps
    prof = plan.profile()
    plan.set_profiling(False)
    launches, total_ms = prof.get("stripe", (0, 0.0))
    # FP64 numerator-and-denominator tiles (samples x stripes per lane) of shapes 0, 1, 2;
    # a work-group covers 64 x TKT samples and 4 x TST stripes, and the state rows are padded
    # to those tiles
    tkt, tst = {0: (4, 8), 1: (2, 12), 2: (2, 8)}[tile]
    sstride = -(-n // (64 * tkt)) * (64 * tkt)
    rows = -(-(s1 - s0) // (4 * tst)) * (4 * tst)
    batches = -(-B // E)
    state = rows * sstride * 8 * 2                      # num + den, FP64
    alg = batches * state * 2 + B * sstride * 2         # read + write per batch, counts once
    gbs = alg / (total_ms / max(1, launches) * 1e-3) / 1e9 if launches else 0.0
    updates = (s1 - s0) * n * B
    res = base_record(args, updates / dt, dt, "f64",
                      {"workload": f"memory-bound striped regime: weighted normalized FP64 "
                                   f"(numerator and denominator stripes), E = {E}, stripes "
                                   f"[{s0}, {s1}) of {n // 2} for {n} samples, coalescent tree "
                                   f"with {(prob.n_nodes + 1) // 2} tips ({B} branches)",
                       "n_samples": n, "branches": B, "stripes": [s0, s1], "emb_batch": E,
                       "tile": tile, "state_bytes": state})
    res["kernels_ms_per_step"] = {k: round(v[1] / args.steps, 3) for k, v in prof.items()}
    res["roofline"] = {"kernel": "k_stripe_fused", "bound": "hbm", "achieved": round(gbs, 1),
                       "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                       "algorithmic_bytes": alg,
                       "avg_launch_ms": round(total_ms / max(1, launches), 3)}
    if launches:
        add_traffic(res["roofline"], f"hbm/{n}x{B}/fp64/den0/tile{tile}/E{E}", ("k_stripe.hip", "api.cpp"),
                    total_ms / launches)
    if not args.no_cpu:
        cpu, pi, pj, want = oracle_sample(prob, "weighted_normalized", args.cpu_seconds, 20050526 + 94,
                                          subset=600)
        res["cpu_baseline"] = cpu
        d = pj - pi
        st = np.where(d <= n // 2, d - 1, n - d - 1)
        keep = (st >= s0) & (st < s1)
        if keep.any():
            res["error_vs_oracle"] = {"fp64": errors(out, n, pi[keep], pj[keep], want[keep])}
    return res


def _sig(x, n=3):
    return float(f"{x:.{n}g}") if isinstance(x, float) else x


def compact_target(rec):
    """The figures of a nested target record (its own run prints the full record): time,
    roofline, comparison, kernel times, CPU baseline and errors, without the descriptive
    strings, so that the one JSON line stays a few kilobytes long."""
    if "error" in rec and "value" not in rec:
        return rec
    out = {k: rec[k] for k in ("value", "ms_per_step", "dtype", "eager_run_ms", "wall_s") if k in rec}
    if "value" in out:
        out["value"] = _sig(out["value"], 5)
    c = rec.get("config", {})
    out["config"] = {k: c[k] for k in ("n_samples", "branches", "jobs", "stripes", "precision", "emb_batch")
                     if k in c}
    if "roofline" in rec:
        r = rec["roofline"]
        out["roofline"] = {k: r[k] for k in ("kernel", "bound", "achieved", "peak", "unit", "frac",
                                             "algorithmic_bytes", "traffic") if k in r}
    if "compare" in rec:
        cm = rec["compare"]
        out["compare"] = {k: cm[k] for k in ("precision", "ms_per_step", "speedup_of_headline") if k in cm}
    if "methods" in rec:
        out["methods_ms_per_step"] = {m: v["ms_per_step"] for m, v in rec["methods"].items()}
    if "kernels_ms_per_step" in rec:
        out["kernels_ms_per_step"] = rec["kernels_ms_per_step"]
    if "end_to_end" in rec:
        out["end_to_end_ms"] = rec["end_to_end"]["ms"]
    if "tuning" in rec:
        out["tuning"] = rec["tuning"].get("used")
    if "cpu_baseline" in rec:
        cb = rec["cpu_baseline"]
        out["cpu_baseline"] = {k: _sig(cb[k], 4) for k in ("value", "cores", "seconds") if k in cb}
        if "one_thread" in cb:
            out["cpu_baseline"]["one_thread_value"] = _sig(cb["one_thread"]["value"], 4)
    if "error_vs_oracle" in rec:
        out["error_vs_oracle"] = {m: {k: _sig(v) for k, v in e.items()} for m, e in rec["error_vs_oracle"].items()}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
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
    extras = set()
    if args.workload == "striped" and args.extras != "none":
        extras = {"mfma", "hbm", "binary_256", "batch", "large_uw", "full_oracle"} if args.extras == "all" \
            else set(x for x in args.extras.split(",") if x)
    args.full_oracle = "full_oracle" in extras and not args.no_cpu
    if args.workload.startswith("large"):
        res = bench_large(args, args.workload.split("-")[1])
    else:
        res = {"striped": bench_striped, "binary_256": bench_binary_256, "mfma": bench_mfma,
               "batch": bench_batch, "hbm": bench_hbm}[args.workload](args)
    if extras - {"full_oracle"}:
        # the other targets, each on its default configuration with a few steps
        res["targets"] = {}
        runs = [("mfma", bench_mfma, ["--workload", "mfma", "--steps", "3", "--warmup", "1",
                                      "--cpu-seconds", "10"]),
                ("hbm", bench_hbm, ["--workload", "hbm", "--steps", "3", "--warmup", "1",
                                    "--cpu-seconds", "5"]),
                ("binary_256", bench_binary_256, ["--workload", "binary_256", "--steps", "20",
                                                  "--warmup", "3"]),
                ("batch", bench_batch, ["--workload", "batch", "--steps", "2", "--warmup", "1",
                                        "--cpu-seconds", "6"]),
                ("large_uw", lambda a: bench_large(a, "uw"), ["--workload", "large-uw", "--steps", "1",
                                                              "--warmup", "0", "--cpu-seconds", "6"])]
        for name, fn, argv in runs:
            if name not in extras:
                continue
            sub = parse(argv + (["--no-cpu"] if args.no_cpu else []))
            log(f"target {name}: {' '.join(argv)}")
            t = time.time()
            try:
                rec = fn(sub)
            except Exception as e:  # a failing extra must not lose the headline line
                rec = {"error": f"{type(e).__name__}: {e}"}
            for k in ("metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "data"):
                rec.pop(k, None)
            rec["wall_s"] = round(time.time() - t, 1)
            res["targets"][name] = compact_target(rec)
            torch.cuda.empty_cache()
    if res.get("targets"):
        for r in (res, res.get("compare", {})):   # described in the module docstring
            if isinstance(r.get("end_to_end"), dict):
                r["end_to_end"].pop("what", None)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
