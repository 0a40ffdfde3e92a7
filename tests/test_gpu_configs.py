"""GPU tests at the shapes of the large workloads, through the C ABI, against the FP64
oracle on seeded pair samples:

* the uneven batch at full size: all 64 generated jobs (200-8,000 samples, 1,000-64,000
  tips), each run weighted normalized on the FP32 striped queue and unweighted on the
  matrix-core queue, in one captured HIP graph, with the knobs the autotuner picks;
* the 113,000-sample workload's shape on a slice of its samples: a 500,000-tip random
  binary tree (999,998 branches), ~1,000 features per sample rarefied to 2,000, 16-bit
  count rows, weighted normalized FP32 striped computed as stripe ranges into an FP32
  condensed output.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle
from synth import batch_job_specs, build_jobs, make_rng, workload_problem

from helpers import condensed_index

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def uf():
    import paper_2005_05826_amd as uf
    return uf


def _pair_sample(n, m, seed):
    rng = make_rng(seed)
    i = rng.integers(0, n, size=m)
    j = rng.integers(0, n, size=m)
    keep = i != j
    return np.minimum(i[keep], j[keep]), np.maximum(i[keep], j[keep])


@pytest.mark.timeout(900)
def test_batch_64_jobs_full_size(uf):
    import torch
    specs = batch_job_specs(n_jobs=64)
    probs = build_jobs(specs)
    print(f"[batch64] generated {len(probs)} jobs, samples {min(p.n_samples for p in probs)}.."
          f"{max(p.n_samples for p in probs)}", flush=True)
    ctx = uf.Context(0)
    # the tuner picks the knobs of the largest job of each kind; jobs in the same size
    # bucket take them, the others keep the defaults
    big = int(np.argmax([p.n_samples * p.n_nodes for p in probs]))
    ctx.autotune([(probs[big], "weighted_normalized", "fp32"), (probs[big], "unweighted", "mfma_bf16x2")])
    t_wn = ctx.tuned("weighted_normalized", "fp32", probs[big].n_samples, probs[big].n_nodes)
    t_uw = ctx.tuned("unweighted", "mfma_bf16x2", probs[big].n_samples, probs[big].n_nodes)
    print(f"[batch64] tuned WN FP32 {t_wn}, UW MFMA {t_uw}", flush=True)
    assert t_wn is not None and t_wn["emb_batch"] <= 128 and t_uw is not None
    jobs, outs = [], []
    for p in probs:
        m = p.n_samples * (p.n_samples - 1) // 2
        for method, prec in (("weighted_normalized", "fp32"), ("unweighted", "mfma_bf16x2")):
            o = torch.full((m,), -1.0, dtype=torch.float64, device="cuda:0")
            outs.append(o)
            jobs.append(dict(problem=p, method=method, precision=prec, out=o))
    b = uf.Batch(ctx, jobs)
    b.capture()
    b.run()
    first = [o.clone() for o in outs]
    for o in outs:
        o.fill_(-3.0)
    b.run()                      # a second replay writes the same bits
    torch.cuda.synchronize()
    worst = {"weighted_normalized": 0.0, "unweighted": 0.0}
    for k, (job, o) in enumerate(zip(jobs, outs)):
        assert torch.equal(o, first[k]), f"job {k}: replays differ"
        p, method = job["problem"], job["method"]
        n = p.n_samples
        pi, pj = _pair_sample(n, 48, seed=4000 + k)
        want = oracle.problem_pairs(p, oracle.WEIGHTED_NORMALIZED if method == "weighted_normalized"
                                    else oracle.UNWEIGHTED, pi, pj)
        got = o[torch.from_numpy(condensed_index(n, pi, pj)).to(o.device)].cpu().numpy()
        err = float(np.abs(got - want).max())
        worst[method] = max(worst[method], err)
        assert err <= 1e-5, (k, n, method, err)
        assert float(o.min()) >= 0.0 and float(o.max()) <= 1.0, (k, "distances outside [0, 1]")
    print(f"[batch64] max_abs_err over sampled pairs: {worst}", flush=True)
    b.close()
    ctx.close()


@pytest.mark.timeout(600)
def test_binary_113000_shape_stripe_ranges_fp32(uf):
    import torch
    prob = workload_problem("binary_113000", n=3000)
    n, B = prob.n_samples, prob.n_nodes - 1
    assert B == 999_998
    totals = np.add.reduceat(prob.counts, prob.indptr[:-1])
    assert totals.max() <= 65535           # so the 16-bit count rows apply
    print(f"[binary_113000 shape] n={n} branches={B} nnz={prob.indices.size}", flush=True)
    ctx = uf.Context(0)
    plan = uf.Plan.from_problem(ctx, prob)
    S = n // 2
    out = torch.full((n * (n - 1) // 2,), -1.0, dtype=torch.float32, device="cuda:0")
    tuning = dict(den_mode=1, tile=2, count_width=2)
    # three uneven ranges that partition the stripes, the way shares of the full matrix run
    cuts = [0, 397, 1100, S]
    for a, c in zip(cuts[:-1], cuts[1:]):
        plan.distance_stripes(a, c, out, "weighted_normalized", "fp32", out_dtype="f32", tuning=tuning)
    torch.cuda.synchronize()
    assert float(out.min()) >= 0.0 and float(out.max()) <= 1.0   # every entry written, in range
    # pairs among 64 random samples (bounds the oracle's walk-up rows at 64 x 10^6)
    rng = make_rng(113)
    pool = np.sort(rng.choice(n, size=64, replace=False))
    a, c = _pair_sample(64, 400, seed=114)
    pi, pj = pool[a], pool[c]
    want = oracle.problem_pairs(prob, oracle.WEIGHTED_NORMALIZED, pi, pj)
    got = out[torch.from_numpy(condensed_index(n, pi, pj)).to(out.device)].double().cpu().numpy()
    err = np.abs(got - want)
    print(f"[binary_113000 shape] {pi.size} pairs max_abs_err={err.max():.3e} mean={err.mean():.3e}",
          flush=True)
    # FP32 path bar plus the FP32 output's own rounding (2^-25 for values in [0, 1])
    assert err.max() <= 1e-5 + 6e-8
    plan.close()
    ctx.close()
