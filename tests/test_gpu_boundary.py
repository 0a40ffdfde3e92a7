"""GPU tests of the boundary calls that the distance path exposes beside plans: the
one-shot embedding-count dump, the context-level autotuner and its cache, and batches
with host outputs and per-job tuned knobs.  Everything goes through the C ABI and is
checked against the FP64 CPU oracle."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle
from synth import batch_job_specs, build_job, workload_problem

from helpers import tiny_problem

pytestmark = pytest.mark.gpu

UW, WN, WU = "unweighted", "weighted_normalized", "weighted_unnormalized"
OMETHOD = {UW: oracle.UNWEIGHTED, WN: oracle.WEIGHTED_NORMALIZED, WU: oracle.WEIGHTED_UNNORMALIZED}
TOL = {"fp64": 1e-12, "fp32": 1e-5, "mfma_bf16x2": 1e-5}


@pytest.fixture(scope="module")
def uf():
    import paper_2005_05826_amd as uf
    return uf


@pytest.fixture(scope="module")
def ctx(uf):
    return uf.Context(0)


COUNT_CASES = {
    "tiny": lambda: tiny_problem(41, max_nodes=30, max_samples=7),
    "binary_256": lambda: workload_problem("binary_256"),
    "coalescent_333": lambda: workload_problem("coalescent_4096", n=333, tips=2500, k=200, depth=900, seed=5),
}


@pytest.mark.parametrize("case", sorted(COUNT_CASES))
def test_debug_embedding_counts_bit_exact(uf, ctx, case):
    prob = COUNT_CASES[case]()
    got = ctx.debug_embedding_counts(prob)                  # [n_nodes - 1][n_samples]
    want = oracle.problem_counts(prob)                      # [n_samples][n_nodes]
    root = int(np.flatnonzero(np.asarray(prob.parent) < 0)[0])
    keep = np.array([v for v in range(prob.n_nodes) if v != root])
    assert got.shape == (prob.n_nodes - 1, prob.n_samples)
    np.testing.assert_array_equal(got, want[:, keep].T)


def test_debug_embedding_counts_rejects_bad_input(uf, ctx):
    prob = tiny_problem(42)
    prob.counts = prob.counts.copy()
    prob.counts[0] = -1
    with pytest.raises(uf.UniFracError) as ei:
        ctx.debug_embedding_counts(prob)
    assert ei.value.status_name == "UF_E_TABLE"


def test_context_autotune_stores_and_uses_knobs(uf):
    ctx = uf.Context(0)       # a fresh context: empty tune cache
    prob = workload_problem("coalescent_4096", n=700, tips=4000, k=300, depth=1500, seed=77)
    n, nodes = prob.n_samples, prob.n_nodes
    assert ctx.tuned(WN, "fp32", n, nodes) is None
    ctx.autotune([(prob, WN, "fp32"), (prob, UW, "mfma_bf16x2"), (prob, UW, "fp64")])
    plan = uf.Plan.from_problem(ctx, prob)
    for method, prec in ((WN, "fp32"), (UW, "mfma_bf16x2"), (UW, "fp64")):
        t = ctx.tuned(method, prec, n, nodes)
        assert t is not None, (method, prec)
        if prec == "fp32":
            # deeper FP32 batches would loosen the in-batch error bound past 1e-5
            assert 1 <= t["emb_batch"] <= 128
        if prec != "mfma_bf16x2":
            assert t["den_mode"] in (0, 1) and t["tile"] in (0, 1, 2)
        # a NULL tuning takes the stored knobs: bit-identical to passing them explicitly
        auto = plan.distance(method, prec)
        explicit = plan.distance(method, prec, tuning=t)
        np.testing.assert_array_equal(auto, explicit)
        want = oracle.problem_condensed(prob, OMETHOD[method])
        err = np.abs(auto - want).max()
        print(f"[autotune {method} {prec}] knobs={t} max_abs_err={err:.3e}", flush=True)
        assert err <= TOL[prec]
    # another size bucket has no entry
    assert ctx.tuned(WN, "fp32", 4 * n, nodes) is None
    plan.close()
    ctx.close()


def _small_jobs():
    specs = batch_job_specs(n_jobs=5, seed=515, n_range=(20, 300), tips_range=(200, 2000))
    kinds = [(WN, "fp32"), (UW, "mfma_bf16x2"), (WU, "fp64"), (UW, "fp32"), (WN, "fp64")]
    out = []
    for spec, (m, p) in zip(specs, kinds):
        spec["p_nonzero"] = 0.2
        spec["depth"] = 200
        out.append((build_job(spec), m, p))
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_host_outputs_equal_device_outputs(uf, ctx, dtype):
    import torch
    jobs = _small_jobs()
    td, nd = (torch.float64, np.float64) if dtype == "f64" else (torch.float32, np.float32)
    dev = [torch.full((p.n_samples * (p.n_samples - 1) // 2,), -1.0, dtype=td, device="cuda:0")
           for p, _, _ in jobs]
    host = [np.full(p.n_samples * (p.n_samples - 1) // 2, -1.0, dtype=nd) for p, _, _ in jobs]
    bd = uf.Batch(ctx, [dict(problem=p, method=m, precision=pr, out=o, out_dtype=dtype)
                        for (p, m, pr), o in zip(jobs, dev)])
    bh = uf.Batch(ctx, [dict(problem=p, method=m, precision=pr, out=o, out_dtype=dtype)
                        for (p, m, pr), o in zip(jobs, host)])
    bd.run()
    bh.run()
    torch.cuda.synchronize()
    for (p, m, pr), d, h in zip(jobs, dev, host):
        np.testing.assert_array_equal(d.cpu().numpy(), h)
        want = oracle.problem_condensed(p, OMETHOD[m])
        tol = TOL[pr] if m != WU else TOL[pr] * max(1.0, float(np.abs(want).max()))
        assert np.abs(h.astype(np.float64) - want).max() <= tol + (6e-8 if dtype == "f32" else 0.0)
    # graph replays write the host outputs again
    bh.capture()
    for h in host:
        h.fill(-5.0)
    bh.run()
    for d, h in zip(dev, host):
        np.testing.assert_array_equal(d.cpu().numpy(), h)
    bd.close()
    bh.close()


def test_batch_takes_per_job_tuned_knobs(uf):
    ctx = uf.Context(0)
    jobs = _small_jobs()
    # tune two of the jobs' kinds: those jobs take the stored knobs, the rest the defaults
    ctx.autotune([(jobs[0][0], WN, "fp32"), (jobs[1][0], UW, "mfma_bf16x2")])
    assert ctx.tuned(WN, "fp32", jobs[0][0].n_samples, jobs[0][0].n_nodes) is not None
    import torch
    outs = [torch.empty(p.n_samples * (p.n_samples - 1) // 2, dtype=torch.float64, device="cuda:0")
            for p, _, _ in jobs]
    b = uf.Batch(ctx, [dict(problem=p, method=m, precision=pr, out=o) for (p, m, pr), o in zip(jobs, outs)])
    b.run()
    for (p, m, pr), o in zip(jobs, outs):
        got = o.cpu().numpy()
        # a batch this small splits each striped job's branches as a single plan does, so a
        # single plan with the same knobs gives the same bits
        t = ctx.tuned(m, pr, p.n_samples, p.n_nodes)
        single = uf.Plan.from_problem(ctx, p).distance(m, pr, tuning=dict(t) if t else dict(tile=2))
        np.testing.assert_array_equal(got, single)
    b.close()
    ctx.close()
