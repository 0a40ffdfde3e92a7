"""GPU tests of batched execution (many uneven jobs, persistent queues, HIP graph replay)
through the C ABI, against the FP64 oracle and against single-job plans."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle
from synth import batch_job_specs, build_job, workload_problem

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5, "mfma_bf16x2": 1e-5}


@pytest.fixture(scope="module")
def uf():
    import paper_2005_05826_amd as uf
    return uf


@pytest.fixture(scope="module")
def ctx(uf):
    return uf.Context(0)


def _jobs():
    # uneven small jobs of the batched workload's kind, covering every path
    specs = batch_job_specs(n_jobs=6, seed=4242, n_range=(2, 400), tips_range=(200, 3000))
    kinds = [("weighted_normalized", "fp32"), ("unweighted", "mfma_bf16x2"),
             ("weighted_normalized", "fp64"), ("unweighted", "fp32"),
             ("unweighted", "mfma_bf16x2"), ("unweighted", "fp64")]
    probs = []
    for spec, (m, p) in zip(specs, kinds):
        spec["p_nonzero"] = 0.2
        spec["depth"] = 200      # small trees: keep the rarefaction depth reachable
        probs.append((build_job(spec), m, p))
    probs.append((workload_problem("binary_256", n=1, tips=50, p_nonzero=0.5, depth=200, seed=3), "weighted_normalized", "fp32"))
    return probs


@pytest.fixture(scope="module")
def jobs():
    return _jobs()


def _outs(jobs, dtype="f64"):
    import torch
    td = torch.float64 if dtype == "f64" else torch.float32
    return [torch.full((max(1, p.n_samples * (p.n_samples - 1) // 2),), -1.0, dtype=td, device="cuda:0")
            for p, _, _ in jobs]


def _want(jobs):
    return [oracle.problem_condensed(p, oracle.UNWEIGHTED if m == "unweighted" else oracle.WEIGHTED_NORMALIZED)
            for p, m, _ in jobs]


def _check(jobs, outs, want, tag):
    import torch
    torch.cuda.synchronize()
    for (p, m, prec), o, w in zip(jobs, outs, want):
        got = o.cpu().numpy()[: w.size].astype(np.float64)
        err = np.abs(got - w).max(initial=0.0)
        # an FP32 output adds its own rounding, at most 2^-25 for distances in [0, 1]
        tol = TOL[prec] + (6e-8 if o.dtype == torch.float32 else 0.0)
        print(f"[{tag}] n={p.n_samples} {m} {prec} max_abs_err={err:.3e}", flush=True)
        assert err <= tol, (tag, p.n_samples, m, prec, err)


@pytest.mark.parametrize("tile,variant", [(0, 0), (2, 1)])
@pytest.mark.parametrize("den_mode", [0, 1])
def test_batch_matches_oracle(uf, ctx, jobs, den_mode, tile, variant):
    outs = _outs(jobs)
    b = uf.Batch(ctx, [dict(problem=p, method=m, precision=pr, out=o) for (p, m, pr), o in zip(jobs, outs)],
                 tuning=dict(den_mode=den_mode, tile=tile, variant=variant))
    b.run()
    _check(jobs, outs, _want(jobs), f"batch den_mode={den_mode} tile={tile} variant={variant}")
    b.close()


@pytest.mark.parametrize("k_split", [1, 0])
def test_batch_equals_single_plans_bitwise(uf, ctx, jobs, k_split):
    # k_split 1: neither side splits branches; 0: this batch is far too small to fill the
    # device, so every striped job splits its branches (and sets its FP64 batch depth) by the
    # single plan's automatic rule
    tuning = dict(den_mode=0, tile=2, k_split=k_split)
    outs = _outs(jobs)
    b = uf.Batch(ctx, [dict(problem=p, method=m, precision=pr, out=o) for (p, m, pr), o in zip(jobs, outs)],
                 tuning=tuning)
    b.run()
    for (p, m, pr), o in zip(jobs, outs):
        if p.n_samples < 2:
            continue
        single = uf.Plan.from_problem(ctx, p).distance(m, pr, tuning=tuning)
        np.testing.assert_array_equal(o.cpu().numpy(), single)
    b.close()


@pytest.mark.parametrize("k_split", [3, 16])
def test_batch_branch_splits(uf, ctx, jobs, k_split):
    """Explicit branch splits in the queues: the oracle's results to the usual bounds, and
    bit for bit those of single plans with the same splits."""
    tuning = dict(den_mode=1, tile=2, k_split=k_split)
    outs = _outs(jobs)
    b = uf.Batch(ctx, [dict(problem=p, method=m, precision=pr, out=o) for (p, m, pr), o in zip(jobs, outs)],
                 tuning=tuning)
    b.capture()
    b.run()
    _check(jobs, outs, _want(jobs), f"batch k_split={k_split}")
    for (p, m, pr), o in zip(jobs, outs):
        if p.n_samples < 2:
            continue
        single = uf.Plan.from_problem(ctx, p).distance(m, pr, tuning=tuning)
        np.testing.assert_array_equal(o.cpu().numpy(), single)
    b.close()


def test_graph_replay_matches_eager(uf, ctx, jobs):
    import torch
    outs = _outs(jobs, "f32")
    b = uf.Batch(ctx, [dict(problem=p, method=m, precision=pr, out=o, out_dtype="f32")
                       for (p, m, pr), o in zip(jobs, outs)])
    b.run()
    eager = [o.clone() for o in outs]
    b.capture()
    for rep in range(3):
        for o in outs:
            o.fill_(-7.0)
        torch.cuda.synchronize()
        b.run()
        for (p, _, _), o, e in zip(jobs, outs, eager):
            # a one-sample job has no pairs: its one-element buffer is never written
            m = p.n_samples * (p.n_samples - 1) // 2
            o, e = o[:m], e[:m]
            if not torch.equal(o, e):
                bad = (o != e)
                print(f"replay {rep}: n={p.n_samples}: {int(bad.sum())} of {m} differ; "
                      f"{int((o[bad] == -7.0).sum())} still hold the fill value", flush=True)
            assert torch.equal(o, e), f"replay {rep} differs from the eager run"
        # unrelated eager work between replays
        x = torch.randn(1 << 16, device="cuda:0")
        (x * 2).sum().item()
    _check(jobs, outs, _want(jobs), "graph f32 out")
    b.close()


def test_batch_errors(uf, ctx, jobs):
    import torch
    p, _, _ = jobs[0]
    out = torch.empty(p.n_samples * (p.n_samples - 1) // 2, dtype=torch.float64, device="cuda:0")
    with pytest.raises(uf.UniFracError) as ei:
        uf.Batch(ctx, [dict(problem=p, method="weighted_normalized", precision="mfma_bf16x2", out=out)])
    assert ei.value.status_name == "UF_E_UNSUPPORTED"
    bad = workload_problem("binary_256", n=5, tips=40, p_nonzero=0.5, depth=200, seed=8)
    bad.parent = bad.parent.copy()
    bad.parent[0] = bad.parent.shape[0] + 5
    with pytest.raises(uf.UniFracError) as ei:
        uf.Batch(ctx, [dict(problem=p, method="unweighted", precision="fp64", out=out),
                       dict(problem=bad, method="unweighted", precision="fp64", out=out)])
    assert ei.value.status_name == "UF_E_TREE"
    with pytest.raises(uf.UniFracError) as ei:
        uf.Batch(ctx, [dict(problem=p, method="unweighted", precision="fp64", out=out)], tuning=dict(k_split=65))
    assert ei.value.status_name == "UF_E_ARG"


@pytest.mark.parametrize("method,prec", [("weighted_normalized", "fp32"), ("unweighted", "mfma_bf16x2"),
                                         ("unweighted", "fp64")])
def test_autotune_picks_valid_knobs_and_caches(uf, ctx, tmp_path, method, prec):
    prob = workload_problem("coalescent_4096", n=700, tips=4000, k=300, depth=1500, seed=77)
    plan = uf.Plan.from_problem(ctx, prob)
    cache = tmp_path / "tune.txt"
    best, ms = plan.autotune(method, prec, reps=2, cache_path=cache)
    assert ms > 0
    got = plan.distance(method, prec, tuning=best)
    want = oracle.problem_condensed(prob, oracle.UNWEIGHTED if method == "unweighted" else oracle.WEIGHTED_NORMALIZED)
    assert np.abs(got - want).max() <= TOL[prec]
    best2, ms2 = plan.autotune(method, prec, reps=2, cache_path=cache)   # served from the cache
    assert best2 == best and ms2 == pytest.approx(ms, rel=1e-5)
    assert len(cache.read_text().strip().splitlines()) == 1


@pytest.mark.parametrize("tile", [0, 1, 2])
@pytest.mark.parametrize("den_mode", [0, 1])
def test_batch_dyadic_bit_identical(uf, ctx, den_mode, tile):
    """The queue-driven kernels on dyadic inputs (lengths m/256, rarefaction depth 256):
    every partial sum is exact, so every job equals the oracle bit for bit."""
    import torch
    probs = [workload_problem("binary_256", n=n, tips=t, p_nonzero=0.3, depth=256, dyadic=True, seed=s)
             for n, t, s in ((170, 500, 301), (33, 900, 302), (260, 300, 303))]
    kinds = [("weighted_normalized", "fp32"), ("unweighted", "fp64"), ("weighted_normalized", "fp64"),
             ("unweighted", "fp32")]
    jobs = [(p, m, pr) for p in probs for m, pr in kinds]
    outs = _outs(jobs)
    b = uf.Batch(ctx, [dict(problem=p, method=m, precision=pr, out=o) for (p, m, pr), o in zip(jobs, outs)],
                 tuning=dict(den_mode=den_mode, tile=tile, emb_batch=64))
    b.run()
    torch.cuda.synchronize()
    for (p, m, pr), o in zip(jobs, outs):
        want = oracle.problem_condensed(p, oracle.UNWEIGHTED if m == "unweighted" else oracle.WEIGHTED_NORMALIZED)
        np.testing.assert_array_equal(o.cpu().numpy(), want)
    b.close()


def test_batch_int32_counts_deep_batches_and_unnormalized(uf, ctx):
    """Paths the small batch above does not reach: sample totals above 65,535 (the int32
    count-row queue), FP32 batches of 512 branches, and weighted-unnormalized jobs."""
    import torch
    big = workload_problem("binary_256", n=150, tips=3000, p_nonzero=0.9, nb_mean=40.0, depth=70000, seed=305)
    small = workload_problem("binary_256", n=120, tips=2500, p_nonzero=0.2, depth=500, seed=306)
    kinds = [("weighted_normalized", "fp32"), ("unweighted", "fp32"), ("weighted_unnormalized", "fp64"),
             ("weighted_unnormalized", "fp32"), ("unweighted", "fp64")]
    jobs = [(p, m, pr) for p in (big, small) for m, pr in kinds]
    outs = _outs(jobs)
    b = uf.Batch(ctx, [dict(problem=p, method=m, precision=pr, out=o) for (p, m, pr), o in zip(jobs, outs)],
                 tuning=dict(emb_batch=512, den_mode=1, tile=2))
    b.run()
    torch.cuda.synchronize()
    om = {"unweighted": oracle.UNWEIGHTED, "weighted_normalized": oracle.WEIGHTED_NORMALIZED,
          "weighted_unnormalized": oracle.WEIGHTED_UNNORMALIZED}
    for (p, m, pr), o in zip(jobs, outs):
        want = oracle.problem_condensed(p, om[m])
        got = o.cpu().numpy()
        err = np.abs(got - want).max()
        # unnormalized values are branch lengths: the bar is relative to max(1, |d|)
        tol = TOL[pr] * (max(1.0, float(np.abs(want).max())) if m == "weighted_unnormalized" else 1.0)
        print(f"[int32/E512] n={p.n_samples} {m} {pr} max_abs_err={err:.3e} (tol {tol:.1e})", flush=True)
        assert err <= tol, (p.n_samples, m, pr, err)
    b.close()


def test_distance_batch_one_shot_equals_batch(uf, ctx, jobs):
    """uf_distance_batch (create, run, wait, destroy in one call) with device and host
    outputs gives the persistent batch's results bit for bit."""
    import torch
    want_outs = _outs(jobs)
    b = uf.Batch(ctx, [dict(problem=p, method=m, precision=pr, out=o) for (p, m, pr), o in zip(jobs, want_outs)])
    b.run()
    torch.cuda.synchronize()
    b.close()
    outs = [o if i % 2 == 0 else np.full(o.numel(), -1.0) for i, o in enumerate(_outs(jobs))]
    uf.distance_batch(ctx, [dict(problem=p, method=m, precision=pr, out=o)
                            for (p, m, pr), o in zip(jobs, outs)])
    for o, w in zip(outs, want_outs):
        got = o if isinstance(o, np.ndarray) else o.cpu().numpy()
        np.testing.assert_array_equal(got, w.cpu().numpy())
    _check(jobs, [torch.from_numpy(o).to("cuda:0") if isinstance(o, np.ndarray) else o for o in outs],
           _want(jobs), "distance_batch")
