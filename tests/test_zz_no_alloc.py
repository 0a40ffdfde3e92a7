"""The no-allocation distance entry point (uf_plan_distance_noalloc) against
uf_plan_distance on the same plans, through the C ABI: two calls in a row on the same
device scratch, the second on a smaller problem."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle
from synth import workload_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def uf():
    import paper_2005_05826_amd as uf
    return uf


@pytest.mark.parametrize("prec,tuning", [("fp64", dict(k_split=3)),
                                          ("fp32", dict(den_mode=1, tile=2, k_split=5)),
                                          ("fp32", dict(den_mode=0, tile=0, k_split=1, emb_batch=64))])
@pytest.mark.parametrize("method", ["weighted_normalized", "unweighted"])
def test_noalloc_matches_plan_distance(uf, method, prec, tuning):
    import torch
    ctx = uf.Context(0)
    big = workload_problem("coalescent_4096", n=700, tips=4000, k=300, depth=1500, seed=77)
    small = workload_problem("binary_256", n=131, tips=900, p_nonzero=0.2, depth=500, seed=78)
    for prob in (big, small):          # the second call reuses the scratch with a smaller input
        plan = uf.Plan.from_problem(ctx, prob)
        n = prob.n_samples
        want = plan.distance(method, prec, tuning=tuning)
        out = torch.full((n * (n - 1) // 2,), -1.0, dtype=torch.float64, device="cuda:0")
        plan.distance_noalloc(out, method, prec, tuning=tuning)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        # same kernels, same knobs, same branch split: the same bits
        np.testing.assert_array_equal(got, want)
        ref = oracle.problem_condensed(prob, oracle.UNWEIGHTED if method == "unweighted"
                                       else oracle.WEIGHTED_NORMALIZED)
        assert np.abs(got - ref).max() <= (1e-12 if prec == "fp64" else 1e-5)
        plan.close()
    ctx.close()


def test_noalloc_f32_output_and_repeat(uf):
    import torch
    ctx = uf.Context(0)
    prob = workload_problem("binary_256", n=300, tips=1500, p_nonzero=0.1, depth=800, seed=79)
    plan = uf.Plan.from_problem(ctx, prob)
    n = prob.n_samples
    want = plan.distance("weighted_normalized", "fp32", out_dtype="f32", tuning=dict(k_split=2))
    out = torch.empty(n * (n - 1) // 2, dtype=torch.float32, device="cuda:0")
    for _ in range(3):
        out.fill_(-1.0)
        plan.distance_noalloc(out, "weighted_normalized", "fp32", out_dtype="f32", tuning=dict(k_split=2))
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), want)
    plan.close()
    ctx.close()


def test_noalloc_rejects_what_it_cannot_hold(uf):
    import torch
    ctx = uf.Context(0)
    # 16-bit count rows of 65,535 nodes x 4,096 samples need 512 MiB, beyond the fixed array
    prob = workload_problem("coalescent_4096")
    plan = uf.Plan.from_problem(ctx, prob)
    n = prob.n_samples
    out = torch.empty(n * (n - 1) // 2, dtype=torch.float64, device="cuda:0")
    with pytest.raises(uf.UniFracError) as ei:
        plan.distance_noalloc(out, "weighted_normalized", "fp32")
    assert ei.value.status_name == "UF_E_ARG" and "bytes of device scratch" in str(ei.value)
    with pytest.raises(uf.UniFracError) as ei:
        plan.distance_noalloc(out, "unweighted", "mfma_bf16x2")
    assert ei.value.status_name == "UF_E_UNSUPPORTED"
    plan.close()
    ctx.close()
