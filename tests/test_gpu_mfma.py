"""GPU parity of the matrix-core (bf16 hi+lo MFMA) unweighted path against the FP64 oracle,
through the C ABI.  Bar: 1e-5 absolute; dyadic lengths m/256 (exact in bf16, exact partial
sums in FP32) must match the oracle bit for bit."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle
from synth import Problem, workload_problem, make_rng

from helpers import condensed_index, tiny_problem

pytestmark = pytest.mark.gpu

UW = "unweighted"
MF = "mfma_bf16x2"


@pytest.fixture(scope="module")
def uf():
    import paper_2005_05826_amd as uf
    return uf


@pytest.fixture(scope="module")
def ctx(uf):
    return uf.Context(0)


def _report(tag, got, want):
    err = np.abs(np.asarray(got, np.float64) - want)
    print(f"[{tag}] n_pairs={want.size} max_abs_err={err.max(initial=0):.3e} "
          f"mean_abs_err={err.mean() if err.size else 0:.3e}", flush=True)
    return err


CASES = {
    "tiny": lambda: tiny_problem(41, max_nodes=30, max_samples=8),
    "binary_256": lambda: workload_problem("binary_256"),
    "n129": lambda: workload_problem("binary_256", n=129, tips=700, p_nonzero=0.2, seed=61),
    "n300": lambda: workload_problem("binary_256", n=300, tips=3000, seed=62),
    "zipf_600": lambda: workload_problem("zipf_25000", n=600, tips=8000, k=400, seed=63),
    "coalescent_513": lambda: workload_problem("coalescent_4096", n=513, tips=3000, k=200, depth=1000, seed=64),
}


@pytest.fixture(scope="module")
def problems():
    return {k: f() for k, f in CASES.items()}


@pytest.mark.parametrize("case", sorted(CASES))
def test_mfma_matches_oracle(uf, ctx, problems, case):
    prob = problems[case]
    plan = uf.Plan.from_problem(ctx, prob)
    got = plan.distance(UW, MF)
    want = oracle.problem_condensed(prob, oracle.UNWEIGHTED)
    err = _report(f"mfma {case}", got, want)
    assert err.max(initial=0.0) <= 1e-5


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("k_chunk", [64, 512, 4096, 16384])
def test_mfma_k_chunk(uf, ctx, problems, k_chunk, variant):
    prob = problems["zipf_600"]
    plan = uf.Plan.from_problem(ctx, prob)
    got = plan.distance(UW, MF, tuning=dict(k_chunk=k_chunk, variant=variant))
    want = oracle.problem_condensed(prob, oracle.UNWEIGHTED)
    err = _report(f"mfma k_chunk={k_chunk} variant={variant}", got, want)
    assert err.max() <= 1e-5


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("n", [2, 3, 127, 128, 257])
def test_mfma_dyadic_bit_identical(uf, ctx, n, variant):
    prob = workload_problem("binary_256", n=n, tips=500, p_nonzero=0.3, dyadic=True, depth=256, seed=200 + n)
    plan = uf.Plan.from_problem(ctx, prob)
    got = plan.distance(UW, MF, tuning=dict(variant=variant))
    want = oracle.problem_condensed(prob, oracle.UNWEIGHTED)
    np.testing.assert_array_equal(got, want)


def test_mfma_identical_samples_exact_zero(uf, ctx):
    base = workload_problem("binary_256", n=200, tips=1500, seed=7)
    rows = [(base.indices[base.indptr[k]:base.indptr[k + 1]], base.counts[base.indptr[k]:base.indptr[k + 1]])
            for k in list(range(base.n_samples)) + [3, 150]]
    indptr = np.zeros(len(rows) + 1, np.int64)
    indptr[1:] = np.cumsum([len(r[0]) for r in rows])
    prob = Problem(**{**base.__dict__, "indptr": indptr, "indices": np.concatenate([r[0] for r in rows]),
                      "counts": np.concatenate([r[1] for r in rows])})
    plan = uf.Plan.from_problem(ctx, prob)
    n = prob.n_samples
    d = plan.distance(UW, MF)
    assert d[condensed_index(n, 3, n - 2)] == 0.0
    assert d[condensed_index(n, 150, n - 1)] == 0.0
    assert np.all(d >= 0) and np.all(d <= 1)


def test_mfma_f32_output_and_single_node(uf, ctx, problems):
    prob = problems["n300"]
    plan = uf.Plan.from_problem(ctx, prob)
    want = oracle.problem_condensed(prob, oracle.UNWEIGHTED)
    got = plan.distance(UW, MF, out_dtype="f32")
    assert got.dtype == np.float32 and np.abs(got - want).max() <= 1e-5
    single = Problem(parent=np.array([-1], np.int32), length=np.zeros(1), feature_node=np.array([0], np.int32),
                     indptr=np.array([0, 1, 2], np.int64), indices=np.array([0, 0], np.int32),
                     counts=np.array([1, 2], np.int32), n_features=1)
    p1 = uf.Plan.from_problem(ctx, single)
    assert p1.distance(UW, MF)[0] == 0.0


def test_mfma_matches_striped_fp64(uf, ctx, problems):
    prob = problems["zipf_600"]
    plan = uf.Plan.from_problem(ctx, prob)
    a = plan.distance(UW, MF)
    b = plan.distance(UW, "fp64")
    assert np.abs(a - b).max() <= 1e-5


def test_mfma_deterministic(uf, ctx, problems):
    plan = uf.Plan.from_problem(ctx, problems["zipf_600"])
    np.testing.assert_array_equal(plan.distance(UW, MF), plan.distance(UW, MF))


@pytest.fixture(scope="module")
def zipf_25000():
    return workload_problem("zipf_25000")


def test_zipf_25000_full_size_sampled(uf, ctx, zipf_25000):
    """25,000 samples on a 300,000-tip tree, default k_chunk 4,096: all outputs in [0, 1],
    a seeded sample of pairs among 160 random samples checked against the oracle."""
    import torch
    plan = uf.Plan.from_problem(ctx, zipf_25000)
    n = zipf_25000.n_samples
    out = torch.empty(n * (n - 1) // 2, dtype=torch.float64, device="cuda:0")
    plan.distance(UW, MF, out=out)
    torch.cuda.synchronize()
    assert bool(((out >= 0) & (out <= 1)).all())
    rng = make_rng(33)
    subset = np.sort(rng.choice(n, size=160, replace=False))
    a = rng.integers(0, subset.size, size=1200)
    b = rng.integers(0, subset.size, size=1200)
    keep = a != b
    pi = np.minimum(subset[a[keep]], subset[b[keep]])
    pj = np.maximum(subset[a[keep]], subset[b[keep]])
    want = oracle.problem_pairs(zipf_25000, oracle.UNWEIGHTED, pi, pj)
    got = out[torch.from_numpy(condensed_index(n, pi, pj)).to("cuda:0")].cpu().numpy()
    err = _report("zipf_25000 mfma sampled", got, want)
    assert err.max() <= 1e-5
