"""GPU tests of generated count rows and presence bits (the path taken when the full rows
do not fit in device memory), forced with a plan memory limit, through the C ABI: the
results equal those of the resident path (the same sums in the same order) and the FP64
oracle."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle
from synth import workload_problem

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


CASES = {
    "coalescent_600": lambda: workload_problem("coalescent_4096", n=600, tips=4000, k=300, depth=1500, seed=72),
    "binary_ragged_257": lambda: workload_problem("binary_256", n=257, seed=71),
}


def _generated(plan):
    return plan.profile().get("generate", (0, 0.0))[0]


def _row_limit(prob, count_width, emb_batch=128):
    """A device-byte limit between what batches of generated rows need and what the full
    count rows need (halfway between rough estimates of the two; the stripe state is
    bounded from above by its largest tile padding)."""
    n, N, nnz = prob.n_samples, prob.n_nodes, int(prob.indices.size)
    cstride = -(-n // 64) * 64
    inputs = (n + 1) * 8 + nnz * 8 + n * 4 + N * 20
    state = (-(-(n // 2) // 96) * 96) * (-(-n // 512) * 512) * 8 * 2
    counts = N * cstride * count_width
    tables = nnz * 8 + N * 8
    buffers = 3 * emb_batch * cstride * count_width   # two row buffers and the sample-major staging
    return inputs + state + n * 16 + (counts + tables + buffers) // 2


@pytest.mark.parametrize("count_width", [4, 2])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("method", [UW, WN])
@pytest.mark.parametrize("case", sorted(CASES))
def test_generated_rows_equal_resident_rows(uf, ctx, case, method, prec, count_width):
    prob = CASES[case]()
    n = prob.n_samples
    resident = uf.Plan.from_problem(ctx, prob)
    limited = uf.Plan.from_problem(ctx, prob)
    limited.set_memory_limit(_row_limit(prob, count_width))
    for tuning in (dict(den_mode=0, tile=2, emb_batch=64), dict(den_mode=1, tile=0, emb_batch=128)):
        tuning = dict(tuning, count_width=count_width, k_split=1)
        want = resident.distance(method, prec, tuning=tuning)
        limited.set_profiling(True)
        got = limited.distance(method, prec, tuning=tuning)
        assert _generated(limited) > 0, "the limit did not force generated rows"
        limited.set_profiling(False)
        if tuning["den_mode"] == 0:
            np.testing.assert_array_equal(got, want)   # same sums, same order
        else:   # per-sample sums are divided batch by batch here
            assert np.abs(got - want).max() <= 1e-13
        ref = oracle.problem_condensed(prob, OMETHOD[method])
        err = np.abs(got - ref).max()
        print(f"[generated {case} {method} {prec} cw={count_width} {tuning}] max_abs_err={err:.3e}", flush=True)
        assert err <= TOL[prec]
    resident.close()
    limited.close()


def test_generated_rows_stripe_ranges_and_unnormalized(uf, ctx):
    prob = CASES["coalescent_600"]()
    n = prob.n_samples
    plan = uf.Plan.from_problem(ctx, prob)
    plan.set_memory_limit(_row_limit(prob, 2))
    tuning = dict(k_split=1, emb_batch=128)
    full = plan.distance(WU, "fp64", tuning=tuning)
    out = np.full(n * (n - 1) // 2, -1.0)
    for a, c in ((0, 100), (100, 233), (233, n // 2)):
        plan.distance_stripes(a, c, out, WU, "fp64", tuning=tuning)
    np.testing.assert_array_equal(out, full)
    ref = oracle.problem_condensed(prob, oracle.WEIGHTED_UNNORMALIZED)
    assert np.abs(full - ref).max() <= 1e-12 * max(1.0, float(np.abs(ref).max()))
    plan.close()


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("k_chunk", [256, 512])
def test_generated_presence_bits_equal_resident(uf, ctx, k_chunk, variant):
    # many samples with few features each: the presence bits outweigh the tables that
    # generate them, so a limit can leave room for chunks of bits but not all of them
    prob = workload_problem("binary_256", n=2000, tips=4000, p_nonzero=0.0125, depth=500, seed=401)
    resident = uf.Plan.from_problem(ctx, prob)
    limited = uf.Plan.from_problem(ctx, prob)
    limited.set_memory_limit(int(3.5 * 2 ** 20))
    tuning = dict(k_chunk=k_chunk, variant=variant)
    want = resident.distance(UW, "mfma_bf16x2", tuning=tuning)
    limited.set_profiling(True)
    got = limited.distance(UW, "mfma_bf16x2", tuning=tuning)
    launches = limited.profile()
    limited.set_profiling(False)
    print(f"[generated bits k_chunk={k_chunk} variant={variant}] launches {launches}", flush=True)
    assert launches.get("generate", (0, 0))[0] >= 2, "the limit did not force chunks of generated bits"
    np.testing.assert_array_equal(got, want)      # chunks of whole flush groups: same sums
    ref = oracle.problem_condensed(prob, oracle.UNWEIGHTED)
    assert np.abs(got - ref).max() <= 1e-5
    resident.close()
    limited.close()


def test_generated_rows_dense_samples(uf, ctx):
    """Samples with 2,044-2,125 distinct tips each, one at or below the 2,048 entries a
    work-group stages in LDS and the others above (they search their entries in place), and
    batch depths that leave a partial last pass of the branch loop."""
    prob = workload_problem("binary_256", n=40, tips=12000, p_nonzero=0.5, depth=2850, seed=403)
    sizes = np.diff(prob.indptr)
    print(f"[dense samples] entries per sample {sizes.min()}..{sizes.max()}", flush=True)
    assert sizes.min() <= 2048 < sizes.max()
    resident = uf.Plan.from_problem(ctx, prob)
    limited = uf.Plan.from_problem(ctx, prob)
    limited.set_memory_limit(_row_limit(prob, 2, emb_batch=300))
    ref = oracle.problem_condensed(prob, oracle.WEIGHTED_NORMALIZED)
    for E in (300, 129):
        tuning = dict(den_mode=0, tile=2, emb_batch=E, count_width=2, k_split=1)
        want = resident.distance(WN, "fp64", tuning=tuning)
        limited.set_profiling(True)
        got = limited.distance(WN, "fp64", tuning=tuning)
        assert _generated(limited) > 0, "the limit did not force generated rows"
        limited.set_profiling(False)
        np.testing.assert_array_equal(got, want)
        assert np.abs(got - ref).max() <= 1e-12
    resident.close()
    limited.close()


def test_limit_too_small_is_reported(uf, ctx):
    prob = CASES["binary_ragged_257"]()
    plan = uf.Plan.from_problem(ctx, prob)
    plan.set_memory_limit(1024)
    with pytest.raises(uf.UniFracError) as ei:
        plan.distance(WN, "fp64")
    assert ei.value.status_name == "UF_E_OOM"
    with pytest.raises(uf.UniFracError) as ei:
        plan.set_memory_limit(-1)
    assert ei.value.status_name == "UF_E_ARG"
    plan.set_memory_limit(0)
    got = plan.distance(WN, "fp64")
    assert np.abs(got - oracle.problem_condensed(prob, oracle.WEIGHTED_NORMALIZED)).max() <= 1e-12
    plan.close()
