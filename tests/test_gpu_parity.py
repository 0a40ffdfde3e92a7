"""GPU parity of the striped hot path against the FP64 CPU oracle, through the C ABI.

Bars: embedding counts bit-exact; FP64 path within 1e-12 absolute; FP32 path within 1e-5
absolute; dyadic inputs (exactly representable partial sums) bit-identical in both."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle
from synth import Problem, workload_problem, make_rng

from helpers import condensed_index, tiny_problem

pytestmark = pytest.mark.gpu

UW, WN = "unweighted", "weighted_normalized"
OMETHOD = {UW: oracle.UNWEIGHTED, WN: oracle.WEIGHTED_NORMALIZED}
TOL = {"fp64": 1e-12, "fp32": 1e-5}


@pytest.fixture(scope="module")
def uf():
    import paper_2005_05826_amd as uf
    return uf


@pytest.fixture(scope="module")
def ctx(uf):
    return uf.Context(0)


def _plan(uf, ctx, prob):
    return uf.Plan.from_problem(ctx, prob)


def _report(tag, got, want):
    err = np.abs(np.asarray(got, np.float64) - want)
    print(f"[{tag}] n_pairs={want.size} max_abs_err={err.max() if err.size else 0:.3e} "
          f"mean_abs_err={err.mean() if err.size else 0:.3e}", flush=True)
    return err


CASES = {
    "tiny_a": lambda: tiny_problem(31, max_nodes=16, max_samples=6),
    "tiny_b": lambda: tiny_problem(32, max_nodes=40, max_samples=9),
    "binary_256": lambda: workload_problem("binary_256"),
    "binary_ragged_257": lambda: workload_problem("binary_256", n=257, seed=71),
    "coalescent_600": lambda: workload_problem("coalescent_4096", n=600, tips=4000, k=300, depth=1500, seed=72),
    "coalescent_513": lambda: workload_problem("coalescent_4096", n=513, tips=3000, k=200, depth=1000, seed=73),
}


@pytest.fixture(scope="module")
def problems():
    return {name: f() for name, f in CASES.items()}


@pytest.mark.parametrize("case", sorted(CASES))
def test_embedding_counts_bit_exact(uf, ctx, problems, case):
    prob = problems[case]
    plan = _plan(uf, ctx, prob)
    got = plan.embedding_counts()
    want = oracle.problem_counts(prob).T
    assert got.shape == want.shape
    np.testing.assert_array_equal(got.astype(np.int64), want)


@pytest.mark.parametrize("case", sorted(CASES))
def test_presence_bits_bit_exact(uf, ctx, problems, case):
    prob = problems[case]
    plan = _plan(uf, ctx, prob)
    got = plan.embedding_presence()
    pres = oracle.problem_counts(prob).T > 0                  # [n_nodes][n]
    n = prob.n_samples
    words = (n + 31) // 32
    padded = np.zeros((pres.shape[0], words * 32), bool)
    padded[:, :n] = pres
    # bit k % 32 of word k // 32
    want = (padded.reshape(pres.shape[0], words, 32).astype(np.uint64)
            << np.arange(32, dtype=np.uint64)).sum(-1)
    np.testing.assert_array_equal(got.astype(np.uint64), want)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("method", [UW, WN])
@pytest.mark.parametrize("case", sorted(CASES))
def test_distance_matches_oracle(uf, ctx, problems, case, method, prec):
    prob = problems[case]
    plan = _plan(uf, ctx, prob)
    got = plan.distance(method, prec)
    want = oracle.problem_condensed(prob, OMETHOD[method])
    err = _report(f"{case} {method} {prec}", got, want)
    assert err.max(initial=0.0) <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("method", [UW, WN])
def test_separable_denominator(uf, ctx, problems, method, prec):
    prob = problems["coalescent_600"]
    plan = _plan(uf, ctx, prob)
    got = plan.distance(method, prec, tuning=dict(den_mode=1))
    want = oracle.problem_condensed(prob, OMETHOD[method])
    err = _report(f"den_mode=1 {method} {prec}", got, want)
    assert err.max() <= TOL[prec]


@pytest.mark.parametrize("tile", [0, 1, 2])
@pytest.mark.parametrize("den_mode", [0, 1])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("method", [UW, WN])
def test_tile_shapes_match_oracle(uf, ctx, problems, method, prec, den_mode, tile):
    # every per-lane tile shape, on a ragged size and on one spanning several tiles
    for case in ("binary_ragged_257", "coalescent_600"):
        prob = problems[case]
        plan = _plan(uf, ctx, prob)
        got = plan.distance(method, prec, tuning=dict(den_mode=den_mode, tile=tile))
        want = oracle.problem_condensed(prob, OMETHOD[method])
        err = _report(f"{case} tile={tile} den_mode={den_mode} {method} {prec}", got, want)
        assert err.max() <= TOL[prec]


@pytest.mark.parametrize("k_split", [1, 2, 5, 16, 0])
@pytest.mark.parametrize("den_mode", [0, 1])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_branch_splits_match_oracle(uf, ctx, problems, prec, den_mode, k_split):
    # the fused kernel's branch splits (separate state copies summed in order), explicit and
    # automatic, on both methods
    prob = problems["coalescent_600"]
    plan = _plan(uf, ctx, prob)
    for method in (UW, WN):
        got = plan.distance(method, prec, tuning=dict(den_mode=den_mode, tile=2, k_split=k_split, emb_batch=64))
        want = oracle.problem_condensed(prob, OMETHOD[method])
        err = _report(f"k_split={k_split} den_mode={den_mode} {method} {prec}", got, want)
        assert err.max() <= TOL[prec]


@pytest.mark.parametrize("k_split", [3, 8, 16])
def test_branch_splits_dyadic_bit_identical(uf, ctx, k_split):
    prob = workload_problem("binary_256", n=300, tips=600, p_nonzero=0.3, depth=256, dyadic=True, seed=91)
    plan = _plan(uf, ctx, prob)
    for method in (UW, WN):
        for prec in ("fp64", "fp32"):
            got = plan.distance(method, prec, tuning=dict(k_split=k_split, emb_batch=16))
            np.testing.assert_array_equal(got, oracle.problem_condensed(prob, OMETHOD[method]))


def test_branch_splits_stripe_range(uf, ctx, problems):
    # a stripe range computed with splits equals the same pairs of the full matrix
    prob = problems["coalescent_600"]
    plan = _plan(uf, ctx, prob)
    full = plan.distance(WN, "fp64", tuning=dict(k_split=1))
    n = prob.n_samples
    out = np.full(n * (n - 1) // 2, -1.0)
    plan.distance_stripes(37, 211, out, WN, "fp64", tuning=dict(k_split=4))
    sel = out != -1.0
    assert sel.sum() > 0
    np.testing.assert_allclose(out[sel], full[sel], rtol=0, atol=1e-12)


@pytest.mark.parametrize("emb_batch", [1, 7, 128])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("method", [UW, WN])
def test_dyadic_inputs_bit_identical(uf, ctx, method, prec, emb_batch):
    # lengths m/256 and rarefaction depth 256: every product and every partial sum of a
    # batch is exactly representable, so all paths must equal the oracle bit for bit
    prob = workload_problem("binary_256", n=300, tips=600, p_nonzero=0.3, depth=256, dyadic=True, seed=90)
    plan = _plan(uf, ctx, prob)
    got = plan.distance(method, prec, tuning=dict(emb_batch=emb_batch))
    want = oracle.problem_condensed(prob, OMETHOD[method])
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 64, 255, 256])
def test_stripe_layout(uf, ctx, n):
    prob = workload_problem("binary_256", n=n, tips=300, p_nonzero=0.3, seed=100 + n)
    plan = _plan(uf, ctx, prob)
    for method in (UW, WN):
        num, den = plan.stripes(method, "fp64")
        S = n // 2
        s, k = np.meshgrid(np.arange(S), np.arange(n), indexing="ij")
        j = (k + s + 1) % n
        with np.errstate(invalid="ignore", divide="ignore"):
            d = np.where(den == 0, 0.0, num / den)
        want = oracle.problem_pairs(prob, OMETHOD[method], k.ravel(), j.ravel()).reshape(S, n)
        assert np.abs(d - want).max(initial=0.0) <= 1e-12
        if n % 2 == 0 and S > 0:     # the doubled last stripe holds equal copies
            np.testing.assert_array_equal(num[S - 1, : n // 2], num[S - 1, n // 2:])


def _single(parent, length, rows, fnode):
    indptr = np.zeros(len(rows) + 1, np.int64)
    indptr[1:] = np.cumsum([len(r) for r in rows])
    idx = np.array([f for r in rows for f, _ in r], np.int32)
    cnt = np.array([c for r in rows for _, c in r], np.int32)
    return Problem(parent=np.array(parent, np.int32), length=np.array(length, np.float64),
                   feature_node=np.array(fnode, np.int32), indptr=indptr, indices=idx,
                   counts=cnt, n_features=len(fnode))


EDGE = {
    "single_node_tree": lambda: _single([-1], [0.0], [[(0, 3)], [(0, 1)], [(0, 2)]], [0]),
    "two_samples": lambda: _single([2, 2, -1], [1.0, 2.0, 0.0], [[(0, 1)], [(1, 5)]], [0, 1]),
    "zero_lengths": lambda: _single([2, 2, -1], [0.0, 0.0, 0.0], [[(0, 1)], [(1, 5)], [(0, 2), (1, 2)]], [0, 1]),
    "dups_unsorted": lambda: _single([3, 3, 4, 4, -1], [1.0, 2.0, 4.0, 3.0, 9.0],
                                     [[(2, 1), (0, 1), (2, 4)], [(1, 2), (2, 2), (1, 1)], [(0, 3), (1, 1)]],
                                     [0, 1, 2]),
    "unary_chain": lambda: _single([1, 2, 3, -1, 3], [0.5, 0.25, 1.0, 0.0, 2.0],
                                   [[(0, 1)], [(1, 1)], [(0, 1), (1, 1)]], [0, 4]),
}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", sorted(EDGE))
def test_edge_cases(uf, ctx, case, prec):
    prob = EDGE[case]()
    plan = _plan(uf, ctx, prob)
    for method in (UW, WN):
        got = plan.distance(method, prec)
        want = oracle.problem_condensed(prob, OMETHOD[method])
        assert np.abs(got - want).max(initial=0.0) <= TOL[prec], (case, method)


def test_one_sample_has_no_pairs(uf, ctx):
    prob = _single([2, 2, -1], [1.0, 2.0, 0.0], [[(0, 1)]], [0, 1])
    plan = _plan(uf, ctx, prob)
    assert plan.distance(UW, "fp64").size == 0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_identical_samples_give_exact_zero(uf, ctx, prec):
    base = workload_problem("binary_256", n=50, tips=400, p_nonzero=0.3, seed=5)
    # append copies of samples 0 and 7
    rows = [(base.indices[base.indptr[k]:base.indptr[k + 1]], base.counts[base.indptr[k]:base.indptr[k + 1]])
            for k in list(range(base.n_samples)) + [0, 7]]
    indptr = np.zeros(len(rows) + 1, np.int64)
    indptr[1:] = np.cumsum([len(r[0]) for r in rows])
    prob = Problem(**{**base.__dict__, "indptr": indptr, "indices": np.concatenate([r[0] for r in rows]),
                      "counts": np.concatenate([r[1] for r in rows])})
    plan = _plan(uf, ctx, prob)
    n = prob.n_samples
    for method in (UW, WN):
        d = plan.distance(method, prec)
        assert d[condensed_index(n, 0, n - 2)] == 0.0
        assert d[condensed_index(n, 7, n - 1)] == 0.0
        assert np.all(d >= 0) and np.all(d <= 1)


def test_deterministic_runs(uf, ctx, problems):
    plan = _plan(uf, ctx, problems["coalescent_600"])
    for prec in ("fp64", "fp32"):
        a = plan.distance(WN, prec)
        b = plan.distance(WN, prec)
        np.testing.assert_array_equal(a, b)


def test_f32_output_and_device_output(uf, ctx, problems):
    import torch
    prob = problems["binary_ragged_257"]
    plan = _plan(uf, ctx, prob)
    want = oracle.problem_condensed(prob, oracle.WEIGHTED_NORMALIZED)
    got32 = plan.distance(WN, "fp64", out_dtype="f32")
    assert got32.dtype == np.float32
    assert np.abs(got32 - want).max() <= 1e-7
    dev = torch.empty(want.size, dtype=torch.float64, device="cuda:0")
    plan.distance(WN, "fp64", out=dev)
    torch.cuda.synchronize()
    assert np.abs(dev.cpu().numpy() - want).max() <= 1e-12


def test_mfma_weighted_is_unsupported(uf, ctx, problems):
    plan = _plan(uf, ctx, problems["tiny_a"])
    with pytest.raises(uf.UniFracError) as ei:
        plan.distance(WN, "mfma_bf16x2")
    assert ei.value.status_name == "UF_E_UNSUPPORTED"


def test_one_shot_distance(uf, ctx, problems):
    prob = problems["tiny_b"]
    got = uf.distance(ctx, prob, UW, "fp64")
    want = oracle.problem_condensed(prob, oracle.UNWEIGHTED)
    assert np.abs(got - want).max() <= 1e-12


def _sampled_pairs(n, n_random, first, seed):
    rng = make_rng(seed)
    i = rng.integers(0, n, size=n_random)
    j = rng.integers(0, n, size=n_random)
    keep = i != j
    i, j = np.minimum(i[keep], j[keep]), np.maximum(i[keep], j[keep])
    fi, fj = np.triu_indices(first, k=1)
    return np.concatenate([i, fi]), np.concatenate([j, fj])


@pytest.fixture(scope="module")
def coalescent_4096():
    return workload_problem("coalescent_4096")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("tuning", [{}, dict(den_mode=1, tile=2)], ids=["default", "bench_headline"])
def test_coalescent_4096_full_size_sampled(uf, ctx, coalescent_4096, prec, tuning):
    """The benchmark workload (4,096 samples, 32,768-tip coalescent tree), with the default
    knobs and with the configuration the benchmark times (separable denominator, tile shape
    2, automatic branch splits): every output checked for range, a seeded sample of pairs
    checked against the oracle."""
    import torch
    plan = _plan(uf, ctx, coalescent_4096)
    n = coalescent_4096.n_samples
    out = torch.empty(n * (n - 1) // 2, dtype=torch.float64, device="cuda:0")
    plan.distance(WN, prec, out=out, tuning=tuning)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.all(got >= 0) and np.all(got <= 1)
    pi, pj = _sampled_pairs(n, 1500, 48, seed=11)
    want = oracle.problem_pairs(coalescent_4096, oracle.WEIGHTED_NORMALIZED, pi, pj)
    err = _report(f"coalescent_4096 WN {prec} {tuning} sampled", got[condensed_index(n, pi, pj)], want)
    assert err.max() <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("method", [UW, WN])
@pytest.mark.parametrize("case", ["binary_ragged_257", "coalescent_513"])
def test_separate_transform_variant(uf, ctx, problems, case, method, prec):
    """variant 1: transform into an embedding buffer, one striped launch per batch"""
    prob = problems[case]
    plan = _plan(uf, ctx, prob)
    want = oracle.problem_condensed(prob, OMETHOD[method])
    for E in (5, 128):
        got = plan.distance(method, prec, tuning=dict(variant=1, emb_batch=E))
        err = _report(f"variant1 E={E} {case} {method} {prec}", got, want)
        assert err.max() <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("den_mode", [0, 1])
def test_stripe_ranges_partition_equals_full(uf, ctx, problems, prec, den_mode):
    """Independent stripe-range chunks (uneven, not tile-aligned) fill the matrix with the
    values of the full computation, bit for bit; host and device outputs."""
    import torch
    prob = problems["coalescent_600"]
    plan = _plan(uf, ctx, prob)
    S = prob.n_samples // 2
    cuts = [0, 5, 37, 40, 161, S]
    for method in (UW, WN):
        full = plan.distance(method, prec, tuning=dict(den_mode=den_mode))
        host = np.full(full.size, -1.0)
        dev = torch.full((full.size,), -1.0, dtype=torch.float64, device="cuda:0")
        for a, b in zip(cuts[:-1], cuts[1:]):
            plan.distance_stripes(a, b, host, method, prec, tuning=dict(den_mode=den_mode))
            plan.distance_stripes(a, b, dev, method, prec, tuning=dict(den_mode=den_mode))
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host, full)
        np.testing.assert_array_equal(dev.cpu().numpy(), full)


def test_stripe_range_leaves_other_pairs(uf, ctx, problems):
    prob = problems["binary_ragged_257"]
    plan = _plan(uf, ctx, prob)
    out = np.full(prob.n_samples * (prob.n_samples - 1) // 2, -3.0)
    plan.distance_stripes(10, 20, out, WN, "fp64")
    n = prob.n_samples
    i, j = oracle.condensed_pairs(n)
    d = j - i
    s = np.where(d <= n // 2, d - 1, n - d - 1)
    inside = (s >= 10) & (s < 20)
    assert np.all(out[~inside] == -3.0)
    want = oracle.problem_pairs(prob, oracle.WEIGHTED_NORMALIZED, i[inside], j[inside])
    assert np.abs(out[inside] - want).max() <= 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ["binary_ragged_257", "coalescent_600", "tiny_b"])
def test_weighted_unnormalized(uf, ctx, problems, case, prec):
    """Weighted unnormalized (numerator only) values are lengths, not fractions: the bar is
    relative to max(1, |d|)."""
    prob = problems[case]
    plan = _plan(uf, ctx, prob)
    want = oracle.problem_condensed(prob, oracle.WEIGHTED_UNNORMALIZED)
    got = plan.distance("weighted_unnormalized", prec)
    err = np.abs(got - want) / np.maximum(1.0, np.abs(want))
    print(f"[wun {case} {prec}] max_rel_err={err.max():.3e}", flush=True)
    assert err.max() <= TOL[prec]
    if prec == "fp64":
        host = np.full(got.size, -1.0)
        S = prob.n_samples // 2
        plan.distance_stripes(0, S // 3, host, "weighted_unnormalized", prec)
        plan.distance_stripes(S // 3, S, host, "weighted_unnormalized", prec)
        np.testing.assert_array_equal(host, got)


@pytest.mark.parametrize("case", ["binary_ragged_257", "coalescent_513", "tiny_b"])
def test_count_width_16_and_32_agree(uf, ctx, problems, case):
    """uint16 count rows (packed two per word) and int32 rows give the same counts and the
    same distances bit for bit."""
    prob = problems[case]
    plan = _plan(uf, ctx, prob)
    want = oracle.problem_counts(prob).T
    np.testing.assert_array_equal(plan.embedding_counts16().astype(np.int64), want)
    for method in (UW, WN):
        for prec in ("fp64", "fp32"):
            a = plan.distance(method, prec, tuning=dict(count_width=2))
            b = plan.distance(method, prec, tuning=dict(count_width=4))
            np.testing.assert_array_equal(a, b)


def test_count_width_16_rejects_large_totals(uf, ctx):
    big = _single([2, 2, -1], [1.0, 2.0, 0.0], [[(0, 70000)], [(1, 5)], [(0, 2), (1, 2)]], [0, 1])
    plan = _plan(uf, ctx, big)
    with pytest.raises(uf.UniFracError) as ei:
        plan.distance(WN, "fp64", tuning=dict(count_width=2))
    assert ei.value.status_name == "UF_E_ARG"
    got = plan.distance(WN, "fp64")          # auto picks int32 rows here
    want = oracle.problem_condensed(big, oracle.WEIGHTED_NORMALIZED)
    assert np.abs(got - want).max() <= 1e-12


@pytest.mark.parametrize("tile", [0, 1, 2])
@pytest.mark.parametrize("den_mode", [0, 1])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("method", [UW, WN])
def test_dyadic_bit_identical_every_form(uf, ctx, method, prec, den_mode, tile):
    """Every tile shape and both denominator forms (numerator and denominator stripes, or
    the per-sample denominator), with automatic branch splits: dyadic inputs leave nothing
    to round, so each must equal the oracle bit for bit."""
    prob = workload_problem("binary_256", n=300, tips=600, p_nonzero=0.3, depth=256, dyadic=True, seed=91)
    plan = _plan(uf, ctx, prob)
    want = oracle.problem_condensed(prob, OMETHOD[method])
    for E in (64, 128):
        got = plan.distance(method, prec, tuning=dict(den_mode=den_mode, tile=tile, emb_batch=E))
        np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("out_dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", ["coalescent_600", "binary_ragged_257"])
def test_stripe_blocks_from_independent_plans_merge(uf, ctx, problems, case, out_dtype):
    """The paper's chunk decomposition: every stripe range computed as a compact block by a
    plan on its own context, then merged into one condensed matrix, reproduces the full
    computation bit for bit (host and device blocks alike)."""
    import torch
    prob = problems[case]
    n = prob.n_samples
    S = n // 2
    tuning = dict(den_mode=1, tile=2, k_split=1)
    td = torch.float64 if out_dtype == "f64" else torch.float32
    full = _plan(uf, ctx, prob).distance(WN, "fp32", out_dtype=out_dtype, tuning=tuning)
    merged = torch.full((n * (n - 1) // 2,), -1.0, dtype=td, device="cuda:0")
    cuts = [0, 7, 64, 65, S]
    for idx, (a, b) in enumerate(zip(cuts[:-1], cuts[1:])):
        c2 = uf.Context(0)
        p2 = uf.Plan.from_problem(c2, prob)
        blk = p2.distance_block(a, b, WN, "fp32", out_dtype=out_dtype, tuning=tuning)
        dblk = torch.empty((b - a) * n, dtype=td, device="cuda:0")
        p2.distance_block(a, b, WN, "fp32", out=dblk, out_dtype=out_dtype, tuning=tuning)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(dblk.cpu().numpy().reshape(b - a, n), blk)
        # row r, column k holds the pair (k, (k + a + r + 1) mod n)
        r = np.repeat(np.arange(b - a), n)
        k = np.tile(np.arange(n), b - a)
        j = (k + a + r + 1) % n
        np.testing.assert_array_equal(blk.ravel(), full[condensed_index(n, np.minimum(k, j), np.maximum(k, j))])
        uf.merge_block(ctx, n, a, b, blk if idx % 2 == 0 else dblk, merged, dtype=out_dtype)
        p2.close()
        c2.close()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(merged.cpu().numpy(), full)


def test_trim_releases_scratch_and_keeps_results(uf, ctx, problems):
    """uf_plan_trim frees the plan's scratch (count rows, stripe state, matrix-core buffers);
    the next call rebuilds it and gives the same distances bit for bit."""
    plan = uf.Plan.from_problem(ctx, problems["coalescent_513"])
    for method, prec in ((WN, "fp32"), (UW, "mfma_bf16x2"), (WN, "fp64")):
        a = plan.distance(method, prec)
        plan.trim()
        b = plan.distance(method, prec)
        np.testing.assert_array_equal(a, b)
    plan.close()
