"""Pins of the CPU oracle against things other than itself: a hand-computed example,
exact rational brute force in a different formulation, library routines the method
reduces to on special trees, and invariants of the distance."""
from __future__ import annotations

import itertools
import json
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.spatial import distance as spd

from oracle import exact, oracle
from synth import Problem, workload_problem, make_rng

from helpers import euler_tour_counts, leaves_of, relabel, table_rows, tiny_problem

UW, WN, WU = oracle.UNWEIGHTED, oracle.WEIGHTED_NORMALIZED, oracle.WEIGHTED_UNNORMALIZED


def _golden(golden_dir):
    with open(os.path.join(golden_dir, "worked_example.json")) as f:
        g = json.load(f)
    samples = np.array(g["samples"], dtype=np.int64)
    n = samples.shape[0]
    rows_i = [np.flatnonzero(r) for r in samples]
    indptr = np.zeros(n + 1, np.int64)
    indptr[1:] = np.cumsum([len(r) for r in rows_i])
    prob = Problem(parent=np.array(g["tree"]["parent"], np.int32),
                   length=np.array(g["tree"]["length"], np.float64),
                   feature_node=np.array(g["features"]["feature_node"], np.int32),
                   indptr=indptr,
                   indices=np.concatenate(rows_i).astype(np.int32),
                   counts=np.concatenate([samples[k][rows_i[k]] for k in range(n)]).astype(np.int32),
                   n_features=samples.shape[1])
    return g, prob


def test_worked_example_oracle(golden_dir):
    g, prob = _golden(golden_dir)
    for key, method in (("unweighted", UW), ("weighted_normalized", WN)):
        want = np.array([float(Fraction(s)) for s in g[key]])
        got = oracle.problem_condensed(prob, method)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-15)


def test_worked_example_exact(golden_dir):
    g, prob = _golden(golden_dir)
    rows = table_rows(prob)
    assert exact.unweighted(prob.parent, prob.length, rows, prob.feature_node) == \
        [Fraction(s) for s in g["unweighted"]]
    assert exact.weighted_normalized(prob.parent, prob.length, rows, prob.feature_node) == \
        [Fraction(s) for s in g["weighted_normalized"]]


def test_worked_example_counts(golden_dir):
    g, prob = _golden(golden_dir)
    c = oracle.problem_counts(prob)
    names = g["tree"]["node_names"]
    for v, name in enumerate(names):
        assert list(c[:, v]) == g["subtree_counts_by_node"][name]


@pytest.mark.parametrize("seed", range(40))
def test_bruteforce_exact(seed):
    prob = tiny_problem(1000 + seed, max_nodes=14, max_samples=6)
    rows = table_rows(prob)
    for method, fn in ((UW, exact.unweighted), (WN, exact.weighted_normalized),
                       (WU, exact.weighted_unnormalized)):
        want = np.array([float(x) for x in fn(prob.parent, prob.length, rows, prob.feature_node)])
        got = oracle.problem_condensed(prob, method)
        # each product L*p rounds once (<= u relative), the compensated sums add < u, the
        # division 0.5u: |rel err| <= ~4.5u = 5e-16 for num/den in FP64
        np.testing.assert_allclose(got, want, rtol=1e-15, atol=1e-300)


@pytest.mark.parametrize("seed", range(10))
def test_walkup_counts_match_euler_tour_and_exact(seed):
    prob = tiny_problem(2000 + seed, max_nodes=40, max_samples=5, max_count=9)
    walk = oracle.problem_counts(prob)
    np.testing.assert_array_equal(walk, euler_tour_counts(prob))
    np.testing.assert_array_equal(walk, np.array(exact.subtree_counts(prob.parent, table_rows(prob),
                                                                      prob.feature_node)))


def test_walkup_counts_invariants_config1_shape():
    prob = workload_problem("binary_256", n=64)
    c = oracle.problem_counts(prob)
    np.testing.assert_array_equal(c, euler_tour_counts(prob))
    root = int(np.flatnonzero(prob.parent < 0)[0])
    tot = np.add.reduceat(prob.counts.astype(np.int64), prob.indptr[:-1])
    np.testing.assert_array_equal(c[:, root], tot)
    child_sum = np.zeros_like(c)
    nz = np.flatnonzero(prob.parent >= 0)
    np.add.at(child_sum.T, prob.parent[nz], c[:, nz].T)
    internal = np.unique(prob.parent[nz])
    np.testing.assert_array_equal(child_sum[:, internal], c[:, internal])


def _star(n_tips, n_samples, seed, unit=True):
    rng = make_rng(seed)
    parent = np.full(n_tips + 1, n_tips, np.int32)
    parent[n_tips] = -1
    length = np.ones(n_tips + 1) if unit else rng.exponential(1.0, n_tips + 1)
    length[n_tips] = 0.0
    dense = rng.integers(0, 6, size=(n_samples, n_tips))
    dense[rng.random(dense.shape) < 0.5] = 0
    dense[:, 0] += (dense.sum(axis=1) == 0)
    rows_i = [np.flatnonzero(r) for r in dense]
    indptr = np.zeros(n_samples + 1, np.int64)
    indptr[1:] = np.cumsum([len(r) for r in rows_i])
    prob = Problem(parent=parent, length=length, feature_node=np.arange(n_tips, dtype=np.int32),
                   indptr=indptr, indices=np.concatenate(rows_i).astype(np.int32),
                   counts=np.concatenate([dense[k][rows_i[k]] for k in range(n_samples)]).astype(np.int32),
                   n_features=n_tips)
    return prob, dense, length[:n_tips]


@pytest.mark.parametrize("unit", [True, False])
def test_star_tree_reduces_to_jaccard_and_braycurtis(unit):
    prob, dense, w = _star(30, 12, 77 if unit else 78, unit=unit)
    pres = dense > 0
    prop = dense / dense.sum(axis=1, keepdims=True)
    uw = oracle.problem_condensed(prob, UW)
    wn = oracle.problem_condensed(prob, WN)
    wu = oracle.problem_condensed(prob, WU)
    k = 0
    for i in range(dense.shape[0]):
        for j in range(i + 1, dense.shape[0]):
            ww = None if unit else w
            assert abs(uw[k] - spd.jaccard(pres[i], pres[j], w=ww)) <= 1e-15
            assert abs(wn[k] - spd.braycurtis(prop[i], prop[j], w=ww)) <= 1e-15
            # weighted unnormalized on a star tree: length-weighted L1 of proportions
            assert abs(wu[k] - spd.cityblock(prop[i], prop[j], w=ww)) <= 1e-14
            k += 1


def _moderate(seed=5, dyadic=False, **kw):
    # 30 % of 300 tips nonzero keeps row totals (~1,800) above the rarefaction depth
    spec = dict(n=40, tips=300, p_nonzero=0.3)
    spec.update(kw)
    if dyadic:
        spec["dyadic"] = True
        spec["depth"] = 512
    return workload_problem("binary_256", seed=seed, **spec)


@pytest.mark.parametrize("method", [UW, WN])
def test_invariants_symmetry_range_identity(method):
    prob = _moderate()
    n = prob.n_samples
    i, j = oracle.condensed_pairs(n)
    d = oracle.problem_pairs(prob, method, i, j)
    dT = oracle.problem_pairs(prob, method, j, i)
    np.testing.assert_array_equal(d, dT)
    assert np.all(d >= 0) and np.all(d <= 1)
    same = oracle.problem_pairs(prob, method, np.arange(n), np.arange(n))
    assert np.all(same == 0.0)


def test_unweighted_triangle_inequality():
    prob = _moderate(seed=9, n=30)
    n = prob.n_samples
    D = np.zeros((n, n))
    i, j = oracle.condensed_pairs(n)
    d = oracle.problem_pairs(prob, UW, i, j)
    D[i, j] = d
    D[j, i] = d
    for a, b, c in itertools.permutations(range(n), 3):
        assert D[a, c] <= D[a, b] + D[b, c] + 1e-15


@pytest.mark.parametrize("method", [UW, WN])
def test_length_power_of_two_scaling_bit_identical(method):
    prob = _moderate(seed=11)
    base = oracle.problem_condensed(prob, method)
    for m in (-3, 5):
        p2 = Problem(**{**prob.__dict__, "length": prob.length * 2.0 ** m})
        np.testing.assert_array_equal(oracle.problem_condensed(p2, method), base)


def test_count_scaling_bit_identical():
    prob = _moderate(seed=12)
    base = oracle.problem_condensed(prob, WN)
    p3 = Problem(**{**prob.__dict__, "counts": prob.counts * 3})
    np.testing.assert_array_equal(oracle.problem_condensed(p3, WN), base)


@pytest.mark.parametrize("method", [UW, WN])
def test_sample_permutation(method):
    prob = _moderate(seed=13, n=25)
    n = prob.n_samples
    perm = make_rng(3).permutation(n)
    i, j = oracle.condensed_pairs(n)
    base = oracle.problem_pairs(prob, method, i, j)
    rows = [(prob.indices[prob.indptr[k]:prob.indptr[k + 1]], prob.counts[prob.indptr[k]:prob.indptr[k + 1]])
            for k in perm]
    indptr = np.zeros(n + 1, np.int64)
    indptr[1:] = np.cumsum([len(r[0]) for r in rows])
    pp = Problem(**{**prob.__dict__, "indptr": indptr,
                    "indices": np.concatenate([r[0] for r in rows]),
                    "counts": np.concatenate([r[1] for r in rows])})
    # pair (a, b) of the permuted table is pair (perm[a], perm[b]) of the original
    got = oracle.problem_pairs(pp, method, i, j)
    want = oracle.problem_pairs(prob, method, perm[i], perm[j])
    np.testing.assert_array_equal(got, want)
    assert base.shape == got.shape


@pytest.mark.parametrize("method", [UW, WN])
def test_relabel_unary_and_empty_tips_dyadic_exact(method):
    prob = _moderate(seed=14, dyadic=True)
    base = oracle.problem_condensed(prob, method)
    N = prob.n_nodes
    # relabel node ids
    perm = make_rng(4).permutation(N)
    p1 = Problem(**{**prob.__dict__, "parent": relabel(prob.parent, perm).astype(np.int32),
                    "length": prob.length[np.argsort(perm)],
                    "feature_node": perm[prob.feature_node].astype(np.int32)})
    np.testing.assert_array_equal(oracle.problem_condensed(p1, method), base)
    # split every tip's branch into a unary chain of two halves, and hang an extra tip with
    # no reads below the root
    tips = prob.feature_node
    parent = np.concatenate([prob.parent, prob.parent[tips], [int(np.flatnonzero(prob.parent < 0)[0])]])
    newmid = np.arange(N, N + tips.shape[0])
    parent[tips] = newmid
    length = np.concatenate([prob.length, prob.length[tips] / 2, [0.75]])
    length[tips] = length[tips] / 2
    p2 = Problem(**{**prob.__dict__, "parent": parent.astype(np.int32), "length": length,
                    "feature_node": np.concatenate([tips, [parent.shape[0] - 1]]).astype(np.int32),
                    "n_features": prob.n_features + 1})
    np.testing.assert_array_equal(oracle.problem_condensed(p2, method), base)


def _ill_conditioned_star(n_tiny: int = 4096):
    """Two samples on a star tree whose branch sums lose every small term under plain
    FP64 summation in node-id order: tip 0 (length 1) holds a read of both samples, tip 1
    (length 1) one of sample 0 only, then n_tiny tips of length 2^-53 a read of sample 0
    only.  Each tiny term is below half an ulp of the running sum, so an uncompensated sum
    drops all of them (a relative error near n_tiny * 2^-54 ~ 2e-13), while the exact
    value, and a compensated sum, keep them."""
    n_tips = 2 + n_tiny
    parent = np.full(n_tips + 1, n_tips, np.int32)
    parent[n_tips] = -1
    length = np.empty(n_tips + 1)
    length[:2] = 1.0
    length[2:n_tips] = 2.0 ** -53
    length[n_tips] = 0.0
    s0 = np.arange(n_tips, dtype=np.int32)
    s1 = np.array([0], np.int32)
    prob = Problem(parent=parent, length=length, feature_node=np.arange(n_tips, dtype=np.int32),
                   indptr=np.array([0, s0.size, s0.size + 1], np.int64),
                   indices=np.concatenate([s0, s1]),
                   counts=np.ones(s0.size + 1, np.int32), n_features=n_tips)
    return prob


def test_compensated_sums_ill_conditioned_exact():
    """The oracle's sums must be compensated: plain summation fails this exact case."""
    prob = _ill_conditioned_star()
    rows = table_rows(prob)
    for method, fn in ((UW, exact.unweighted), (WN, exact.weighted_normalized),
                       (WU, exact.weighted_unnormalized)):
        want = fn(prob.parent, prob.length, rows, prob.feature_node)[0]
        got = oracle.problem_condensed(prob, method)[0]
        # the exact value differs from what plain summation gives by ~2e-13 relative;
        # compensated FP64 stays within a few ulp
        assert abs(Fraction(float(got)) - want) <= Fraction(1, 10 ** 15) * abs(want), method


def test_zero_length_tree_gives_zero():
    prob = tiny_problem(5, max_nodes=10)
    p0 = Problem(**{**prob.__dict__, "length": np.zeros_like(prob.length)})
    assert np.all(oracle.problem_condensed(p0, UW) == 0)
    assert np.all(oracle.problem_condensed(p0, WN) == 0)


# --------------------------------------------------------------------- planted mistakes

MUTANTS = {
    "unnormalized divides": ("            out[p] = N;\n", "            out[p] = (D == 0.0) ? 0.0 : N / D;\n"),
    "abs dropped": ("L * fabs(pi - pj)", "L * (pi - pj)"),
    "den drops q": ("L * (pi + pj)", "L * (pi)"),
    "xor as and": ("(x != y) ? L : 0.0", "(x && y) ? L : 0.0"),
    "root branch kept": ("if (parent[v] < 0) continue;            /* the root has no branch */", ""),
    "wrong total": ("double pj = (double)cj[v] / tj;", "double pj = (double)cj[v] / ti;"),
    "tip not counted": ("row[v] += c;\n                v = parent[v];", "v = parent[v];\n                if (v >= 0) row[v] += c;"),
    "no compensation": ("double N = num + num_c, D = den + den_c;", "double N = num, D = den;"),
    "Neumaier branch swapped": ("if (fabs(*sum) >= fabs(x))", "if (fabs(*sum) < fabs(x))"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistakes_are_caught(name, tmp_path, golden_dir):
    """Compile a copy of the oracle with one plausible mistake and check that the pins
    above reject it (on the CPU, in a temporary directory)."""
    import ctypes
    import subprocess
    src = open(os.path.join(os.path.dirname(oracle.__file__), "uf_oracle.c")).read()
    old, new = MUTANTS[name]
    assert old in src, name
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / "mut.so"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", str(mut), "-o", str(so), "-lm"])
    lib = ctypes.CDLL(str(so))
    saved = oracle._lib
    try:
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        lib.uf_oracle_counts.argtypes = [i32, P, i32, i32, P, P, P, P, i32, P, P]
        lib.uf_oracle_pairs.argtypes = [i32, P, P, i32, P, P, i32, i64, P, P, P, i32]
        lib.uf_oracle_max_threads.restype = ctypes.c_int
        oracle._lib = lib
        caught = False
        try:
            test_worked_example_oracle(golden_dir)
        except AssertionError:
            caught = True
        for seed in range(10):
            if caught:
                break
            try:
                test_bruteforce_exact(seed)
            except AssertionError:
                caught = True
        if not caught:
            try:
                test_compensated_sums_ill_conditioned_exact()
            except AssertionError:
                caught = True
        assert caught, f"mutant '{name}' survived the pins"
    finally:
        oracle._lib = saved


# ------------------------------------------------------------------------- Mantel statistic

def test_mantel_pearson_matches_scipy():
    from scipy.stats import pearsonr
    from oracle import mantel as M
    rng = make_rng(21)
    for _ in range(5):
        x = rng.random(300)
        y = 0.3 * x + rng.random(300)
        assert abs(M.pearson(x, y) - pearsonr(x, y)[0]) <= 1e-14


def test_mantel_permutation_pins():
    from itertools import permutations as all_perms
    from oracle import mantel as M
    n = 5
    rng = make_rng(22)
    x = rng.random(n * (n - 1) // 2)
    y = x + 0.5 * rng.random(x.size)
    ident = [np.arange(n)]
    r, p, rp = M.mantel(x, y, n, ident)
    assert rp[0] == pytest.approx(r, abs=1e-15) and p == 1.0
    r1, _, _ = M.mantel(x, x, n, [])
    assert r1 == pytest.approx(1.0, abs=1e-15)
    # relabelling y by sigma and testing with sigma^-1 restores the original matrix
    sigma = rng.permutation(n)
    inv = np.argsort(sigma)
    ys = M.relabel(y, n, sigma)
    assert M.pearson(x, M.relabel(ys, n, inv)) == pytest.approx(r, abs=1e-15)
    # full enumeration: the exact permutation distribution contains the observed value
    perms = [np.array(q) for q in all_perms(range(n))]
    _, p_all, rp_all = M.mantel(x, y, n, perms)
    assert np.any(np.isclose(rp_all, r)) and 1 / 121 <= p_all <= 1
