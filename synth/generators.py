"""Seeded generators for the synthetic UniFrac workloads.

Every random number comes from numpy's Philox-4x64 counter-based generator (Salmon et al.,
"Parallel random numbers: as easy as 1, 2, 3", SC 2011), so a given seed yields the same
arrays on every machine and for every thread count.

The paper measures on the Earth Microbiome Project table and on a 113,721-sample table,
neither of which is available here; these generators stand in for them with trees, length
and count distributions of the same kind (sparse, over-dispersed counts rarefied to a fixed
depth, on trees with hundreds of thousands of tips).

Representation shared by all consumers:
  parent[N]        int32, parent node id, -1 for the (single) root
  length[N]        float64, length of the branch above each node (0.0 at the root)
  feature_node[F]  int32, node id of the tip that feature f sits on (tips = leaves)
  indptr[n+1]      int64, CSR row pointers (one row per sample)
  indices[nnz]     int32, feature ids
  counts[nnz]      int32, counts (> 0)
"""
from __future__ import annotations

import os
from dataclasses import dataclass, field

import numpy as np

MASTER_SEED = 20050526


def make_rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(int(seed)))


@dataclass
class Problem:
    parent: np.ndarray
    length: np.ndarray
    feature_node: np.ndarray
    indptr: np.ndarray
    indices: np.ndarray
    counts: np.ndarray
    n_features: int
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.parent.shape[0])

    @property
    def n_samples(self) -> int:
        return int(self.indptr.shape[0] - 1)

    def dense_table(self) -> np.ndarray:
        """Dense [n_samples][n_features] int64 table (small problems only)."""
        out = np.zeros((self.n_samples, self.n_features), dtype=np.int64)
        rows = np.repeat(np.arange(self.n_samples), np.diff(self.indptr))
        np.add.at(out, (rows, self.indices), self.counts)
        return out


# ----------------------------------------------------------------------------- trees

def random_binary_tree(n_tips: int, rng: np.random.Generator) -> tuple[np.ndarray, np.ndarray]:
    """Uniform random rooted binary tree by edge attachment (Remy's procedure).

    Starting from a single tip, each step picks one of the current edges uniformly (the
    edges above every node, counting an edge above the root) and splits it with a new
    internal node that also carries a new tip.  Returns (parent, tips) with 2*n_tips-1
    nodes; tips are listed in creation order.
    """
    if n_tips < 1:
        raise ValueError("n_tips must be >= 1")
    n_nodes = 2 * n_tips - 1
    parent = np.full(n_nodes, -1, dtype=np.int64)
    tips = np.empty(n_tips, dtype=np.int64)
    tips[0] = 0
    u = rng.random(n_tips)
    root = 0
    cur = 1
    par = parent  # local alias for the loop
    for step in range(1, n_tips):
        x = int(u[step] * cur)
        if x >= cur:
            x = cur - 1
        m = cur
        t = cur + 1
        cur += 2
        par[m] = par[x]
        if x == root:
            root = m
        par[x] = m
        par[t] = m
        tips[step] = t
    return parent.astype(np.int32), tips.astype(np.int32)


def coalescent_tree(n_tips: int, rng: np.random.Generator) -> tuple[np.ndarray, np.ndarray]:
    """Random coalescent topology: repeatedly merge two uniformly chosen lineages.

    Tips are nodes 0..n_tips-1, internal nodes are created in merge order and the last one
    is the root.
    """
    if n_tips < 1:
        raise ValueError("n_tips must be >= 1")
    n_nodes = 2 * n_tips - 1
    parent = np.full(n_nodes, -1, dtype=np.int64)
    lineages = list(range(n_tips))
    u = rng.random((max(n_tips - 1, 0), 2))
    m = n_tips
    for step in range(n_tips - 1):
        size = len(lineages)
        a = int(u[step, 0] * size)
        a = min(a, size - 1)
        na = lineages[a]
        lineages[a] = lineages[-1]
        lineages.pop()
        size -= 1
        b = int(u[step, 1] * size)
        b = min(b, size - 1)
        nb = lineages[b]
        parent[na] = m
        parent[nb] = m
        lineages[b] = m
        m += 1
    return parent.astype(np.int32), np.arange(n_tips, dtype=np.int32)


def exp_lengths(parent: np.ndarray, mean: float, rng: np.random.Generator) -> np.ndarray:
    """i.i.d. Exp(mean) branch lengths, 0.0 at the root."""
    length = rng.exponential(mean, size=parent.shape[0])
    length[parent < 0] = 0.0
    return length.astype(np.float64)


def dyadic_lengths(parent: np.ndarray, rng: np.random.Generator, max_m: int = 255,
                   shift: int = 8) -> np.ndarray:
    """Lengths m * 2**-shift with m uniform in 1..max_m (exact in bf16 when max_m <= 256)."""
    m = rng.integers(1, max_m + 1, size=parent.shape[0])
    length = m.astype(np.float64) * 2.0 ** (-shift)
    length[parent < 0] = 0.0
    return length


# ----------------------------------------------------------------------------- counts

def ztnb(size: int, mean: float, alpha: float, rng: np.random.Generator) -> np.ndarray:
    """Zero-truncated negative binomial: mean `mean`, variance mean + alpha*mean^2 before
    truncation; zeros are redrawn."""
    r = 1.0 / alpha
    p = r / (r + mean)
    out = rng.negative_binomial(r, p, size=size).astype(np.int64)
    bad = np.flatnonzero(out == 0)
    while bad.size:
        out[bad] = rng.negative_binomial(r, p, size=bad.size)
        bad = bad[out[bad] == 0]
    return out


def rarefy_rows(rows_idx: list[np.ndarray], rows_cnt: list[np.ndarray], depth: int,
                rng: np.random.Generator) -> tuple[list[np.ndarray], list[np.ndarray]]:
    """Subsample each row without replacement to exactly `depth` reads (multivariate
    hypergeometric); features that lose all reads are dropped."""
    out_i, out_c = [], []
    for idx, cnt in zip(rows_idx, rows_cnt):
        sub = rng.multivariate_hypergeometric(cnt.astype(np.int64), depth, method="marginals")
        keep = sub > 0
        out_i.append(idx[keep])
        out_c.append(sub[keep])
    return out_i, out_c


def _to_csr(rows_idx, rows_cnt):
    lens = np.array([len(r) for r in rows_idx], dtype=np.int64)
    indptr = np.zeros(len(rows_idx) + 1, dtype=np.int64)
    np.cumsum(lens, out=indptr[1:])
    if len(rows_idx):
        indices = np.concatenate(rows_idx).astype(np.int32)
        counts = np.concatenate(rows_cnt).astype(np.int32)
    else:
        indices = np.zeros(0, np.int32)
        counts = np.zeros(0, np.int32)
    return indptr, indices, counts


_MAX_REDRAWS = 1000


def _redraw_guard(attempt: int):
    if attempt >= _MAX_REDRAWS:
        raise ValueError("rarefaction depth is out of reach for this table shape "
                         f"({_MAX_REDRAWS} redraws of one sample fell below it)")


def table_sparse_nb(n_samples: int, n_features: int, p_nonzero: float, nb_mean: float,
                    nb_alpha: float, depth: int | None, rng: np.random.Generator):
    """Each feature is nonzero in a sample with probability p_nonzero, with a ZTNB count;
    rows are rarefied to `depth` (a row whose total is below depth is redrawn)."""
    rows_idx, rows_cnt = [], []
    for _ in range(n_samples):
        for attempt in range(_MAX_REDRAWS + 1):
            _redraw_guard(attempt)
            k = int(rng.binomial(n_features, p_nonzero))
            if k == 0:
                continue
            idx = np.sort(rng.choice(n_features, size=k, replace=False))
            cnt = ztnb(k, nb_mean, nb_alpha, rng)
            if depth is None or cnt.sum() >= depth:
                break
        rows_idx.append(idx)
        rows_cnt.append(cnt)
    if depth is not None:
        rows_idx, rows_cnt = rarefy_rows(rows_idx, rows_cnt, depth, rng)
    return _to_csr(rows_idx, rows_cnt)


def table_fixed_nb(n_samples: int, n_features: int, k_per_sample: int, nb_mean: float,
                   nb_alpha: float, depth: int | None, rng: np.random.Generator):
    """About k_per_sample distinct features per sample drawn uniformly, ZTNB counts,
    rarefied to `depth` (rows below depth are redrawn)."""
    k_per_sample = min(k_per_sample, n_features)
    rows_idx, rows_cnt = [], []
    for _ in range(n_samples):
        for attempt in range(_MAX_REDRAWS + 1):
            _redraw_guard(attempt)
            idx = np.sort(rng.choice(n_features, size=k_per_sample, replace=False))
            cnt = ztnb(k_per_sample, nb_mean, nb_alpha, rng)
            if depth is None or cnt.sum() >= depth:
                break
        rows_idx.append(idx)
        rows_cnt.append(cnt)
    if depth is not None:
        rows_idx, rows_cnt = rarefy_rows(rows_idx, rows_cnt, depth, rng)
    return _to_csr(rows_idx, rows_cnt)


def table_zipf_presence(n_samples: int, n_features: int, k_per_sample: int, zipf_s: float,
                        rng: np.random.Generator):
    """Exactly k_per_sample distinct features per sample, drawn one after another without
    replacement with probability proportional to rank**-zipf_s (ranks are a seeded
    permutation of the features); every count is 1."""
    k_per_sample = min(k_per_sample, n_features)
    perm = rng.permutation(n_features)            # perm[r] = feature of rank r+1
    w = np.arange(1, n_features + 1, dtype=np.float64) ** (-zipf_s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    rows_idx, rows_cnt = [], []
    for _ in range(n_samples):
        chosen = np.empty(0, dtype=np.int64)
        draw = max(4 * k_per_sample, 64)
        while chosen.size < k_per_sample:
            r = np.searchsorted(cdf, rng.random(draw), side="right")
            r = np.minimum(r, n_features - 1)
            allr = np.concatenate([chosen, r])
            _, first = np.unique(allr, return_index=True)
            chosen = allr[np.sort(first)]
            draw *= 2
        ranks = chosen[:k_per_sample]
        idx = np.sort(perm[ranks])
        rows_idx.append(idx)
        rows_cnt.append(np.ones(k_per_sample, dtype=np.int64))
    return _to_csr(rows_idx, rows_cnt)


# ----------------------------------------------------------------------------- workloads

# Named synthetic workloads; seed_offset fixes each one's default seed (MASTER_SEED + offset).
WORKLOADS = {
    # 256 samples, random binary tree with 2,048 tips, Exp(0.05) lengths, 95 % zeros,
    # ZTNB(20, 0.5) counts rarefied to 1,000; FP64 unweighted + weighted normalized.
    "binary_256": dict(n=256, tips=2048, tree="binary", mean_len=0.05, table="sparse_nb",
                       p_nonzero=0.05, nb_mean=20.0, nb_alpha=0.5, depth=1000, seed_offset=1),
    # 4,096 samples, coalescent tree with 32,768 tips, ~800 features/sample, ZTNB(10, 0.3)
    # rarefied to 5,000; weighted normalized, FP64 vs FP32.
    "coalescent_4096": dict(n=4096, tips=32768, tree="coalescent", mean_len=0.05, table="fixed_nb",
                            k=800, nb_mean=10.0, nb_alpha=0.3, depth=5000, seed_offset=2),
    # 25,000 samples, random binary tree with 300,000 tips, Exp(0.02), 1,500 present
    # features/sample with Zipf(1.1) prevalence; unweighted (MFMA vs FP64 striped).
    "zipf_25000": dict(n=25000, tips=300000, tree="binary", mean_len=0.02, table="zipf_presence",
                       k=1500, zipf_s=1.1, seed_offset=3),
    # 113,000 samples, random binary tree with 500,000 tips, ~1,000 features/sample,
    # ZTNB(8, 0.3) rarefied to 2,000.
    "binary_113000": dict(n=113000, tips=500000, tree="binary", mean_len=0.02, table="fixed_nb",
                          k=1000, nb_mean=8.0, nb_alpha=0.3, depth=2000, seed_offset=5),
}


def _build(spec: dict, rng: np.random.Generator) -> Problem:
    tips_n = int(spec["tips"])
    if spec["tree"] == "binary":
        parent, tips = random_binary_tree(tips_n, rng)
    elif spec["tree"] == "coalescent":
        parent, tips = coalescent_tree(tips_n, rng)
    else:
        raise ValueError(spec["tree"])
    if spec.get("dyadic"):
        length = dyadic_lengths(parent, rng)
    else:
        length = exp_lengths(parent, float(spec["mean_len"]), rng)
    n = int(spec["n"])
    kind = spec["table"]
    if kind == "sparse_nb":
        indptr, indices, counts = table_sparse_nb(n, tips_n, spec["p_nonzero"], spec["nb_mean"],
                                                  spec["nb_alpha"], spec.get("depth"), rng)
    elif kind == "fixed_nb":
        indptr, indices, counts = table_fixed_nb(n, tips_n, int(spec["k"]), spec["nb_mean"],
                                                 spec["nb_alpha"], spec.get("depth"), rng)
    elif kind == "zipf_presence":
        indptr, indices, counts = table_zipf_presence(n, tips_n, int(spec["k"]), spec["zipf_s"], rng)
    else:
        raise ValueError(kind)
    return Problem(parent=parent, length=length, feature_node=tips.astype(np.int32),
                   indptr=indptr, indices=indices, counts=counts, n_features=tips_n,
                   meta=dict(spec))


def workload_problem(name: str, seed: int | None = None, **overrides) -> Problem:
    """The synthetic problem of the named workload, optionally with fields overridden (e.g.
    n=300, tips=3000 for a scaled-down case of the same kind)."""
    spec = dict(WORKLOADS[name])
    spec.update(overrides)
    if seed is None:
        seed = MASTER_SEED + spec["seed_offset"]
    spec["seed"] = int(seed)
    spec["workload"] = name
    return _build(spec, make_rng(seed))


def batch_job_specs(n_jobs: int = 64, seed: int | None = None, n_range=(200, 8000),
                    tips_range=(1000, 64000)) -> list[dict]:
    """Specs of the uneven batch: n ~ U{n_range}, tips ~ U{tips_range}, everything else as
    the 256-sample binary-tree workload.  Job j is generated from seed + 1000*j."""
    if seed is None:
        seed = MASTER_SEED + 4
    rng = make_rng(seed)
    ns = rng.integers(n_range[0], n_range[1] + 1, size=n_jobs)
    ts = rng.integers(tips_range[0], tips_range[1] + 1, size=n_jobs)
    specs = []
    for j in range(n_jobs):
        spec = dict(WORKLOADS["binary_256"])
        spec.update(n=int(ns[j]), tips=int(ts[j]), seed=int(seed + 1000 * (j + 1)), job=j)
        specs.append(spec)
    return specs


def build_job(spec: dict) -> Problem:
    return _build(spec, make_rng(spec["seed"]))


def build_jobs(specs: list[dict], workers: int = 0) -> list[Problem]:
    """build_job for every spec, in a pool of fresh interpreter processes (spawned, so no
    state of the calling process, such as an open GPU, is inherited).  Every job comes from
    its own seed, so the result does not depend on the number of workers.  workers <= 0:
    one per CPU, at most 16; 1: in this process."""
    if workers <= 0:
        workers = min(16, os.cpu_count() or 1, len(specs))
    if workers <= 1 or len(specs) <= 1:
        return [build_job(s) for s in specs]
    import multiprocessing as mp
    # largest jobs first so the pool's tail is short; results go back in spec order
    order = sorted(range(len(specs)), key=lambda j: -int(specs[j]["n"]) * int(specs[j]["tips"]))
    # the workers are closed and joined, not terminated: they exit by themselves once the
    # work is done, with no signal (a profiler preloaded into them may not survive one)
    pool = mp.get_context("spawn").Pool(workers)
    try:
        built = pool.map(build_job, [specs[j] for j in order], chunksize=1)
    except BaseException:
        pool.terminate()
        raise
    pool.close()
    pool.join()
    out: list = [None] * len(specs)
    for j, prob in zip(order, built):
        out[j] = prob
    return out


def permutations(n: int, n_perm: int, seed: int) -> np.ndarray:
    """[n_perm][n] int32, each row a uniform random permutation of 0..n-1."""
    rng = make_rng(seed)
    return np.stack([rng.permutation(n) for _ in range(n_perm)]).astype(np.int32) if n_perm \
        else np.zeros((0, n), np.int32)
