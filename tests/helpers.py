"""Small helpers shared by the tests: tiny random trees and tables, Euler-tour counts,
and conversions between CSR tables and per-sample dicts.  No UniFrac arithmetic here
beyond the independent Euler-tour count method used as a pin."""
from __future__ import annotations

import numpy as np

from synth import Problem, make_rng


def random_recursive_tree(n_nodes: int, rng) -> np.ndarray:
    """Each new node attaches below a uniformly chosen earlier node: any shape, with
    multifurcations and unary chains."""
    parent = np.full(n_nodes, -1, dtype=np.int32)
    for v in range(1, n_nodes):
        parent[v] = int(rng.integers(0, v))
    return parent


def leaves_of(parent: np.ndarray) -> np.ndarray:
    has_child = np.zeros(parent.shape[0], dtype=bool)
    has_child[parent[parent >= 0]] = True
    return np.flatnonzero(~has_child).astype(np.int32)


def relabel(parent: np.ndarray, perm: np.ndarray) -> np.ndarray:
    """New tree where old node v becomes node perm[v]."""
    newp = np.full_like(parent, -1)
    for v, p in enumerate(parent):
        newp[perm[v]] = -1 if p < 0 else perm[p]
    return newp


def tiny_problem(seed: int, max_nodes: int = 16, max_samples: int = 6, max_count: int = 5,
                 zero_p: float = 0.5, dyadic: bool = False) -> Problem:
    rng = make_rng(seed)
    n_nodes = int(rng.integers(2, max_nodes + 1))
    parent = random_recursive_tree(n_nodes, rng)
    if dyadic:
        length = rng.integers(0, 256, size=n_nodes).astype(np.float64) / 256.0
    else:
        length = rng.exponential(0.5, size=n_nodes)
        length[rng.random(n_nodes) < 0.1] = 0.0
    # the root has no branch: give it a nonzero length that every implementation must ignore
    length[parent < 0] = 0.75
    tips = leaves_of(parent)
    n_samples = int(rng.integers(2, max_samples + 1))
    rows_i, rows_c = [], []
    for _ in range(n_samples):
        while True:
            c = rng.integers(1, max_count + 1, size=tips.shape[0])
            c[rng.random(tips.shape[0]) < zero_p] = 0
            if c.sum() > 0:
                break
        nz = np.flatnonzero(c)
        rows_i.append(nz)
        rows_c.append(c[nz])
    indptr = np.zeros(n_samples + 1, np.int64)
    indptr[1:] = np.cumsum([len(r) for r in rows_i])
    return Problem(parent=parent, length=length, feature_node=tips,
                   indptr=indptr, indices=np.concatenate(rows_i).astype(np.int32),
                   counts=np.concatenate(rows_c).astype(np.int32), n_features=tips.shape[0])


def table_rows(prob: Problem) -> list[dict]:
    rows = []
    for k in range(prob.n_samples):
        d = {}
        for e in range(prob.indptr[k], prob.indptr[k + 1]):
            f = int(prob.indices[e])
            d[f] = d.get(f, 0) + int(prob.counts[e])
        rows.append(d)
    return rows


def euler_tour_counts(prob: Problem) -> np.ndarray:
    """[n_samples][n_nodes] counts from prefix sums over tips in depth-first order: the
    tips below v occupy a contiguous range [lo(v), hi(v)) of that order."""
    parent = np.asarray(prob.parent)
    n = parent.shape[0]
    children = [[] for _ in range(n)]
    root = -1
    for v in range(n):
        if parent[v] < 0:
            root = v
        else:
            children[parent[v]].append(v)
    lo = np.zeros(n, np.int64)
    hi = np.zeros(n, np.int64)
    tip_pos = {}
    pos = 0
    stack = [(root, False)]
    while stack:
        v, done = stack.pop()
        if done:
            hi[v] = pos
            continue
        lo[v] = pos
        if not children[v]:
            tip_pos[v] = pos
            pos += 1
            hi[v] = pos
            continue
        stack.append((v, True))
        for c in reversed(children[v]):
            stack.append((c, False))
    n_tips = pos
    dense = np.zeros((prob.n_samples, n_tips), np.int64)
    fn = np.asarray(prob.feature_node)
    rows = np.repeat(np.arange(prob.n_samples), np.diff(prob.indptr))
    cols = np.array([tip_pos[int(fn[f])] for f in prob.indices], dtype=np.int64)
    np.add.at(dense, (rows, cols), np.asarray(prob.counts, np.int64))
    prefix = np.zeros((prob.n_samples, n_tips + 1), np.int64)
    np.cumsum(dense, axis=1, out=prefix[:, 1:])
    return prefix[:, hi] - prefix[:, lo]


def condensed_index(n: int, i, j):
    i = np.asarray(i, np.int64)
    j = np.asarray(j, np.int64)
    return n * i - i * (i + 1) // 2 + (j - i - 1)
