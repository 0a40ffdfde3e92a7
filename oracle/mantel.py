"""Plain FP64 Mantel statistic for two condensed distance matrices (numpy).

TEST INFRASTRUCTURE ONLY.  Pearson's r over all pairs, and the two-sided permutation
p-value (1 + #{|r_perm| >= |r|}) / (1 + n_perm), where each permutation relabels the
samples of the second matrix.  The permutations are inputs, so the GPU and this code test
the same relabellings.
"""
from __future__ import annotations

import numpy as np


def pearson(x, y) -> float:
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    xm = x - x.mean()
    ym = y - y.mean()
    den = np.sqrt(np.dot(xm, xm) * np.dot(ym, ym))
    return float(np.dot(xm, ym) / den) if den > 0 else 0.0


def relabel(y, n: int, perm) -> np.ndarray:
    """Condensed y' with y'_ij = y_{perm[i], perm[j]}."""
    i, j = np.triu_indices(n, k=1)
    a, b = np.asarray(perm)[i], np.asarray(perm)[j]
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    return np.asarray(y)[n * lo - lo * (lo + 1) // 2 + (hi - lo - 1)]


def mantel(x, y, n: int, perms):
    r = pearson(x, y)
    rp = np.array([pearson(x, relabel(y, n, p)) for p in perms])
    p = (1 + np.count_nonzero(np.abs(rp) >= abs(r))) / (1 + len(rp)) if len(rp) else 1.0
    return r, p, rp
