"""Python front end of the FP64 CPU oracle (uf_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the benchmark's CPU
baseline, never by the library.  It does not import the GPU package and the GPU package
does not import it.

The arithmetic lives in uf_oracle.c (walk-up counts, per pair and per branch Neumaier sums
in FP64).  This module only marshals arrays, picks which samples a set of pairs touches,
and lays results out in condensed (scipy squareform) order: row i ascending, then j > i.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "uf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

UNWEIGHTED = 0
WEIGHTED_NORMALIZED = 1
WEIGHTED_UNNORMALIZED = 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    lib.uf_oracle_counts.argtypes = [i32, P, i32, i32, P, P, P, P, i32, P, P]
    lib.uf_oracle_counts.restype = ctypes.c_int
    lib.uf_oracle_pairs.argtypes = [i32, P, P, i32, P, P, i32, i64, P, P, P, i32]
    lib.uf_oracle_pairs.restype = ctypes.c_int
    lib.uf_oracle_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def max_threads() -> int:
    return int(_load().uf_oracle_max_threads())


def walkup_counts(parent, indptr, indices, counts, n_features, feature_node=None, samples=None):
    """[len(samples)][n_nodes] int64 walk-up counts (all samples if `samples` is None)."""
    lib = _load()
    parent = np.ascontiguousarray(parent, np.int32)
    indptr = np.ascontiguousarray(indptr, np.int64)
    indices = np.ascontiguousarray(indices, np.int32)
    counts = np.ascontiguousarray(counts, np.int32)
    fn = None if feature_node is None else np.ascontiguousarray(feature_node, np.int32)
    n_samples = indptr.shape[0] - 1
    sel = np.arange(n_samples, dtype=np.int32) if samples is None else \
        np.ascontiguousarray(samples, np.int32)
    out = np.empty((sel.shape[0], parent.shape[0]), dtype=np.int64)
    rc = lib.uf_oracle_counts(parent.shape[0], _ptr(parent), n_samples, int(n_features),
                              _ptr(indptr), _ptr(indices), _ptr(counts), _ptr(fn),
                              sel.shape[0], _ptr(sel), _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle counts failed with code {rc}")
    return out


def distance_pairs(parent, length, indptr, indices, counts, n_features, method, pi, pj,
                   feature_node=None, n_threads: int = 0):
    """FP64 distances for the sample pairs (pi[p], pj[p])."""
    lib = _load()
    parent = np.ascontiguousarray(parent, np.int32)
    length = np.ascontiguousarray(length, np.float64)
    pi = np.asarray(pi, np.int64)
    pj = np.asarray(pj, np.int64)
    used, inv = np.unique(np.concatenate([pi, pj]), return_inverse=True)
    a = np.ascontiguousarray(inv[: pi.shape[0]], np.int32)
    b = np.ascontiguousarray(inv[pi.shape[0]:], np.int32)
    rows = walkup_counts(parent, indptr, indices, counts, n_features, feature_node, used)
    indptr = np.asarray(indptr, np.int64)
    cs = np.concatenate([[0], np.cumsum(np.asarray(counts, np.int64))])
    tot_all = cs[indptr[1:]] - cs[indptr[:-1]]
    tot = np.ascontiguousarray(tot_all[used], np.int64)
    out = np.empty(pi.shape[0], dtype=np.float64)
    rc = lib.uf_oracle_pairs(parent.shape[0], _ptr(parent), _ptr(length), rows.shape[0],
                             _ptr(rows), _ptr(tot), int(method), pi.shape[0], _ptr(a), _ptr(b),
                             _ptr(out), int(n_threads))
    if rc != 0:
        raise ValueError(f"oracle pairs failed with code {rc}")
    return out


def condensed_pairs(n: int):
    """(i, j) index arrays of the condensed order: i ascending, then j > i ascending."""
    i, j = np.triu_indices(n, k=1)
    return i.astype(np.int64), j.astype(np.int64)


def distance_condensed(parent, length, indptr, indices, counts, n_features, method,
                       feature_node=None, n_threads: int = 0):
    n = int(np.asarray(indptr).shape[0] - 1)
    i, j = condensed_pairs(n)
    return distance_pairs(parent, length, indptr, indices, counts, n_features, method, i, j,
                          feature_node=feature_node, n_threads=n_threads)


def problem_condensed(prob, method, n_threads: int = 0):
    """Condensed distances of a synth.Problem-like object (attributes parent, length,
    indptr, indices, counts, n_features, feature_node)."""
    return distance_condensed(prob.parent, prob.length, prob.indptr, prob.indices, prob.counts,
                              prob.n_features, method, feature_node=prob.feature_node,
                              n_threads=n_threads)


def problem_pairs(prob, method, pi, pj, n_threads: int = 0):
    return distance_pairs(prob.parent, prob.length, prob.indptr, prob.indices, prob.counts,
                          prob.n_features, method, pi, pj, feature_node=prob.feature_node,
                          n_threads=n_threads)


def problem_counts(prob, samples=None):
    return walkup_counts(prob.parent, prob.indptr, prob.indices, prob.counts, prob.n_features,
                         prob.feature_node, samples)
