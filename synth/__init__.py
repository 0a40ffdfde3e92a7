"""Seeded synthetic inputs (trees, branch lengths, sample x feature count tables).

This package draws random inputs only.  It holds none of the UniFrac arithmetic, so both
the CPU oracle's tests and the GPU library can consume the same arrays without sharing
any of the method's code.
"""
from .generators import (  # noqa: F401
    MASTER_SEED,
    Problem,
    make_rng,
    random_binary_tree,
    coalescent_tree,
    exp_lengths,
    dyadic_lengths,
    ztnb,
    rarefy_rows,
    table_sparse_nb,
    table_fixed_nb,
    table_zipf_presence,
    workload_problem,
    batch_job_specs,
    WORKLOADS,
    build_job,
    build_jobs,
    permutations,
)
