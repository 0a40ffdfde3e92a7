"""Host logic of bench.py that needs no GPU: the one-GPU guard, the condensed index and the
sizing of the oracle sample behind the CPU baseline."""
from __future__ import annotations

import json
import os
import subprocess
import sys

import numpy as np

import bench
from synth import workload_problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    rec = json.loads(r.stdout.strip().splitlines()[-1])
    assert rec["n_gpus"] == 2 and "one GPU" in rec["error"]


def test_cond_index_is_squareform_order():
    n = 37
    i, j = np.triu_indices(n, k=1)
    np.testing.assert_array_equal(bench.cond_index(n, i.astype(np.int64), j.astype(np.int64)),
                                  np.arange(n * (n - 1) // 2))


def test_sample_pairs_are_ordered_distinct_and_in_range():
    rng = np.random.Generator(np.random.Philox(5))
    pi, pj = bench.sample_pairs(rng, 50, 4000)
    assert pi.size == pj.size and pi.size > 3000
    assert np.all(pi < pj) and pi.min() >= 0 and pj.max() < 50


def test_oracle_sample_grows_to_the_target_and_reports_its_size():
    prob = workload_problem("binary_256", n=64, tips=300, p_nonzero=0.3, seed=11)
    cpu, pi, pj, want = bench.oracle_sample(prob, "weighted_normalized", 0.5, 123)
    assert cpu["kind"] == "oracle" and cpu["cores"] >= 1
    assert cpu["unit"] == "pair-branch updates/s" and cpu["value"] > 0
    # the sample run took at least half the target or hit the size cap
    assert cpu["seconds"] >= 0.25 or pi.size >= 2_000_000
    assert want.shape == pi.shape and np.all((want >= 0) & (want <= 1))
    assert cpu["one_thread"]["pairs"] >= 16 and cpu["one_thread"]["value"] > 0
    assert str(pi.size) in cpu["sample"]


def test_nested_target_records_keep_their_figures_compactly():
    rec = {"metric": "m", "value": 441765807614559.3, "unit": "pair-branch updates/s", "steps": 3,
           "warmup": 1, "ms_per_step": 424.415, "dtype": "bf16",
           "config": {"workload": "x" * 200, "n_samples": 25000, "branches": 599998, "precision": "mfma_bf16x2"},
           "full_matrix_wall_ms": 424.415, "kernels_ms_per_step": {"mfma": 414.3},
           "roofline": {"kernel": "k_mfma_gemm", "bound": "mfma", "achieved": 1810.19, "peak": 2500.0,
                        "unit": "TFLOP/s", "frac": 0.7241, "traffic": 300525769216,
                        "traffic_detail": {"profile": "p" * 80}},
           "compare": {"precision": "fp64", "ms_per_step": 27704.0, "speedup_of_headline": 65.3,
                       "kernels_ms_per_step": {"stripe": 27676.8}},
           "end_to_end": {"ms": 819.2, "runs": 1, "what": "w" * 150},
           "cpu_baseline": {"value": 3969486239.6, "unit": "u", "cores": 16, "kind": "oracle",
                            "sample": "s" * 200, "seconds": 5.79, "one_thread": {"value": 124926253.6}},
           "error_vs_oracle": {"mfma_bf16x2": {"max_abs": 3.07580687142206e-07, "mean_abs": 6.1e-08,
                                               "pairs": 38301}},
           "wall_s": 68.9}
    out = bench.compact_target(rec)
    assert out["ms_per_step"] == 424.415 and out["roofline"]["frac"] == 0.7241
    assert out["roofline"]["traffic"] == 300525769216 and "traffic_detail" not in out["roofline"]
    assert out["compare"]["speedup_of_headline"] == 65.3 and out["end_to_end_ms"] == 819.2
    assert out["cpu_baseline"]["cores"] == 16 and out["cpu_baseline"]["one_thread_value"] > 0
    assert out["error_vs_oracle"]["mfma_bf16x2"]["max_abs"] == 3.08e-07
    assert out["config"] == {"n_samples": 25000, "branches": 599998, "precision": "mfma_bf16x2"}
    assert len(json.dumps(out)) < 1000
    err = {"error": "RuntimeError: boom", "wall_s": 1.0}
    assert bench.compact_target(err) == err
