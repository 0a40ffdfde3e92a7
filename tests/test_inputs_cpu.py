"""Every synthetic input the GPU tests build can be generated (CPU only), so a generator
problem never costs a GPU run."""
from __future__ import annotations

import pytest

import test_gpu_batch
import test_gpu_mfma
import test_gpu_parity


@pytest.mark.parametrize("name", sorted(test_gpu_parity.CASES))
def test_parity_cases_build(name):
    assert test_gpu_parity.CASES[name]().n_samples >= 1


@pytest.mark.parametrize("name", sorted(test_gpu_parity.EDGE))
def test_edge_cases_build(name):
    assert test_gpu_parity.EDGE[name]().n_samples >= 1


@pytest.mark.parametrize("name", sorted(test_gpu_mfma.CASES))
def test_mfma_cases_build(name):
    assert test_gpu_mfma.CASES[name]().n_samples >= 1


def test_batch_jobs_build():
    jobs = test_gpu_batch._jobs()
    assert len(jobs) == 7 and any(p.n_samples == 1 for p, _, _ in jobs)
