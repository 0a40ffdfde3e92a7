"""GPU Mantel statistic (uf_mantel) against the numpy FP64 version, same permutations."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import mantel as M
from oracle import oracle
from synth import workload_problem, permutations

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def uf():
    import paper_2005_05826_amd as uf
    return uf


@pytest.fixture(scope="module")
def ctx(uf):
    return uf.Context(0)


def test_mantel_matches_numpy(uf, ctx):
    import torch
    prob = workload_problem("binary_256", n=120, tips=800, p_nonzero=0.2, seed=31)
    plan = uf.Plan.from_problem(ctx, prob)
    n = prob.n_samples
    x = plan.distance("weighted_normalized", "fp64")
    y = plan.distance("unweighted", "fp64")
    perms = permutations(n, 50, seed=5)
    r, p, rp = M.mantel(x, y, n, perms)
    dx = torch.from_numpy(x).cuda()
    dy = torch.from_numpy(y).cuda()
    dp = torch.from_numpy(perms).cuda()
    gr, gp, grp = uf.mantel(ctx, dx, dy, n, dp)
    assert abs(gr - r) <= 1e-12
    np.testing.assert_allclose(grp, rp, rtol=0, atol=1e-12)
    assert gp == p
    # FP32 striped vs FP64: the paper's precision criterion (Mantel R^2 >= 0.99999)
    x32 = torch.from_numpy(plan.distance("weighted_normalized", "fp32")).cuda()
    r32, _, _ = uf.mantel(ctx, x32, dx, n)
    assert r32 * r32 >= 0.99999


def test_mantel_rejects_bad_permutations(uf, ctx):
    import torch
    n = 10
    x = torch.rand(n * (n - 1) // 2, dtype=torch.float64, device="cuda:0")
    bad = torch.from_numpy(np.tile(np.arange(n, dtype=np.int32), (2, 1))).cuda()
    bad[1, 3] = 4      # repeated label
    with pytest.raises(uf.UniFracError) as ei:
        uf.mantel(ctx, x, x, n, bad)
    assert ei.value.status_name == "UF_E_ARG"
    bad[1, 3] = 99     # out of range
    with pytest.raises(uf.UniFracError):
        uf.mantel(ctx, x, x, n, bad)
