"""Host logic of the hierarchy optimisation loop: the log-uniform tau draw
and the batch sampling (no GPU)."""
from __future__ import annotations

import math

import numpy as np
import pytest

from paper_2406_12080_amd import optimize, synth


def test_log_uniform_tau_is_uniform_in_log_tau():
    rng = np.random.default_rng(0)
    tau = optimize.log_uniform_tau(rng, 200_000, 3.0, 15.0)
    assert tau.min() >= 3.0 and tau.max() <= 15.0
    u = (np.log(tau) - math.log(3.0)) / (math.log(15.0) - math.log(3.0))
    # deciles of a uniform variable
    q = np.quantile(u, np.linspace(0.1, 0.9, 9))
    assert np.abs(q - np.linspace(0.1, 0.9, 9)).max() < 5e-3
    # the geometric mean of the range is the median
    assert abs(np.median(tau) - math.sqrt(45.0)) < 0.05
    with pytest.raises(ValueError):
        optimize.log_uniform_tau(rng, 3, 0.0, 1.0)


def test_sample_draws_distinct_views_with_their_own_tau():
    opt = optimize.HierarchyOptimizer.__new__(optimize.HierarchyOptimizer)
    opt.views = [synth.look_at((3 * math.cos(a), 0, 3 * math.sin(a)), (0, 0, 0), (0, 1, 0), 64, 48, 0.0)
                 for a in np.linspace(0, 6, 10)]
    opt.batch, opt.tau_range, opt.rng = 4, (2.0, 16.0), np.random.default_rng(3)
    seen = set()
    for _ in range(50):
        idx, views = opt.sample()
        assert len(set(idx.tolist())) == 4
        for i, v in zip(idx, views):
            assert 2.0 <= v.tau <= 16.0
            assert np.array_equal(v.eye, opt.views[i].eye)
        seen |= set(idx.tolist())
    assert seen == set(range(10))
    opt.batch = 32  # more than the pool: every view once
    idx, _ = opt.sample()
    assert sorted(idx.tolist()) == list(range(10))
