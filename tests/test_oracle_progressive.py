"""Pins of the progressive-sampling oracle."""
import math

import numpy as np
import pytest

from oracle.progressive import hoeffding_eps, progressive
from paper_2301_06499_amd import inputs as gen


@pytest.mark.parametrize("n", [100, 10_000, 1_000_000])
@pytest.mark.parametrize("eps", [0.3, 0.1, 0.05])
def test_theorem_sample_size(n, eps):
    # the error-bound theorem: s = ln(n) / eps^2 seeds give error at most eps
    # with probability at least 1 - 2 / n^2
    s = math.ceil(math.log(n) / eps ** 2)
    delta = 2.0 / n ** 2
    assert hoeffding_eps(s, delta) <= eps * (1 + 1e-12)
    assert hoeffding_eps(s - 1, delta) > eps * (1 - 1e-12) or s == 1


@pytest.mark.parametrize("s", [20, 200])
def test_half_width_covers_bernoulli_means(s):
    # values in [0, 1]: the mean of s fair coin flips strays from 1/2 by at
    # least eps in at most a delta fraction of trials; half of eps does not
    # cover (so the width is not off by a factor of two)
    rng = np.random.default_rng(5 + s)
    delta = 0.1
    trials = 20_000
    means = rng.integers(0, 2, size=(trials, s)).mean(axis=1)
    eps = hoeffding_eps(s, delta)
    assert np.mean(np.abs(means - 0.5) >= eps) <= delta
    assert np.mean(np.abs(means - 0.5) >= eps / 2) > delta


@pytest.mark.parametrize("n,group,target", [(50, 4, 10.0), (101, 8, 20.0), (64, 1, 40.0)])
def test_cycle_stops_at_the_closed_form_sample(n, group, target):
    # a cycle: every seed reaches every node, D = floor(n/2), alpha = 1, so
    # the run stops at the first multiple of `group` with D eps(s) <= target
    g = gen.cycle_graph(n)
    delta = 0.05
    pool = np.arange(n, dtype=np.int32) % n
    pool = np.concatenate([pool, pool, pool, pool])
    res = progressive(g.n, g.src, g.dst, pool, group, target, delta, g.undirected)
    D = n // 2
    s = group
    while D * math.sqrt(math.log(2 / delta) / (2 * s)) > target:
        s += group
    assert res["met"] and res["seeds"] == s and res["groups"] == s // group
    assert res["D"] == D and res["alpha"] == 1.0
    assert res["counts"][0] == s and res["counts"].sum() == s * n


def test_pool_runs_out():
    g = gen.path_graph(40)
    res = progressive(g.n, g.src, g.dst, np.arange(6, dtype=np.int32), 4, 0.01, 0.05, g.undirected)
    assert not res["met"] and res["seeds"] == 6 and res["groups"] == 2


def test_no_arcs_stops_at_once():
    res = progressive(5, np.zeros(0, np.int32), np.zeros(0, np.int32), np.arange(5, dtype=np.int32), 2, 0.0, 0.05, True)
    assert res["met"] and res["seeds"] == 2 and res["D"] == 0 and res["bound"] == 0.0
