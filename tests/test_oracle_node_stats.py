"""Pins of the per-node statistics oracle."""
import numpy as np
import pytest

import oracle
from oracle.node_stats import node_stats
from paper_2301_06499_amd import inputs as gen


def test_path_every_node_a_seed():
    # undirected path 0..L-1, every node a seed: u reaches all L nodes and
    # sum_v |u - v| = u(u+1)/2 + (L-1-u)(L-u)/2
    L = 23
    g = gen.path_graph(L)
    reached, ds = node_stats(L, g.src, g.dst, np.arange(L), g.undirected)
    u = np.arange(L)
    assert reached.tolist() == [L] * L
    assert ds.tolist() == (u * (u + 1) // 2 + (L - 1 - u) * (L - u) // 2).tolist()


def test_star_and_cycle():
    k = 9   # star: centre 0, leaves 1..k (undirected)
    g = gen.star_graph(k + 1)
    reached, ds = node_stats(k + 1, g.src, g.dst, np.arange(k + 1), g.undirected)
    assert reached.tolist() == [k + 1] * (k + 1)
    assert ds[0] == k and ds[1:].tolist() == [1 + 2 * (k - 1)] * k
    n = 12   # cycle: every node the same, sum_v d(u, v) = n^2 / 4 for even n
    c = gen.cycle_graph(n)
    reached, ds = node_stats(n, c.src, c.dst, np.arange(n), c.undirected)
    assert set(ds.tolist()) == {n * n // 4} and set(reached.tolist()) == {n}


@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("undirected,transpose", [(False, False), (True, False), (False, True)])
def test_against_matrix_powers_and_counts(seed, undirected, transpose):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 40))
    src = rng.integers(0, n, 2 * n)
    dst = rng.integers(0, n, 2 * n)
    seeds = rng.integers(0, n, 7)
    counts, dist = oracle.brute_force_counts(n, src, dst, seeds, undirected, transpose)
    d = dist[:, seeds]                       # [u][i] = d(u, x_i)
    reached, ds = node_stats(n, src, dst, seeds, undirected, transpose)
    assert reached.tolist() == (d >= 0).sum(axis=1).tolist()
    assert ds.tolist() == np.where(d >= 0, d, 0).sum(axis=1).tolist()
    # Algorithm 1's totals
    assert int(reached.sum()) == int(counts.sum())
    assert int(ds.sum()) == int(sum(r * int(c) for r, c in enumerate(counts)))
    # after k rounds only distances up to k
    for k in range(len(counts)):
        rk, dk = node_stats(n, src, dst, seeds, undirected, transpose, rounds=k)
        assert int(rk.sum()) == int(counts[:k + 1].sum())
        assert int(dk.sum()) == int(sum(r * int(c) for r, c in enumerate(counts[:k + 1])))
