"""Pins of the PROPAGATE-S oracle (Algorithm 2) against independent facts."""
import numpy as np
import pytest

import oracle
from oracle.propagate_s import propagate_s


def _random_graph(rng, n, m):
    src = rng.integers(0, n, m)
    dst = rng.integers(0, n, m)
    return src, dst


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("undirected,transpose", [(False, False), (True, False), (False, True)])
def test_matches_all_pairs_distances(seed, undirected, transpose):
    # Section 3: c[r] counts the pairs (u, x_i) with d(u, x_i) = r; the
    # boolean matrix powers know nothing of Algorithm 2's passes or breaks
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 30))
    src, dst = _random_graph(rng, n, int(rng.integers(0, 3 * n)))
    seeds = rng.integers(0, n, int(rng.integers(1, 9)))   # duplicates allowed
    counts, D, _ = propagate_s(n, src, dst, seeds, undirected, transpose)
    want, _ = oracle.brute_force_counts(n, src, dst, seeds, undirected, transpose)
    assert counts.tolist() == want.tolist()
    assert D == len(want) - 1


def test_path_closed_form():
    # arcs u -> u+1: u reaches the last node L-1 at distance L-1-u
    L = 9
    src, dst = np.arange(L - 1), np.arange(1, L)
    counts, D, _ = propagate_s(L, src, dst, [L - 1], undirected=False)
    assert counts.tolist() == [1] * L and D == L - 1
    # from node 0 nothing else reaches it along the arcs
    counts, D, _ = propagate_s(L, src, dst, [0], undirected=False)
    assert counts.tolist() == [1] and D == 0


def test_star_and_early_break():
    # leaves 1..k point to the centre 0; the centre as seed is found by every
    # leaf in pass 1, each after examining its one arc
    k = 7
    src, dst = np.arange(1, k + 1), np.zeros(k, dtype=np.int64)
    counts, D, examined = propagate_s(k + 1, src, dst, [0], undirected=False)
    assert counts.tolist() == [1, k] and D == 1
    # pass 1 examines the k arcs; pass 2 finds every node set and examines none
    assert examined == k


def test_early_break_stops_at_the_first_hit():
    # node 0 has arcs to 1, 2, 3 in that order; seeds at 1: the break after
    # the first arc leaves the other two unexamined
    src, dst = np.array([0, 0, 0]), np.array([1, 2, 3])
    _, _, examined = propagate_s(4, src, dst, [1], undirected=False)
    assert examined == 1


def test_empty_graph():
    counts, D, examined = propagate_s(5, [], [], [0, 3, 3], undirected=True)
    assert counts.tolist() == [3] and D == 0 and examined == 0


def test_stored_arc_set_keeps_the_counts():
    # merging duplicates, dropping self-loops and sorting the lists changes
    # only which arcs the early break examines
    rng = np.random.default_rng(11)
    for _ in range(5):
        n = int(rng.integers(2, 25))
        src, dst = _random_graph(rng, n, 3 * n)
        seeds = rng.integers(0, n, 4)
        a, Da, _ = propagate_s(n, src, dst, seeds, False)
        b, Db, _ = propagate_s(n, src, dst, seeds, False, stored=True)
        assert a.tolist() == b.tolist() and Da == Db
