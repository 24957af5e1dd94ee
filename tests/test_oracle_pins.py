"""Pins for the CPU oracle, against what the paper and the mathematics fix.

Each test names what it pins and why a plausible mistake in the oracle would
fail it: closed forms on textbook graphs (a wrong index or direction changes
them), brute force over every digraph on 4 labelled nodes, a step-by-step
dense run of Algorithm 1, union-find components, and invariants stated in
the proof of Theorem 1.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_2301_06499_amd import inputs as gen


def run(g, seeds, **kw):
    return oracle.propagate(g.n, g.src, g.dst, seeds, g.undirected, **kw)


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", [1, 2, 3, 7, 40])
def test_path_per_seed_counts_closed_form(n):
    """Undirected path, seed at p: c_i[r] = [p-r >= 0] + [p+r <= n-1] (r >= 1)."""
    g = gen.path_graph(n)
    seeds = np.arange(n, dtype=np.int32)
    out = run(g, seeds, seed_counts=True)
    assert out["D"] == n - 1
    sc = out["seed_counts"]
    for i, p in enumerate(seeds):
        assert sc[0, i] == 1
        for r in range(1, n):
            assert sc[r, i] == int(p - r >= 0) + int(p + r <= n - 1)
    # all nodes as seeds: c[r] = 2 (n - r)
    for r in range(1, n):
        assert out["counts"][r] == 2 * (n - r)
    assert out["counts"][0] == n


@pytest.mark.parametrize("n", [3, 4, 9, 10])
def test_cycle_closed_form(n):
    g = gen.cycle_graph(n)
    seeds = np.array([0, n // 2, n - 1], dtype=np.int32)
    out = run(g, seeds, seed_counts=True)
    assert out["D"] == n // 2
    for i in range(3):
        for r in range(1, n // 2 + 1):
            want = 1 if (n % 2 == 0 and r == n // 2) else 2
            assert out["seed_counts"][r, i] == want


@pytest.mark.parametrize("n", [2, 5, 12])
def test_star_closed_form(n):
    g = gen.star_graph(n)
    out = run(g, np.array([0, 1], dtype=np.int32), seed_counts=True)
    sc = out["seed_counts"]
    assert sc[1, 0] == n - 1                       # hub seed
    assert sc[1, 1] == 1                           # leaf seed
    if n > 2:
        assert sc[2, 1] == n - 2
        assert out["D"] == 2
    assert sc[:, 0].sum() == n and sc[:, 1].sum() == n


@pytest.mark.parametrize("n", [2, 6])
def test_complete_closed_form(n):
    g = gen.complete_graph(n)
    out = run(g, np.arange(n, dtype=np.int32))
    assert out["D"] == 1
    assert list(out["counts"]) == [n, n * (n - 1)]
    m = oracle.metrics(out["counts"], n, n)
    assert m["avg_dist"] == 1.0 and m["alpha"] == 1.0 and m["diameter"] == 1


@pytest.mark.parametrize("a,b", [(1, 1), (1, 5), (4, 3), (7, 7)])
def test_grid_manhattan_counts(a, b):
    """Grid distances are Manhattan distances; counted directly per seed."""
    g = gen.grid_graph(a, b)
    seeds = np.arange(a * b, dtype=np.int32)
    out = run(g, seeds, seed_counts=True)
    assert out["D"] == a + b - 2
    xs, ys = np.meshgrid(np.arange(a), np.arange(b))
    xs, ys = xs.ravel(), ys.ravel()
    for i, x in enumerate(seeds):
        d = np.abs(xs - xs[x]) + np.abs(ys - ys[x])
        for r in range(out["D"] + 1):
            assert out["seed_counts"][r, i] == np.count_nonzero(d == r)
    # total distance sum with all nodes as seeds
    sd = sum(r * int(c) for r, c in enumerate(out["counts"]))
    assert sd == (b * b * a * (a * a - 1)) // 3 + (a * a * b * (b * b - 1)) // 3


def test_directed_path_direction():
    """Arc u -> v means u ORs in v's signature: bit of x_i reaches nodes 0..x_i."""
    n = 9
    g = gen.path_graph(n, directed=True)
    seeds = np.array([0, 4, 8], dtype=np.int32)
    fw = run(g, seeds, seed_counts=True, final_sig=True)
    tr = run(g, seeds, seed_counts=True, transpose=True)
    assert fw["D"] == tr["D"] == n - 1
    for i, x in enumerate(seeds):
        for r in range(1, n):
            assert fw["seed_counts"][r, i] == (1 if r <= x else 0)
            assert tr["seed_counts"][r, i] == (1 if r <= n - 1 - x else 0)
    # node u holds seed bit i iff u <= x_i
    for u in range(n):
        for i, x in enumerate(seeds):
            assert bool(fw["final_sig"][u, 0] >> np.uint64(i) & np.uint64(1)) == (u <= x)


def test_directed_cycle():
    n = 8
    g = gen.cycle_graph(n, directed=True)
    out = run(g, np.array([3], dtype=np.int32), seed_counts=True)
    assert out["D"] == n - 1
    assert list(out["seed_counts"][:, 0]) == [1] * n


# ---------------------------------------------------------------- brute force

def test_all_digraphs_on_four_nodes():
    """Every one of the 4096 labelled digraphs on 4 nodes, against matrix powers."""
    n = 4
    pairs = [(u, v) for u in range(n) for v in range(n) if u != v]
    seeds = np.arange(n, dtype=np.int32)
    sub = np.array([2, 0], dtype=np.int32)
    for mask in range(1 << len(pairs)):
        arcs = [pairs[k] for k in range(len(pairs)) if mask >> k & 1]
        src = np.array([a for a, _ in arcs], dtype=np.int32)
        dst = np.array([b for _, b in arcs], dtype=np.int32)
        want, _ = oracle.brute_force_counts(n, src, dst, seeds, False)
        got = oracle.propagate(n, src, dst, seeds, False, nthreads=1)["counts"]
        assert list(got) == list(want), arcs
        want2, _ = oracle.brute_force_counts(n, src, dst, sub, False)
        got2 = oracle.propagate(n, src, dst, sub, False, nthreads=2)["counts"]
        assert list(got2) == list(want2), arcs


@pytest.mark.parametrize("trial", range(12))
def test_random_small_graphs_vs_matrix_powers(trial):
    rng = np.random.default_rng(1000 + trial)
    n = int(rng.integers(1, 64))
    m = int(rng.integers(0, 3 * n + 1))
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)      # loops and duplicates on purpose
    und = bool(trial % 2)
    s = int(rng.integers(1, n + 1))
    seeds = rng.integers(0, n, s).astype(np.int32)     # repeats allowed
    for tr in (False, True):
        want, dist = oracle.brute_force_counts(n, src, dst, seeds, und, transpose=tr)
        got = oracle.propagate(n, src, dst, seeds, und, transpose=tr, dist=True, nthreads=3)
        assert list(got["counts"]) == list(want)
        # d(u, x_i) from matrix powers equals the BFS distance column
        assert np.array_equal(got["dist"].T, dist[:, seeds])


@pytest.mark.parametrize("trial", range(8))
def test_literal_algorithm1_matches_bfs(trial):
    """Dense synchronous Algorithm 1 equals one BFS per seed, round by round."""
    rng = np.random.default_rng(7 + trial)
    n = int(rng.integers(2, 48))
    m = int(rng.integers(0, 4 * n))
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    und = trial % 3 == 0
    s = int(rng.integers(1, 130))                      # crosses a word boundary
    seeds = rng.integers(0, n, s).astype(np.int32)
    for tr in (False, True):
        counts, hist = oracle.dense_rounds(n, src, dst, seeds, und, transpose=tr)
        rounds = list(range(len(hist)))
        got = oracle.propagate(n, src, dst, seeds, und, transpose=tr, sig_rounds=rounds,
                               seed_counts=True, final_sig=True)
        assert list(got["counts"]) == list(counts)
        for k, r in enumerate(rounds):
            assert np.array_equal(got["sigs"][k], oracle.bits_from_matrix(hist[r]))
        assert np.array_equal(got["final_sig"], oracle.bits_from_matrix(hist[-1]))
        assert np.array_equal(got["seed_counts"].sum(axis=1), got["counts"])


def test_undirected_final_signatures_are_components():
    """bit_i(u) = [u and x_i in the same component] (union-find)."""
    rng = np.random.default_rng(5)
    n, m = 300, 240
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x
    for a, b in zip(src.tolist(), dst.tolist()):
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[ra] = rb
    seeds = rng.choice(n, 100, replace=False).astype(np.int32)
    out = oracle.propagate(n, src, dst, seeds, True, final_sig=True)
    for u in range(n):
        for i, x in enumerate(seeds.tolist()):
            bit = int(out["final_sig"][u, i >> 6] >> np.uint64(i & 63) & np.uint64(1))
            assert bit == int(find(u) == find(x))


# ---------------------------------------------------------------- invariants

def test_invariants_monotone_and_bounded():
    """Bits never revert; sum of counts equals final popcount; D <= true diameter."""
    g, seeds = gen.workload_er(seed=3)
    out = oracle.propagate(g.n, g.src, g.dst, seeds, True, sig_rounds=[0, 1, 2, 3, 4, 5, 50],
                           final_sig=True, seed_counts=True)
    sigs = out["sigs"]
    for k in range(sigs.shape[0] - 1):
        assert np.array_equal(sigs[k] & sigs[k + 1], sigs[k])
    pop = int(np.unpackbits(out["final_sig"].view(np.uint8)).sum())
    assert pop == int(out["counts"].sum())
    assert np.array_equal(sigs[-1], out["final_sig"])
    assert all(c > 0 for c in out["counts"])
    # per-round count equals the popcount growth between consecutive rounds
    for k in range(1, 6):
        grow = int(np.unpackbits((sigs[k] ^ sigs[k - 1]).view(np.uint8)).sum())
        want = int(out["counts"][k]) if k <= out["D"] else 0
        assert grow == want


def test_disjoint_union_counts_add():
    a = gen.grid_graph(5, 4)
    b = gen.path_graph(9)
    sa = np.array([0, 7, 19], dtype=np.int32)
    sb = np.array([2, 8, 8], dtype=np.int32)
    oa = run(a, sa)
    ob = run(b, sb)
    src = np.concatenate([a.src, b.src + a.n]).astype(np.int32)
    dst = np.concatenate([a.dst, b.dst + a.n]).astype(np.int32)
    # seeds of b get bits of their own: run the union with both seed lists
    ou = oracle.propagate(a.n + b.n, src, dst, np.concatenate([sa, sb + a.n]), True)
    L = max(len(oa["counts"]), len(ob["counts"]))
    pa = np.pad(oa["counts"], (0, L - len(oa["counts"])))
    pb = np.pad(ob["counts"], (0, L - len(ob["counts"])))
    assert list(ou["counts"]) == list(pa + pb)


def test_edge_cases():
    # isolated seeds: nothing propagates
    out = oracle.propagate(5, np.zeros(0, np.int32), np.zeros(0, np.int32),
                           np.array([1, 3], np.int32), False)
    assert out["D"] == 0 and list(out["counts"]) == [2]
    # a single node
    out = oracle.propagate(1, np.zeros(0, np.int32), np.zeros(0, np.int32), np.array([0], np.int32), True)
    assert list(out["counts"]) == [1]
    # self-loops and duplicate arcs change nothing
    src = np.array([0, 0, 1, 1, 2], np.int32)
    dst = np.array([1, 1, 1, 2, 2], np.int32)
    a = oracle.propagate(3, src, dst, np.array([2], np.int32), False)
    b = oracle.propagate(3, np.array([0, 1], np.int32), np.array([1, 2], np.int32), np.array([2], np.int32), False)
    assert list(a["counts"]) == list(b["counts"]) == [1, 1, 1]
    with pytest.raises(RuntimeError):
        oracle.propagate(3, np.array([0], np.int32), np.array([5], np.int32), np.array([0], np.int32), False)
