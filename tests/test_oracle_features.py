"""Pins of the scheduler-feature oracle (oracle/features.py): closed forms on
paths and stars, and an independent derivation from Algorithm 1's dense
signature matrices with a set-based predecessor count."""
import math

import numpy as np
import pytest

import oracle
from oracle import features
from paper_2301_06499_amd import inputs


def feats_from_dist(n, src, dst, seeds, undirected, transpose, modes):
    out = oracle.propagate(n, src, dst, seeds, undirected, transpose=transpose, dist=True)
    D = out["D"]
    indeg, m = features.stored_indegree(n, src, dst, undirected, transpose)
    changed = features.changed_sets(out["dist"], D + 2)
    return features.round_features(n, len(seeds), indeg, m, out["counts"], changed, modes), out


def test_undirected_path_closed_form():
    n = 9
    src = np.arange(n - 1, dtype=np.int32)
    dst = src + 1
    modes = [2] + [k % 2 for k in range(1, n + 1)]
    f, out = feats_from_dist(n, src, dst, np.array([0], np.int32), True, False, modes)
    assert out["D"] == n - 1
    m = 2 * (n - 1)
    for k in range(n):   # round k changes node k alone
        deg = 1 if k in (0, n - 1) else 2
        exp = [1 / n, deg / m, k / n, 1 / n, 0.25, math.log2(k + 2) / 16, math.log2(deg + 1) / 16,
               1.0 if modes[k] == 0 else 0.0]
        np.testing.assert_allclose(f[k], exp, rtol=1e-15, atol=0)
    # round n finds nothing
    np.testing.assert_allclose(f[n], [0, 0, (n - 1) / n, 0, 0, math.log2(n + 2) / 16, 0, modes[n] == 0],
                               rtol=1e-15, atol=0)


def test_star_from_center_closed_form():
    leaves = 12
    n = leaves + 1
    src = np.zeros(leaves, np.int32)
    dst = np.arange(1, n, dtype=np.int32)
    seeds = np.array([0, 0, 3], np.int32)   # a repeated seed and a leaf
    s = 3
    f, out = feats_from_dist(n, src, dst, seeds, True, False, [2, 0, 1, 0])
    # round 0: nodes {0, 3}; round 1: every leaf (3 included) gains seeds 0 and 1, the centre
    # gains seed 2; round 2: the other 11 leaves gain seed 2
    assert list(out["counts"]) == [3, 2 * leaves + 1, leaves - 1]
    np.testing.assert_allclose(f[0][:2], [2 / n, (leaves + 1) / (2 * leaves)], rtol=1e-15)
    np.testing.assert_allclose(f[1][:5], [n / n, (leaves + leaves) / (2 * leaves), 25 / (n * s), 25 / (n * s),
                                          min(25 / 3, 4) / 4], rtol=1e-15)
    np.testing.assert_allclose(f[2][:5], [11 / n, 11 / (2 * leaves), 36 / (n * s), 11 / (n * s), (11 / 25) / 4],
                               rtol=1e-15)


@pytest.mark.parametrize("undirected,transpose", [(False, False), (False, True), (True, False)])
def test_against_dense_signatures(undirected, transpose):
    g = inputs.erdos_renyi_gnm(40, 70, seed=7 + transpose)
    src = np.concatenate([g.src, [3, 5, 5]]).astype(np.int32)   # a self-loop and a duplicate arc
    dst = np.concatenate([g.dst, [3, 9, 9]]).astype(np.int32)
    seeds = inputs.sample_seeds(40, 10, seed=11)
    rng = np.random.default_rng(1)
    modes = [2] + list(rng.integers(0, 2, size=60))
    f, out = feats_from_dist(40, src, dst, seeds, undirected, transpose, modes)
    counts, hist = oracle.dense_rounds(40, src, dst, seeds, undirected, transpose)
    # predecessor sets by brute force over the input pairs
    preds = [set() for _ in range(40)]
    for a, b in zip(src.tolist(), dst.tolist()):
        pairs = [(a, b), (b, a)] if undirected else [(a, b)]
        for u, v in pairs:
            if transpose:
                u, v = v, u
            if u != v:
                preds[v].add(u)
    indeg = np.array([len(p) for p in preds])
    m = sum(indeg)
    changed = [hist[0].any(axis=1)] + [(hist[k] ^ hist[k - 1]).any(axis=1) for k in range(1, len(hist))]
    c = list(counts) + [0] * 4
    exp = features.round_features(40, 10, indeg, m, c, np.array(changed), modes)
    assert len(exp) == len(f)
    np.testing.assert_array_equal(f, exp)
