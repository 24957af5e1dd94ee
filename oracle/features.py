"""Per-round scheduler features, from exact distances (float64 numpy).

TEST INFRASTRUCTURE ONLY (see the package header): checks the eight
features the device computes at the end of each round for the direction
scheduler.

Round k of Algorithm 1 (PROPAGATE-P) changes the nodes u with d(u, x_i) = k
for some seed x_i (round 0: the seed nodes).  A push from a changed node v
reaches its predecessors, the u with an arc u -> v (Sig(u) takes Sig(v));
the arc set is the stored one: self-loops dropped, duplicates merged, both
directions for an undirected input, reversed for a transposed one.  With
C_k the nodes changed in round k, c[k] its new pairs and m the stored arcs,
the features of round k + 1 are

    f0 = |C_k| / n                   f1 = a_k / m,  a_k = sum_{v in C_k} indeg(v)
    f2 = (c[1] + ... + c[k]) / (n s) f3 = c[k] / (n s)
    f4 = min(c[k] / max(c[k-1], 1), 4) / 4   with c[-1] = 0
    f5 = log2(k + 2) / 16            f6 = log2(a_k / max(|C_k|, 1) + 1) / 16
    f7 = 1 if round k pulled else 0

Pins (``tests/test_oracle_features.py``): closed forms on paths and stars,
and agreement with features derived from the dense signature matrices of
``dense_rounds``.
"""
from __future__ import annotations

import math

import numpy as np


def stored_indegree(n, src, dst, undirected, transpose):
    """(indeg [n], m): predecessor counts and size of the stored arc set."""
    a = np.asarray(src, dtype=np.int64)
    b = np.asarray(dst, dtype=np.int64)
    if transpose:
        a, b = b, a
    if undirected:
        a, b = np.concatenate([a, b]), np.concatenate([b, a])
    keep = a != b
    key = np.unique(a[keep] * n + b[keep])
    heads = key % n   # v of each arc u -> v
    return np.bincount(heads, minlength=n).astype(np.int64), int(key.size)


def changed_sets(dist, rounds):
    """C_0 .. C_{rounds-1} as boolean masks [rounds][n] from dist [s][n]."""
    dist = np.asarray(dist)
    return np.stack([(dist == k).any(axis=0) for k in range(rounds)])


def round_features(n, s, indeg, m, counts, changed, modes, pull_mode=0):
    """Rows 1 .. len(changed) of the feature log: row k+1 from round k's state.

    counts: c[0..] (zero past the end); changed: masks of C_0..; modes: the
    direction of each round (any value other than ``pull_mode`` counts as not
    pulling, round 0 included).
    """
    c = [int(x) for x in counts]
    rows = []
    reached = 0
    for k in range(len(changed)):
        ck = c[k] if k < len(c) else 0
        prev = (c[k - 1] if k - 1 < len(c) else 0) if k > 0 else 0
        if k > 0:
            reached += ck
        fn = int(np.count_nonzero(changed[k]))
        fa = int(indeg[changed[k]].sum())
        pairs = float(n) * float(s)
        grow = float(ck) / float(max(prev, 1))
        rows.append([
            fn / float(n),
            fa / float(max(m, 1)),
            float(reached) / pairs,
            float(ck) / pairs,
            min(grow, 4.0) / 4.0,
            math.log2(k + 2.0) / 16.0,
            math.log2(float(fa) / float(max(fn, 1)) + 1.0) / 16.0,
            1.0 if int(modes[k]) == pull_mode else 0.0,
        ])
    return np.array(rows, dtype=np.float64)
