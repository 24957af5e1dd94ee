"""PROPAGATE-S (Algorithm 2): the seeds one at a time, one bit per node.

TEST INFRASTRUCTURE ONLY (see the package header): the product never
imports this module.

What Algorithm 2 computes, stated from distances (Section 3 and Section 4's
description of the sequential form), not from its printed steps:
  * For a seed x, let d(u) be the length of a shortest directed path from u
    to x along the arcs (u takes the bits of the heads of its arcs, as in
    Algorithm 1).  Pass k >= 1 of the seed sets exactly the nodes with
    d(u) = k, so the per-pass counts summed over the seeds are Algorithm 1's
    c[k]; c[0] = s counts the seeds themselves.  The seed's last pass is the
    first that sets nothing, pass ecc(x) + 1, ecc(x) = max of the finite d.
  * The early break: in pass k every node not set before the pass (d(u) >= k,
    or unreachable) walks its successor list in order up to the first
    successor set before the pass (d(v) <= k - 1), which it examines too; a
    node that meets none examines its whole list.  The arcs examined are
    summed over passes and seeds.

Readings of the printed listing, which cannot run as printed: the signature
is cleared for every seed and the pass count for every pass; c[0] = s, pass
k >= 1 adds into c[k], and D_LB is the last pass that set a node (the
numbering under which the counts are Algorithm 1's).

Pins (``tests/test_oracle_propagate_s.py``): all-pairs distances by
boolean matrix powers on random small graphs (directed, undirected,
transposed, self-loops, duplicate arcs and seeds, isolated nodes); closed
forms on paths and stars, with the arcs the early break examines; the
empty graph.
"""
from __future__ import annotations

import numpy as np


def successor_lists(n, src, dst, undirected, transpose=False, stored=False):
    """Arc lists of the propagation direction: u takes Sig(v) for an arc u -> v.

    stored: the arc set a graph library would store -- self-loops dropped,
    duplicates merged, each list in increasing node order -- which fixes the
    order the early break sees (the counts do not depend on it)."""
    succ = [[] for _ in range(int(n))]
    pairs = list(zip(np.asarray(src, dtype=np.int64).tolist(), np.asarray(dst, dtype=np.int64).tolist()))
    if undirected:
        pairs = pairs + [(v, u) for u, v in pairs]
    for u, v in pairs:
        if transpose:
            u, v = v, u
        succ[u].append(v)
    if stored:
        succ = [sorted(set(v for v in lst if v != u)) for u, lst in enumerate(succ)]
    return succ


def _distances_to(n, succ, x):
    """d(u) for every u: shortest path u -> x along the arcs (-1 if none), by BFS from x
    over the predecessor lists."""
    pred = [[] for _ in range(n)]
    for u, lst in enumerate(succ):
        for v in lst:
            pred[v].append(u)
    dist = [-1] * n
    dist[x] = 0
    frontier = [x]
    while frontier:
        nxt = []
        for v in frontier:
            for u in pred[v]:
                if dist[u] < 0:
                    dist[u] = dist[v] + 1
                    nxt.append(u)
        frontier = nxt
    return dist


def propagate_s(n, src, dst, seeds, undirected, transpose=False, stored=False):
    """(c [D_LB + 1] int64, D_LB, arcs examined) of Algorithm 2, from distances (small graphs only)."""
    n = int(n)
    succ = successor_lists(n, src, dst, undirected, transpose, stored)
    seeds = [int(x) for x in np.asarray(seeds).tolist()]
    counts = [len(seeds)]
    d_lb = 0
    examined = 0
    for x in seeds:
        dist = _distances_to(n, succ, x)
        ecc = max(dist)
        for k in range(1, ecc + 1):   # pass k sets the nodes at distance k
            while len(counts) <= k:
                counts.append(0)
            counts[k] += sum(1 for d in dist if d == k)
        d_lb = max(d_lb, ecc)
        for k in range(1, ecc + 2):   # passes 1 .. ecc + 1, the last setting nothing
            for u in range(n):
                if 0 <= dist[u] < k:
                    continue          # set before pass k: not walked
                lst = succ[u]
                first = next((i for i, v in enumerate(lst) if 0 <= dist[v] <= k - 1), None)
                examined += len(lst) if first is None else first + 1
    return np.asarray(counts, dtype=np.int64), d_lb, examined
