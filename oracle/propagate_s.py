"""PROPAGATE-S (Algorithm 2): the seeds one at a time, one bit per node.

TEST INFRASTRUCTURE ONLY (see the package header): the product never
imports this module.

Algorithm 2 keeps a single n-bit signature Sig of the whole graph for the
seed x_i being processed.  Sig(x_i) = 1 at the start.  Each pass copies Sig
into NewSig; every node u with Sig(u) = 0 ORs into NewSig(u) the bits Sig(v)
of the heads v of its arcs u -> v, one arc after the other, and stops at the
first arc that sets it (the early break).  The pass then counts the bits of
NewSig XOR Sig, commits NewSig, and the seed is done at the first pass that
counts nothing.  CountAll[k] sums over the seeds the nodes found at pass k.
The arc direction and the counts are those of Algorithm 1: Sig(u) takes the
bits of u's successors, and CountAll equals Algorithm 1's c[r].

Readings of the printed listing, which cannot run as printed: Sig is cleared
for every seed and Count for every pass; CountAll[0] = s counts the seeds
themselves, pass k >= 1 adds into CountAll[k], and D_LB is the last pass
that found a node (the numbering under which the counts are Algorithm 1's).

Pins (``tests/test_oracle_propagate_s.py``): all-pairs distances by
boolean matrix powers on random small graphs (directed, undirected,
transposed, self-loops, duplicate arcs and seeds, isolated nodes); closed
forms on paths and stars; the empty graph.
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


def propagate_s(n, src, dst, seeds, undirected, transpose=False, stored=False):
    """(CountAll [D_LB + 1] int64, D_LB, arcs examined) by Algorithm 2, pure Python (small graphs only)."""
    n = int(n)
    succ = successor_lists(n, src, dst, undirected, transpose, stored)
    seeds = [int(x) for x in np.asarray(seeds).tolist()]
    count_all = [len(seeds)]
    d_lb = 0
    examined = 0
    for x in seeds:
        sig = bytearray(n)            # Sig, cleared for this seed
        sig[x] = 1
        k = 0
        while True:
            k += 1
            new_sig = bytearray(sig)  # NewSig = Sig
            for u in range(n):
                if sig[u]:
                    continue
                for v in succ[u]:
                    examined += 1
                    new_sig[u] |= sig[v]
                    if new_sig[u]:
                        break         # the early break
            count = sum(1 for a, b in zip(new_sig, sig) if a != b)
            sig = new_sig
            if count == 0:
                break
            while len(count_all) <= k:
                count_all.append(0)
            count_all[k] += count
            d_lb = max(d_lb, k)
    return np.asarray(count_all, dtype=np.int64), d_lb, examined
