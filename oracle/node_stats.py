"""Per-node outputs for centrality estimates (exact integers).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper names per-node centralities as future work and defines none.  The
per-node quantities the propagation determines are plain definitions: for a
node u and the sampled seeds x_1..x_s,

    reached(u)  = #{ i : d(u, x_i) is finite }            (seed bits u holds)
    dist_sum(u) = sum over those i of d(u, x_i)

(d along the propagation direction, as for the counts; a repeated seed counts
once per occurrence).  After k rounds only distances up to k are known, so
the partial values count the i with d(u, x_i) <= k.  Sampled closeness or
harmonic estimates are left to the caller.

Pins (``tests/test_oracle_node_stats.py``): closed forms on paths, cycles
and stars; all-pairs distances by boolean matrix powers; the per-node sums
add up to Algorithm 1's counts (sum_u reached(u) = R[D], sum_u dist_sum(u) =
sum_r r c[r]).
"""
from __future__ import annotations

import numpy as np

from . import propagate as _propagate


def node_stats(n, src, dst, seeds, undirected, transpose=False, rounds=None):
    """(reached int32 [n], dist_sum int64 [n]); rounds: only distances <= rounds."""
    res = _propagate(n, src, dst, seeds, undirected, transpose=transpose, dist=True)
    d = np.asarray(res["dist"], dtype=np.int64)          # [s][n], -1 unreachable
    ok = d >= 0
    if rounds is not None:
        ok &= d <= int(rounds)
    reached = ok.sum(axis=0).astype(np.int32)
    dist_sum = np.where(ok, d, 0).sum(axis=0).astype(np.int64)
    return reached, dist_sum
