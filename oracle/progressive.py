"""Progressive sampling with a Hoeffding stopping rule (float64 / exact integers).

TEST INFRASTRUCTURE ONLY (see the package header).

Section 4 (error bounds) bounds each metric through per-seed random
variables with a known range: for n values X_i in [0, b], Hoeffding's
inequality gives P(|mean - E| >= b eps) <= delta with
eps = sqrt(ln(2 / delta) / (2 s)).  The average distance's variable lies in
[0, Delta / alpha] (part i of the error-bound theorem), the connectivity
rate's in [0, 1] (part iv).  The paper suggests growing the sample
progressively until a criterion is met but gives none; the reading here:

  * seeds come from a caller's pool, in its order, `group` at a time;
  * after each group the counts of all seeds so far are summed, alpha is
    this build's estimator (T - s) / (s (n - 1)) and Delta the sample's D;
  * the run stops at the first group after which eps * D / alpha (the
    average distance's half-width with the sample's Delta and alpha put in
    for the unknown ones) is at most `target`, or when the pool runs out.
    With D = 0 the bound is 0.

Pins (``tests/test_oracle_progressive.py``): the paper's sample size
ln(n) / eps^2 at delta = 2 / n^2 (the error-bound theorem); coverage of the
half-width on Bernoulli(1/2) samples, the case Hoeffding's bound is nearest
to; the stopping sample on cycles, where every seed sees the same
neighbourhood (alpha = 1, D = floor(n / 2)); the pool running out.
"""
from __future__ import annotations

import math

import numpy as np

from . import metrics as _metrics
from . import propagate as _propagate


def hoeffding_eps(s: int, delta: float) -> float:
    """Half-width for the mean of s values in [0, 1] at confidence 1 - delta."""
    return math.sqrt(math.log(2.0 / delta) / (2.0 * s))


def progressive(n, src, dst, pool, group, target, delta, undirected, transpose=False, cap=None):
    """The sampling run: dict with counts (summed, [D+1]), seeds, groups, met, D, alpha, eps, bound."""
    pool = np.asarray(pool, dtype=np.int32)
    total = np.zeros(0, dtype=np.int64)
    used = 0
    groups = 0
    out = None
    while used < len(pool):
        g = pool[used:used + group]
        res = _propagate(n, src, dst, g, undirected, transpose=transpose, cap=cap)
        c = np.asarray(res["counts"], dtype=np.int64)
        if len(c) > len(total):
            total = np.concatenate([total, np.zeros(len(c) - len(total), dtype=np.int64)])
        total[:len(c)] += c
        used += len(g)
        groups += 1
        m = _metrics(total, n, used)
        D = int(m["diameter"])
        alpha = float(m["alpha"])
        eps = hoeffding_eps(used, delta)
        bound = 0.0 if D == 0 else (eps * float(D) / alpha if alpha > 0.0 else math.inf)
        out = {"counts": total[:D + 1].copy(), "seeds": used, "groups": groups, "met": bound <= target,
               "D": D, "alpha": alpha, "eps": eps, "bound": bound}
        if bound <= target:
            break
    return out
