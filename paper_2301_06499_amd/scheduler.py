"""Learned direction scheduler: measured round costs, labels, training, evaluation.

A round of PROPAGATE-P (Algorithm 1) yields the same signatures whether it
pulls or pushes, so the direction of each round is a pure cost decision.
The decision is not local: a push that follows a pull first has to find
the nodes the pull changed (a scan of every node), so a pull now makes the
next push dearer.  This module

  * measures, for every round r of a propagation, the cost c[r][p][a] of
    running round r in direction a after round r-1 ran in direction p (two
    runs kept one round apart, one per previous direction, plus a scratch
    copy; ``pp_time_round`` times one forced round);
  * solves the two-state dynamic programme over those costs for the best
    schedule and its cost-to-go V[r][p];
  * labels each (round, previous direction) with the effective cost of
    each direction, c[r][p][a] + V[r+1][a] - min_b V[r+1][b]: the round's
    own time plus what the choice adds to the rest of the run, so that the
    direction with the smaller label is the optimal one;
  * fits the library's cost model to the logarithm of those labels with
    the library's device training kernels, and scores schedules on the
    measured costs.

Everything numeric on the propagation path runs in the HIP library; this
module marshals arrays and does the host-side bookkeeping of labels.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import pp

PULL, PUSH = pp.MODE_PULL, pp.MODE_PUSH


@dataclass
class CostTable:
    """Measured costs of one propagation: feat [R][8] (feature 7 left 0) and
    cost [R][2][2] in ms, cost[r][p][a] = round r+1 in direction a after a
    round in direction p (row r = 0 is the first round, after the
    initialisation, whose two p rows are equal)."""
    feat: np.ndarray
    cost: np.ndarray

    def __len__(self) -> int:
        return int(self.feat.shape[0])


def _timed(run, mode):
    try:
        return pp.pp_time_round(run, mode)
    except pp.PPError as e:
        if e.code == pp.PP_ESTATE:   # converged: no round left
            return None
        raise


def measure(graph: pp.Graph, seeds, max_rounds: int = 0, stream=None) -> CostTable:
    """Costs of every round in both directions after both kinds of previous round."""
    opts = pp.options(max_rounds=max_rounds)
    after_pull = pp.pp_seeds_init(graph, seeds, opts=opts, stream=stream)
    scratch = pp.pp_run_snapshot(after_pull)
    after_push = None
    feats, costs = [], []
    try:
        while True:
            # from the state after a pull (the initialisation, for the first round)
            pp.pp_run_restore(scratch, after_pull)
            got = _timed(after_pull, PULL)
            if got is None:
                break
            f, c_pull = got
            _, c_push = _timed(scratch, PUSH)
            row = np.zeros((2, 2))
            if after_push is None:
                # first round: one previous state; the pushed copy becomes the push branch
                row[PULL] = row[PUSH] = (c_pull, c_push)
                after_push = pp.pp_run_snapshot(scratch)
                f = f.copy()
            else:
                row[PULL] = (c_pull, c_push)
                pp.pp_run_restore(scratch, after_push)
                f2, c_pull2 = _timed(scratch, PULL)
                _, c_push2 = _timed(after_push, PUSH)
                row[PUSH] = (c_pull2, c_push2)
                if not np.array_equal(f[:7], f2[:7]):
                    raise RuntimeError("round features depend on the schedule")
            f[7] = 0.0
            feats.append(f)
            costs.append(row)
    finally:
        for r in (after_pull, after_push, scratch):
            if r is not None:
                r.free()
    return CostTable(np.array(feats, np.float32).reshape(-1, pp.MLP_IN), np.array(costs).reshape(-1, 2, 2))


def optimal_schedule(t: CostTable):
    """Two-state dynamic programme: (V [R+1][2] cost-to-go, best total, best directions)."""
    R = len(t)
    V = np.zeros((R + 1, 2))
    for r in range(R - 1, -1, -1):
        for p in (PULL, PUSH):
            V[r, p] = min(t.cost[r, p, a] + V[r + 1, a] for a in (PULL, PUSH))
    p = PUSH   # the first round's rows are equal
    plan = []
    for r in range(R):
        a = min((PULL, PUSH), key=lambda a: t.cost[r, p, a] + V[r + 1, a])
        plan.append(a)
        p = a
    return V, float(V[0, PUSH]), np.array(plan, np.int32)


@dataclass
class Samples:
    """Training samples: features x [N][8] and targets t [N][2] (log ms)."""
    x: np.ndarray
    t: np.ndarray

    def __len__(self) -> int:
        return int(self.x.shape[0])

    @staticmethod
    def concat(parts) -> "Samples":
        parts = list(parts)
        return Samples(np.concatenate([p.x for p in parts]), np.concatenate([p.t for p in parts]))


def label(t: CostTable) -> Samples:
    """One sample per (round, previous direction): features with feature 7 set
    to the previous direction, targets log(c[r][p][a] + V[r+1][a] - min V[r+1])."""
    V, _, _ = optimal_schedule(t)
    xs, ys = [], []
    for r in range(len(t)):
        extra = V[r + 1] - V[r + 1].min()
        for p in ((PUSH,) if r == 0 else (PULL, PUSH)):
            f = t.feat[r].copy()
            f[7] = 1.0 if p == PULL else 0.0
            xs.append(f)
            ys.append(np.log(t.cost[r, p] + extra))
    return Samples(np.array(xs, np.float32), np.array(ys, np.float32))


def init_params(seed: int) -> np.ndarray:
    """He-normal weights, zero biases (seeded)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in [(pp.MLP_IN, pp.MLP_HID), (pp.MLP_HID, pp.MLP_HID), (pp.MLP_HID, pp.MLP_OUT)]:
        parts.append(rng.normal(scale=math.sqrt(2.0 / fan_in), size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    p = np.concatenate(parts).astype(np.float32)
    assert p.shape == (pp.MLP_PARAMS,)
    return p


def train(samples: Samples, steps: int = 3000, lr: float = 3e-3, seed: int = 0):
    """Fit the cost model on the device; returns (params, loss before each step)."""
    return pp.pp_mlp_train(init_params(seed), samples.x, samples.t, steps, lr)


def heuristic_policy(push_div: int = 8):
    """The fixed heuristic: push while frontier arcs * push_div < arcs (feature 1)."""
    return lambda r, f: PUSH if f[1] * push_div < 1.0 else PULL


def model_policy(params, t: CostTable):
    """The cost model's decisions over a table's rounds (pull when y0 <= y1),
    evaluated by the library for both values of feature 7 at once."""
    x = np.repeat(t.feat, 2, axis=0)
    x[0::2, 7] = 0.0
    x[1::2, 7] = 1.0
    y = pp.pp_mlp_forward(params, x).reshape(len(t), 2, 2)
    pick = np.where(y[:, :, 0] <= y[:, :, 1], PULL, PUSH)   # [round][feature 7]
    return lambda r, f: int(pick[r, int(f[7])])


def policy_cost(t: CostTable, choose) -> tuple[float, np.ndarray]:
    """Measured cost of a feature-driven schedule choose(r, f) over the table
    (feature 7 follows the schedule's own previous direction)."""
    p = PUSH
    total = 0.0
    plan = []
    for r in range(len(t)):
        f = t.feat[r].copy()
        f[7] = 1.0 if (r > 0 and p == PULL) else 0.0
        a = choose(r, f)
        total += float(t.cost[r, p, a])
        plan.append(a)
        p = a
    return total, np.array(plan, np.int32)


def timed_run(graph: pp.Graph, seeds, scheduler: int, params=None, repeats: int = 3, push_div: int = 0,
              stream=None, pull_k: int = 0):
    """Best wall time (ms) of a whole propagation with graph replay, the counts, D and the mode log.

    The library's calls return after the device work they ask for (the
    convergence check reads the control block back), so host clocks bracket
    the device time.
    """
    opts = pp.options(scheduler=scheduler, push_div=push_div, pull_k=pull_k)
    run = pp.pp_seeds_init(graph, seeds, opts=opts, stream=stream)
    try:
        if params is not None:
            pp.pp_run_set_mlp(run, params)
        best = math.inf
        counts = D = None
        for _ in range(repeats):
            pp.pp_seeds_reset(run, seeds)
            t0 = time.perf_counter()
            counts, D = pp.pp_propagate_until_converged(run)
            best = min(best, (time.perf_counter() - t0) * 1e3)
        modes, _ = pp.pp_get_round_log(run, int(D.max()) + 2)
        return best, counts, D, modes
    finally:
        run.free()
