"""Learned scheduler: measured round costs, labels, training, evaluation.

A round of PROPAGATE-P (Algorithm 1) yields the same signatures whatever
action runs it, so the action of each round is a pure cost decision.  The
model's actions (its outputs, in order) are a dense pull, a push over direct
slots per frontier entry, a push over flattened arc ranges, and a sparse
pull.  The decision is not local: a sparse round that follows a pull first
has to find the nodes the pull changed (a scan of every node), so a pull now
makes the next sparse round dearer.  This module

  * measures, for every round r of a propagation, the cost c[r][p][a] of
    running round r with action a after a round that pulled (p = 0) or did
    not (p = 1) (two runs kept one round apart, one per previous kind, plus
    a scratch copy restored before each forced round; ``pp_time_round``
    times one forced round);
  * solves the two-state dynamic programme over those costs for the best
    schedule and its cost-to-go V[r][p];
  * labels each (round, previous kind) with the effective cost of each
    action, c[r][p][a] + V[r+1][q(a)] - min_q V[r+1][q] (q(a): the kind of
    round a is): the round's own time plus what the choice adds to the rest
    of the run, so that the action with the smallest label is optimal;
  * fits the library's cost model to the logarithm of those labels with the
    library's device training kernels, and scores schedules on the measured
    costs.

Everything numeric on the propagation path runs in the HIP library; this
module marshals arrays and does the host-side bookkeeping of labels.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import pp

# model outputs -> the library's round actions
ACTIONS = (pp.MODE_PULL, pp.MODE_PUSH, pp.MODE_PUSH_FLAT, pp.MODE_SPULL)
A_PULL, A_PUSH, A_FLAT, A_SPULL = 0, 1, 2, 3
NACT = len(ACTIONS)
# the previous round's kind: pulled, or sparse (a push or a sparse pull)
PULL, SPARSE = 0, 1
PUSH = SPARSE
FLAT_MIN = 16384   # the fixed rule's tiling: flattened ranges from this many frontier entries


def kind(a: int) -> int:
    """The kind of round an action makes (the next round's previous kind)."""
    return PULL if a == A_PULL else SPARSE


@dataclass
class CostTable:
    """Measured costs of one propagation: feat [R][8] (feature 7 left 0) and
    cost [R][2][4] in ms, cost[r][p][a] = round r+1 with action a after a
    round of kind p (row r = 0 is the first round, after the initialisation,
    whose two p rows are equal); n nodes (feature 0 is the frontier over n)."""
    feat: np.ndarray
    cost: np.ndarray
    n: int = 1

    def __len__(self) -> int:
        return int(self.feat.shape[0])


def _timed(run, mode):
    try:
        return pp.pp_time_round(run, mode)
    except pp.PPError as e:
        if e.code == pp.PP_ESTATE:   # converged: no round left
            return None
        raise


def measure(graph: pp.Graph, seeds, max_rounds: int = 0, stream=None, opts=None) -> CostTable:
    """Costs of every round under every action after both kinds of previous round."""
    o = opts if opts is not None else pp.options(max_rounds=max_rounds)
    after_pull = pp.pp_seeds_init(graph, seeds, opts=o, stream=stream)
    scratch = pp.pp_run_snapshot(after_pull)
    after_sparse = None
    feats, costs = [], []
    try:
        while True:
            row = np.zeros((2, NACT))
            # after a pull (the initialisation, for the first round): the sparse
            # actions on restored copies, the pull on the run itself (advancing it)
            f = None
            for a in (A_PUSH, A_FLAT, A_SPULL):
                pp.pp_run_restore(scratch, after_pull)
                got = _timed(scratch, ACTIONS[a])
                if got is None:
                    break
                f, row[PULL, a] = got
                if a == A_PUSH and after_sparse is None:
                    after_sparse = pp.pp_run_snapshot(scratch)   # the first round's sparse branch
            if f is None:
                break
            f = f.copy()
            _, row[PULL, A_PULL] = _timed(after_pull, ACTIONS[A_PULL])
            if len(costs) == 0:
                row[SPARSE] = row[PULL]
            else:
                for a in (A_PULL, A_FLAT, A_SPULL):
                    pp.pp_run_restore(scratch, after_sparse)
                    f2, row[SPARSE, a] = _timed(scratch, ACTIONS[a])
                    if not np.array_equal(f[:7], f2[:7]):
                        raise RuntimeError("round features depend on the schedule")
                _, row[SPARSE, A_PUSH] = _timed(after_sparse, ACTIONS[A_PUSH])
            f[7] = 0.0
            feats.append(f)
            costs.append(row)
    finally:
        for r in (after_pull, after_sparse, scratch):
            if r is not None:
                r.free()
    return CostTable(np.array(feats, np.float32).reshape(-1, pp.MLP_IN), np.array(costs).reshape(-1, 2, NACT),
                     graph.nodes)


def measure_replay(graph: pp.Graph, seeds, opts=None, repeats: int = 3, stream=None) -> CostTable:
    """Costs of every round under every allowed action after both kinds of round,
    from whole propagations on the ordinary path (graph replay) that follow fixed
    plans: each round's device-clock duration (pp_get_round_times), the median of
    `repeats` propagations per plan after one to warm up.  The plans: every
    action throughout (c[r][kind(a)][a]), and dense pulls alternating with each
    sparse action in both phases (c[r][pull][a] and c[r][sparse][pull]).  The
    features come from a propagation under the heuristic (they do not depend on
    the schedule but for feature 7, which the labels set).  With the run's
    sparse_pull at 0 the sparse pull is not allowed and gets a prohibitive cost
    (ten times the dearest measured round); at 1 the pushes get it."""
    o = pp.Options.from_buffer_copy(opts) if opts is not None else pp.options()
    o.scheduler = pp.PP_SCHED_PLAN
    o.time_kernels = 0
    run = pp.pp_seeds_init(graph, seeds, opts=o, stream=stream)
    try:
        pp.pp_run_set_plan(run, [])   # the heuristic
        pp.pp_seeds_reset(run, seeds)
        counts0, D0 = pp.pp_propagate_until_converged(run)
        R = int(D0[0]) + 1            # rounds 1..R, the last one finding nothing
        cap = R + 2
        feat = pp.pp_get_round_features(run, cap)[1:R + 1].copy()
        feat[:, 7] = 0.0
        allowed = [a for a in range(NACT) if (a != A_SPULL or o.sparse_pull != 0) and
                   (a not in (A_PUSH, A_FLAT) or o.sparse_pull != 1)]
        cost = np.full((R, 2, NACT), np.nan)

        def run_plan(plan):
            pp.pp_run_set_plan(run, plan)
            times = []
            for k in range(repeats + 1):
                pp.pp_seeds_reset(run, seeds)
                c, D = pp.pp_propagate_until_converged(run)
                if int(D[0]) != int(D0[0]) or list(c[0]) != list(counts0[0]):
                    raise RuntimeError("a plan changed the counts")
                if k:
                    times.append(pp.pp_get_round_times(run, cap))
            return np.median(np.array(times, dtype=np.float64), axis=0)

        for a in allowed:
            t = run_plan(np.full(cap, a, np.int32))
            cost[0, :, a] = t[1]
            for r in range(2, R + 1):
                cost[r - 1, kind(a), a] = t[r]
        if A_PULL in allowed:
            for x in allowed:
                if x == A_PULL:
                    continue
                for parity in (0, 1):
                    plan = np.array([A_PULL if r % 2 == parity else x for r in range(cap)], np.int32)
                    t = run_plan(plan)
                    for r in range(2, R + 1):
                        cost[r - 1, kind(int(plan[r - 1])), int(plan[r])] = t[r]
        worst = np.nanmax(cost)
        cost[np.isnan(cost)] = 10.0 * worst   # actions the run does not allow
        return CostTable(feat.astype(np.float32), cost, graph.nodes)
    finally:
        run.free()


def replay_plan(graph: pp.Graph, seeds, plan, opts=None, repeats: int = 3, stream=None):
    """Best wall time (ms) of whole propagations that follow a fixed plan of actions
    (cost-model action indices per round), with the counts and D."""
    o = pp.Options.from_buffer_copy(opts) if opts is not None else pp.options()
    o.scheduler = pp.PP_SCHED_PLAN
    run = pp.pp_seeds_init(graph, seeds, opts=o, stream=stream)
    try:
        pp.pp_run_set_plan(run, np.concatenate([[0], np.asarray(plan, np.int32)]))   # plan[i] is round i + 1
        best = math.inf
        counts = D = None
        for _ in range(repeats + 1):
            pp.pp_seeds_reset(run, seeds)
            t0 = time.perf_counter()
            counts, D = pp.pp_propagate_until_converged(run)
            best = min(best, (time.perf_counter() - t0) * 1e3)
        return best, counts, D
    finally:
        run.free()


def optimal_schedule(t: CostTable):
    """Two-state dynamic programme: (V [R+1][2] cost-to-go, best total, best actions)."""
    R = len(t)
    V = np.zeros((R + 1, 2))
    for r in range(R - 1, -1, -1):
        for p in (PULL, SPARSE):
            V[r, p] = min(t.cost[r, p, a] + V[r + 1, kind(a)] for a in range(NACT))
    p = SPARSE   # the first round's rows are equal
    plan = []
    for r in range(R):
        a = min(range(NACT), key=lambda a: (t.cost[r, p, a] + V[r + 1, kind(a)], a))
        plan.append(a)
        p = kind(a)
    return V, float(V[0, SPARSE]), np.array(plan, np.int32)


@dataclass
class Samples:
    """Training samples: features x [N][8] and targets t [N][4] (log ms)."""
    x: np.ndarray
    t: np.ndarray

    def __len__(self) -> int:
        return int(self.x.shape[0])

    @staticmethod
    def concat(parts) -> "Samples":
        parts = list(parts)
        return Samples(np.concatenate([p.x for p in parts]), np.concatenate([p.t for p in parts]))


def label(t: CostTable) -> Samples:
    """One sample per (round, previous kind): features with feature 7 set to
    whether the previous round pulled, targets log(c[r][p][a] + V[r+1][q(a)] -
    min V[r+1]) for every action a."""
    V, _, _ = optimal_schedule(t)
    xs, ys = [], []
    for r in range(len(t)):
        extra = np.array([V[r + 1, kind(a)] for a in range(NACT)]) - V[r + 1].min()
        for p in ((SPARSE,) if r == 0 else (PULL, SPARSE)):
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


def heuristic_policy(push_div: int = 8, n: int | None = None):
    """The fixed rule: a sparse round while frontier arcs * push_div < arcs (feature
    1), as a push over flattened ranges from FLAT_MIN frontier entries (feature 0
    times n; direct slots when n is not given)."""
    def choose(r, f):
        if f[1] * push_div >= 1.0:
            return A_PULL
        return A_FLAT if (n is not None and round(float(f[0]) * n) >= FLAT_MIN) else A_PUSH
    return choose


def model_policy(params, t: CostTable, allowed=(A_PULL, A_PUSH, A_FLAT)):
    """The cost model's decisions over a table's rounds (the allowed output with
    the least value, the first of equal ones), evaluated by the library for both
    values of feature 7 at once."""
    x = np.repeat(t.feat, 2, axis=0)
    x[0::2, 7] = 0.0
    x[1::2, 7] = 1.0
    y = pp.pp_mlp_forward(params, x).reshape(len(t), 2, NACT)
    allowed = list(allowed)
    pick = np.array(allowed)[np.argmin(y[:, :, allowed], axis=2)]   # [round][feature 7]
    return lambda r, f: int(pick[r, int(f[7])])


def policy_cost(t: CostTable, choose) -> tuple[float, np.ndarray]:
    """Measured cost of a feature-driven schedule choose(r, f) -> action over the
    table (feature 7 follows the schedule's own previous kind)."""
    p = SPARSE
    total = 0.0
    plan = []
    for r in range(len(t)):
        f = t.feat[r].copy()
        f[7] = 1.0 if (r > 0 and p == PULL) else 0.0
        a = choose(r, f)
        total += float(t.cost[r, p, a])
        plan.append(a)
        p = kind(a)
    return total, np.array(plan, np.int32)


def wall_times(graph: pp.Graph, seeds, scheduler: int, params=None, reps: int = 9, warm: int = 2, push_div: int = 0,
               pull_k: int = 0, plan=None, stream=None):
    """Wall times (ms) of `reps` whole propagations on one run after `warm` untimed
    ones (graph capture included there), with the counts and D of the last.
    plan: cost-model actions per round (from round 1) for PP_SCHED_PLAN."""
    opts = pp.options(scheduler=scheduler, push_div=push_div, pull_k=pull_k)
    run = pp.pp_seeds_init(graph, seeds, opts=opts, stream=stream)
    try:
        if params is not None:
            pp.pp_run_set_mlp(run, params)
        if plan is not None:
            pp.pp_run_set_plan(run, np.concatenate([[0], np.asarray(plan, np.int32)]))
        out = []
        counts = D = None
        for k in range(warm + reps):
            pp.pp_seeds_reset(run, seeds)
            t0 = time.perf_counter()
            counts, D = pp.pp_propagate_until_converged(run)
            if k >= warm:
                out.append((time.perf_counter() - t0) * 1e3)
        return np.array(out), counts, D
    finally:
        run.free()


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
