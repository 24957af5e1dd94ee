"""Host-side logic of the learned scheduler (no GPU): the dynamic programme
against brute force over every schedule, the labels' argmin against the
programme's plan, and policy scoring."""
import itertools

import numpy as np
import pytest

from paper_2301_06499_amd import scheduler
from paper_2301_06499_amd.scheduler import PULL, PUSH


def random_table(seed, R):
    rng = np.random.default_rng(seed)
    cost = rng.uniform(0.01, 1.0, size=(R, 2, 2))
    cost[0, PULL] = cost[0, PUSH]
    feat = rng.uniform(0, 1, size=(R, 8)).astype(np.float32)
    feat[:, 7] = 0
    return scheduler.CostTable(feat, cost)


def brute_force(t):
    best, arg = np.inf, None
    for plan in itertools.product((PULL, PUSH), repeat=len(t)):
        p, tot = PUSH, 0.0
        for r, a in enumerate(plan):
            tot += t.cost[r, p, a]
            p = a
        if tot < best:
            best, arg = tot, plan
    return best, arg


@pytest.mark.parametrize("seed", range(6))
def test_dynamic_programme_is_optimal(seed):
    t = random_table(seed, 9)
    V, best, plan = scheduler.optimal_schedule(t)
    bf, _ = brute_force(t)
    assert best == pytest.approx(bf, rel=1e-12)
    got, _ = scheduler.policy_cost(t, lambda r, f: int(plan[r]))
    assert got == pytest.approx(best, rel=1e-12)
    # no feature-driven policy beats it
    for pol in (scheduler.heuristic_policy(8), scheduler.heuristic_policy(2), lambda r, f: PULL,
                lambda r, f: PUSH):
        assert scheduler.policy_cost(t, pol)[0] >= best - 1e-12


def test_labels_pick_the_optimal_direction():
    t = random_table(11, 30)
    V, best, plan = scheduler.optimal_schedule(t)
    s = scheduler.label(t)
    assert len(s) == 1 + 2 * (len(t) - 1)
    # following the labels' argmin, with feature 7 from the own history, is optimal
    rows = {}
    k = 0
    for r in range(len(t)):
        for p in ((PUSH,) if r == 0 else (PULL, PUSH)):
            rows[(r, p)] = s.t[k]
            assert s.x[k, 7] == (1.0 if p == PULL else 0.0)
            k += 1
    p, tot = PUSH, 0.0
    for r in range(len(t)):
        y = rows[(r, PUSH if r == 0 else p)]
        a = PULL if y[0] <= y[1] else PUSH
        tot += t.cost[r, p, a]
        p = a
    assert tot == pytest.approx(best, rel=1e-6)


def test_switch_cost_makes_the_greedy_choice_wrong():
    """A pull that is cheaper now but forces a dear push later loses to pushing on."""
    R = 4
    cost = np.zeros((R, 2, 2))
    cost[:, PUSH, PUSH] = 1.0      # push after push
    cost[:, PULL, PUSH] = 5.0      # push after a pull rescans every node
    cost[:, :, PULL] = 0.9         # a pull, after anything
    t = scheduler.CostTable(np.zeros((R, 8), np.float32), cost)
    _, best, plan = scheduler.optimal_schedule(t)
    assert best == pytest.approx(3.6)          # pulling throughout
    cost[:, :, PULL] = 1.5
    t = scheduler.CostTable(np.zeros((R, 8), np.float32), cost)
    _, best, plan = scheduler.optimal_schedule(t)
    assert list(plan) == [PUSH] * R and best == pytest.approx(4.0)
