"""Host-side logic of the learned scheduler (no GPU): the dynamic programme
against brute force over every schedule, the labels' argmin against the
programme's plan, and policy scoring."""
import itertools

import numpy as np
import pytest

from paper_2301_06499_amd import scheduler
from paper_2301_06499_amd.scheduler import A_FLAT, A_PULL, A_PUSH, A_SPULL, NACT, PULL, SPARSE, kind


def random_table(seed, R):
    rng = np.random.default_rng(seed)
    cost = rng.uniform(0.01, 1.0, size=(R, 2, NACT))
    cost[0, PULL] = cost[0, SPARSE]
    feat = rng.uniform(0, 1, size=(R, 8)).astype(np.float32)
    feat[:, 7] = 0
    return scheduler.CostTable(feat, cost, 100000)


def brute_force(t):
    best, arg = np.inf, None
    for plan in itertools.product(range(NACT), repeat=len(t)):
        p, tot = SPARSE, 0.0
        for r, a in enumerate(plan):
            tot += t.cost[r, p, a]
            p = kind(a)
        if tot < best:
            best, arg = tot, plan
    return best, arg


@pytest.mark.parametrize("seed", range(6))
def test_dynamic_programme_is_optimal(seed):
    t = random_table(seed, 7)
    V, best, plan = scheduler.optimal_schedule(t)
    bf, _ = brute_force(t)
    assert best == pytest.approx(bf, rel=1e-12)
    got, _ = scheduler.policy_cost(t, lambda r, f: int(plan[r]))
    assert got == pytest.approx(best, rel=1e-12)
    # no feature-driven policy beats it
    for pol in (scheduler.heuristic_policy(8, t.n), scheduler.heuristic_policy(2), lambda r, f: A_PULL,
                lambda r, f: A_PUSH, lambda r, f: A_FLAT, lambda r, f: A_SPULL):
        assert scheduler.policy_cost(t, pol)[0] >= best - 1e-12


def test_labels_pick_the_optimal_action():
    t = random_table(11, 30)
    V, best, plan = scheduler.optimal_schedule(t)
    s = scheduler.label(t)
    assert len(s) == 1 + 2 * (len(t) - 1) and s.t.shape[1] == NACT
    # following the labels' argmin, with feature 7 from the own history, is optimal
    rows = {}
    k = 0
    for r in range(len(t)):
        for p in ((SPARSE,) if r == 0 else (PULL, SPARSE)):
            rows[(r, p)] = s.t[k]
            assert s.x[k, 7] == (1.0 if p == PULL else 0.0)
            k += 1
    p, tot = SPARSE, 0.0
    for r in range(len(t)):
        y = rows[(r, SPARSE if r == 0 else p)]
        a = int(np.argmin(y))
        tot += t.cost[r, p, a]
        p = kind(a)
    assert tot == pytest.approx(best, rel=1e-6)


def test_switch_cost_makes_the_greedy_choice_wrong():
    """A pull that is cheaper now but forces a dear sparse round later loses to staying sparse."""
    R = 4
    cost = np.zeros((R, 2, NACT))
    cost[:, SPARSE, A_PUSH] = 1.0      # push after a sparse round
    cost[:, PULL, A_PUSH] = 5.0        # push after a pull rescans every node
    cost[:, :, A_FLAT] = 9.0           # the other sparse actions dearer here
    cost[:, :, A_SPULL] = 9.0
    cost[:, :, A_PULL] = 0.9           # a pull, after anything
    t = scheduler.CostTable(np.zeros((R, 8), np.float32), cost)
    _, best, plan = scheduler.optimal_schedule(t)
    assert best == pytest.approx(3.6)          # pulling throughout
    cost[:, :, A_PULL] = 1.5
    t = scheduler.CostTable(np.zeros((R, 8), np.float32), cost)
    _, best, plan = scheduler.optimal_schedule(t)
    assert list(plan) == [A_PUSH] * R and best == pytest.approx(4.0)


def test_heuristic_policy_tiling_follows_the_frontier_size():
    n = 1 << 20
    pol = scheduler.heuristic_policy(8, n)
    f = np.zeros(8, np.float32)
    f[1] = 0.2                                  # frontier arcs >= arcs / 8: pull
    assert pol(0, f) == A_PULL
    f[1] = 0.05
    f[0] = np.float32(100 / n)                  # a small frontier: direct slots
    assert pol(0, f) == A_PUSH
    f[0] = np.float32(20000 / n)                # from 16384 entries: flattened ranges
    assert pol(0, f) == A_FLAT
