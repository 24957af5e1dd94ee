"""GPU tests of the learned direction scheduler.

The cost model's forward pass, gradient and Adam steps against the float64
oracle (fp32 arithmetic on the device: tolerances below); the eight
per-round features against the oracle's exact values; the in-kernel
decision against the oracle's model on the logged features; and the rule
that a schedule never changes an output bit.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from oracle import features as ofeat
from oracle import mlp as omlp
from paper_2301_06499_amd import inputs as gen
from paper_2301_06499_amd import pp
from paper_2301_06499_amd import scheduler

pytestmark = pytest.mark.gpu

# fp32 feature values are float32(exact double): allow one float ulp
FEAT_RTOL = 2.5e-7


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rand_params(seed, scale=0.4):
    return np.random.default_rng(seed).normal(scale=scale, size=pp.MLP_PARAMS).astype(np.float32)


def threshold_params(theta, k=8.0):
    """Pull iff feature 1 >= theta: y0 = k (theta - f1), the other outputs 0 (a
    sparse round then takes the first of them, a push over direct slots)."""
    w = {name: np.zeros(shape) for name, shape in omlp.SHAPES}
    w["W1"][0, 1] = 1.0
    w["W2"][0, 0] = 1.0
    w["W3"][0, 0] = -k
    w["b3"][0] = k * theta
    return omlp.pack(w).astype(np.float32)


# ------------------------------------------------------------ the model

@pytest.mark.parametrize("n", [1, 255, 1000])
def test_forward_matches_oracle(n):
    say("mlp forward", n)
    p = rand_params(n)
    x = np.random.default_rng(100 + n).uniform(0, 1, size=(n, 8)).astype(np.float32)
    y = pp.pp_mlp_forward(p, x)
    want = omlp.forward(p.astype(np.float64), x.astype(np.float64))
    scale = np.abs(want).max() + 1.0
    # 8 + 32 + 32 fp32 products per output: a few ulp of the largest term
    np.testing.assert_allclose(y, want, rtol=0, atol=2e-5 * scale)


@pytest.mark.parametrize("n", [3, 777])
def test_loss_and_gradient_match_oracle(n):
    say("mlp grad", n)
    p = rand_params(7 + n)
    rng = np.random.default_rng(n)
    x = rng.uniform(0, 1, size=(n, 8)).astype(np.float32)
    t = rng.normal(size=(n, pp.MLP_OUT)).astype(np.float32)
    loss, g = pp.pp_mlp_loss_grad(p, x, t)
    wl, wg = omlp.loss_grad(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64))
    assert loss == pytest.approx(wl, rel=1e-5)
    np.testing.assert_allclose(g, wg, rtol=1e-4, atol=1e-5 * np.abs(wg).max())


def test_training_follows_oracle_adam_and_is_reproducible():
    say("mlp train")
    rng = np.random.default_rng(3)
    teacher = rand_params(11, 0.5).astype(np.float64)
    x = rng.uniform(0, 1, size=(600, 8)).astype(np.float32)
    t = omlp.forward(teacher, x.astype(np.float64)).astype(np.float32)
    p0 = scheduler.init_params(5)
    p, losses = pp.pp_mlp_train(p0, x, t, 40, 3e-3)
    p2, losses2 = pp.pp_mlp_train(p0, x, t, 40, 3e-3)
    assert np.array_equal(p, p2) and np.array_equal(losses, losses2)   # fixed reduction order
    wp, wl = omlp.adam(p0.astype(np.float64), x.astype(np.float64), t.astype(np.float64), 40, 3e-3)
    np.testing.assert_allclose(losses, wl, rtol=2e-3)
    # Adam's sign-like steps can flip on a gradient within rounding of zero:
    # nearly every parameter must still follow the float64 path
    close = np.abs(p - wp) <= 1e-4 + 1e-3 * np.abs(wp)
    assert close.mean() > 0.99, close.mean()
    _, long = pp.pp_mlp_train(p0, x, t, 800, 3e-3)
    assert long[-1] < 0.1 * long[0]


# ------------------------------------------------------------ features and decisions

def oracle_features(n, src, dst, seeds, undirected, modes, rows, want):
    indeg, m = ofeat.stored_indegree(n, src, dst, undirected, False)
    changed = ofeat.changed_sets(want["dist"], rows)
    return ofeat.round_features(n, len(seeds), indeg, m, want["counts"], changed, modes)


CASES = [("er", lambda: gen.erdos_renyi_gnm(3000, 9000, 5), 100),
         ("grid", lambda: gen.grid_with_shortcuts(60, 50, gen.Fraction(1, 10), 12, 3), 64),
         ("rmat", lambda: gen.rmat(12, 8, 9), 130)]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("persistent", [False, True])
def test_round_features_match_oracle(case, persistent):
    name, make, s = CASES[case]
    g = make()
    seeds = gen.sample_seeds(g.n, s, 17 + case)
    say("features", name, "persistent", persistent)
    want = oracle.propagate(g.n, g.src, g.dst, seeds, g.undirected, dist=True)
    D = want["D"]
    cap = D + 4
    graph = pp.pp_csr_build(g.n, g.src, g.dst, undirected=g.undirected)
    opts = pp.options(scheduler=pp.PP_SCHED_FUZZ, fuzz_seed=case, max_rounds=cap, persistent=persistent)
    run = pp.pp_seeds_init(graph, seeds, opts=opts)
    counts, Dg = pp.pp_propagate_until_converged(run)
    assert int(Dg[0]) == D and list(counts[0]) == list(want["counts"])
    modes, _ = pp.pp_get_round_log(run, cap)
    feat = pp.pp_get_round_features(run, cap)
    rows = D + 2   # rounds 0 .. D+1 each write the next round's row
    exp = oracle_features(g.n, g.src, g.dst, seeds, g.undirected, modes, rows, want)
    assert len(set(modes[1:D + 2].tolist())) == 2   # both directions were taken
    np.testing.assert_allclose(feat[1:rows + 1], exp, rtol=FEAT_RTOL, atol=0)


@pytest.mark.parametrize("which", ["threshold", "random0", "random1", "unset"])
@pytest.mark.parametrize("persistent", [False, True])
def test_mlp_decisions_and_outputs(which, persistent):
    g = gen.grid_with_shortcuts(90, 70, gen.Fraction(1, 10), 20, 4)
    s = 96
    seeds = gen.sample_seeds(g.n, s, 23)
    say("mlp decisions", which, "persistent", persistent)
    want = oracle.propagate(g.n, g.src, g.dst, seeds, g.undirected, seed_counts=True, final_sig=True)
    D = want["D"]
    cap = D + 4
    if which == "threshold":
        params = threshold_params(0.05)
    elif which == "unset":
        params = None
    else:
        params = rand_params(int(which[-1]) + 40, scale=1.0)
    graph = pp.pp_csr_build(g.n, g.src, g.dst, undirected=True)
    opts = pp.options(scheduler=pp.PP_SCHED_MLP, max_rounds=cap, persistent=persistent, seed_counts=True)
    run = pp.pp_seeds_init(graph, seeds, opts=opts)
    if params is not None:
        pp.pp_run_set_mlp(run, params)
    counts, Dg = pp.pp_propagate_until_converged(run)
    assert int(Dg[0]) == D and list(counts[0]) == list(want["counts"])
    sig = pp.pp_get_signatures(run)
    assert np.array_equal(sig[:, :want["final_sig"].shape[1]], want["final_sig"])
    assert np.array_equal(pp.pp_get_seed_counts(run, D + 1)[0], want["seed_counts"])
    modes, _ = pp.pp_get_round_log(run, cap)
    feat = pp.pp_get_round_features(run, cap)
    # the logged mode of each action: the persistent engine's pushes use direct slots
    logged = {0: pp.MODE_PULL, 1: pp.MODE_PUSH, 2: pp.MODE_PUSH if persistent else pp.MODE_PUSH_FLAT,
              3: pp.MODE_SPULL}
    checked = 0
    for r in range(1, D + 2):
        f = feat[r].astype(np.float64)
        if params is None:
            # no weights: the heuristic (push while frontier arcs * 8 < arcs; this
            # graph's frontiers are far below the flattened tiling's 16384 entries)
            exp = 1 if f[1] * 8 < 1.0 else 0
            if abs(f[1] * 8 - 1.0) < 1e-6:
                continue
        else:
            y = omlp.forward(params.astype(np.float64), f.reshape(1, 8))[0]
            allowed = (0, 1, 2)
            a = omlp.decide(params.astype(np.float64), f, allowed)
            # a near tie may go either way in fp32; an exact one (outputs with no
            # weights) goes to the first of the equal outputs on both sides
            if any(0 < abs(y[b] - y[a]) < 1e-4 * (1 + abs(y[a])) for b in allowed if b != a):
                continue
            exp = logged[a]
        assert modes[r] == exp, (r, modes[r], exp, f)
        checked += 1
    assert checked >= D - 2
    if which == "threshold":
        assert 0 in modes[1:D + 2] and 1 in modes[1:D + 2]


def test_forced_rounds_keep_results():
    g, seeds = gen.workload_er(2)
    say("forced rounds", g.n)
    want = oracle.propagate(g.n, g.src, g.dst, seeds, g.undirected, dist=True)
    D = want["D"]
    graph = pp.pp_csr_build(g.n, g.src, g.dst, undirected=g.undirected)
    run = pp.pp_seeds_init(graph, seeds, opts=pp.options(max_rounds=D + 4))
    rng = np.random.default_rng(4)
    forced, xs, ts = [], [], []
    while True:
        mode = [pp.MODE_PULL, pp.MODE_PUSH, pp.MODE_PUSH_FLAT, pp.MODE_SPULL][int(rng.integers(0, 4))]
        try:
            f, ms = pp.pp_time_round(run, mode)
        except pp.PPError as e:
            assert e.code == pp.PP_ESTATE
            break
        forced.append(mode)
        xs.append(f)
        ts.append(ms)
    assert len(xs) == D + 1
    assert np.all(np.isfinite(ts)) and np.all(np.array(ts) > 0)
    counts, Dg = pp.pp_propagate_until_converged(run)
    assert int(Dg[0]) == D and list(counts[0]) == list(want["counts"])
    modes, _ = pp.pp_get_round_log(run, D + 4)
    assert list(modes[1:D + 2]) == forced
    feat = pp.pp_get_round_features(run, D + 4)
    np.testing.assert_array_equal(np.array(xs), feat[1:D + 2])
    exp = oracle_features(g.n, g.src, g.dst, seeds, g.undirected, modes, D + 2, want)
    np.testing.assert_allclose(np.array(xs), exp[:D + 1], rtol=FEAT_RTOL, atol=0)
    with pytest.raises(pp.PPError):
        pp.pp_time_round(run, 2)


def test_trained_scheduler_keeps_results():
    """Costs measured on two grids, a model trained on the device, a third grid run with it."""
    parts = []
    for k in range(2):
        g = gen.grid_with_shortcuts(200, 200, gen.Fraction(1, 10), 30, 50 + k)
        graph = pp.pp_csr_build(g.n, g.src, g.dst, undirected=True)
        table = scheduler.measure(graph, gen.sample_seeds(g.n, 128, k))
        _, best, plan = scheduler.optimal_schedule(table)
        heur, _ = scheduler.policy_cost(table, scheduler.heuristic_policy())
        assert best <= heur + 1e-9
        parts.append(scheduler.label(table))
    samples = scheduler.Samples.concat(parts)
    say("trained scheduler samples", len(samples))
    params, losses = scheduler.train(samples, steps=1500)
    assert np.isfinite(losses).all() and losses[-1] < 0.5 * losses[0]
    g = gen.grid_with_shortcuts(200, 200, gen.Fraction(1, 10), 30, 60)
    seeds = gen.sample_seeds(g.n, 128, 9)
    want = oracle.propagate(g.n, g.src, g.dst, seeds, True)
    graph = pp.pp_csr_build(g.n, g.src, g.dst, undirected=True)
    ms, counts, D, modes = scheduler.timed_run(graph, seeds, pp.PP_SCHED_MLP, params, repeats=1)
    assert int(D[0]) == want["D"] and list(counts[0]) == list(want["counts"])
    assert math.isfinite(ms)


def grid_tables(side, seeds_per, ks, shortcuts=60):
    tables, graphs = [], []
    for k in ks:
        g = gen.grid_with_shortcuts(side, side, gen.Fraction(1, 10), shortcuts, 70 + k)
        graph = pp.pp_csr_build(g.n, g.src, g.dst, undirected=True)
        sd = gen.sample_seeds(g.n, seeds_per, k)
        tables.append(scheduler.measure_replay(graph, sd))
        graphs.append((graph, sd))
    return tables, graphs


@pytest.fixture(scope="module")
def trained_on_grids():
    """Round costs of three 768^2 grids with deletions and shortcuts (s = 128) under every
    action after both kinds of round, from replayed propagations that follow fixed
    plans; a model trained on the first two."""
    tables, graphs = grid_tables(768, 128, (2, 3, 1))
    params, losses = scheduler.train(scheduler.Samples.concat(scheduler.label(t) for t in tables[:2]), steps=4000)
    yield tables, graphs, params, losses
    for graph, _ in graphs:
        graph.free()


def test_learned_schedule_gains_on_held_out_costs(trained_on_grids):
    """The trained model's schedule against the fixed rule's (the heuristic's direction
    threshold and tiling threshold), both priced on the measured round costs of the
    held-out graph: the model must be strictly cheaper and near the optimum."""
    tables, _, params, losses = trained_on_grids
    held = tables[2]
    _, best, _ = scheduler.optimal_schedule(held)
    heur, hplan = scheduler.policy_cost(held, scheduler.heuristic_policy(8, held.n))
    learned, plan = scheduler.policy_cost(held, scheduler.model_policy(params, held))
    say("held-out costs ms: optimal %.3f heuristic %.3f learned %.3f (loss %.3f -> %.4f); actions %s" % (
        best, heur, learned, losses[0], losses[-1], np.bincount(plan, minlength=4).tolist()))
    assert best <= learned + 1e-9 and best <= heur + 1e-9
    assert learned < heur
    assert learned <= best * 1.03


def test_learned_scheduler_gains_in_wall_time(trained_on_grids):
    """The same held-out graph run end to end (graph replay, after warm-up runs): the
    learned scheduler's median wall time must be below the default-threshold
    heuristic's.  Reported beside them: the heuristic at its autotuned threshold,
    and the measured table's optimal plan replayed (PP_SCHED_PLAN)."""
    tables, graphs, params, _ = trained_on_grids
    graph, seeds = graphs[2]
    h_ms, hc, hD = scheduler.wall_times(graph, seeds, pp.PP_SCHED_HEURISTIC, reps=11)
    l_ms, lc, lD = scheduler.wall_times(graph, seeds, pp.PP_SCHED_MLP, params, reps=11)
    assert int(hD[0]) == int(lD[0]) and list(hc[0]) == list(lc[0])   # the same counts every way
    tuned, _ = pp.pp_autotune(graph, seeds, reps=2)
    t_ms, _, _ = scheduler.wall_times(graph, seeds, pp.PP_SCHED_HEURISTIC, reps=7, push_div=int(tuned.push_div),
                                      pull_k=int(tuned.pull_k))
    _, _, plan = scheduler.optimal_schedule(tables[2])
    o_ms, oc, _ = scheduler.wall_times(graph, seeds, pp.PP_SCHED_PLAN, plan=plan, reps=7)
    assert list(oc[0]) == list(hc[0])
    hm, lm, tm, om = (float(np.median(x)) for x in (h_ms, l_ms, t_ms, o_ms))
    say("held-out wall ms (median): heuristic %.3f learned %.3f tuned threshold %.3f (push_div %d, pull_k %d); "
        "the table's optimal plan replayed %.3f" % (hm, lm, tm, tuned.push_div, tuned.pull_k, om))
    assert lm < hm


def test_plan_scheduler_keeps_results_and_follows_the_plan():
    """PP_SCHED_PLAN: every action the plan names runs in its round (the log says so),
    the rounds beyond the plan follow the heuristic, and no bit changes; each round's
    device-clock time is positive."""
    g, seeds = gen.workload_er(3)
    want = oracle.propagate(g.n, g.src, g.dst, seeds, True, seed_counts=True, final_sig=True)
    D = want["D"]
    G = pp.pp_csr_build(g.n, g.src, g.dst, undirected=True)
    for sparse in (0, 2):
        run = pp.pp_seeds_init(G, seeds, opts=pp.options(scheduler=pp.PP_SCHED_PLAN, sparse_pull=sparse,
                                                          seed_counts=True, max_rounds=D + 4))
        acts = [1, 0, 2, 3, 0, 1, 2][:D]
        pp.pp_run_set_plan(run, [-1] + acts)
        pp.pp_seeds_reset(run, seeds)
        counts, Dg = pp.pp_propagate_until_converged(run)
        assert int(Dg[0]) == D and list(counts[0]) == list(want["counts"])
        assert np.array_equal(pp.pp_get_seed_counts(run, D + 1)[0], want["seed_counts"])
        assert np.array_equal(pp.pp_get_signatures(run), want["final_sig"])
        modes, _ = pp.pp_get_round_log(run, D + 2)
        logged = {0: pp.MODE_PULL, 1: pp.MODE_PUSH, 2: pp.MODE_PUSH_FLAT, 3: pp.MODE_SPULL}
        for r, a in enumerate(acts, start=1):
            if a == 3 and sparse == 0:
                continue   # not allowed: the heuristic's choice
            assert int(modes[r]) == logged[a], (r, a, modes[r])
        t = pp.pp_get_round_times(run, D + 3)
        assert t[0] == 0 and np.all(t[1:D + 2] > 0) and t[D + 2] == 0
        run.free()
