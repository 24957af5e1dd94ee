"""GPU parity of runs with seed groups (several groups of one graph's seeds in
the same launches, each with its own row width, direction, counts and
convergence) and with a seed order, against the oracle, element by element.

Outputs must be those of a single group in the caller's bit order: per-round
counts, D, per-seed counts and final signatures, for ragged groups, more than
512 seeds, the by-reach grouping (a group of seeds without predecessors
converges after its first round), batches of graphs, every direction policy,
rounds one at a time, device seed lists, snapshots and the learned scheduler.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2301_06499_amd import inputs as gen
from paper_2301_06499_amd import pp

pytestmark = pytest.mark.gpu

SCHEDS = [pp.PP_SCHED_PULL, pp.PP_SCHED_PUSH, pp.PP_SCHED_HEURISTIC, pp.PP_SCHED_FUZZ]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def pad_words(sig, W):
    if sig.shape[1] == W:
        return sig
    out = np.zeros((sig.shape[0], W), dtype=np.uint64)
    out[:, :sig.shape[1]] = sig
    return out


def check(g, seeds, want=None, **kw):
    s = len(seeds)
    if want is None:
        want = oracle.propagate(g.n, g.src, g.dst, seeds, g.undirected, seed_counts=True, final_sig=True)
    G = pp.pp_csr_build(g.n, g.src, g.dst, undirected=g.undirected, keep_order=kw.pop("keep_order", False))
    opts = pp.options(seed_counts=True, max_rounds=want["D"] + 4, **kw)
    r = pp.pp_seeds_init(G, seeds, opts=opts)
    counts, D = pp.pp_propagate_until_converged(r)
    assert int(D[0]) == want["D"]
    assert list(counts[0]) == list(want["counts"])
    assert np.array_equal(pp.pp_get_seed_counts(r, want["D"] + 1)[0], want["seed_counts"])
    assert np.array_equal(pp.pp_get_signatures(r), pad_words(want["final_sig"], r.words))
    return r, G, want


GRAPHS = [lambda: gen.path_graph(60), lambda: gen.star_graph(700), lambda: gen.grid_graph(17, 11),
          lambda: gen.path_graph(40, directed=True), lambda: gen.rmat(12, 16, 3),
          lambda: gen.erdos_renyi_gnm(900, 2500, 4)]
SPLITS = [(130, 3), (65, 2), (300, 2), (256, 4), (200, 1), (64, 64)]


@pytest.mark.parametrize("gi", range(len(GRAPHS)))
@pytest.mark.parametrize("split", range(len(SPLITS)))
@pytest.mark.parametrize("order", [0, 1])
def test_groups_match_oracle(gi, split, order):
    g = GRAPHS[gi]()
    s, k = SPLITS[split]
    seeds = gen.sample_seeds(g.n, min(s, g.n), 5 + gi, distinct=False)
    if len(seeds) < s:
        seeds = np.resize(seeds, s)
    sched = SCHEDS[(gi + split) % 4]
    say("groups", g.name, "s", s, "k", k, "order", order, "sched", sched)
    r, _, _ = check(g, seeds, scheduler=sched, seed_groups=k, seed_order=order, fuzz_seed=gi)
    assert r.groups == k


@pytest.mark.parametrize("s", [513, 700, 1024, 4096])
def test_more_than_512_seeds(s):
    """s > 512: ceil(s / 512) groups by default (up to 64-word reported rows)."""
    g = gen.rmat(11, 8, 9) if s < 4096 else gen.erdos_renyi_gnm(5000, 15000, 3)
    seeds = gen.sample_seeds(g.n, s, 31, distinct=False)
    say("wide", g.name, "s", s)
    r, _, _ = check(g, seeds, scheduler=pp.PP_SCHED_FUZZ, fuzz_seed=s)
    assert r.groups == (s + 511) // 512 and r.words == 1 << max(0, (s + 63) // 64 - 1).bit_length()


@pytest.mark.parametrize("sched", SCHEDS)
@pytest.mark.parametrize("sparse", [0, 1, 2])
def test_by_reach_on_rmat(sched, sparse):
    """R-MAT: about half the seeds have no predecessor.  By reach, those fill the last
    group, which converges at round 1 while the first runs on; the groups' own logs
    show it."""
    g = gen.rmat(14, 16, 77)
    pred = np.bincount(g.dst[g.src != g.dst], minlength=g.n) > 0
    # 100 seeds with a predecessor and 156 without, interleaved (a uniform sample of a
    # graph this small has about 63% of the first kind; R-MAT 20: 50%, 26: 36%)
    pool = gen.sample_seeds(g.n, 2000, 8)
    lv, dd = pool[pred[pool]][:100], pool[~pred[pool]][:156]
    seeds = np.empty(256, np.int32)
    pick = np.zeros(256, bool)
    pick[np.linspace(0, 255, 100).astype(int)] = True
    seeds[pick], seeds[~pick] = lv, dd
    live = int(pred[seeds].sum())
    assert live == 100
    say("by reach rmat14 live", live, "sched", sched, "sparse", sparse)
    r, _, want = check(g, seeds, scheduler=sched, seed_groups=pp.PP_GROUPS_BY_REACH, sparse_pull=sparse,
                       fuzz_seed=4)
    k = r.groups
    sg = -(-256 // k)
    assert sg >= live and k >= 2
    modes_last, _ = pp.pp_get_group_log(r, k - 1, want["D"] + 2)
    assert [int(m) for m in modes_last[:3]] == [2, int(modes_last[1]), -1]   # init, one round, nothing after
    modes0, _ = pp.pp_get_group_log(r, 0, want["D"] + 2)
    assert all(int(m) in (0, 1, 3, 4) for m in modes0[1:want["D"] + 2])


@pytest.mark.parametrize("sched", [pp.PP_SCHED_PULL, pp.PP_SCHED_PUSH, pp.PP_SCHED_HEURISTIC])
def test_resets_after_groups_that_added_nothing(sched):
    """A reset clears only the seeds' rows of a group whose last propagation
    added no bit after round 0.  Seed sets that put live seeds into such groups
    and take them out again, on one run: every count, per-seed count and final
    signature against the oracle after each reset, including a reset after a
    propagation stopped after one round (which clears every group in full)."""
    g = gen.rmat(14, 16, 77)
    pred = np.bincount(g.dst[g.src != g.dst], minlength=g.n) > 0
    pool = gen.sample_seeds(g.n, 6000, 9)
    lv, dd = pool[pred[pool]], pool[~pred[pool]]
    assert len(lv) >= 600 and len(dd) >= 450
    few = [np.concatenate([lv[:40], dd[:216]]), np.concatenate([dd[216:416], lv[40:96]])]
    many = [lv[100:356], lv[356:612]]
    sets = [few[0], many[0], few[1], many[1], few[0]]
    sets = [np.ascontiguousarray(s, dtype=np.int32) for s in sets]
    wants = [oracle.propagate(g.n, g.src, g.dst, sd, False, seed_counts=True, final_sig=True) for sd in sets]
    G = pp.pp_csr_build(g.n, g.src, g.dst)
    opts = pp.options(seed_counts=True, max_rounds=max(w["D"] for w in wants) + 4, scheduler=sched,
                      seed_groups=pp.PP_GROUPS_BY_REACH)

    def run_to_end(r, want, i):
        counts, D = pp.pp_propagate_until_converged(r)
        assert int(D[0]) == want["D"], i
        assert list(counts[0]) == list(want["counts"]), i
        assert np.array_equal(pp.pp_get_seed_counts(r, want["D"] + 1)[0], want["seed_counts"]), i
        assert np.array_equal(pp.pp_get_signatures(r), pad_words(want["final_sig"], r.words)), i

    say("resets after dead groups, sched", sched)
    r = pp.pp_seeds_init(G, sets[0], opts=opts)
    assert r.groups == 4   # 40 seeds with a predecessor: groups of 64, three of them dead
    run_to_end(r, wants[0], 0)
    for i in range(1, len(sets)):
        say("  set", i)
        pp.pp_seeds_reset(r, sets[i])
        run_to_end(r, wants[i], i)
    say("  stopped after one round, then a reset")
    pp.pp_seeds_reset(r, sets[2])
    pp.pp_propagate_round(r)
    pp.pp_seeds_reset(r, sets[3])
    run_to_end(r, wants[3], "after a stop")
    r.free()
    G.free()


@pytest.mark.parametrize("persistent_first", [False])
def test_batch_of_graphs_with_groups(persistent_first):
    graphs = [gen.grid_graph(20, 15), gen.path_graph(300), gen.rmat(10, 8, 4), gen.star_graph(900),
              gen.cycle_graph(7, directed=True)]
    s = 150
    seeds = []
    for k_, g in enumerate(graphs):
        sd = gen.sample_seeds(g.n, min(s, g.n), 20 + k_)
        seeds.append(np.resize(sd, s))
    wants = [oracle.propagate(g.n, g.src, g.dst, sd, g.undirected, seed_counts=True, final_sig=True)
             for g, sd in zip(graphs, seeds)]
    n, src, dst, offs, allseeds = gen.union_of(graphs, seeds)
    G = pp.pp_csr_build(n, src, dst, node_offsets=offs)
    for sched in SCHEDS:
        for k, order in ((3, 1), (2, 0), (pp.PP_GROUPS_BY_REACH, 1)):
            say("batch groups", sched, k, order)
            r = pp.pp_seeds_init(G, allseeds, s=s, opts=pp.options(scheduler=sched, seed_counts=True, max_rounds=400,
                                                                   fuzz_seed=2, seed_groups=k, seed_order=order))
            counts, D = pp.pp_propagate_until_converged(r)
            sc = pp.pp_get_seed_counts(r, 400)
            sig = pp.pp_get_signatures(r)
            for j, w in enumerate(wants):
                assert int(D[j]) == w["D"], j
                assert list(counts[j][:w["D"] + 1]) == list(w["counts"]), j
                assert np.array_equal(sc[j][:w["D"] + 1], w["seed_counts"]), j
                assert np.array_equal(sig[offs[j]:offs[j + 1]], pad_words(w["final_sig"], r.words)), j
            r.free()


@pytest.mark.parametrize("k", [2, 3])
def test_round_by_round_snapshot_and_device_seeds(k):
    from hipmem import DeviceArray
    g, seeds = gen.workload_er(1)
    want = oracle.propagate(g.n, g.src, g.dst, seeds, True, sig_rounds=list(range(0, 16)), seed_counts=True,
                            final_sig=True)
    say("groups rounds", k, "D", want["D"])
    G = pp.pp_csr_build(g.n, g.src, g.dst, undirected=True)
    r = pp.pp_seeds_init(G, seeds, opts=pp.options(scheduler=pp.PP_SCHED_FUZZ, fuzz_seed=9, max_rounds=64,
                                                    seed_groups=k, seed_order=1, seed_counts=True))
    assert np.array_equal(pp.pp_get_signatures(r), pad_words(want["sigs"][0], r.words))
    got = [len(seeds)]
    snap = None
    for step in range(1, want["D"] + 2):
        nb, conv = pp.pp_propagate_round(r)
        got.append(int(nb[0]))
        assert np.array_equal(pp.pp_get_signatures(r), pad_words(want["sigs"][min(step, 15)], r.words)), step
        assert conv == (step == want["D"] + 1)
        if step == 2:
            snap = pp.pp_run_snapshot(r)
    assert got[:-1] == list(want["counts"]) and got[-1] == 0
    # restored after round 2, the run ends the same
    pp.pp_run_restore(r, snap)
    counts, D = pp.pp_propagate_until_converged(r)
    assert list(counts[0]) == list(want["counts"])
    assert np.array_equal(pp.pp_get_seed_counts(r, want["D"] + 1)[0], want["seed_counts"])
    # device seeds for a reset: another seed list, mapped and ordered on the device
    s2 = gen.sample_seeds(g.n, len(seeds), 77)
    w2 = oracle.propagate(g.n, g.src, g.dst, s2, True, seed_counts=True, final_sig=True)
    pp.pp_seeds_reset(r, DeviceArray(s2.astype(np.int32)))
    counts, D = pp.pp_propagate_until_converged(r)
    assert list(counts[0]) == list(w2["counts"])
    assert np.array_equal(pp.pp_get_seed_counts(r, w2["D"] + 1)[0], w2["seed_counts"])
    assert np.array_equal(pp.pp_get_signatures(r), pad_words(w2["final_sig"], r.words))
    bad = DeviceArray(np.where(np.arange(len(s2)) == 3, g.n + 5, s2).astype(np.int32))
    pp.pp_seeds_reset(r, bad)
    with pytest.raises(pp.PPError) as e:
        pp.pp_propagate_until_converged(r)
    assert e.value.code == pp.PP_ERANGE


def test_learned_scheduler_and_forced_rounds_with_groups():
    from test_gpu_scheduler import rand_params, threshold_params
    g = gen.rmat(13, 16, 21)
    seeds = gen.sample_seeds(g.n, 256, 4)
    want = oracle.propagate(g.n, g.src, g.dst, seeds, False, seed_counts=True, final_sig=True)
    G = pp.pp_csr_build(g.n, g.src, g.dst)
    for params in (threshold_params(0.125), rand_params(5, 0.4)):
        r = pp.pp_seeds_init(G, seeds, opts=pp.options(scheduler=pp.PP_SCHED_MLP, seed_counts=True, max_rounds=64,
                                                        seed_groups=pp.PP_GROUPS_BY_REACH))
        pp.pp_run_set_mlp(r, params)
        counts, D = pp.pp_propagate_until_converged(r)
        assert list(counts[0]) == list(want["counts"])
        assert np.array_equal(pp.pp_get_seed_counts(r, want["D"] + 1)[0], want["seed_counts"])
        assert np.array_equal(pp.pp_get_signatures(r), pad_words(want["final_sig"], r.words))
        r.free()
    # every direction forced in round 2, in every group at once
    r = pp.pp_seeds_init(G, seeds, opts=pp.options(max_rounds=64, seed_groups=2, seed_order=1))
    pp.pp_propagate_round(r)
    snap = pp.pp_run_snapshot(r)
    for mode in (pp.MODE_PULL, pp.MODE_PUSH, pp.MODE_SPULL):
        pp.pp_run_restore(r, snap)
        f, ms = pp.pp_time_round(r, mode)
        assert ms > 0
        counts, D = pp.pp_propagate_until_converged(r)
        assert list(counts[0]) == list(want["counts"])
        assert np.array_equal(pp.pp_get_signatures(r), pad_words(want["final_sig"], r.words))


def test_group_errors():
    g = gen.path_graph(100)
    G = pp.pp_csr_build(g.n, g.src, g.dst, undirected=True)
    seeds = np.arange(0, 100, dtype=np.int32)
    for bad in (dict(seed_groups=65), dict(seed_groups=-2), dict(seed_order=2),
                dict(seed_groups=2, persistent=True), dict(seed_order=1, persistent=True),
                dict(seed_groups=2, node_stats=True)):
        with pytest.raises(pp.PPError) as e:
            pp.pp_seeds_init(G, seeds, opts=pp.options(**bad))
        assert e.value.code == pp.PP_EINVAL, bad
    with pytest.raises(pp.PPError) as e:      # 4 seeds cannot fill 3 groups of 2
        pp.pp_seeds_init(G, seeds[:4], opts=pp.options(seed_groups=3))
    assert e.value.code == pp.PP_EINVAL
    with pytest.raises(pp.PPError) as e:      # 600 seeds in one group
        pp.pp_seeds_init(G, np.resize(seeds, 600), opts=pp.options(seed_groups=1))
    assert e.value.code == pp.PP_EINVAL
    with pytest.raises(pp.PPError) as e:
        pp.pp_seeds_init(G, np.resize(seeds, 4097))
    assert e.value.code == pp.PP_EINVAL
    r = pp.pp_seeds_init(G, seeds, opts=pp.options(seed_groups=2))
    with pytest.raises(pp.PPError) as e:
        pp.pp_get_group_log(r, 2, 8)
    assert e.value.code == pp.PP_EINVAL
