"""GPU parity: the HIP path against the CPU oracle, element by element.

Integer work, so the bar is bit-exact: per-round counts, per-seed counts,
signatures (final and at sampled rounds), D, and the metrics (same exact
integer formulas on both sides).  Every direction policy is checked, since
the push/pull choice may never change an output bit.
"""
import sys

import numpy as np
import pytest

import oracle
import oracle.propagate_s
from paper_2301_06499_amd import inputs as gen
from paper_2301_06499_amd import pp

pytestmark = pytest.mark.gpu

SCHEDS = [pp.PP_SCHED_PULL, pp.PP_SCHED_PUSH, pp.PP_SCHED_HEURISTIC, pp.PP_SCHED_FUZZ]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def pad_words(sig, W):
    """Oracle signatures [n][ceil(s/64)] padded to the library's W words."""
    if sig.shape[1] == W:
        return sig
    out = np.zeros((sig.shape[0], W), dtype=np.uint64)
    out[:, :sig.shape[1]] = sig
    return out


def check_run(n, src, dst, seeds, undirected, transpose=False, sched=pp.PP_SCHED_HEURISTIC,
              fuzz_seed=0, use_graph=True, want=None, max_rounds=0, persistent=False, keep_order=False,
              pull_k=0, sparse_pull=0):
    s = len(seeds)
    if want is None:
        want = oracle.propagate(n, src, dst, seeds, undirected, transpose=transpose,
                                seed_counts=True, final_sig=True)
    g = pp.pp_csr_build(n, src, dst, undirected=undirected, transpose=transpose, keep_order=keep_order)
    cap = max_rounds or want["D"] + 4
    opts = pp.options(scheduler=sched, seed_counts=True, max_rounds=cap, fuzz_seed=fuzz_seed,
                      use_graph=use_graph, persistent=persistent, pull_k=pull_k, sparse_pull=sparse_pull)
    r = pp.pp_seeds_init(g, seeds, opts=opts)
    counts, D = pp.pp_propagate_until_converged(r)
    assert int(D[0]) == want["D"]
    assert list(counts[0]) == list(want["counts"])
    sig = pp.pp_get_signatures(r)
    assert np.array_equal(sig, pad_words(want["final_sig"], r.words))
    sc = pp.pp_get_seed_counts(r, want["D"] + 1)[0]
    assert np.array_equal(sc, want["seed_counts"])
    return r, g, counts[0]


# ------------------------------------------------------------ closed forms

CLOSED = [gen.path_graph(50), gen.cycle_graph(31), gen.cycle_graph(32), gen.star_graph(3000),
          gen.complete_graph(40), gen.grid_graph(13, 9), gen.path_graph(30, directed=True),
          gen.cycle_graph(17, directed=True), gen.path_graph(1), gen.path_graph(2)]


@pytest.mark.parametrize("gi", range(len(CLOSED)))
@pytest.mark.parametrize("sched", SCHEDS)
@pytest.mark.parametrize("persistent", [False, True])
def test_closed_form_graphs(gi, sched, persistent):
    g = CLOSED[gi]
    s = min(g.n, 512)
    seeds = gen.sample_seeds(g.n, s, 3 + gi)
    say("closed", g.name, "s", s, "sched", sched)
    check_run(g.n, g.src, g.dst, seeds, g.undirected, sched=sched, fuzz_seed=gi, persistent=persistent)


@pytest.mark.parametrize("sched", SCHEDS)
def test_transposed_direction(sched):
    g = gen.path_graph(40, directed=True)
    seeds = np.array([0, 5, 39, 20], np.int32)
    say("transpose", sched)
    r, _, counts = check_run(g.n, g.src, g.dst, seeds, False, transpose=True, sched=sched)
    # seed x reaches x+1..n-1 along reversed arcs: c_i[r] = 1 for r <= n-1-x
    assert counts[1] == 3


# ------------------------------------------------------------ random graphs

@pytest.mark.parametrize("trial", range(24))
def test_random_graphs_word_boundaries(trial):
    rng = np.random.default_rng(500 + trial)
    s = [1, 63, 64, 65, 127, 129, 200, 256, 300, 448, 511, 512][trial % 12]
    n = int(rng.integers(max(2, s // 4), 3000))
    m = int(rng.integers(0, 8 * n))
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    und = bool(trial % 3 == 0)
    tr = bool(trial % 4 == 1)
    seeds = rng.integers(0, n, s).astype(np.int32)          # repeats allowed
    sched = SCHEDS[trial % 4]
    pers = trial % 2 == 1
    k = 2 if (not pers and trial % 4 == 2) else 0
    say("random", trial, "n", n, "m", m, "s", s, "und", und, "tr", tr, "sched", sched, "pull_k", k)
    check_run(n, src, dst, seeds, und, transpose=tr, sched=sched, fuzz_seed=trial, persistent=pers, pull_k=k)


@pytest.mark.parametrize("sched", SCHEDS)
@pytest.mark.parametrize("persistent", [False, True])
@pytest.mark.parametrize("keep_order", [False, True])
def test_rmat_with_hubs(sched, persistent, keep_order):
    """R-MAT scale 14: nodes with more arcs than a pull tile holds (hub chunks);
    stored in hub-first order (results reported by input id) or in input order."""
    g = gen.rmat(14, 16, 77)
    seeds = gen.sample_seeds(g.n, 256, 8)
    say("rmat14", sched, "persistent", persistent, "keep_order", keep_order)
    check_run(g.n, g.src, g.dst, seeds, False, sched=sched, fuzz_seed=5, persistent=persistent,
              keep_order=keep_order, pull_k=2 if (keep_order and not persistent) else 0)


@pytest.mark.parametrize("keep_order", [False, True])
def test_device_arcs_seeds_and_signatures(keep_order):
    """Device-resident input arcs, device seeds for a reset, signatures into device memory."""
    from hipmem import DeviceArray
    g = gen.rmat(12, 16, 5)
    s1 = gen.sample_seeds(g.n, 100, 1)
    s2 = gen.sample_seeds(g.n, 100, 2)
    say("device io", keep_order)
    w1 = oracle.propagate(g.n, g.src, g.dst, s1, False, final_sig=True)
    w2 = oracle.propagate(g.n, g.src, g.dst, s2, False, final_sig=True)
    dsrc, ddst = DeviceArray(g.src.astype(np.int32)), DeviceArray(g.dst.astype(np.int32))
    G = pp.pp_csr_build(g.n, dsrc, ddst, keep_order=keep_order)
    host_G = pp.pp_csr_build(g.n, g.src, g.dst, keep_order=keep_order)
    assert G.arcs == host_G.arcs
    r = pp.pp_seeds_init(G, s1)
    c, D = pp.pp_propagate_until_converged(r)
    assert list(c[0]) == list(w1["counts"])
    out = DeviceArray(dtype=np.uint64, count=g.n * r.words)
    pp.pp_get_signatures(r, out)
    assert np.array_equal(out.to_host().reshape(g.n, r.words), pad_words(w1["final_sig"], r.words))
    pp.pp_seeds_reset(r, DeviceArray(s2.astype(np.int32)))
    c, D = pp.pp_propagate_until_converged(r)
    assert list(c[0]) == list(w2["counts"])
    assert np.array_equal(pp.pp_get_signatures(r), pad_words(w2["final_sig"], r.words))
    bad = DeviceArray(np.where(np.arange(100) == 7, g.n, s2).astype(np.int32))
    pp.pp_seeds_reset(r, bad)   # checked on the device: reported by the next wait
    with pytest.raises(pp.PPError) as e:
        pp.pp_propagate_until_converged(r)
    assert e.value.code == pp.PP_ERANGE
    pp.pp_seeds_reset(r, s1)
    c, D = pp.pp_propagate_until_converged(r)
    assert list(c[0]) == list(w1["counts"])


def test_empty_and_isolated():
    say("empty")
    check_run(10, np.zeros(0, np.int32), np.zeros(0, np.int32), np.array([3, 3, 9], np.int32), False)
    check_run(5, np.array([0, 1, 2], np.int32), np.array([0, 1, 2], np.int32), np.array([4], np.int32), True)


# ------------------------------------------------------------ round by round

@pytest.mark.parametrize("sched", [pp.PP_SCHED_PULL, pp.PP_SCHED_PUSH, pp.PP_SCHED_FUZZ])
@pytest.mark.parametrize("persistent", [False, True])
def test_er_workload_round_by_round(sched, persistent):
    """The ER workload, signatures after every round, and the metrics."""
    g, seeds = gen.workload_er(1)
    want = oracle.propagate(g.n, g.src, g.dst, seeds, True, sig_rounds=list(range(0, 16)),
                            seed_counts=True, final_sig=True)
    say("er rounds", sched, "D", want["D"], "persistent", persistent)
    G = pp.pp_csr_build(g.n, g.src, g.dst, undirected=True)
    r = pp.pp_seeds_init(G, seeds, opts=pp.options(scheduler=sched, seed_counts=True, max_rounds=64,
                                                    fuzz_seed=9, persistent=persistent))
    assert np.array_equal(pp.pp_get_signatures(r), want["sigs"][0])
    got = [len(seeds)]
    for k in range(1, want["D"] + 2):
        nb, conv = pp.pp_propagate_round(r)
        got.append(int(nb[0]))
        assert np.array_equal(pp.pp_get_signatures(r), want["sigs"][min(k, 15)]), k
        assert conv == (k == want["D"] + 1)
    assert got[:-1] == list(want["counts"]) and got[-1] == 0
    counts, D = pp.pp_propagate_until_converged(r)
    m_gpu = pp.pp_estimate_metrics(counts[0], g.n, len(seeds))
    m_cpu = oracle.metrics(want["counts"], g.n, len(seeds))
    for k, v in m_cpu.items():
        assert m_gpu[k] == v


def test_snapshot_restore_and_graph_replay():
    g, seeds = gen.workload_er(2)
    want = oracle.propagate(g.n, g.src, g.dst, seeds, True, final_sig=True)
    G = pp.pp_csr_build(g.n, g.src, g.dst, undirected=True)
    r = pp.pp_seeds_init(G, seeds, opts=pp.options(scheduler=pp.PP_SCHED_FUZZ, fuzz_seed=3, max_rounds=64))
    pp.pp_propagate_round(r)
    pp.pp_propagate_round(r)
    snap = pp.pp_run_snapshot(r)
    c1, D1 = pp.pp_propagate_until_converged(r)
    sig1 = pp.pp_get_signatures(r)
    pp.pp_run_restore(r, snap)
    assert r.round == 3
    c2, D2 = pp.pp_propagate_until_converged(r)
    assert np.array_equal(c1, c2) and np.array_equal(sig1, pp.pp_get_signatures(r))
    assert list(c1[0]) == list(want["counts"])
    # the same run replayed without graph capture, one round per sync
    r2 = pp.pp_seeds_init(G, seeds, opts=pp.options(scheduler=pp.PP_SCHED_FUZZ, fuzz_seed=3, max_rounds=64,
                                                     use_graph=False, rounds_per_sync=1))
    c3, _ = pp.pp_propagate_until_converged(r2)
    assert np.array_equal(c1, c3)
    say("snapshot ok")


@pytest.mark.parametrize("persistent", [False, True])
def test_round_cap_reports_not_converged(persistent):
    g = gen.path_graph(200)
    seeds = np.array([0], np.int32)
    G = pp.pp_csr_build(g.n, g.src, g.dst, undirected=True)
    r = pp.pp_seeds_init(G, seeds, opts=pp.options(max_rounds=50, persistent=persistent))
    with pytest.raises(pp.PPError) as e:
        pp.pp_propagate_until_converged(r)
    assert e.value.code == pp.PP_ENOTCONV
    counts, D = pp.pp_propagate_until_converged(r, raise_on_cap=False)
    assert list(counts[0][:50]) == [1] * 50


# ------------------------------------------------------------ batches

def test_batched_union_matches_solo_runs():
    graphs = [gen.grid_graph(20, 15), gen.path_graph(300), gen.rmat(10, 8, 4), gen.star_graph(2500),
              gen.cycle_graph(7, directed=True), gen.path_graph(1)]
    s = 64
    offs = [0]
    srcs, dsts, seeds = [], [], []
    wants = []
    for k, g in enumerate(graphs):
        sd = gen.sample_seeds(g.n, min(s, g.n), 20 + k)
        if len(sd) < s:
            sd = np.resize(sd, s)
        wants.append(oracle.propagate(g.n, g.src, g.dst, sd, g.undirected, seed_counts=True, final_sig=True))
        src, dst = g.src.astype(np.int64), g.dst.astype(np.int64)
        if g.undirected:
            src, dst = np.concatenate([src, dst]), np.concatenate([dst, src])
        srcs.append(src + offs[-1])
        dsts.append(dst + offs[-1])
        seeds.append(sd + offs[-1])
        offs.append(offs[-1] + g.n)
    n = offs[-1]
    # every direction policy on both engines, and sparse rounds as sparse pulls
    # (or mixed with pushes) on the per-round engine
    cases = [(sc_, p_, 0) for sc_ in SCHEDS for p_ in (False, True)] + \
            [(sc_, False, sp) for sc_ in (pp.PP_SCHED_PUSH, pp.PP_SCHED_HEURISTIC, pp.PP_SCHED_FUZZ) for sp in (1, 2)]
    for sched, persistent, sparse in cases:
        say("batch", sched, "persistent", persistent, "sparse_pull", sparse)
        G = pp.pp_csr_build(n, np.concatenate(srcs).astype(np.int32), np.concatenate(dsts).astype(np.int32),
                            node_offsets=offs)
        r = pp.pp_seeds_init(G, np.concatenate(seeds), s=s,
                             opts=pp.options(scheduler=sched, seed_counts=True, max_rounds=400, fuzz_seed=1,
                                             persistent=persistent, sparse_pull=sparse))
        counts, D = pp.pp_propagate_until_converged(r)
        sc = pp.pp_get_seed_counts(r, 400)
        sig = pp.pp_get_signatures(r)
        for k, w in enumerate(wants):
            assert int(D[k]) == w["D"], k
            assert list(counts[k][:w["D"] + 1]) == list(w["counts"]), k
            assert not counts[k][w["D"] + 1:].any()
            assert np.array_equal(sc[k][:w["D"] + 1], w["seed_counts"]), k
            # every graph's final signatures, also of graphs that converged long before the last
            assert np.array_equal(sig[offs[k]:offs[k + 1]], pad_words(w["final_sig"], r.words)), k


# ------------------------------------------------------------ short lists

PULL_NPL = 6   # the pull's one-lane-per-node limit (successors per node)


def capped_degree_graph(n, dmax, seed):
    """A directed graph with out-degree at most dmax, a quarter of the nodes at
    exactly dmax (distinct successors, no self-loops)."""
    rng = np.random.default_rng(seed)
    deg = rng.integers(0, dmax + 1, n)
    deg[rng.random(n) < 0.25] = dmax
    src, dst = [], []
    for u in range(n):
        off = 1 + rng.choice(n - 1, int(deg[u]), replace=False)
        src.append(np.full(len(off), u))
        dst.append((u + off) % n)
    return np.concatenate(src).astype(np.int32), np.concatenate(dst).astype(np.int32)


@pytest.mark.parametrize("dmax", [1, PULL_NPL, PULL_NPL + 1])
@pytest.mark.parametrize("s", [40, 64, 100, 128])
def test_short_list_pull(dmax, s):
    """Graphs whose every node has at most PULL_NPL successors and no high-degree
    chunk take the pull's short-list form at one- and two-word rows; one more
    successor on some node takes the general form.  Both against the oracle, with
    every round a pull and with the heuristic's mix."""
    n = 2500
    src, dst = capped_degree_graph(n, dmax, 900 + dmax)
    seeds = gen.sample_seeds(n, s, 31 + s)
    want = oracle.propagate(n, src, dst, seeds, False, seed_counts=True, final_sig=True)
    for sched in (pp.PP_SCHED_PULL, pp.PP_SCHED_HEURISTIC):
        say("short lists dmax", dmax, "s", s, "sched", sched)
        check_run(n, src, dst, seeds, False, sched=sched, want=want)


def test_short_list_pull_batch():
    """A batch of lattices, paths and cycles (every list short) whose members
    converge at different rounds: the pull's short-list form copies the rows of
    a converged member and gathers for the others."""
    graphs = [gen.grid_graph(30, 20), gen.path_graph(400), gen.cycle_graph(9, directed=True),
              gen.grid_graph(5, 5), gen.path_graph(1), gen.cycle_graph(150)]
    s = 100
    offs, srcs, dsts, seeds, wants = [0], [], [], [], []
    for k, g in enumerate(graphs):
        sd = np.resize(gen.sample_seeds(g.n, min(s, g.n), 60 + k), s)
        wants.append(oracle.propagate(g.n, g.src, g.dst, sd, g.undirected, seed_counts=True, final_sig=True))
        src, dst = g.src.astype(np.int64), g.dst.astype(np.int64)
        if g.undirected:
            src, dst = np.concatenate([src, dst]), np.concatenate([dst, src])
        srcs.append(src + offs[-1])
        dsts.append(dst + offs[-1])
        seeds.append(sd + offs[-1])
        offs.append(offs[-1] + g.n)
    G = pp.pp_csr_build(offs[-1], np.concatenate(srcs).astype(np.int32), np.concatenate(dsts).astype(np.int32),
                        node_offsets=offs)
    for sched, persistent in ((pp.PP_SCHED_PULL, False), (pp.PP_SCHED_HEURISTIC, False), (pp.PP_SCHED_PULL, True)):
        say("short-list batch", sched, "persistent", persistent)
        r = pp.pp_seeds_init(G, np.concatenate(seeds), s=s,
                             opts=pp.options(scheduler=sched, seed_counts=True, max_rounds=600, persistent=persistent))
        counts, D = pp.pp_propagate_until_converged(r)
        sc = pp.pp_get_seed_counts(r, 600)
        sig = pp.pp_get_signatures(r)
        for k, w in enumerate(wants):
            assert int(D[k]) == w["D"], k
            assert list(counts[k][:w["D"] + 1]) == list(w["counts"]), k
            assert np.array_equal(sc[k][:w["D"] + 1], w["seed_counts"]), k
            assert np.array_equal(sig[offs[k]:offs[k + 1]], pad_words(w["final_sig"], r.words)), k
        r.free()


# ------------------------------------------------------------ nodes without successors

@pytest.mark.parametrize("form", ["plain", "persistent", "groups"])
def test_rows_of_nodes_without_successors(form):
    """A graph whose nodes mostly have no successor, with rows beyond the
    last-level cache (R-MAT scale 18 among 2^22 nodes, s = 512): the pull leaves
    such rows alone, relying on the initialisation having written them into
    both buffers.  Three seed sets on one run, the second after a reset, the
    third after a reset from a restored snapshot of the first: every count,
    per-seed count and signature against the oracle (a seed bit left over from
    an earlier seed set, or a row missing from one buffer, would show in c[0],
    the signatures or the per-seed counts)."""
    g = gen.rmat(18, 8, 11)
    n = 1 << 22
    rng = np.random.default_rng(40)
    sets = [rng.choice(n, 512, replace=False).astype(np.int32) for _ in range(3)]
    sets[2][:64] = sets[0][:64]   # some seeds again, most not
    wants = [oracle.propagate(n, g.src, g.dst, sd, False, seed_counts=True, final_sig=True) for sd in sets]
    G = pp.pp_csr_build(n, g.src, g.dst)
    cap = max(w["D"] for w in wants) + 4
    opts = pp.options(seed_counts=True, max_rounds=cap, persistent=form == "persistent",
                      seed_groups=pp.PP_GROUPS_BY_REACH if form == "groups" else 0)

    def check(r, want, k):
        counts, D = pp.pp_propagate_until_converged(r)
        assert int(D[0]) == want["D"], k
        assert list(counts[0]) == list(want["counts"]), k
        assert np.array_equal(pp.pp_get_seed_counts(r, want["D"] + 1)[0], want["seed_counts"]), k
        assert np.array_equal(pp.pp_get_signatures(r), pad_words(want["final_sig"], r.words)), k

    say("dead rows", form, "set 0")
    r = pp.pp_seeds_init(G, sets[0], opts=opts)
    check(r, wants[0], 0)
    snap = pp.pp_run_snapshot(r)
    say("dead rows", form, "set 1 after a reset")
    pp.pp_seeds_reset(r, sets[1])
    check(r, wants[1], 1)
    say("dead rows", form, "set 2 after a restore and a reset")
    pp.pp_run_restore(r, snap)
    pp.pp_seeds_reset(r, sets[2])
    check(r, wants[2], 2)
    snap.free()
    r.free()
    G.free()


# ------------------------------------------------------------ full size

def test_rmat26_full_size_sampled_seeds():
    """R-MAT scale 26, s = 512, in the benchmark's launch configurations: one group of
    eight-word rows, whose pushes run at their widest (one block per 2^17 arcs, 8192
    blocks), and seed groups by reach (two groups of four-word rows, the benchmark's
    headline form).

    Per-round totals come from the GPU only (the two forms must agree); the oracle
    checks 8 sampled seeds one by one (per-seed counts and the seeds' signature bit
    columns over all 2^26 nodes) in both forms, and the totals are checked against
    the per-seed counts' sums.
    """
    g, seeds = gen.workload_rmat(26, 16, 512, 1)
    say("rmat26 build", g.n)
    G = pp.pp_csr_build(g.n, g.src, g.dst)
    runs = {}
    for name, groups in (("one group", 0), ("groups by reach", pp.PP_GROUPS_BY_REACH)):
        r = pp.pp_seeds_init(G, seeds, opts=pp.options(seed_counts=True, max_rounds=256, seed_groups=groups))
        counts, D = pp.pp_propagate_until_converged(r)
        Dg = int(D[0])
        modes, _ = pp.pp_get_round_log(r, Dg + 2)
        say("rmat26", name, "groups", r.groups, "D", Dg, "modes", list(modes[1:Dg + 2]))
        ran = [int(m) for m in modes[1:Dg + 2]]
        assert (pp.MODE_PUSH in ran or pp.MODE_PUSH_FLAT in ran) and pp.MODE_PULL in ran
        assert r.groups == (1 if groups == 0 else 2)
        sc = pp.pp_get_seed_counts(r, Dg + 1)[0]
        assert np.array_equal(sc.sum(axis=1).astype(np.int64), counts[0])
        runs[name] = (counts[0].copy(), Dg, sc, pp.pp_get_signatures(r))
        r.free()
    G.free()
    (c1, D1, _, _), (c2, D2, _, _) = runs["one group"], runs["groups by reach"]
    assert D1 == D2 and list(c1) == list(c2)
    pick = np.unique(np.linspace(0, 511, 8).astype(np.int64))
    say("rmat26 oracle", list(pick))
    want = oracle.propagate(g.n, g.src, g.dst, seeds[pick], False, seed_counts=True, dist=True)
    for name, (counts, Dg, sc, sig) in runs.items():
        for j, i in enumerate(pick):
            col = want["seed_counts"][:, j]
            L = max(len(col), Dg + 1)
            assert np.array_equal(np.pad(sc[:, i], (0, L - Dg - 1)), np.pad(col, (0, L - len(col)))), (name, i)
            bits = (sig[:, i >> 6] >> np.uint64(i & 63)) & np.uint64(1)
            assert np.array_equal(bits.astype(bool), want["dist"][j] >= 0), (name, i)
    say("rmat26 ok", list(c1))


def test_autotune_candidates_keep_results():
    """Every autotuner candidate runs the same propagation; the tuned options reproduce it."""
    g = gen.rmat(13, 16, 21)
    seeds = gen.sample_seeds(g.n, 128, 4)
    say("autotune rmat13")
    want = oracle.propagate(g.n, g.src, g.dst, seeds, False, final_sig=True)
    G = pp.pp_csr_build(g.n, g.src, g.dst)
    best, table = pp.pp_autotune(G, seeds, reps=2)
    assert len(table) == 13
    assert {(t["pull_k"], t["push_div"]) for t in table if not t["persistent"] and not t["sparse_pull"]} == \
        {(k, d) for k in (2, 4) for d in (4, 8, 16, 32)}
    assert {(t["pull_k"], t["push_div"]) for t in table if t["sparse_pull"]} == {(4, d) for d in (4, 8, 16, 32)}
    assert sum(1 for t in table if t["persistent"]) == 1
    assert all(np.isfinite(t["ms"]) and t["ms"] > 0 for t in table)
    best_ms = min(t["ms"] for t in table)
    assert any(t["ms"] == best_ms and t["pull_k"] == best.pull_k and t["push_div"] == best.push_div
               and t["persistent"] == best.persistent and t["sparse_pull"] == best.sparse_pull for t in table)
    for k in (2, 4):
        for pers, sparse in (((False, 0), (True, 0), (False, 1)) if k == 4 else ((False, 0),)):
            opts = pp.options(pull_k=k, persistent=pers, push_div=best.push_div, max_rounds=want["D"] + 4,
                              sparse_pull=sparse)
            r = pp.pp_seeds_init(G, seeds, opts=opts)
            c, D = pp.pp_propagate_until_converged(r)
            assert int(D[0]) == want["D"] and list(c[0]) == list(want["counts"])
            assert np.array_equal(pp.pp_get_signatures(r), pad_words(want["final_sig"], r.words))
    with pytest.raises(pp.PPError):
        pp.pp_seeds_init(G, seeds, opts=pp.options(pull_k=3))
    with pytest.raises(pp.PPError):
        pp.pp_seeds_init(G, seeds, opts=pp.options(pull_k=2, persistent=True))


@pytest.mark.parametrize("case", range(4))
def test_exact_neighbourhood_function(case):
    """Every node a seed, in groups: the counts equal all-pairs distances (brute force)."""
    g = [gen.erdos_renyi_gnm(300, 700, 2), gen.grid_with_shortcuts(20, 15, gen.Fraction(1, 10), 5, 1),
         gen.rmat(9, 8, 4), gen.path_graph(130)][case]
    group = [64, 100, 512, 7][case]
    say("exact", g.name, "group", group)
    want, dist = oracle.brute_force_counts(g.n, g.src, g.dst, np.arange(g.n), g.undirected)
    G = pp.pp_csr_build(g.n, g.src, g.dst, undirected=g.undirected)
    counts, D = pp.pp_exact_counts(G, group=group)
    assert D == len(want) - 1 and list(counts) == list(want)
    m = pp.pp_estimate_metrics(counts, g.n, g.n)
    assert m["reachable_pairs"] == float(int((dist >= 0).sum()))
    with pytest.raises(pp.PPError):
        pp.pp_exact_counts(G, group=513)


# ------------------------------------------------------------ PROPAGATE-S

S_CASES = [("er", lambda: gen.erdos_renyi_gnm(400, 1200, 5), 64),
           ("rmat", lambda: gen.rmat(12, 8, 6), 100),
           ("grid", lambda: gen.grid_with_shortcuts(40, 30, gen.Fraction(1, 10), 20, 2), 77),
           ("path", lambda: gen.path_graph(300), 5),
           ("dpath", lambda: gen.path_graph(120, directed=True), 9),
           ("star", lambda: gen.star_graph(2000), 33)]


@pytest.mark.parametrize("case", range(len(S_CASES)))
@pytest.mark.parametrize("concurrent", [0, 1, 7])
@pytest.mark.parametrize("keep_order", [False, True])
def test_propagate_s_counts(case, concurrent, keep_order):
    """Algorithm 2 on the device: the same per-round counts and D as the BFS oracle, for every
    number of seeds in flight (batches with a ragged last one) and both storage orders."""
    name, make, s = S_CASES[case]
    g = make()
    seeds = gen.sample_seeds(g.n, s, 13 + case)
    seeds[1] = seeds[0]   # a duplicate seed counts twice
    say("propagate_s", name, "n", g.n, "s", s, "concurrent", concurrent, "keep_order", keep_order)
    want = oracle.propagate(g.n, g.src, g.dst, seeds, g.undirected)
    G = pp.pp_csr_build(g.n, g.src, g.dst, undirected=g.undirected, keep_order=keep_order)
    counts, D, examined = pp.pp_propagate_s(G, seeds, concurrent=concurrent)
    assert D == want["D"] and list(counts) == list(want["counts"])
    assert 0 < examined <= (D + 1) * s * G.arcs


@pytest.mark.parametrize("case", range(4))
def test_propagate_s_literal_algorithm(case):
    """Small graphs against the literal Algorithm 2 oracle, early-break work included: with the
    stored order kept, every node walks the same sorted list and stops at the same arc."""
    rng = np.random.default_rng(40 + case)
    n = [40, 60, 25, 50][case]
    src = rng.integers(0, n, 3 * n).astype(np.int32)
    dst = rng.integers(0, n, 3 * n).astype(np.int32)
    undirected, transpose = [(False, False), (True, False), (False, True), (True, True)][case]
    seeds = rng.integers(0, n, 6).astype(np.int32)
    say("propagate_s literal", case)
    want, Dw, ex = oracle.propagate_s.propagate_s(n, src, dst, seeds, undirected, transpose, stored=True)
    G = pp.pp_csr_build(n, src, dst, undirected=undirected, transpose=transpose, keep_order=True)
    for conc in (0, 2):
        counts, D, examined = pp.pp_propagate_s(G, seeds, concurrent=conc)
        assert D == Dw and list(counts) == list(want) and examined == ex


def test_propagate_s_long_lists_and_errors():
    """Nodes with more successors than one lane walks (the wave-per-node launch), the log's
    end, bad seeds and batches."""
    hub = gen.star_graph(5000)   # undirected: the centre's list is 4999 long
    seeds = np.array([3, 0, 4998, 17], np.int32)
    want = oracle.propagate(hub.n, hub.src, hub.dst, seeds, hub.undirected)
    G = pp.pp_csr_build(hub.n, hub.src, hub.dst, undirected=True)
    counts, D, _ = pp.pp_propagate_s(G, seeds)
    assert D == want["D"] and list(counts) == list(want["counts"])
    # the early break inside a long list: the centre stops at the arc to the seed
    # leaf (arc x of its sorted list), exactly as the literal algorithm does;
    # hits at several offsets within a step of the wave-wide walk
    GK = pp.pp_csr_build(hub.n, hub.src, hub.dst, undirected=True, keep_order=True)
    for x in (1, 16, 17, 63, 64, 65, 300, 4999):
        one = np.array([x], np.int32)
        wc, wD, wex = oracle.propagate_s.propagate_s(hub.n, hub.src, hub.dst, one, True, stored=True)
        counts, D, examined = pp.pp_propagate_s(GK, one)
        assert D == wD and list(counts) == list(wc) and examined == wex == x + 2 * 4998, x
    P = gen.path_graph(64)
    GP = pp.pp_csr_build(P.n, P.src, P.dst, undirected=True)
    with pytest.raises(pp.PPError) as e:
        pp.pp_propagate_s(GP, np.array([0], np.int32), cap_rounds=10)
    assert e.value.code == pp.PP_ENOTCONV
    with pytest.raises(pp.PPError) as e:
        pp.pp_propagate_s(GP, np.array([64], np.int32))
    assert e.value.code == pp.PP_ERANGE
    B = pp.pp_csr_build(4, np.array([0, 2], np.int32), np.array([1, 3], np.int32), node_offsets=[0, 2, 4])
    with pytest.raises(pp.PPError) as e:
        pp.pp_propagate_s(B, np.array([0], np.int32))
    assert e.value.code == pp.PP_EINVAL


# ------------------------------------------------------------ per-node statistics

NS_CASES = [("er", lambda: gen.erdos_renyi_gnm(500, 1500, 8), 70),
            ("rmat", lambda: gen.rmat(11, 8, 3), 130),
            ("grid", lambda: gen.grid_with_shortcuts(25, 20, gen.Fraction(1, 10), 8, 6), 64),
            ("dpath", lambda: gen.path_graph(90, directed=True), 10)]


@pytest.mark.parametrize("case", range(len(NS_CASES)))
@pytest.mark.parametrize("sched", SCHEDS)
@pytest.mark.parametrize("keep_order", [False, True])
def test_node_stats(case, sched, keep_order):
    """Per-node reach counts and distance sums after convergence and after each of the
    first rounds, against the oracle's BFS distances, for every direction policy."""
    import oracle.node_stats as ons
    name, make, s = NS_CASES[case]
    g = make()
    seeds = gen.sample_seeds(g.n, s, 21 + case)
    seeds[2] = seeds[1]
    say("node_stats", name, "sched", sched, "keep_order", keep_order)
    want = oracle.propagate(g.n, g.src, g.dst, seeds, g.undirected)
    G = pp.pp_csr_build(g.n, g.src, g.dst, undirected=g.undirected, keep_order=keep_order)
    r = pp.pp_seeds_init(G, seeds, opts=pp.options(scheduler=sched, fuzz_seed=case, node_stats=True,
                                                    max_rounds=want["D"] + 4))
    for k in range(0, 4):
        if k:
            pp.pp_propagate_round(r)
        wr, wd = ons.node_stats(g.n, g.src, g.dst, seeds, g.undirected, rounds=k)
        gr, gd = pp.pp_get_node_stats(r)
        assert np.array_equal(gr, wr) and np.array_equal(gd, wd), k
    pp.pp_propagate_until_converged(r)
    wr, wd = ons.node_stats(g.n, g.src, g.dst, seeds, g.undirected)
    gr, gd = pp.pp_get_node_stats(r)
    assert np.array_equal(gr, wr) and np.array_equal(gd, wd)
    # a reset starts the sums again; extra no-op replays after convergence add nothing
    pp.pp_seeds_reset(r, seeds)
    pp.pp_propagate_until_converged(r)
    pp.pp_propagate_round(r)
    gr, gd = pp.pp_get_node_stats(r)
    assert np.array_equal(gr, wr) and np.array_equal(gd, wd)


@pytest.mark.parametrize("sched", [pp.PP_SCHED_FUZZ, pp.PP_SCHED_HEURISTIC])
def test_node_stats_batched_union(sched):
    """Per-node sums on a batch of graphs that converge at different rounds, each
    graph's slice against the oracle's BFS distances of that graph alone."""
    import oracle.node_stats as ons
    graphs = [gen.path_graph(120), gen.rmat(10, 8, 4), gen.grid_graph(9, 7), gen.cycle_graph(31, directed=True)]
    s = 16
    offs, srcs, dsts, seeds, wants = [0], [], [], [], []
    for k, g in enumerate(graphs):
        sd = gen.sample_seeds(g.n, s, 40 + k)
        wants.append(ons.node_stats(g.n, g.src, g.dst, sd, g.undirected))
        src, dst = g.src.astype(np.int64), g.dst.astype(np.int64)
        if g.undirected:
            src, dst = np.concatenate([src, dst]), np.concatenate([dst, src])
        srcs.append(src + offs[-1])
        dsts.append(dst + offs[-1])
        seeds.append(sd + offs[-1])
        offs.append(offs[-1] + g.n)
    say("node_stats batch", sched)
    G = pp.pp_csr_build(offs[-1], np.concatenate(srcs).astype(np.int32), np.concatenate(dsts).astype(np.int32),
                        node_offsets=offs)
    r = pp.pp_seeds_init(G, np.concatenate(seeds).astype(np.int32), s=s,
                         opts=pp.options(scheduler=sched, fuzz_seed=7, node_stats=True, max_rounds=300))
    pp.pp_propagate_until_converged(r)
    gr, gd = pp.pp_get_node_stats(r)
    for k, (wr, wd) in enumerate(wants):
        assert np.array_equal(gr[offs[k]:offs[k + 1]], wr), k
        assert np.array_equal(gd[offs[k]:offs[k + 1]], wd), k


def test_node_stats_errors():
    g = gen.path_graph(20)
    G = pp.pp_csr_build(g.n, g.src, g.dst, undirected=True)
    r = pp.pp_seeds_init(G, np.array([0, 5], np.int32))
    with pytest.raises(pp.PPError) as e:
        pp.pp_get_node_stats(r)
    assert e.value.code == pp.PP_ESTATE
    with pytest.raises(pp.PPError) as e:
        pp.pp_seeds_init(G, np.array([0, 5], np.int32), opts=pp.options(node_stats=True, persistent=True))
    assert e.value.code == pp.PP_EINVAL


# ------------------------------------------------------------ progressive sampling

@pytest.mark.parametrize("case", range(4))
def test_progressive_sample(case):
    """Seed groups until the Hoeffding half-width meets the target: the same groups, the
    same summed counts and the same float64 figures as the oracle (exact integers, one
    rounding each, the same libm), including a run whose pool runs out."""
    import oracle.progressive as prog
    g, group, target, delta = [(gen.erdos_renyi_gnm(2000, 6000, 3), 64, 0.5, 0.05),
                               (gen.rmat(12, 8, 9), 100, 1.2, 0.1),
                               (gen.cycle_graph(301), 17, 25.0, 0.05),
                               (gen.grid_with_shortcuts(30, 30, gen.Fraction(1, 10), 10, 4), 32, 0.01, 0.05)][case]
    rng = np.random.default_rng(70 + case)
    pool = rng.integers(0, g.n, 600).astype(np.int32)
    say("progressive", g.name, "group", group, "target", target)
    want = prog.progressive(g.n, g.src, g.dst, pool, group, target, delta, g.undirected)
    G = pp.pp_csr_build(g.n, g.src, g.dst, undirected=g.undirected)
    got = pp.pp_progressive_sample(G, pool, group, target, delta)
    assert list(got["counts"]) == list(want["counts"])
    for k in ("seeds", "groups", "met", "D", "alpha", "eps", "bound"):
        assert got[k] == want[k], k
    assert got["met"] == (case != 3) and got["groups"] > 1


def test_grid4096_full_size():
    """The 4096^2 grid with deletions and shortcuts, s = 128, at full size: per-round
    counts, per-seed counts, D and every signature against the oracle (all 128 BFS
    on the host), with the heuristic, a pseudo-random schedule and the learned
    scheduler (a threshold model at another threshold than the heuristic's, and
    random weights); sparse rounds as pushes, as sparse pulls, or either."""
    from test_gpu_scheduler import rand_params, threshold_params
    g, seeds = gen.workload_grid_shortcuts(4096, 128, 1)
    say("grid4096 oracle", g.n)
    want = oracle.propagate(g.n, g.src, g.dst, seeds, True, final_sig=True, seed_counts=True)
    G = pp.pp_csr_build(g.n, g.src, g.dst, undirected=True)
    cases = [(pp.PP_SCHED_HEURISTIC, 0, None), (pp.PP_SCHED_FUZZ, 0, None), (pp.PP_SCHED_HEURISTIC, 1, None),
             (pp.PP_SCHED_FUZZ, 2, None), (pp.PP_SCHED_MLP, 0, threshold_params(1.0 / 12.0)),
             (pp.PP_SCHED_MLP, 2, rand_params(17, 0.3))]
    for sched, sparse, params in cases:
        say("grid4096 run", sched, "sparse_pull", sparse, "model", params is not None)
        r = pp.pp_seeds_init(G, seeds, opts=pp.options(scheduler=sched, fuzz_seed=3, max_rounds=want["D"] + 4,
                                                        sparse_pull=sparse, seed_counts=True))
        if params is not None:
            pp.pp_run_set_mlp(r, params)
        counts, D = pp.pp_propagate_until_converged(r)
        assert int(D[0]) == want["D"] and list(counts[0]) == list(want["counts"])
        assert np.array_equal(pp.pp_get_seed_counts(r, want["D"] + 1)[0], want["seed_counts"])
        assert np.array_equal(pp.pp_get_signatures(r), pad_words(want["final_sig"], r.words))
        if params is not None:
            modes, _ = pp.pp_get_round_log(r, want["D"] + 2)
            ran = [int(m) for m in modes[1:want["D"] + 2]]
            say("grid4096 learned: pulls", ran.count(pp.MODE_PULL), "of", len(ran))
            if sparse == 0:   # the threshold model mixes both directions on this graph
                assert pp.MODE_PULL in ran and pp.MODE_PUSH in ran
        r.free()


# ------------------------------------------------------------ sparse pull

SPARSE_SCHEDS = [pp.PP_SCHED_PUSH, pp.PP_SCHED_HEURISTIC, pp.PP_SCHED_FUZZ]


@pytest.mark.parametrize("gi", range(len(CLOSED)))
@pytest.mark.parametrize("sched", SPARSE_SCHEDS)
@pytest.mark.parametrize("sparse", [1, 2])
def test_sparse_pull_closed_forms(gi, sched, sparse):
    """Sparse rounds as sparse pulls (1) or mixed with pushes (2): the star and the
    complete graph take the long-list path, the lattices and paths the gather."""
    g = CLOSED[gi]
    s = min(g.n, 512)
    seeds = gen.sample_seeds(g.n, s, 3 + gi)
    say("sparse closed", g.name, "s", s, "sched", sched, "sparse_pull", sparse)
    r, _, counts = check_run(g.n, g.src, g.dst, seeds, g.undirected, sched=sched, fuzz_seed=gi,
                             sparse_pull=sparse)
    modes, _ = pp.pp_get_round_log(r, len(counts) + 1)
    if sched == pp.PP_SCHED_PUSH and sparse == 1:
        assert all(int(m) == pp.MODE_SPULL for m in modes[1:len(counts) + 1])


@pytest.mark.parametrize("trial", range(16))
def test_sparse_pull_random_graphs(trial):
    """Random multigraphs at every signature width, sparse rounds as sparse pulls."""
    rng = np.random.default_rng(900 + trial)
    s = [1, 64, 65, 128, 200, 256, 300, 512][trial % 8]
    n = int(rng.integers(max(2, s // 4), 3000))
    m = int(rng.integers(0, 8 * n))
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    und = bool(trial % 3 == 0)
    tr = bool(trial % 4 == 1)
    seeds = rng.integers(0, n, s).astype(np.int32)
    sched = SPARSE_SCHEDS[trial % 3]
    sparse = 1 + trial % 2
    say("sparse random", trial, "n", n, "m", m, "s", s, "sched", sched, "sparse_pull", sparse)
    check_run(n, src, dst, seeds, und, transpose=tr, sched=sched, fuzz_seed=trial, sparse_pull=sparse,
              pull_k=2 if trial % 5 == 0 else 0)


@pytest.mark.parametrize("sched", SPARSE_SCHEDS)
@pytest.mark.parametrize("keep_order", [False, True])
def test_sparse_pull_rmat_with_hubs(sched, keep_order):
    """R-MAT scale 14 (lists far longer than the gather limit), sparse pulls."""
    g = gen.rmat(14, 16, 77)
    seeds = gen.sample_seeds(g.n, 256, 8)
    say("sparse rmat14", sched, "keep_order", keep_order)
    check_run(g.n, g.src, g.dst, seeds, False, sched=sched, fuzz_seed=5, keep_order=keep_order, sparse_pull=1)


@pytest.mark.parametrize("sparse", [1, 2])
def test_sparse_pull_round_by_round(sparse):
    """The ER workload one round at a time: the signatures after every round."""
    g, seeds = gen.workload_er(1)
    want = oracle.propagate(g.n, g.src, g.dst, seeds, True, sig_rounds=list(range(0, 16)),
                            seed_counts=True, final_sig=True)
    say("sparse er rounds", sparse, "D", want["D"])
    G = pp.pp_csr_build(g.n, g.src, g.dst, undirected=True)
    r = pp.pp_seeds_init(G, seeds, opts=pp.options(scheduler=pp.PP_SCHED_FUZZ, seed_counts=True, max_rounds=64,
                                                    fuzz_seed=9, sparse_pull=sparse))
    got = [len(seeds)]
    for k in range(1, want["D"] + 2):
        nb, conv = pp.pp_propagate_round(r)
        got.append(int(nb[0]))
        assert np.array_equal(pp.pp_get_signatures(r), want["sigs"][min(k, 15)]), k
        assert conv == (k == want["D"] + 1)
    assert got[:-1] == list(want["counts"]) and got[-1] == 0
    modes, arcs = pp.pp_get_round_log(r, want["D"] + 2)
    assert set(int(m) for m in modes[1:want["D"] + 2]) <= {pp.MODE_PULL, pp.MODE_PUSH, pp.MODE_SPULL}
    if sparse == 1:
        assert pp.MODE_PUSH not in [int(m) for m in modes[1:want["D"] + 2]]


@pytest.mark.parametrize("case", range(len(NS_CASES)))
def test_sparse_pull_node_stats(case):
    """Per-node sums with sparse pulls, against the oracle's BFS distances."""
    import oracle.node_stats as ons
    name, make, s = NS_CASES[case]
    g = make()
    seeds = gen.sample_seeds(g.n, s, 21 + case)
    say("sparse node_stats", name)
    G = pp.pp_csr_build(g.n, g.src, g.dst, undirected=g.undirected)
    r = pp.pp_seeds_init(G, seeds, opts=pp.options(scheduler=pp.PP_SCHED_PUSH, node_stats=True, sparse_pull=1,
                                                    max_rounds=g.n + 2))
    pp.pp_propagate_until_converged(r)
    wr, wd = ons.node_stats(g.n, g.src, g.dst, seeds, g.undirected)
    gr, gd = pp.pp_get_node_stats(r)
    assert np.array_equal(gr, wr) and np.array_equal(gd, wd)


def test_sparse_pull_forced_rounds_snapshot_and_errors():
    """pp_time_round in each direction, from snapshots: the same bits every way; the
    mode log records the sparse pulls; bad options are rejected."""
    g, seeds = gen.workload_er(2)
    want = oracle.propagate(g.n, g.src, g.dst, seeds, True, final_sig=True)
    G = pp.pp_csr_build(g.n, g.src, g.dst, undirected=True)
    r = pp.pp_seeds_init(G, seeds, opts=pp.options(max_rounds=64, sparse_pull=1))
    pp.pp_propagate_round(r)
    snap = pp.pp_run_snapshot(r)
    results = []
    for mode in (pp.MODE_PULL, pp.MODE_PUSH, pp.MODE_SPULL):
        pp.pp_run_restore(r, snap)
        pp.pp_time_round(r, mode)
        modes, _ = pp.pp_get_round_log(r, 4)
        assert int(modes[2]) == (pp.MODE_PULL if mode == pp.MODE_PULL else pp.MODE_SPULL), mode
        c, _ = pp.pp_propagate_until_converged(r)
        results.append((list(c[0]), pp.pp_get_signatures(r)))
    for c, sig in results:
        assert c == list(want["counts"])
        assert np.array_equal(sig, pad_words(want["final_sig"], sig.shape[1]))
    # a push run forced into a sparse pull, and back
    r2 = pp.pp_seeds_init(G, seeds, opts=pp.options(max_rounds=64))
    pp.pp_propagate_round(r2)
    pp.pp_time_round(r2, pp.MODE_SPULL)
    pp.pp_time_round(r2, pp.MODE_PUSH)
    modes, _ = pp.pp_get_round_log(r2, 4)
    assert [int(m) for m in modes[2:4]] == [pp.MODE_SPULL, pp.MODE_PUSH]
    c, _ = pp.pp_propagate_until_converged(r2)
    assert list(c[0]) == list(want["counts"])
    for bad in (dict(sparse_pull=3), dict(sparse_pull=-1), dict(sparse_pull=1, persistent=True)):
        with pytest.raises(pp.PPError) as e:
            pp.pp_seeds_init(G, seeds, opts=pp.options(**bad))
        assert e.value.code == pp.PP_EINVAL, bad
    with pytest.raises(pp.PPError) as e:
        pp.pp_time_round(r2, 2)
    assert e.value.code == pp.PP_EINVAL
