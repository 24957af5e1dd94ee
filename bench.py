#!/usr/bin/env python
"""Throughput of the PROPAGATE-P hot path on one MI355X.

One step = Algorithm 1 end to end on one batch of synthetic input: the seed
initialisation (pp_seeds_reset) and the synchronous rounds until the first
round with no new bit (pp_propagate_until_converged), with the per-round
counts copied to the host.  The graph is built once, before timing (the
paper does not time graph loading either); the seed list is already in HBM.

Metric: edge-words OR'd per second, full-scan accounting: every executed
round (D + 1 of them) is credited with m arcs x s/64 words, as Algorithm 1
scans every arc every round.  The edge-words the kernels actually touched
(push rounds touch only the frontier's arcs) are reported beside it.

Prints one JSON line.  `roofline` covers the dense pull kernel (HIP events
around each launch, on the run's stream, over the timed steps);
`cpu_baseline` times the CPU oracle (one BFS per seed, all host cores) on
the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, published
METRIC = "edge-words OR'd/sec (edges x s/64 per round) and achieved HBM GB/s vs peak, bit-exact"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name: str):
    from paper_2301_06499_amd import inputs
    if name == "rmat20":
        g, seeds = inputs.workload_rmat(20, 16, 256, 1)
        return g, seeds, {"workload": "rmat_scale20_ef16_s256", "generator": "R-MAT a,b,c,d=.57,.19,.19,.05, "
                          "self-loops and duplicates removed, all 2^20 nodes kept", "seeds": 256}
    if name == "rmat26":
        g, seeds = inputs.workload_rmat(26, 16, 512, 1)
        return g, seeds, {"workload": "rmat_scale26_ef16_s512", "generator": "R-MAT a,b,c,d=.57,.19,.19,.05, "
                          "self-loops and duplicates removed, all 2^26 nodes kept", "seeds": 512}
    if name.startswith("rmat:"):   # rmat:SCALE:SEEDS, edge factor 16
        scale, s = (int(x) for x in name.split(":")[1:3])
        g, seeds = inputs.workload_rmat(scale, 16, s, 1)
        return g, seeds, {"workload": f"rmat_scale{scale}_ef16_s{s}", "seeds": s}
    if name.startswith("grid:"):   # grid:SIDE, the lattice workload without the cost-model training
        side = int(name.split(":")[1])
        g, seeds = inputs.workload_grid_shortcuts(side, 128, 1)
        return g, seeds, {"workload": f"grid{side}x{side}_del10pct_sc1000_lcc_s128", "seeds": 128}
    if name == "er":
        g, seeds = inputs.workload_er(1)
        return g, seeds, {"workload": "er_n10000_m50000_lcc_s64", "seeds": 64}
    raise SystemExit(f"unknown workload {name}")


# workloads whose dense pull launches have counter figures under profiles/ (one seed
# group, and seed groups by reach)
TRAFFIC_PROFILES = {("rmat20", False): ["k_pull_rmat20_s256"], ("rmat20", True): ["k_pull_rmat20_s256_groups"],
                    ("rmat26", False): ["k_pull_rmat26_s512"], ("rmat26", True): ["k_pull_rmat26_s512_groups"],
                    ("grid:4096", False): ["k_pull_short_grid4096_s128"], ("grid:4096", True): ["k_pull_short_grid4096_s128"]}


PULL_NPL = 6   # successors per node up to which the pull gathers one node per lane


def pull_kernel(W: int, pull_k: int, form: str = "") -> str:
    """The dense pull kernel's name for rows of W words and pull_k arcs per lane;
    form (pull_form): "short" (the short-list form, for rows of one or two
    words) or "dead" (rows of nodes without successors left alone), both at
    the default pull_k."""
    if pull_k == 2:
        return f"k_pull<{W}, 2, false>"
    if form == "short" and W <= 2:
        return f"k_pull_short<{W}>"
    return f"k_pull<{W}, 0, {'true' if form == 'dead' else 'false'}>"


def pull_form(pp, G, W: int) -> str:
    """The form of the pull the library launches on G for rows of W words, by the
    library's own rule: "short" when no stored node has more than PULL_NPL
    successors (rows of one or two words), "dead" when a quarter of the nodes
    or more have none and the two row buffers exceed 256 MiB, else ""."""
    rp = np.zeros(G.nodes + 1, np.int64)
    pp._check(pp.lib().pp_graph_get_csr(G.handle, pp._np_ptr(rp), None, None, None, None))
    deg = np.diff(rp)
    if W <= 2 and (G.nodes == 0 or int(deg.max()) <= PULL_NPL):
        return "short"
    if int((deg == 0).sum()) * 4 >= G.nodes and 16.0 * W * G.nodes > 256.0 * 1048576.0:
        return "dead"
    return ""


def traffic_for(profiles, kernel: str):
    """The first of the workload's counter summaries that covers this kernel, if any."""
    for p in profiles:
        t = measured_traffic(p, kernel)
        if t is not None:
            return t
    return None


def measured_traffic(profile: str, kernel: str):
    """HBM bytes per launch from the committed counter summary, if the kernel is unchanged.

    profiles/<profile>_traffic.json holds FETCH_SIZE + WRITE_SIZE per launch
    (scaled by a copy of known size), the kernel it covers and the hash of the
    kernel sources the counters were taken on; another kernel or hash means the
    figure does not apply.
    """
    import hashlib
    path = os.path.join(ROOT, "profiles", profile + "_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel") != kernel:
        return None
    csrc = os.path.join(ROOT, "paper_2301_06499_amd", "csrc")
    src = b"".join(open(os.path.join(csrc, f), "rb").read() for f in ("pp_kernels.hip", "pp_internal.h"))
    if hashlib.sha256(src).hexdigest() != rec.get("source_sha256"):
        return None
    return int(rec["fetch_bytes_per_launch"]) + int(rec["write_bytes_per_launch"])


def bench_batch(args, torch, pp):
    """The 64-graph batch (R-MAT, grids, paths; 64 seeds each) in one launch vs plain runs.

    Batched: the disjoint union, every graph run by its own cluster of
    co-resident blocks in one cooperative launch (each graph converges on its
    own).  Plain: each graph alone, per-round launches, fixed-threshold
    heuristic.  Both give the same per-graph counts (checked here).
    """
    from paper_2301_06499_amd import inputs
    t0 = time.perf_counter()
    graphs, seeds = inputs.workload_batch(1, 64)
    n, usrc, udst, offs, allseeds = inputs.union_of(graphs, seeds)
    log(f"[bench] generated the batch in {time.perf_counter() - t0:.1f} s: {len(graphs)} graphs, n={n}")
    stream = torch.cuda.Stream()
    GB = pp.pp_csr_build(n, usrc, udst, node_offsets=offs, stream=stream)
    torch.cuda.synchronize()
    calibration_copy(args, torch)
    dseeds = torch.from_numpy(allseeds).to("cuda")
    engines = {}
    chosen = [e for e in (("clustered", True), ("union", False)) if e[0] in args.batch_engines.split(",")]
    if not chosen:
        raise SystemExit("--batch-engines names neither clustered nor union")
    for name, persistent in chosen:
        run = pp.pp_seeds_init(GB, allseeds, s=64, opts=pp.options(max_rounds=25000, persistent=persistent),
                               stream=stream)

        def step():
            pp.pp_seeds_reset(run, dseeds)
            return pp.pp_propagate_until_converged(run)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            counts, D = step()
        torch.cuda.synchronize()
        engines[name] = ((time.perf_counter() - t0) / args.steps, counts, D)
        if args.round_log and not persistent:
            rounds = int(D.max()) + 2
            write_round_log(args.round_log, pp, run, GB, counts.sum(axis=0), int(D.max()),
                            [pp.pp_get_group_log(run, 0, rounds + 1)])
        run.free()
        log(f"[bench] batch, {name} engine: {engines[name][0] * 1e3:.2f} ms per step")
    if len(engines) == 2:
        assert np.array_equal(engines["union"][1], engines["clustered"][1])
    best = min(engines, key=lambda k: engines[k][0])
    t_batch, counts, D = engines[best]
    if args.no_plain:   # the batched engines only (for profiling them)
        print(json.dumps({"engines_ms_per_step": {k: round(v[0] * 1000.0, 3) for k, v in engines.items()},
                          "note": "batched engines only (--no-plain)"}), flush=True)
        GB.free()
        return
    # stored arcs per graph, from solo builds (also used by the plain runs)
    solo_graphs, solo_runs, arcs_g = [], [], []
    for g, sd in zip(graphs, seeds):
        Gs = pp.pp_csr_build(g.n, g.src, g.dst, undirected=g.undirected, stream=stream)
        solo_graphs.append(Gs)
        arcs_g.append(Gs.arcs)
        solo_runs.append(pp.pp_seeds_init(Gs, sd, opts=pp.options(max_rounds=25000), stream=stream))
    nominal = float(sum(arcs_g[k] * (int(D[k]) + 1) for k in range(len(graphs))))   # W = 1
    plain_steps = max(1, min(args.steps, 2))
    plain_counts = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(plain_steps):
        plain_counts = []
        for r_, sd in zip(solo_runs, seeds):
            pp.pp_seeds_reset(r_, sd)
            c, _ = pp.pp_propagate_until_converged(r_)
            plain_counts.append(c[0])
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / plain_steps
    for k, c in enumerate(plain_counts):
        assert list(c) == list(counts[k][:int(D[k]) + 1]), f"graph {k}: batched and plain counts differ"
    out = {
        "metric": METRIC,
        "value": nominal / t_batch,
        "unit": "edge-words/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(t_batch * 1000.0, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": "batch64: 22 R-MAT (scale 10-16, edge factor 8-16), 21 grids (64^2..512^2), "
                               "21 paths (1000..20000 edges), 64 seeds each",
                   "graphs": len(graphs), "nodes": n, "arcs": int(GB.arcs), "words": 1,
                   "max_rounds": int(D.max()) + 1,
                   "engine": {"clustered": "one persistent launch, each graph on its own block range",
                              "union": "per-round launches over the disjoint union, graph replay"}[best]},
        "engines_ms_per_step": {k: round(v[0] * 1000.0, 3) for k, v in engines.items()},
        "plain": {"ms_per_step": round(t_plain * 1000.0, 3), "value": nominal / t_plain,
                  "engine": "64 solo runs, per-round launches, fixed-threshold heuristic"},
        "speedup_vs_plain": round(t_plain / t_batch, 2),
        "roofline": None,
    }
    print(json.dumps(out), flush=True)
    # every handle goes back before the process ends, not at interpreter teardown
    for r_ in solo_runs:
        r_.free()
    for g_ in solo_graphs:
        g_.free()
    GB.free()
    torch.cuda.synchronize()


def bench_grid(args, torch, pp):
    """Large-diameter grid with the learned direction scheduler vs the fixed heuristic.

    The cost model is trained on this method's own round timings: every round
    of two training graphs (same family, other generator seeds) is priced under
    every action after both kinds of previous round by replaying fixed plans on
    the ordinary path, the best schedule of each is solved exactly, and the
    model is fitted to the resulting per-round action costs by the library's
    device training kernels.  The held-out graph (generator seed 1) is then run
    to convergence with the heuristic, the model, the heuristic at its
    autotuned threshold and the optimal plan of its own measured costs; all
    give the same counts (checked here).
    """
    from paper_2301_06499_amd import inputs
    from paper_2301_06499_amd import scheduler as S
    side = args.grid_side
    tables = []
    t_prep = time.perf_counter()
    for gs in (2, 3):
        g, sd = inputs.workload_grid_shortcuts(side, 128, gs)
        Gt = pp.pp_csr_build(g.n, g.src, g.dst, undirected=True)
        tables.append(S.measure_replay(Gt, sd, repeats=2))
        Gt.free()
        log(f"[bench] priced {len(tables[-1])} rounds of training graph {gs} under every action")
    samples = S.Samples.concat(S.label(t) for t in tables)
    t0 = time.perf_counter()
    params, losses = S.train(samples, steps=4000)
    t_train = time.perf_counter() - t0
    log(f"[bench] trained on {len(samples)} samples in {t_train:.2f} s, loss {losses[0]:.3f} -> {losses[-1]:.5f}")
    g, seeds = inputs.workload_grid_shortcuts(side, 128, 1)
    G = pp.pp_csr_build(g.n, g.src, g.dst, undirected=True)
    held = S.measure_replay(G, seeds, repeats=2)
    _, best_ms, best_plan = S.optimal_schedule(held)
    t_prep = time.perf_counter() - t_prep
    reps = max(1, args.steps)
    runs = {}
    for name, sch, params_ in (("heuristic", pp.PP_SCHED_HEURISTIC, None), ("learned", pp.PP_SCHED_MLP, params),
                               ("pull_only", pp.PP_SCHED_PULL, None), ("push_only", pp.PP_SCHED_PUSH, None)):
        S.timed_run(G, seeds, sch, params_, repeats=max(1, args.warmup))
        runs[name] = S.timed_run(G, seeds, sch, params_, repeats=reps)
        log(f"[bench] {name}: {runs[name][0]:.3f} ms")
    # the fixed threshold at its best for this graph (autotuned push threshold and tile)
    tuned, tuned_table = pp.pp_autotune(G, seeds, reps=2)
    runs["heuristic_tuned"] = S.timed_run(G, seeds, pp.PP_SCHED_HEURISTIC, None, repeats=reps,
                                          push_div=int(tuned.push_div), pull_k=int(tuned.pull_k))
    log(f"[bench] heuristic with the tuned threshold {tuned.push_div}: {runs['heuristic_tuned'][0]:.3f} ms")
    t_opt, c_opt, D_opt = S.replay_plan(G, seeds, best_plan, repeats=reps)
    runs["optimal_plan"] = (t_opt, c_opt, D_opt, None)
    log(f"[bench] the held-out table's optimal plan replayed: {t_opt:.3f} ms")
    (t_h, c_h, D_h, m_h), (t_l, c_l, D_l, m_l) = runs["heuristic"], runs["learned"]
    for name, (_, c_x, D_x, _) in runs.items():
        assert int(D_x[0]) == int(D_l[0]) and list(c_x[0]) == list(c_l[0]), f"{name} changed the counts"
    rounds = int(D_l[0]) + 1
    W = 2
    nominal = float(G.arcs) * W * rounds
    out = {
        "metric": METRIC,
        "value": nominal / (t_l / 1000.0),
        "unit": "edge-words/s",
        "n_gpus": 1, "steps": reps, "warmup": args.warmup,
        "ms_per_step": round(t_l, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"grid{side}x{side}_del10pct_sc1000_lcc_s128", "nodes": G.nodes, "arcs": G.arcs,
                   "words": W, "rounds": rounds, "scheduler": "learned (MLP 8-32-32-4: dense pull, push over direct slots, push over "
                                "flattened ranges, sparse pull), heuristic fallback",
                   "timing": "best of steps, whole propagation with graph replay, host clock around "
                             "synchronous library calls"},
        "heuristic": {"ms_per_step": round(t_h, 4), "value": nominal / (t_h / 1000.0),
                      "pulls": int((m_h[1:rounds + 1] == pp.MODE_PULL).sum())},
        "learned": {"pulls": int((m_l[1:rounds + 1] == pp.MODE_PULL).sum()),
                    "training_samples": len(samples), "train_s": round(t_train, 3),
                    "final_loss": float(losses[-1])},
        "speedup_vs_heuristic": round(t_h / t_l, 4),
        "pull_only_ms": round(runs["pull_only"][0], 4),
        "push_only_ms": round(runs["push_only"][0], 4),
        "heuristic_tuned": {"ms_per_step": round(runs["heuristic_tuned"][0], 4), "push_div": int(tuned.push_div),
                            "pull_k": int(tuned.pull_k),
                            "pulls": int((runs["heuristic_tuned"][3][1:rounds + 1] == pp.MODE_PULL).sum())},
        "optimal_plan_replayed_ms": round(t_opt, 4),
        "held_out_table_ms": {"optimal": round(best_ms, 3),
                              "heuristic": round(S.policy_cost(held, S.heuristic_policy(8, held.n))[0], 3),
                              "learned": round(S.policy_cost(held, S.model_policy(params, held))[0], 3),
                              "all_pull": round(S.policy_cost(held, lambda r, f: S.A_PULL)[0], 3)},
        "prep_s": round(t_prep, 1),
        "roofline": None,
    }
    print(json.dumps(out), flush=True)
    G.free()


def bench_progressive(args, torch, pp, g, seeds, cfg):
    """Progressive sampling on the workload's graph: seed groups of the workload's s from a
    pool of 16 s distinct seeds until the average distance's Hoeffding half-width (the
    sample's D and alpha) meets --target; the run checked against the oracle's."""
    from paper_2301_06499_amd import inputs
    import oracle.progressive as prog
    s = len(seeds)
    pool = inputs.sample_seeds(g.n, min(g.n, 16 * s), 7)
    G = pp.pp_csr_build(g.n, g.src, g.dst, undirected=g.undirected)
    group = min(s, 512)
    for _ in range(args.warmup):
        pp.pp_progressive_sample(G, pool, group, args.target, args.delta)
    times = []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        got = pp.pp_progressive_sample(G, pool, group, args.target, args.delta)
        times.append(time.perf_counter() - t0)
    t = sum(times) / len(times)
    t0 = time.perf_counter()
    want = prog.progressive(g.n, g.src, g.dst, pool, group, args.target, args.delta, g.undirected)
    t_oracle = time.perf_counter() - t0
    exact = list(want["counts"]) == list(got["counts"]) and all(
        want[k] == got[k] for k in ("seeds", "groups", "met", "D", "alpha", "eps", "bound"))
    m = pp.pp_estimate_metrics(got["counts"], g.n, got["seeds"])
    rounds = int(got["D"]) + 1
    nominal = float(G.arcs) * (got["seeds"] / 64.0) * rounds
    out = {"metric": "edge-words OR'd/sec (edges x s/64 per round), progressive sampling", "value": nominal / t,
           "unit": "edge-words/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(t * 1000.0, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "u64", "data": "synthetic",
           "config": dict(cfg, method="progressive sampling, Hoeffding stop", group=group, pool=len(pool),
                          target=args.target, delta=args.delta),
           "stop": {k: (bool(v) if k == "met" else v) for k, v in got.items() if k != "counts"},
           "estimates": {k: m[k] for k in ("avg_dist", "eff_diam", "diameter", "alpha", "reachable_pairs")},
           "roofline": None,
           "cpu_baseline": {"value": nominal / t_oracle, "unit": "edge-words/s", "cores": __import__("oracle").default_threads(),
                            "kind": "oracle", "sample": f"the whole run ({got['seeds']} seeds) by per-seed BFS in {t_oracle:.2f} s"},
           "check": {"against": "the oracle's progressive run (same pool)", "result": "bit-exact" if exact else "MISMATCH"}}
    print(json.dumps(out), flush=True)
    G.free()
    if not exact:
        raise SystemExit("progressive sampling differs from the oracle")


def calibration_copy(args, torch):
    """A plain device copy of known size, for scaling the traffic counters."""
    if not args.copy_calibration:
        return
    nb = args.copy_calibration << 20
    a = torch.empty(nb // 4, dtype=torch.int32, device="cuda").fill_(1)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    log(f"[bench] calibration copy of {nb} bytes read + {nb} bytes written")
    del a, b


def bench_propagate_s(args, torch, pp, g, seeds, cfg):
    """PROPAGATE-S (Algorithm 2) on the same workload: time per propagation of all seeds,
    with the same nominal accounting as PROPAGATE-P, and its counts against the oracle."""
    import oracle
    stream = torch.cuda.Stream()
    G = pp.pp_csr_build(g.n, g.src, g.dst, undirected=g.undirected, stream=stream)
    torch.cuda.synchronize()
    calibration_copy(args, torch)
    s = len(seeds)
    for _ in range(args.warmup):
        pp.pp_propagate_s(G, seeds, concurrent=args.concurrent, stream=stream)
    times = []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        counts, D, examined = pp.pp_propagate_s(G, seeds, concurrent=args.concurrent, stream=stream)
        times.append(time.perf_counter() - t0)
    t = sum(times) / len(times)
    want = oracle.propagate(g.n, g.src, g.dst, seeds, g.undirected)
    exact = want["D"] == D and list(want["counts"]) == list(counts)
    rounds = D + 1
    nominal = float(G.arcs) * (s / 64.0) * rounds
    nw = (g.n + 63) // 64
    # per examined arc its 4-byte successor id and the 8-byte signature word
    # holding the successor's bit; per pass and seed every word read and written
    bytes_total = examined * 12.0 + rounds * s * nw * 16.0
    achieved = bytes_total / t / 1e9
    out = {"metric": "edge-words OR'd/sec (edges x s/64 per round), PROPAGATE-S", "value": nominal / t,
           "unit": "edge-words/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(t * 1000.0, 4), "ms_per_step_min": round(min(times) * 1000.0, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
           "config": dict(cfg, method="PROPAGATE-S (Algorithm 2)", nodes=int(G.nodes), arcs=int(G.arcs), rounds=rounds,
                          concurrent=args.concurrent or min(s, 256)),
           "arcs_examined": int(examined),
           "arcs_examined_per_s": examined / t,
           "full_scan_arcs": int(G.arcs) * rounds * s,
           "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": 8000.0, "unit": "GB/s",
                        "frac": round(achieved / 8000.0, 4), "traffic": None, "kernel": "k_seq_pass",
                        "bytes_per_step": bytes_total,
                        "timing": "host clock around the synchronous call (every pass launch and check included)"},
           "check": {"against": "oracle per-seed BFS, every seed", "result": "bit-exact" if exact else "MISMATCH"}}
    print(json.dumps(out), flush=True)
    G.free()
    if not exact:
        raise SystemExit("PROPAGATE-S counts differ from the oracle")


def host_info() -> dict:
    """CPU model, usable cores and memory of the host the oracle ran on."""
    info = {"nproc": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["cpu"] = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                info["mem_gib"] = round(int(line.split()[1]) / 2**20, 1)
                break
    except OSError:
        pass
    return info


def oracle_sample(g, seeds, idx, nominal_edge_words: float, single_thread: bool):
    """The oracle (not tuned) on the host cores for the seeds idx: its exact per-seed
    counts and final signature columns (for the check), and its time, scaled to the
    whole seed set, as cpu_baseline."""
    import oracle
    nth = oracle.default_threads()
    s, k = len(seeds), len(idx)
    t0 = time.perf_counter()
    want = oracle.propagate(g.n, g.src, g.dst, seeds[idx], g.undirected, seed_counts=True, final_sig=True,
                            nthreads=nth)
    t1 = time.perf_counter() - t0
    t_full = t1 * s / k
    base = {"value": nominal_edge_words / t_full, "unit": "edge-words/s", "cores": min(nth, k), "kind": "oracle",
            "sample": f"per-seed BFS over {k} of {s} seeds in {t1:.2f} s (predecessor lists built inside the "
                      f"timed call), scaled by {s}/{k} to the full seed set ({t_full:.2f} s)",
            "host": host_info()}
    if single_thread:   # one thread on a few seeds, for the per-core figure
        k1 = min(s, 8)
        t0 = time.perf_counter()
        oracle.propagate(g.n, g.src, g.dst, seeds[:k1], g.undirected, nthreads=1)
        base["single_thread_value"] = nominal_edge_words / ((time.perf_counter() - t0) * s / k1)
        base["single_thread_sample"] = f"{k1} seeds on one thread, scaled by {s}/{k1}"
    return want, base


def compare(want, idx, counts, sc, sig, D, whole: bool) -> dict:
    """The timed run's results against the oracle's for the seeds idx (all seeds when whole)."""
    s = sc.shape[1]
    res = {"against": "oracle per-seed BFS", "seeds_checked": len(idx) if whole else [int(i) for i in idx]}
    res["totals_vs_per_seed_sums"] = "equal" if np.array_equal(sc.sum(axis=1).astype(np.int64), counts) else "DIFFER"
    ok_counts, ok_cols = True, True
    L = max(D + 1, want["seed_counts"].shape[0])
    for j, i in enumerate(idx):
        mine = np.pad(sc[:, i], (0, L - sc.shape[0]))
        theirs = np.pad(want["seed_counts"][:, j], (0, L - want["seed_counts"].shape[0]))
        ok_counts &= bool(np.array_equal(mine, theirs))
        bit = (sig[:, i >> 6] >> np.uint64(i & 63)) & np.uint64(1)
        wbit = (want["final_sig"][:, j >> 6] >> np.uint64(j & 63)) & np.uint64(1)
        ok_cols &= bool(np.array_equal(bit, wbit))
    res["per_seed_counts"] = "bit-exact" if ok_counts else "MISMATCH"
    res["signature_columns"] = "bit-exact" if ok_cols else "MISMATCH"
    if whole:
        res["counts"] = "bit-exact" if (want["D"] == D and list(want["counts"]) == list(counts)) else "MISMATCH"
    good = ok_counts and ok_cols and res["totals_vs_per_seed_sums"] == "equal" and res.get("counts", "bit-exact") == "bit-exact"
    res["result"] = "bit-exact" if good else "MISMATCH"
    return res


def write_round_log(path, pp, run, G, counts, D, logs):
    """Per-round figures of seed group 0 for per-kernel byte models: the direction of
    each round, the frontier it walked (entries and arcs, from the scheduler's features
    computed at the end of the round before) and the bits it added."""
    rounds = D + 2
    feat = pp.pp_get_round_features(run, rounds + 1)
    n, m = G.nodes, G.arcs
    modes, arcs = logs[0]
    rec = {"n": n, "m": m, "words": run.words, "group_words": run.group_words, "groups": run.groups, "D": D,
           "rounds": [{"r": r, "mode": int(modes[r]), "arcs": int(arcs[r]),
                       "entries": int(round(float(feat[r][0]) * n)), "entry_arcs": int(round(float(feat[r][1]) * m)),
                       "count": int(counts[r]) if r < len(counts) else 0} for r in range(1, rounds)]}
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "a") as f:
        f.write(json.dumps(rec) + "\n")


def time_propagation(args, torch, pp, G, seeds, opts, stream, params=None):
    """K timed steps (seed reset + propagation to convergence, counts on the host) on one
    run, then the same K steps on a second run with HIP events around every pull launch.
    params: the cost model's weights, for runs with the learned scheduler."""
    dseeds = torch.from_numpy(seeds.astype(np.int32)).to("cuda")
    run = pp.pp_seeds_init(G, seeds, opts=opts, stream=stream)
    opts_t = pp.Options.from_buffer_copy(opts)
    opts_t.time_kernels = 1
    run_t = pp.pp_seeds_init(G, seeds, opts=opts_t, stream=stream)
    if params is not None:
        pp.pp_run_set_mlp(run, params)
        pp.pp_run_set_mlp(run_t, params)

    def step(r):
        pp.pp_seeds_reset(r, dseeds)
        return pp.pp_propagate_until_converged(r)

    for _ in range(args.warmup):
        step(run)
    torch.cuda.synchronize()
    per_step = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        counts, D = step(run)
        per_step.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    cap = 4097
    for _ in range(args.warmup):
        step(run_t)
    torch.cuda.synchronize()
    ms_before = pp.pp_get_kernel_times(run_t, cap).astype(np.float64)
    t1 = time.perf_counter()
    for _ in range(args.steps):
        counts_t, D_t = step(run_t)
    torch.cuda.synchronize()
    elapsed_t = time.perf_counter() - t1
    ms_after = pp.pp_get_kernel_times(run_t, cap).astype(np.float64)
    assert int(D_t[0]) == int(D[0]) and list(counts_t[0]) == list(counts[0])
    logs = [pp.pp_get_group_log(run_t, j, cap) for j in range(run.groups)]   # (modes, arcs) per seed group
    if args.round_log:
        write_round_log(args.round_log, pp, run_t, G, counts[0], int(D[0]), logs)
    out = {"counts": counts[0], "D": int(D[0]), "elapsed": elapsed, "elapsed_t": elapsed_t, "per_step": per_step,
           "pull_ms": (ms_after - ms_before) / args.steps, "logs": logs, "words": run.words,
           "group_words": run.group_words, "groups": run.groups, "dseeds": dseeds,
           "form": pull_form(pp, G, run.group_words)}
    run.free()
    run_t.free()
    return out


def step_figures(args, pp, T, m, n, s, wl, opts):
    """Throughput, roofline of the dense pull launches and the round record of one timed run.

    Each round's pull launch covers every seed group; its algorithmic bytes are
    those of the groups that pulled in that round (group logs), per group
      per arc gathered: 4 B column index + 8Wg B source row
      per node: 8 B row offset (int64) + 8Wg B own row read + 8Wg B new row written."""
    rounds = T["D"] + 1
    Wg = T["group_words"]
    by_reach = bool(opts.seed_groups == pp.PP_GROUPS_BY_REACH)
    nominal = m * (s / 64.0) * rounds
    touched = sum(float(a[1:rounds + 1].sum()) * Wg for _, a in T["logs"])
    pull_rounds, bytes_pull = [], 0.0
    for r in range(1, rounds + 1):
        pulled = [float(a[r]) for md, a in T["logs"] if md[r] == pp.MODE_PULL]
        if pulled:
            pull_rounds.append(r)
            bytes_pull += sum(x * (4 + 8 * Wg) + n * (8 + 16 * Wg) for x in pulled)
    t_pull = sum(T["pull_ms"][r] for r in pull_rounds) / 1000.0
    achieved = bytes_pull / t_pull / 1e9 if t_pull > 0 else 0.0
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": (traffic_for(TRAFFIC_PROFILES[(wl, by_reach)], pull_kernel(Wg, opts.pull_k, T["form"]))
                        if ((wl, by_reach) in TRAFFIC_PROFILES and not opts.persistent and
                            args.sparse_pull == 0 and args.push_div == 0 and args.scheduler == "heuristic")
                        else None),
            "kernel": f"k_batch<{Wg}> pull phase" if opts.persistent else pull_kernel(Wg, opts.pull_k, T["form"]),
            "timing": ("device clock between grid barriers" if opts.persistent else
                       "HIP events around each launch, on the run's stream, over a second timed region of "
                       "the same steps"),
            "ms_per_step_with_events": round(T["elapsed_t"] * 1000.0 / args.steps, 4),
            "launches_per_step": len(pull_rounds),
            "avg_launch_ms": round(t_pull * 1000.0 / max(1, len(pull_rounds)), 4),
            "bytes_per_launch": round(bytes_pull / max(1, len(pull_rounds)))}
    if roof["traffic"] and pull_rounds and t_pull > 0:
        # the counted HBM traffic (FETCH_SIZE + WRITE_SIZE per launch) over the same
        # launch time, against the same peak
        roof["traffic_frac"] = round(roof["traffic"] / (t_pull / len(pull_rounds)) / 1e9 / HBM_PEAK_GBS, 4)
    code = {pp.MODE_PULL: "P", pp.MODE_PUSH: "S", pp.MODE_PUSH_FLAT: "F", pp.MODE_SPULL: "Q"}
    modes = ["".join(code.get(int(md[r]), "-") for r in range(1, rounds + 1)) for md, _ in T["logs"]]
    return {"value": nominal * args.steps / T["elapsed"], "unit": "edge-words/s",
            "ms_per_step": round(T["elapsed"] * 1000.0 / args.steps, 4),
            "ms_per_step_min": round(min(T["per_step"]) * 1000.0, 4),
            "ms_per_step_median": round(float(np.median(T["per_step"])) * 1000.0, 4),
            "touched_edge_words_per_s": touched * args.steps / T["elapsed"], "roofline": roof,
            "run": {"words": T["words"], "seed_groups": T["groups"], "group_words": Wg, "rounds": rounds,
                    "modes": modes[0] if len(modes) == 1 else modes}}


def learned_object(args, torch, pp, G, g, seeds, base_opts, stream, T, res):
    """The same propagation with the learned scheduler: the cost model trained on the
    round costs of another seed sample of the same graph (every allowed action after
    both kinds of round, replayed on the ordinary path), then timed on the run's seeds.
    Also the training table's costs of the fixed rule, the model and the optimal plan."""
    from paper_2301_06499_amd import inputs, scheduler
    t0 = time.perf_counter()
    train_seeds = inputs.sample_seeds(g.n, len(seeds), 7)
    table = scheduler.measure_replay(G, train_seeds, opts=base_opts, repeats=2, stream=stream)
    params, loss = scheduler.train(scheduler.label(table), steps=3000)
    _, opt_ms, opt_plan = scheduler.optimal_schedule(table)
    heur_ms, heur_plan = scheduler.policy_cost(table, scheduler.heuristic_policy(8, G.nodes))
    model_ms, model_plan = scheduler.policy_cost(table, scheduler.model_policy(params, table))
    train_s = time.perf_counter() - t0
    opts = pp.Options.from_buffer_copy(base_opts)
    opts.scheduler = pp.PP_SCHED_MLP
    L = time_propagation(args, torch, pp, G, seeds, opts, stream, params=params)
    if L["D"] != T["D"] or list(L["counts"]) != list(T["counts"]):
        raise SystemExit("the learned scheduler's counts differ from the heuristic's")
    ms = L["elapsed"] * 1000.0 / args.steps
    code = "PSFQ"
    out = {"ms_per_step": round(ms, 4), "ms_per_step_median": round(float(np.median(L["per_step"])) * 1000.0, 4),
           "vs_heuristic_same_groups": round(res["ms_per_step"] / ms, 4),
           "modes": ["".join({pp.MODE_PULL: "P", pp.MODE_PUSH: "S", pp.MODE_PUSH_FLAT: "F",
                              pp.MODE_SPULL: "Q"}.get(int(md[r]), "-") for r in range(1, L["D"] + 2))
                     for md, _ in L["logs"]],
           "counts": "equal to the heuristic's",
           "training": {"seeds": "another uniform sample of the same size (sampler seed 7)",
                        "rounds": len(table), "samples": 2 * len(table) - 1, "final_loss": round(float(loss[-1]), 5),
                        "seconds": round(train_s, 1),
                        "table_ms": {"heuristic": round(heur_ms, 3), "model": round(model_ms, 3),
                                     "optimal": round(opt_ms, 3)},
                        "plans": {"heuristic": "".join(code[a] for a in heur_plan),
                                  "model": "".join(code[a] for a in model_plan),
                                  "optimal": "".join(code[a] for a in opt_plan)}}}
    if "plain" in res:
        out["vs_plain"] = round(res["plain"]["ms_per_step"] / ms, 4)
    log(f"[bench] learned scheduler: {out['ms_per_step']} ms per step (heuristic {res['ms_per_step']})")
    return out, L, opts, params


def propagation_line(args, torch, pp, g, seeds, cfg, wl, sample, stream, base_opts, plain_opts=None,
                     learned=False):
    """Builds the graph, times the propagation (and the plain form beside it when
    plain_opts is given), checks it: one result object.

    sample: indices of the seeds the oracle checks one by one (and times for
    cpu_baseline); all of them for a whole-seed-set check."""
    t0 = time.perf_counter()
    G = pp.pp_csr_build(g.n, g.src, g.dst, undirected=g.undirected, stream=stream)
    log(f"[bench] {cfg['workload']}: csr_build {time.perf_counter() - t0:.1f} s, n={G.nodes} arcs={G.arcs}")
    torch.cuda.synchronize()
    calibration_copy(args, torch)
    m, n, s = G.arcs, G.nodes, len(seeds)
    T = time_propagation(args, torch, pp, G, seeds, base_opts, stream)
    counts, Dv = T["counts"], T["D"]
    res = step_figures(args, pp, T, m, n, s, wl, base_opts)
    res["config"] = dict(cfg, nodes=n, arcs=m, words=T["words"], rounds=Dv + 1, diameter_lb=Dv,
                         scheduler=args.scheduler, engine="persistent" if base_opts.persistent else "rounds",
                         pull_k=int(base_opts.pull_k) or 4, push_div=int(base_opts.push_div) or 8,
                         sparse_pull=int(base_opts.sparse_pull), seed_groups=T["groups"],
                         group_words=T["group_words"],
                         seed_order="by reach" if (base_opts.seed_order or base_opts.seed_groups == pp.PP_GROUPS_BY_REACH)
                         else "as given")
    log(f"[bench] {cfg['workload']}: {res['ms_per_step']} ms per step, {T['groups']} seed group(s)")
    if plain_opts is not None:
        P = time_propagation(args, torch, pp, G, seeds, plain_opts, stream)
        if P["D"] != Dv or list(P["counts"]) != list(counts):
            raise SystemExit("the plain form's counts differ from the seed groups'")
        res["plain"] = step_figures(args, pp, P, m, n, s, wl, plain_opts)
        res["plain"]["note"] = "the same graph and seeds as one group of s seeds, same scheduler"
        res["plain"]["pull_k"] = int(plain_opts.pull_k) or 4
        res["speedup_vs_plain"] = round(P["elapsed"] / T["elapsed"], 4)
        log(f"[bench] {cfg['workload']}: plain {res['plain']['ms_per_step']} ms per step")
    if learned:
        # the configuration's own form: seed groups plus the learned scheduler is
        # the line's value; the same groups under the fixed heuristic stand beside it
        lo, L, lopts, lparams = learned_object(args, torch, pp, G, g, seeds, base_opts, stream, T, res)
        keys = ("value", "unit", "ms_per_step", "ms_per_step_min", "ms_per_step_median", "touched_edge_words_per_s",
                "roofline", "run")
        res["heuristic"] = {k: res[k] for k in keys}
        res["heuristic"]["note"] = "the same seed groups under the fixed-threshold heuristic"
        res.update(step_figures(args, pp, L, m, n, s, wl, lopts))
        res["config"]["scheduler"] = ("learned: MLP 8-32-32-4 trained on the replayed round costs of another seed "
                                      "sample of the same graph, the heuristic as fallback")
        if "plain" in res:
            res["speedup_vs_plain"] = round(P["elapsed"] / L["elapsed"], 4)
        res["learned"] = lo
    if args.no_check and args.no_cpu_baseline:
        G.free()
        return res
    # the check: the line's own form (with the learned scheduler when it is the
    # value) with per-seed counts (untimed) against the timed counts, its totals
    # against its per-seed sums, and the sampled seeds against the oracle
    opts_c = pp.Options.from_buffer_copy(lopts if learned else base_opts)
    opts_c.seed_counts = 1
    chk = pp.pp_seeds_init(G, seeds, opts=opts_c, stream=stream)
    if learned:
        pp.pp_run_set_mlp(chk, lparams)
    pp.pp_seeds_reset(chk, T["dseeds"])
    c2, D2 = pp.pp_propagate_until_converged(chk)
    sc = pp.pp_get_seed_counts(chk, Dv + 1)[0]
    sig = pp.pp_get_signatures(chk)
    chk.free()
    G.free()
    log(f"[bench] {cfg['workload']}: oracle on {len(sample)} of {s} seeds")
    nominal = m * (s / 64.0) * (Dv + 1)
    want, base = oracle_sample(g, seeds, sample, nominal, single_thread=g.n <= (1 << 22))
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = base
    check = compare(want, sample, counts, sc, sig, Dv, whole=len(sample) == s)
    check["check_run_counts_vs_timed"] = "equal" if (int(D2[0]) == Dv and list(c2[0]) == list(counts)) else "DIFFER"
    if check["check_run_counts_vs_timed"] != "equal":
        check["result"] = "MISMATCH"
    res["check"] = check
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat26",
                    help="rmat26 (the default: the largest single-GPU configuration, with R-MAT 20 as a "
                         "secondary object in the same line), rmat20, er, grid:SIDE, rmat:SCALE:SEEDS, "
                         "grid4096 (learned scheduler), batch64 (the 64-graph batch)")
    ap.add_argument("--no-secondary", action="store_true", help="rmat26: skip the R-MAT 20 object")
    ap.add_argument("--groups", default="reach",
                    help="seed groups of the timed run: 'reach' (the default: groups sized so that the seeds "
                         "with a predecessor fill whole groups first), 'plain' (one group), or a number; "
                         "with more than one group the plain form is timed beside it")
    ap.add_argument("--scheduler", default="heuristic", choices=["heuristic", "pull", "push"])
    ap.add_argument("--grid-side", type=int, default=4096, help="side of the grid4096 workload")
    ap.add_argument("--persistent", action="store_true",
                    help="all rounds in one cooperative launch instead of launches per round")
    ap.add_argument("--check-seeds", type=int, default=16,
                    help="seeds the oracle checks one by one on graphs above 2^22 nodes (all seeds below)")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--tune", action="store_true",
                    help="run options from the autotuner (measured before the timed steps, cached per workload)")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--method", default="p", choices=["p", "s", "progressive"],
                    help="p: PROPAGATE-P (the default, the headline line); s: PROPAGATE-S, one bit per node "
                         "and seed; progressive: seed groups until the average distance's Hoeffding half-width "
                         "meets --target (each its own JSON line)")
    ap.add_argument("--target", type=float, default=1.0, help="progressive: half-width target (hops)")
    ap.add_argument("--node-stats", action="store_true",
                    help="also keep the per-node reach and distance sums (one extra pass per round) in the "
                         "timed runs (their values are checked against the oracle by the GPU tests)")
    ap.add_argument("--hip-malloc", action="store_true",
                    help="the library's own hipMalloc / hipFree for its device memory instead of PyTorch's caching "
                         "allocator (the default here, through pp_set_allocator): releasing gigabytes with hipFree "
                         "slows the GPU work of the next seconds by a few percent, which would reach every form "
                         "timed after the first")
    ap.add_argument("--pull-k", type=int, default=0, choices=[0, 2, 4],
                    help="arcs per lane of the dense pull's tiles (0: the library's default, 4)")
    ap.add_argument("--push-div", type=int, default=0,
                    help="heuristic: push while frontier arcs x push_div < arcs (0: the library's default)")
    ap.add_argument("--sparse-pull", type=int, default=0, choices=[0, 1, 2],
                    help="sparse rounds: 0 push, 1 sparse pull, 2 either per round (pseudo-random)")
    ap.add_argument("--delta", type=float, default=0.05, help="progressive: 1 - confidence")
    ap.add_argument("--concurrent", type=int, default=0, help="PROPAGATE-S: seeds in flight (0: min(s, 256))")
    ap.add_argument("--no-learned", action="store_true",
                    help="rmat26: skip the learned-scheduler run (cost model trained on another seed sample's "
                         "replayed round costs)")
    ap.add_argument("--batch-engines", default="clustered,union",
                    help="batch64: the batched engines to run, comma-separated (clustered, union)")
    ap.add_argument("--no-plain", action="store_true",
                    help="batch64: time the two batched engines only, without the 64 solo runs")
    ap.add_argument("--round-log", default="", metavar="PATH",
                    help="append each timed propagation's per-round figures (direction, frontier entries "
                         "and arcs, new bits; seed group 0) as one JSON line to PATH")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device with a plain torch copy, so that a "
                         "hardware-counter run has a kernel of known traffic to scale against")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the propagation runs on a single MI355X and has no multi-GPU "
              "path in this build (seed groups would shard across GPUs with one final all-reduce of the "
              "per-round counts). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    t_start = time.perf_counter()

    import torch
    from paper_2301_06499_amd import pp

    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    torch.cuda.set_device(0)
    if not args.hip_malloc:
        pp.use_torch_allocator(torch)
    sched = {"heuristic": pp.PP_SCHED_HEURISTIC, "pull": pp.PP_SCHED_PULL, "push": pp.PP_SCHED_PUSH}[args.scheduler]
    if args.workload == "batch64":
        return bench_batch(args, torch, pp)
    if args.workload == "grid4096":
        return bench_grid(args, torch, pp)

    t0 = time.perf_counter()
    g, seeds, cfg = workload(args.workload)
    log(f"[bench] generated {cfg['workload']} in {time.perf_counter() - t0:.1f} s")
    if args.method == "s":
        return bench_propagate_s(args, torch, pp, g, seeds, cfg)
    if args.method == "progressive":
        return bench_progressive(args, torch, pp, g, seeds, cfg)
    stream = torch.cuda.Stream()                       # default priority
    def make_opts(groups):
        sg = {"reach": pp.PP_GROUPS_BY_REACH, "plain": 0}.get(groups, None)
        sg = int(groups) if sg is None else sg
        return pp.options(scheduler=sched, max_rounds=4096, persistent=args.persistent, node_stats=args.node_stats,
                          sparse_pull=args.sparse_pull, push_div=args.push_div, seed_groups=sg, pull_k=args.pull_k)

    grouped = args.groups != "plain" and not args.persistent and not args.node_stats
    base = make_opts(args.groups if grouped else "plain")
    plain = make_opts("plain") if grouped else None
    tuned = None
    if args.tune:
        from paper_2301_06499_amd import autotune
        t0 = time.perf_counter()
        Gt = pp.pp_csr_build(g.n, g.src, g.dst, undirected=g.undirected, stream=stream)
        base, tuned = autotune.tune(Gt, seeds, base=base, reps=3, name=cfg["workload"])
        Gt.free()
        tuned = {k: v for k, v in tuned.items() if k != "candidates"} | {"tune_s": round(time.perf_counter() - t0, 2)}
        log(f"[bench] tuned options {tuned}")
    s = len(seeds)
    sample = (np.arange(s) if g.n <= (1 << 22) else
              np.unique(np.linspace(0, s - 1, min(s, args.check_seeds)).astype(np.int64)))
    head = propagation_line(args, torch, pp, g, seeds, cfg, args.workload, sample, stream, base, plain,
                            learned=(args.workload == "rmat26" and not args.no_learned and sched == pp.PP_SCHED_HEURISTIC
                                     and not args.persistent and not args.node_stats))
    head["config"]["tuned"] = tuned
    out = {"metric": METRIC, "value": head["value"], "unit": "edge-words/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "ms_per_step_min": head["ms_per_step_min"],
           "ms_per_step_median": head["ms_per_step_median"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u64", "data": "synthetic", "config": head["config"],
           "touched_edge_words_per_s": head["touched_edge_words_per_s"], "roofline": head["roofline"],
           "run": head["run"]}
    for k in ("heuristic", "plain", "speedup_vs_plain", "learned", "cpu_baseline", "check"):
        if k in head:
            out[k] = head[k]
    del g
    if args.workload == "rmat26" and not args.no_secondary:
        g2, seeds2, cfg2 = workload("rmat20")
        out["rmat20"] = propagation_line(args, torch, pp, g2, seeds2, cfg2, "rmat20", np.arange(len(seeds2)),
                                         stream, base, plain)
        out["rmat20"]["note"] = "secondary: R-MAT scale 20, s = 256, every seed checked against the oracle"
    if args.node_stats:
        out["node_stats_note"] = "per-node sums kept in every timed round (their check runs in the GPU tests)"
    out["hip_runtime"] = pp.hip_runtime()
    out["allocator"] = "hipMalloc (the library's own)" if args.hip_malloc else "PyTorch's caching allocator (pp_set_allocator)"
    out["wall_s"] = round(time.perf_counter() - t_start, 1)
    print(json.dumps(out), flush=True)
    bad = [k for k, v in (("headline", out.get("check")), ("rmat20", out.get("rmat20", {}).get("check")))
           if v is not None and v.get("result") != "bit-exact"]
    if bad:
        raise SystemExit(f"check failed: {bad}")


if __name__ == "__main__":
    main()
