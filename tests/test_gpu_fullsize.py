"""GPU parity at the workloads' full sizes, element by element against the oracle.

* R-MAT scale 20, s = 256, in the benchmark's launch configuration: every
  per-round count, every seed's per-round counts, the final signatures, and
  the signatures after rounds 1, 2, floor(D/2) and D.
* The same workload in a process that loads PyTorch first and hands the
  library a PyTorch stream and device seeds, as the benchmark does (the
  library then runs on PyTorch's bundled HIP runtime).
* The 64-graph batch on both batch engines (clustered persistent launch and
  per-round launches over the union): each graph's D, counts, per-seed counts
  and final signatures against that graph's own oracle run.
* A batch whose large graphs run on clusters of several blocks starting at
  non-zero block offsets (persistent engine), every direction policy.
* The 4096^2 grid under the learned scheduler is in test_gpu_parity.py
  (test_grid4096_full_size), with the oracle run it shares with the other
  policies.
"""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2301_06499_amd import inputs as gen
from paper_2301_06499_amd import pp

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def pad_words(sig, W):
    if sig.shape[1] == W:
        return sig
    out = np.zeros((sig.shape[0], W), dtype=np.uint64)
    out[:, :sig.shape[1]] = sig
    return out


def test_rmat20_every_seed_and_round_signatures():
    g, seeds = gen.workload_rmat(20, 16, 256, 1)
    say("rmat20 oracle", g.n)
    want = oracle.propagate(g.n, g.src, g.dst, seeds, False, seed_counts=True, final_sig=True,
                            sig_rounds=list(range(1, 13)))
    D = want["D"]
    assert 2 <= D < 12
    G = pp.pp_csr_build(g.n, g.src, g.dst)
    # the benchmark's options: heuristic directions, graph replay, adaptive batches
    r = pp.pp_seeds_init(G, seeds, opts=pp.options(seed_counts=True, max_rounds=256))
    counts, Dg = pp.pp_propagate_until_converged(r)
    assert int(Dg[0]) == D
    assert list(counts[0]) == list(want["counts"])
    assert np.array_equal(pp.pp_get_seed_counts(r, D + 1)[0], want["seed_counts"])
    assert np.array_equal(pp.pp_get_signatures(r), want["final_sig"])
    r.free()
    # one round at a time: the signatures after rounds 1, 2, floor(D/2), D
    r = pp.pp_seeds_init(G, seeds, opts=pp.options(max_rounds=256))
    check = sorted({1, 2, D // 2, D})
    for k in range(1, D + 2):
        nb, conv = pp.pp_propagate_round(r)
        assert int(nb[0]) == (int(want["counts"][k]) if k <= D else 0), k
        if k in check:
            assert np.array_equal(pp.pp_get_signatures(r), want["sigs"][k - 1]), k
        assert conv == (k == D + 1)
    say("rmat20 D", D, "rounds checked", check)


TORCH_FIRST = r'''
import json, sys
import numpy as np
import torch
torch.cuda.set_device(0)
torch.zeros(1, device="cuda")              # PyTorch's HIP runtime first, as in the benchmark
sys.path.insert(0, sys.argv[1])
import oracle
from paper_2301_06499_amd import inputs as gen
from paper_2301_06499_amd import pp
g, seeds = gen.workload_rmat(20, 16, 256, 1)
stream = torch.cuda.Stream()
G = pp.pp_csr_build(g.n, g.src, g.dst, stream=stream)
dseeds = torch.from_numpy(seeds.astype(np.int32)).to("cuda")
r = pp.pp_seeds_init(G, seeds, opts=pp.options(seed_counts=True, max_rounds=256), stream=stream)
res = []
for rep in range(3):                         # resets from device seeds, as the timed steps do
    pp.pp_seeds_reset(r, dseeds)
    counts, D = pp.pp_propagate_until_converged(r)
    res.append((list(map(int, counts[0])), int(D[0])))
sc = pp.pp_get_seed_counts(r, res[0][1] + 1)[0]
sig = pp.pp_get_signatures(r)
want = oracle.propagate(g.n, g.src, g.dst, seeds, False, seed_counts=True, final_sig=True)
ok = {"counts": all(c == list(map(int, want["counts"])) and d == want["D"] for c, d in res),
      "seed_counts": bool(np.array_equal(sc, want["seed_counts"])),
      "signatures": bool(np.array_equal(sig, want["final_sig"]))}
print(json.dumps({"runtime": pp.hip_runtime(), "ok": ok}), flush=True)
'''


@pytest.mark.timeout(900)
def test_rmat20_with_pytorch_loaded_first():
    """The benchmark's runtime configuration: PyTorch's HIP runtime, a PyTorch stream, device seeds."""
    say("rmat20 torch-first subprocess")
    p = subprocess.run([sys.executable, "-u", "-c", TORCH_FIRST, ROOT], capture_output=True, text=True,
                       timeout=840, cwd=ROOT)
    assert p.returncode == 0, p.stderr[-3000:]
    rec = json.loads(p.stdout.strip().splitlines()[-1])
    say("runtime", rec["runtime"], rec["ok"])
    assert rec["runtime"] and "torch" in rec["runtime"], rec
    assert all(rec["ok"].values()), rec


def batch_against_oracle(graphs, seeds, s, opts_list, cap):
    wants = [oracle.propagate(g.n, g.src, g.dst, sd, g.undirected, seed_counts=True, final_sig=True)
             for g, sd in zip(graphs, seeds)]
    n, src, dst, offs, allseeds = gen.union_of(graphs, seeds)
    G = pp.pp_csr_build(n, src, dst, node_offsets=offs)
    Dmax = max(w["D"] for w in wants)
    for opts in opts_list:
        say("batch", len(graphs), "graphs: persistent", opts.persistent, "sched", opts.scheduler)
        r = pp.pp_seeds_init(G, allseeds, s=s, opts=opts)
        counts, D = pp.pp_propagate_until_converged(r)
        sc = pp.pp_get_seed_counts(r, Dmax + 1)
        sig = pp.pp_get_signatures(r)
        for k, w in enumerate(wants):
            assert int(D[k]) == w["D"], k
            assert list(counts[k][:w["D"] + 1]) == list(w["counts"]), k
            assert not counts[k][w["D"] + 1:].any(), k
            assert np.array_equal(sc[k][:w["D"] + 1], w["seed_counts"]), k
            assert not sc[k][w["D"] + 1:].any(), k
            assert np.array_equal(sig[offs[k]:offs[k + 1]], pad_words(w["final_sig"], r.words)), k
        r.free()
        del sc, sig
    G.free()


def test_batch64_both_engines():
    """The 64-graph workload (R-MAT 10-16, grids 64^2-512^2, paths up to 20 000 edges), 64 seeds each."""
    graphs, seeds = gen.workload_batch(1, 64)
    opts = [pp.options(seed_counts=True, max_rounds=25000, persistent=True),
            pp.options(seed_counts=True, max_rounds=25000, persistent=False)]
    batch_against_oracle(graphs, seeds, 64, opts, 25000)


@pytest.mark.parametrize("sched", [pp.PP_SCHED_HEURISTIC, pp.PP_SCHED_PULL, pp.PP_SCHED_PUSH, pp.PP_SCHED_FUZZ])
def test_clusters_of_several_blocks(sched):
    """A small graph first, then graphs of 2-7 times 64 Ki arcs plus nodes: the persistent
    engine gives each of those a cluster of several blocks, at a non-zero first block."""
    graphs = [gen.path_graph(500), gen.rmat(14, 16, 9), gen.grid_graph(300, 300), gen.star_graph(1000),
              gen.rmat(13, 8, 2), gen.grid_with_shortcuts(200, 150, gen.Fraction(1, 10), 30, 4)]
    seeds = [gen.sample_seeds(g.n, 100, 60 + k) for k, g in enumerate(graphs)]
    for g in graphs[1:3]:
        assert g.n + (2 if g.undirected else 1) * len(g.src) > 2 * 65536
    batch_against_oracle(graphs, seeds, 100, [pp.options(scheduler=sched, seed_counts=True, max_rounds=1200,
                                                         persistent=True, fuzz_seed=11)], 1200)
