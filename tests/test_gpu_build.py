"""The adjacency build on the device against the build on host threads: the
same successor rows, predecessor rows and storage order, array for array, on
graphs with self-loops, duplicate arcs, hubs, empty rows, batches of graphs,
both directions and both orders; device-resident input; the range checks.

The host build is the one every other parity test has exercised against the
oracle; the graph a run sees is these arrays, so equal arrays give equal
results.  A propagation on a device-built graph is checked against the oracle
too."""
import sys

import numpy as np
import pytest

import oracle
from hipmem import DeviceArray
from paper_2301_06499_amd import inputs as gen
from paper_2301_06499_amd import pp

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def csr_both(n, src, dst, **kw):
    gh = pp.pp_csr_build(n, src, dst, build="host", **kw)
    gd = pp.pp_csr_build(n, src, dst, build="device", **kw)
    a, b = pp.pp_graph_get_csr(gh), pp.pp_graph_get_csr(gd)
    assert gh.arcs == gd.arcs
    for name, x, y in zip(("rp", "col", "trp", "tcol", "perm"), a, b):
        assert np.array_equal(x, y), name
    return gh, gd, a


def multigraph(seed, n, m, loops=0.05, dups=0.2):
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    k = rng.random(m) < loops
    dst[k] = src[k]                                      # self-loops
    j = rng.integers(0, m, int(m * dups))
    src = np.concatenate([src, src[j]])                  # repeated arcs
    dst = np.concatenate([dst, dst[j]])
    return src, dst


CASES = [
    ("random multigraph", lambda: (5000,) + multigraph(1, 5000, 40000), {}),
    ("random multigraph undirected", lambda: (3000,) + multigraph(2, 3000, 20000), {"undirected": True}),
    ("random multigraph transposed", lambda: (3000,) + multigraph(3, 3000, 20000), {"transpose": True}),
    ("random multigraph in input order", lambda: (3000,) + multigraph(4, 3000, 20000), {"keep_order": True}),
    ("rmat with hubs", lambda: (lambda g: (g.n, g.src, g.dst))(gen.rmat(14, 16, 77)), {}),
    ("rmat with hubs, the rest in input order", lambda: (lambda g: (g.n, g.src, g.dst))(gen.rmat(14, 16, 77)),
     {"hubs_only": True}),
    ("grid, input order (no hubs)", lambda: (lambda g: (g.n, g.src, g.dst))(gen.grid_graph(60, 45)),
     {"undirected": True, "hubs_only": True}),
    ("grid", lambda: (lambda g: (g.n, g.src, g.dst))(gen.grid_graph(60, 45)), {"undirected": True}),
    ("star", lambda: (lambda g: (g.n, g.src, g.dst))(gen.star_graph(3000)), {"undirected": True}),
    ("isolated nodes only", lambda: (100, np.zeros(0, np.int32), np.zeros(0, np.int32)), {}),
    ("self-loops only", lambda: (10, np.arange(10, dtype=np.int32), np.arange(10, dtype=np.int32)), {}),
    ("one node", lambda: (1, np.zeros(3, np.int32), np.zeros(3, np.int32)), {}),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_device_build_equals_host_build(case):
    name, make, kw = CASES[case]
    n, src, dst = make()
    say("build", name, "n", n, "pairs", len(src))
    gh, gd, (rp, col, trp, tcol, perm) = csr_both(n, src, dst, **kw)
    # the arrays themselves: rows sorted and without repeats or self-loops
    for u in range(0, n, max(1, n // 200)):
        row = col[rp[u]:rp[u + 1]]
        assert np.all(np.diff(row) > 0) and not np.any(row == u)
    assert rp[-1] == gd.arcs == trp[-1]


def test_storage_orders_give_the_oracle_results():
    """The three storage orders of one graph (hubs first then breadth-first, hubs
    first then input order, input order): the same results as the oracle,
    reported by input id, and different stored arrays."""
    g = gen.rmat(12, 16, 9)
    seeds = gen.sample_seeds(g.n, 200, 4)
    want = oracle.propagate(g.n, g.src, g.dst, seeds, False, seed_counts=True, final_sig=True)
    perms = []
    for kw in ({}, {"hubs_only": True}, {"keep_order": True}):
        say("order", kw)
        G = pp.pp_csr_build(g.n, g.src, g.dst, **kw)
        perms.append(pp.pp_graph_get_csr(G)[4])
        r = pp.pp_seeds_init(G, seeds, opts=pp.options(seed_counts=True, max_rounds=want["D"] + 4))
        counts, D = pp.pp_propagate_until_converged(r)
        assert int(D[0]) == want["D"] and list(counts[0]) == list(want["counts"])
        assert np.array_equal(pp.pp_get_seed_counts(r, want["D"] + 1)[0], want["seed_counts"])
        sig = pp.pp_get_signatures(r)
        assert np.array_equal(sig[:, :want["final_sig"].shape[1]], want["final_sig"])
        r.free()
        G.free()
    assert not np.array_equal(perms[0], perms[1]) and np.array_equal(perms[2], np.arange(g.n))
    # hubs first in both orders that move nodes: the same node stored first
    assert int(np.argmin(perms[0])) == int(np.argmin(perms[1]))


def test_batch_of_graphs():
    graphs = [gen.grid_graph(20, 15), gen.path_graph(300), gen.rmat(10, 8, 4), gen.star_graph(900),
              gen.cycle_graph(7, directed=True)]
    n, src, dst, offs, _ = gen.union_of(graphs, [np.zeros(1, np.int32)] * len(graphs))   # both arcs of an edge
    say("build batch", n, len(src))
    csr_both(n, src, dst, node_offsets=offs)


def test_device_input_and_range_errors():
    src, dst = multigraph(7, 4000, 30000)
    gh, _, want = csr_both(4000, src, dst)
    ds, dd = DeviceArray(src), DeviceArray(dst)
    gdev = pp.pp_csr_build(4000, ds, dd, build="device")
    got = pp.pp_graph_get_csr(gdev)
    for name, x, y in zip(("rp", "col", "trp", "tcol", "perm"), want, got):
        assert np.array_equal(x, y), name
    # ids outside [0, n) and arcs across graphs, from the host and from the device
    bad = dst.copy()
    bad[12345] = 4000
    for build in ("host", "device"):
        with pytest.raises(pp.PPError) as e:
            pp.pp_csr_build(4000, src, bad, build=build)
        assert e.value.code == pp.PP_ERANGE and "12345" in str(e.value)
        with pytest.raises(pp.PPError) as e:
            pp.pp_csr_build(4000, DeviceArray(src), DeviceArray(bad), build=build)
        assert e.value.code == pp.PP_ERANGE and "12345" in str(e.value)
        with pytest.raises(pp.PPError) as e:
            pp.pp_csr_build(4, np.array([0, 1], np.int32), np.array([1, 2], np.int32), node_offsets=[0, 2, 4],
                            build=build)
        assert e.value.code == pp.PP_ERANGE
    with pytest.raises(ValueError):
        pp.pp_csr_build(10, src[:5] % 10, dst[:5] % 10, build="nope")
    with pytest.raises(pp.PPError) as e:
        pp._check(pp.lib().pp_csr_build(10, 0, None, None, pp.PP_BUILD_ON_HOST | pp.PP_BUILD_ON_DEVICE, None, 1,
                                           None, pp.ctypes.byref(pp.ctypes.c_void_p())))
    assert e.value.code == pp.PP_EINVAL


def test_large_default_build_and_propagation():
    """R-MAT scale 21 (above the size from which the device build is the default):
    the default build equals the host build, and a propagation on it equals the
    oracle's."""
    g = gen.rmat(21, 16, 5)
    assert len(g.src) >= pp.DEVICE_BUILD_MIN
    say("large build", g.n, len(g.src))
    gh = pp.pp_csr_build(g.n, g.src, g.dst, build="host")
    gd = pp.pp_csr_build(g.n, g.src, g.dst)
    for name, x, y in zip(("rp", "col", "trp", "tcol", "perm"), pp.pp_graph_get_csr(gh), pp.pp_graph_get_csr(gd)):
        assert np.array_equal(x, y), name
    gh.free()
    seeds = gen.sample_seeds(g.n, 128, 3)
    want = oracle.propagate(g.n, g.src, g.dst, seeds, False, seed_counts=True, final_sig=True)
    r = pp.pp_seeds_init(gd, seeds, opts=pp.options(seed_counts=True, max_rounds=want["D"] + 4))
    counts, D = pp.pp_propagate_until_converged(r)
    assert int(D[0]) == want["D"] and list(counts[0]) == list(want["counts"])
    assert np.array_equal(pp.pp_get_seed_counts(r, want["D"] + 1)[0], want["seed_counts"])
    assert np.array_equal(pp.pp_get_signatures(r), want["final_sig"])
    r.free()
    gd.free()
