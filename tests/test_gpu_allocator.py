"""The caller's device allocator (pp_set_allocator): every block the library
allocates comes from it and goes back to it, results unchanged."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2301_06499_amd import inputs as gen
from paper_2301_06499_amd import pp
from hipmem import hip

pytestmark = pytest.mark.gpu


class CountingAllocator:
    """hipMalloc / hipFree through the HIP runtime's C interface, with a ledger."""

    def __init__(self):
        self.live, self.allocs, self.releases, self.streams = {}, 0, 0, set()

    def alloc(self, n, stream):
        p = ctypes.c_void_p()
        if hip().hipMalloc(ctypes.byref(p), n) != 0:
            return 0
        assert p.value % 256 == 0
        self.live[p.value] = n
        self.allocs += 1
        self.streams.add(stream)
        return p.value

    def release(self, p, stream):
        assert p in self.live, "a block this allocator did not give"
        del self.live[p]
        self.releases += 1
        assert hip().hipFree(ctypes.c_void_p(p)) == 0


def test_blocks_come_from_and_go_back_to_the_callers_allocator():
    a = CountingAllocator()
    g = gen.rmat(12, 8, 3)
    seeds = gen.sample_seeds(g.n, 130, 4)
    want = oracle.propagate(g.n, g.src, g.dst, seeds, False, seed_counts=True, final_sig=True)
    pp.pp_set_allocator(a.alloc, a.release)
    try:
        G = pp.pp_csr_build(g.n, g.src, g.dst)
        r = pp.pp_seeds_init(G, seeds, opts=pp.options(seed_counts=True, node_stats=True,
                                                        max_rounds=want["D"] + 4))
        assert a.allocs > 20 and sum(a.live.values()) > 8 * g.n * r.words
        counts, D = pp.pp_propagate_until_converged(r)
        assert int(D[0]) == want["D"] and list(counts[0]) == list(want["counts"])
        assert np.array_equal(pp.pp_get_signatures(r)[:, :2], want["final_sig"][:, :2])
        snap = pp.pp_run_snapshot(r)
        pp.pp_get_node_stats(r)                     # temporaries of a single call
        before = a.allocs
        pp.pp_mlp_forward(np.zeros(pp.MLP_PARAMS, np.float32), np.zeros((5, pp.MLP_IN), np.float32))
        assert a.allocs > before                    # the cost model's buffers too
        # cleared while blocks are out: new ones come from hipMalloc, the old go back to `a`
        pp.pp_set_allocator(None, None)
        n_before = a.allocs
        r2 = pp.pp_seeds_init(G, seeds, opts=pp.options(max_rounds=want["D"] + 4))
        assert a.allocs == n_before
        c2, _ = pp.pp_propagate_until_converged(r2)
        assert list(c2[0]) == list(want["counts"])
        for obj in (r2, snap, r, G):
            obj.free()
        assert a.live == {} and a.releases == a.allocs
    finally:
        pp.pp_set_allocator(None, None)


def test_failed_allocation_is_reported():
    g = gen.path_graph(100)
    G = pp.pp_csr_build(g.n, g.src, g.dst, undirected=True)
    pp.pp_set_allocator(lambda n, st: 0, lambda p, st: None)
    try:
        with pytest.raises(pp.PPError) as e:
            pp.pp_seeds_init(G, np.array([0, 50], np.int32))
        assert e.value.code == pp.PP_ENOMEM
    finally:
        pp.pp_set_allocator(None, None)
    # a block off the 256-byte alignment is handed back and reported
    a = CountingAllocator()
    pp.pp_set_allocator(lambda n, st: a.alloc(n + 256, st) + 64, lambda p, st: a.release(p - 64, st))
    try:
        with pytest.raises(pp.PPError) as e:
            pp.pp_seeds_init(G, np.array([0, 50], np.int32))
        assert e.value.code == pp.PP_ENOMEM and "aligned" in str(e.value)
    finally:
        pp.pp_set_allocator(None, None)
    assert a.live == {} and a.allocs >= 1
    r = pp.pp_seeds_init(G, np.array([0, 50], np.int32))
    c, D = pp.pp_propagate_until_converged(r)
    assert int(D[0]) == 99   # node 99 lies 99 hops from seed 0
