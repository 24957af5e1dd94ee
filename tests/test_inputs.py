"""The seeded input generators: determinism, sizes and distributions."""
from fractions import Fraction

import numpy as np

from paper_2301_06499_amd import inputs as gen


def test_splitmix64_published_first_outputs():
    """SplitMix64 with state 0: the first outputs of the reference generator."""
    x = gen.splitmix64(0, np.arange(3, dtype=np.uint64))
    assert [int(v) for v in x] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_er_gnm_exact_and_deterministic():
    g1 = gen.erdos_renyi_gnm(500, 2000, 7)
    g2 = gen.erdos_renyi_gnm(500, 2000, 7)
    assert np.array_equal(g1.src, g2.src) and np.array_equal(g1.dst, g2.dst)
    assert g1.m_input == 2000
    assert np.all(g1.src < g1.dst)                   # canonical, no loops
    keys = g1.src.astype(np.int64) * 500 + g1.dst
    assert np.unique(keys).size == 2000              # distinct


def test_rmat_quadrant_frequencies():
    g = gen.rmat(12, 4, 3)
    # top-level bit frequencies follow (a+b, c+d) for src and (a+c, b+d) for dst
    top_s = (g.src >> 11) & 1
    top_d = (g.dst >> 11) & 1
    m = g.m_input
    for got, p in ((top_s.mean(), 0.24), (top_d.mean(), 0.24), ((top_s & top_d).mean(), 0.05)):
        assert abs(got - p) < 5 * np.sqrt(p * (1 - p) / m)
    assert g.src.max() < 4096 and g.dst.max() < 4096
    g2 = gen.rmat(12, 4, 3, chunk=1000)             # chunking does not change draws
    assert np.array_equal(g.src, g2.src) and np.array_equal(g.dst, g2.dst)


def test_rmat_thresholds():
    t1, t2, t3 = gen.rmat_thresholds()
    assert t1 == (57 * 2**32) // 100 and t2 == (76 * 2**32) // 100 and t3 == (95 * 2**32) // 100


def test_grid_shortcuts():
    g = gen.grid_with_shortcuts(30, 20, Fraction(1, 10), 15, 5)
    E = 29 * 20 + 30 * 19
    assert g.m_input == E - E // 10 + 15
    sc_s, sc_d = g.src[-15:], g.dst[-15:]
    d = np.abs(sc_s % 30 - sc_d % 30) + np.abs(sc_s // 30 - sc_d // 30)
    assert np.all(d > 1)


def test_largest_component_relabel():
    # two components: {0,1,2} and {3,4,5,6}; keep the second, relabelled 0..3
    src = np.array([0, 1, 3, 4, 5], np.int32)
    dst = np.array([1, 2, 4, 5, 6], np.int32)
    g = gen.largest_component(gen.Graph(7, src, dst, True))
    assert g.n == 4 and list(g.src) == [0, 1, 2] and list(g.dst) == [1, 2, 3]
    # a tie goes to the component holding the smallest id
    g = gen.largest_component(gen.Graph(4, np.array([2, 0], np.int32), np.array([3, 1], np.int32), True))
    assert g.n == 2 and list(g.src) == [0]


def test_seed_sampling():
    s = gen.sample_seeds(1000, 256, 1)
    assert s.size == 256 and np.unique(s).size == 256 and s.min() >= 0 and s.max() < 1000
    assert np.array_equal(s, gen.sample_seeds(1000, 256, 1))
    assert np.array_equal(np.sort(gen.sample_seeds(10, 10, 3)), np.arange(10))


def test_workload_er_shape():
    g, seeds = gen.workload_er(1)
    assert 9000 < g.n <= 10000 and seeds.size == 64 and np.unique(seeds).size == 64


def test_native_rmat_matches_numpy():
    """The C generator and the numpy one give the same edge list."""
    for scale, ef, seed in [(10, 8, 3), (13, 16, 1), (14, 4, 99)]:
        a = gen.rmat(scale, ef, seed, native=False, chunk=1 << 12)
        b = gen.rmat(scale, ef, seed, native=True)
        assert np.array_equal(a.src, b.src) and np.array_equal(a.dst, b.dst)
