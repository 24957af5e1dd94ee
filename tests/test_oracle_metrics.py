"""Pins for the oracle's estimators (Algorithm 1 closing steps, Section 3 metrics)."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2301_06499_amd import inputs as gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_kv(path):
    out = {}
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if "=" in line:
            k, v = (x.strip() for x in line.split("=", 1))
            out[k] = int(v)
    return out


def _graph(kind, n):
    return {"path": gen.path_graph, "cycle": gen.cycle_graph, "star": gen.star_graph,
            "complete": gen.complete_graph}[kind](n)


def test_closed_form_average_distance_and_diameter():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "closed_forms.txt"))
            if l.strip() and not l.startswith("#")]
    for kind, n, num, den, diam in rows:
        n, num, den, diam = int(n), int(num), int(den), int(diam)
        g = _graph(kind, n)
        out = oracle.propagate(g.n, g.src, g.dst, np.arange(n, dtype=np.int32), True)
        m = oracle.metrics(out["counts"], n, n)
        assert m["diameter"] == diam, kind
        assert m["avg_dist"] == float(num) / float(den) or math.isclose(m["avg_dist"], num / den, rel_tol=1e-15)
        assert m["alpha"] == 1.0
        assert m["reachable_pairs"] == float(n * n)
        # self-pairs kept in the denominator: sum d / n^2
        sd = Fraction(num, den) * n * (n - 1)
        assert math.isclose(m["avg_dist_paper"], float(sd / (n * n)), rel_tol=1e-15)


def test_twitch_pairs_pin():
    """A connected undirected graph gives (n/s) R[D] = n^2 for any seed set.

    Uses the paper's printed Twitch figures: n = 168114 and 28262316996 pairs.
    The graph is a stand-in with the same n (a star; any connected undirected
    graph has the same pair count); the seeds are 256 uniform nodes.
    """
    gd = _read_kv(os.path.join(GOLDEN, "twitch_reachable_pairs.txt"))
    n = gd["n"]
    assert gd["exact_pairs"] == n * n
    # a star spans all n nodes with diameter 2, which keeps the 256 searches cheap
    hub = np.zeros(n - 1, dtype=np.int32)
    leaves = np.arange(1, n, dtype=np.int32)
    seeds = gen.sample_seeds(n, gd["seeds"], 11)
    out = oracle.propagate(n, hub, leaves, seeds, True)
    m = oracle.metrics(out["counts"], n, gd["seeds"])
    assert m["reachable_pairs"] == float(gd["exact_pairs"]) == float(gd["propagate_s_pairs"])
    assert m["alpha"] == float(gd["alpha"])


def test_effective_diameter_exact_threshold():
    # R = [10, 40, 90, 100]: tau*T = 90 -> k* = 2 exactly at the boundary
    m = oracle.metrics([10, 30, 50, 10], n=50, s=10)
    assert m["eff_diam"] == 2.0
    assert m["diameter"] == 3
    assert m["eff_diam_interp"] == 1.0 + (90 - 40) / (10 * 5)   # = 2.0, crossing exactly at 2
    m = oracle.metrics([10, 30, 49, 11], n=50, s=10)           # R[2] = 89 < 90
    assert m["eff_diam"] == 3.0
    assert m["eff_diam_interp"] == 2.0 + float(900 - 890) / float(10 * 11)
    # tau = 1 gives the diameter (Thm 3 proof: diameter = effective diameter at tau 1)
    m = oracle.metrics([4, 8, 0, 0], n=20, s=4, tau_num=1, tau_den=1)
    assert m["eff_diam"] == 1.0 == m["diameter"]


@pytest.mark.parametrize("case", range(6))
def test_interpolated_eff_diam_is_the_inverse_of_the_cumulative_count(case):
    """The interpolated effective diameter is the hop at which the piecewise-linear
    cumulative pair count R (hops 0..D, linear between hops) reaches tau R[D]: the
    library routine numpy.interp inverts it independently of the oracle's exact
    integer arithmetic.  R is strictly increasing up to D (a pair at distance d puts
    pairs at every shorter distance on its path), as numpy.interp needs."""
    g, seeds = [
        (gen.erdos_renyi_gnm(300, 700, 3), gen.sample_seeds(300, 40, 1)),
        (gen.rmat(10, 8, 4), gen.sample_seeds(1024, 64, 2)),
        (gen.grid_graph(20, 13), gen.sample_seeds(260, 30, 3)),
        (gen.path_graph(77), gen.sample_seeds(77, 77, 4)),
        (gen.cycle_graph(40, directed=True), gen.sample_seeds(40, 9, 5)),
        (gen.star_graph(50), gen.sample_seeds(50, 12, 6))][case]
    g_n = g.n
    out = oracle.propagate(g_n, g.src, g.dst, seeds, g.undirected)
    counts = out["counts"]
    R = np.cumsum(counts)
    assert np.all(np.diff(R) > 0)
    hops = np.arange(len(R), dtype=np.float64)
    for num, den in [(9, 10), (1, 2), (99, 100), (1, 3), (1, 1)]:
        m = oracle.metrics(counts, g_n, len(seeds), num, den)
        want = float(np.interp(num / den * float(R[-1]), R.astype(np.float64), hops))
        assert m["eff_diam_interp"] == pytest.approx(want, rel=1e-12, abs=1e-12), (num, den)


def test_interpolated_eff_diam_monotone_in_tau():
    g, seeds = gen.workload_er(seed=2)
    out = oracle.propagate(g.n, g.src, g.dst, seeds, True)
    prev = -1.0
    for num in range(1, 20):
        m = oracle.metrics(out["counts"], g.n, len(seeds), num, 20)
        assert m["eff_diam_interp"] >= prev
        assert m["eff_diam_interp"] <= m["eff_diam"] <= m["eff_diam_interp"] + 1
        prev = m["eff_diam_interp"]


def test_metric_edge_cases():
    m = oracle.metrics([3], n=7, s=3)          # isolated seeds
    assert m["diameter"] == 0 and m["avg_dist"] == 0.0 and m["alpha"] == 0.0
    assert m["eff_diam"] == 0.0 and m["reachable_pairs"] == 7.0 and m["rounds_executed"] == 1
    m = oracle.metrics([1], n=1, s=1)
    assert m["alpha"] == 0.0 and m["reachable_pairs"] == 1.0
    with pytest.raises(ValueError):
        oracle.metrics([1], n=1, s=0)
    with pytest.raises(ValueError):
        oracle.metrics([1, 2], n=4, s=1, tau_num=11, tau_den=10)
    # trailing zero rounds do not change anything
    a = oracle.metrics([5, 7, 3], n=40, s=5)
    b = oracle.metrics([5, 7, 3, 0, 0], n=40, s=5)
    assert a == b


def test_exact_mode_equals_all_pairs():
    """s = n: estimates equal the all-pairs values (exact neighbourhood function)."""
    rng = np.random.default_rng(3)
    n = 40
    src = rng.integers(0, n, 70).astype(np.int32)
    dst = rng.integers(0, n, 70).astype(np.int32)
    seeds = np.arange(n, dtype=np.int32)
    out = oracle.propagate(n, src, dst, seeds, False)
    _, dist = oracle.brute_force_counts(n, src, dst, seeds, False)
    reach = dist >= 0
    off = reach & ~np.eye(n, dtype=bool)
    m = oracle.metrics(out["counts"], n, n)
    assert m["reachable_pairs"] == float(reach.sum())
    assert m["alpha"] == float(off.sum()) / float(n * (n - 1))
    assert m["avg_dist"] == float(dist[off].sum()) / float(off.sum())
    assert m["diameter"] == int(dist.max())


@pytest.mark.slow
def test_theorem3_error_bounds_hold():
    """Hoeffding bounds of Theorem 3 on a 2000-node ER graph (statistical, loose).

    With eps = sqrt(ln n / s): |avg error| <= eps * Delta / alpha,
    |alpha error| <= eps, |eff. diameter error| <= eps / alpha~.
    Each holds with probability >= 1 - 2/n^2; 5 seed draws are checked.
    """
    g = gen.largest_component(gen.erdos_renyi_gnm(2000, 6000, 9))
    n = g.n
    full = oracle.propagate(n, g.src, g.dst, np.arange(n, dtype=np.int32), True)
    ex = oracle.metrics(full["counts"], n, n)
    for trial in range(5):
        s = 128
        seeds = gen.sample_seeds(n, s, 50 + trial)
        est = oracle.metrics(oracle.propagate(n, g.src, g.dst, seeds, True)["counts"], n, s)
        eps = math.sqrt(math.log(n) / s)
        alpha = ex["alpha"]
        at = alpha * (n - 1) / n
        assert abs(est["avg_dist"] - ex["avg_dist"]) <= eps * ex["diameter"] / alpha
        assert abs(est["alpha"] - alpha) <= eps
        assert abs(est["eff_diam_interp"] - ex["eff_diam_interp"]) <= eps / at
        assert abs(est["diameter"] - ex["diameter"]) <= ex["diameter"]   # lower bound only
        assert est["diameter"] <= ex["diameter"]
