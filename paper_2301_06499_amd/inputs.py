"""Seeded synthetic graph and seed-set generators.

This module is the only code shared by the HIP path's tests/benchmark and the
CPU oracle: it produces edge lists and seed lists, and holds none of the
propagation or estimation arithmetic.

Every random draw comes from SplitMix64 (Steele, Lea and Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014) used in its
counter-based form: draw ``i`` of stream ``seed`` is
``mix64(seed + (i + 1) * 0x9E3779B97F4A7C15)`` where ``mix64`` is the
variant-13 finaliser (shifts 30/27/31).  A draw is therefore a pure function
of (seed, i), so results do not depend on batch sizes or thread counts.

The paper's evaluation graphs (social networks and web crawls) are not
available; these generators are stand-ins with the same structural regimes:
R-MAT for heavy-tailed directed graphs, 2-D grids with shortcuts for long
diameters, Erdos-Renyi for the small case, and closed-form graphs (path,
cycle, star, complete) for checks.

Edge lists are returned as ``(src, dst)`` int32 numpy arrays.  For undirected
graphs each edge appears once; callers pass the ``undirected`` flag to the
consumer, which adds the reverse arc.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from fractions import Fraction

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK32 = np.uint64(0xFFFFFFFF)


def splitmix64(seed: int, idx) -> np.ndarray:
    """Counter-based SplitMix64: draw number ``idx`` (array of uint64) of stream ``seed``."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (idx + np.uint64(1)) * GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def subseed(seed: int, tag: int) -> int:
    """Independent stream seed for a given purpose (tag) of a generator seed."""
    return int(splitmix64(seed, np.array([tag], dtype=np.uint64))[0])


def _below(x32: np.ndarray, n: int) -> np.ndarray:
    """Map uniform 32-bit draws to [0, n) by multiply-high (bias <= n / 2^32)."""
    return ((x32 & _MASK32) * np.uint64(n)) >> np.uint64(32)


@dataclass
class Graph:
    """An edge list plus the facts consumers need to interpret it."""
    n: int
    src: np.ndarray
    dst: np.ndarray
    undirected: bool
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m_input(self) -> int:
        return int(self.src.shape[0])


# --------------------------------------------------------------------------
# closed-form graphs
# --------------------------------------------------------------------------

def path_graph(nodes: int, directed: bool = False) -> Graph:
    """Path 0-1-...-(nodes-1); directed form has arcs i -> i+1."""
    i = np.arange(max(nodes - 1, 0), dtype=np.int32)
    return Graph(nodes, i, i + 1, not directed, f"path{nodes}{'d' if directed else ''}")


def cycle_graph(nodes: int, directed: bool = False) -> Graph:
    i = np.arange(nodes, dtype=np.int32)
    return Graph(nodes, i, ((i + 1) % nodes).astype(np.int32), not directed,
                 f"cycle{nodes}{'d' if directed else ''}")


def star_graph(nodes: int) -> Graph:
    """Hub 0 joined to leaves 1..nodes-1 (undirected)."""
    leaves = np.arange(1, nodes, dtype=np.int32)
    return Graph(nodes, np.zeros_like(leaves), leaves, True, f"star{nodes}")


def complete_graph(nodes: int) -> Graph:
    u, v = np.triu_indices(nodes, k=1)
    return Graph(nodes, u.astype(np.int32), v.astype(np.int32), True, f"complete{nodes}")


def grid_graph(a: int, b: int) -> Graph:
    """a x b 4-neighbour lattice; node (x, y) has id y*a + x."""
    return _lattice(a, b)


def _lattice(a: int, b: int) -> Graph:
    ids = np.arange(a * b, dtype=np.int64).reshape(b, a)
    hs, hd = ids[:, :-1].ravel(), ids[:, 1:].ravel()
    vs, vd = ids[:-1, :].ravel(), ids[1:, :].ravel()
    src = np.concatenate([hs, vs]).astype(np.int32)
    dst = np.concatenate([hd, vd]).astype(np.int32)
    return Graph(a * b, src, dst, True, f"grid{a}x{b}")


# --------------------------------------------------------------------------
# random graphs
# --------------------------------------------------------------------------

def _distinct_pairs(n: int, count: int, seed: int, reject=None, ordered=False):
    """Draw ``count`` distinct non-loop pairs uniformly, in draw order.

    Unordered pairs are canonicalised as (min, max).  ``reject(u, v)`` may
    veto extra pairs (vectorised, returns a bool mask of pairs to drop).
    """
    if count == 0:
        return np.zeros(0, np.int32), np.zeros(0, np.int32)
    keys_kept = np.zeros(0, dtype=np.int64)
    order_kept = np.zeros(0, dtype=np.int64)
    drawn = 0
    batch = max(1024, 2 * count)
    while keys_kept.shape[0] < count:
        idx = np.arange(drawn, drawn + batch, dtype=np.uint64)
        x = splitmix64(seed, idx)
        u = _below(x >> np.uint64(32), n).astype(np.int64)
        v = _below(x, n).astype(np.int64)
        ok = u != v
        if reject is not None:
            ok &= ~reject(u, v)
        if not ordered:
            u, v = np.minimum(u, v), np.maximum(u, v)
        keys = u * n + v
        order = idx.astype(np.int64)
        keys, order = keys[ok], order[ok]
        allk = np.concatenate([keys_kept, keys])
        allo = np.concatenate([order_kept, order])
        uk, first = np.unique(allk, return_index=True)
        sel = np.sort(first)
        keys_kept, order_kept = allk[sel], allo[sel]
        drawn += batch
    keys_kept = keys_kept[:count]
    return (keys_kept // n).astype(np.int32), (keys_kept % n).astype(np.int32)


def erdos_renyi_gnm(n: int, m: int, seed: int) -> Graph:
    """Undirected G(n, m): m distinct non-loop unordered pairs, uniform."""
    src, dst = _distinct_pairs(n, m, subseed(seed, 1))
    return Graph(n, src, dst, True, f"er_n{n}_m{m}_s{seed}")


def rmat_thresholds(a=Fraction(57, 100), b=Fraction(19, 100), c=Fraction(19, 100)):
    """Integer thresholds floor(p * 2^32) for the cumulative quadrant probabilities."""
    t1 = (a * 2**32).__floor__()
    t2 = ((a + b) * 2**32).__floor__()
    t3 = ((a + b + c) * 2**32).__floor__()
    return int(t1), int(t2), int(t3)


_GEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gen")
_GEN_SRC = os.path.join(_GEN_DIR, "rmat_gen.c")
_GEN_LIB = os.path.join(_GEN_DIR, "librmat_gen.so")
_gen_lib = None


def build_native(force: bool = True) -> str:
    """Compile the native R-MAT generator (plain C, pthreads) with gcc."""
    if force or not os.path.exists(_GEN_LIB):
        tmp = _GEN_LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-pthread", _GEN_SRC, "-o", tmp])
        os.replace(tmp, _GEN_LIB)
    return _GEN_LIB


def _native():
    global _gen_lib
    if _gen_lib is None:
        if not os.path.exists(_GEN_LIB):
            build_native(force=False)
        lib = ctypes.CDLL(_GEN_LIB)
        U64, P = ctypes.c_uint64, ctypes.c_void_p
        lib.rmat_edges.restype = ctypes.c_int
        lib.rmat_edges.argtypes = [ctypes.c_int, ctypes.c_int64, U64, U64, U64, U64, P, P, ctypes.c_int]
        _gen_lib = lib
    return _gen_lib


def _host_threads() -> int:
    try:
        return max(1, min(64, len(os.sched_getaffinity(0))))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def rmat(scale: int, edge_factor: int, seed: int, chunk: int = 1 << 22,
         a=Fraction(57, 100), b=Fraction(19, 100), c=Fraction(19, 100), native: bool | None = None) -> Graph:
    """Directed R-MAT edge list (Chakrabarti, Zhan, Faloutsos 2004), no noise.

    Edge k, level l (0 = most significant bit) uses the 32-bit half
    (high half for even l) of draw k*ceil(scale/2) + l//2, compared against
    integer thresholds; quadrant a=(0,0), b=(0,1), c=(1,0), d=(1,1) sets the
    (src, dst) bits at position scale-1-l.  Duplicates and self-loops are kept
    here; the consumer removes them.  ``native`` (default: from scale 15 on)
    uses the C generator of the same definition on every host core.
    """
    m = edge_factor << scale
    if native is None:
        native = scale >= 15
    if native:
        t = rmat_thresholds(a, b, c)
        src = np.empty(m, dtype=np.int32)
        dst = np.empty(m, dtype=np.int32)
        rc = _native().rmat_edges(scale, m, seed & 0xFFFFFFFFFFFFFFFF, t[0], t[1], t[2],
                                  src.ctypes.data_as(ctypes.c_void_p), dst.ctypes.data_as(ctypes.c_void_p),
                                  _host_threads())
        if rc != 0:
            raise RuntimeError(f"rmat_edges failed with {rc}")
        return Graph(1 << scale, src, dst, False, f"rmat{scale}_ef{edge_factor}_s{seed}",
                     {"scale": scale, "edge_factor": edge_factor})
    t1, t2, t3 = (np.uint64(t) for t in rmat_thresholds(a, b, c))
    per_edge = (scale + 1) // 2
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    for lo in range(0, m, chunk):
        hi = min(m, lo + chunk)
        k = np.arange(lo, hi, dtype=np.uint64) * np.uint64(per_edge)
        s = np.zeros(hi - lo, dtype=np.uint64)
        d = np.zeros(hi - lo, dtype=np.uint64)
        x = None
        for lvl in range(scale):
            if lvl % 2 == 0:
                x = splitmix64(seed, k + np.uint64(lvl // 2))
                u = x >> np.uint64(32)
            else:
                u = x & _MASK32
            bit = np.uint64(scale - 1 - lvl)
            sb = (u >= t2).astype(np.uint64)              # quadrants c, d
            db = ((u >= t1) & (u < t2)) | (u >= t3)       # quadrants b, d
            s |= sb << bit
            d |= db.astype(np.uint64) << bit
        src[lo:hi] = s.astype(np.int32)
        dst[lo:hi] = d.astype(np.int32)
    return Graph(1 << scale, src, dst, False, f"rmat{scale}_ef{edge_factor}_s{seed}",
                 {"scale": scale, "edge_factor": edge_factor})


def grid_with_shortcuts(a: int, b: int, delete_frac: Fraction, shortcuts: int, seed: int) -> Graph:
    """a x b lattice, exactly floor(delete_frac*E) edges removed, plus random shortcuts.

    Deleted edges are the floor(delete_frac*E) smallest (draw, index) keys.
    Shortcuts are distinct uniformly random pairs that are not lattice
    neighbours.
    """
    g = _lattice(a, b)
    E = g.src.shape[0]
    ndel = int((Fraction(delete_frac) * E).__floor__())
    keys = splitmix64(subseed(seed, 2), np.arange(E, dtype=np.uint64))
    order = np.lexsort((np.arange(E), keys))
    keep = np.ones(E, dtype=bool)
    keep[order[:ndel]] = False
    src, dst = g.src[keep], g.dst[keep]

    def adjacent(u, v):
        ux, uy = u % a, u // a
        vx, vy = v % a, v // a
        return (np.abs(ux - vx) + np.abs(uy - vy)) == 1

    su, sv = _distinct_pairs(a * b, shortcuts, subseed(seed, 3), reject=adjacent)
    return Graph(a * b, np.concatenate([src, su]).astype(np.int32),
                 np.concatenate([dst, sv]).astype(np.int32), True,
                 f"grid{a}x{b}_del{delete_frac}_sc{shortcuts}_s{seed}",
                 {"deleted": ndel, "shortcuts": shortcuts})


# --------------------------------------------------------------------------
# structure helpers (input preparation, not part of the method)
# --------------------------------------------------------------------------

def largest_component(g: Graph) -> Graph:
    """Keep the largest weakly connected component, relabelled stably by id.

    Ties between equally large components go to the one holding the smallest
    node id.
    """
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    n = g.n
    A = sp.coo_matrix((np.ones(g.src.shape[0], dtype=np.int8), (g.src, g.dst)), shape=(n, n)).tocsr()
    ncomp, lab = connected_components(A, directed=True, connection="weak")
    sizes = np.bincount(lab, minlength=ncomp)
    best = sizes.max()
    # smallest node id among the largest components
    first_node = np.full(ncomp, n, dtype=np.int64)
    np.minimum.at(first_node, lab, np.arange(n))
    cand = np.where(sizes == best)[0]
    comp = cand[np.argmin(first_node[cand])]
    keep = lab == comp
    newid = np.cumsum(keep) - 1
    em = keep[g.src] & keep[g.dst]
    return Graph(int(keep.sum()), newid[g.src[em]].astype(np.int32), newid[g.dst[em]].astype(np.int32),
                 g.undirected, g.name + "_lcc", dict(g.meta, n_before_lcc=n))


def sample_seeds(n: int, s: int, seed: int, distinct: bool = True) -> np.ndarray:
    """s seed node ids in [0, n), uniform; distinct ones by rejection, in draw order."""
    if distinct and s > n:
        raise ValueError("cannot draw more distinct seeds than nodes")
    st = subseed(seed, 4)
    if not distinct:
        x = splitmix64(st, np.arange(s, dtype=np.uint64))
        return _below(x >> np.uint64(32), n).astype(np.int32)
    out, seen, drawn = [], set(), 0
    while len(out) < s:
        x = splitmix64(st, np.arange(drawn, drawn + 4 * s + 16, dtype=np.uint64))
        drawn += 4 * s + 16
        for v in _below(x >> np.uint64(32), n).tolist():
            if v not in seen:
                seen.add(v)
                out.append(v)
                if len(out) == s:
                    break
    return np.asarray(out, dtype=np.int32)


# --------------------------------------------------------------------------
# the benchmark workloads
# --------------------------------------------------------------------------

def workload_er(seed: int = 1):
    """ER G(10000, 50000) undirected, largest component, 64 distinct seeds."""
    g = largest_component(erdos_renyi_gnm(10000, 50000, seed))
    return g, sample_seeds(g.n, 64, seed)


def workload_rmat(scale: int = 20, edge_factor: int = 16, s: int = 256, seed: int = 1):
    """Directed R-MAT (a,b,c,d = .57,.19,.19,.05), all 2^scale nodes kept, s seeds."""
    g = rmat(scale, edge_factor, subseed(seed, 5))
    return g, sample_seeds(g.n, s, seed)


def workload_grid_shortcuts(side: int = 4096, s: int = 128, seed: int = 1):
    """side x side lattice, 10% of edges deleted, 1000 shortcuts, largest component."""
    g = largest_component(grid_with_shortcuts(side, side, Fraction(1, 10), 1000, seed))
    return g, sample_seeds(g.n, s, seed)


def workload_batch(seed: int = 1, s: int = 64):
    """The 64 uneven graphs of the batched workload: R-MAT, grids and paths."""
    graphs = []
    for k in range(22):
        graphs.append(rmat(10 + k % 7, 8 + 4 * (k % 3), subseed(seed, 100 + k)))
    for k in range(21):
        side = 64 + (k * 448) // 20
        graphs.append(grid_graph(side, side))
    for k in range(21):
        graphs.append(path_graph(1000 + (k * 19000) // 20 + 1))
    seeds = [sample_seeds(g.n, s, subseed(seed, 200 + i)) for i, g in enumerate(graphs)]
    return graphs, seeds


def union_of(graphs, seeds):
    """A batch as one disjoint union: (n, src, dst, node_offsets, seeds) with
    every undirected edge written as its two arcs and graph k's node ids and
    seeds shifted by node_offsets[k] (input plumbing only)."""
    offs, srcs, dsts, sds = [0], [], [], []
    for g, sd in zip(graphs, seeds):
        src, dst = g.src.astype(np.int64), g.dst.astype(np.int64)
        if g.undirected:
            src, dst = np.concatenate([src, dst]), np.concatenate([dst, src])
        srcs.append(src + offs[-1])
        dsts.append(dst + offs[-1])
        sds.append(np.asarray(sd, dtype=np.int64) + offs[-1])
        offs.append(offs[-1] + g.n)
    cat = (lambda xs: np.concatenate(xs).astype(np.int32)) if graphs else (lambda xs: np.zeros(0, np.int32))
    return offs[-1], cat(srcs), cat(dsts), offs, cat(sds)
