"""CPU oracle for PROPAGATE-P seed-bitset propagation.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package's ``smoke()`` check and
the benchmark's CPU-baseline leg may import this package.  The product (the
HIP library and its binding) never calls it, and the two share no code: the
only common inputs come from the seeded generators, which hold none of the
method's arithmetic.

Contents
--------
``propagate``       per-seed BFS (plain C, ``bfs_oracle.c``): exact per-round
                    counts c[r], per-seed counts c_i[r], signatures at chosen
                    rounds, final signatures.  Paper: Section 3 definitions of
                    N(u, r) and d(u, v); Algorithm 1 (PROPAGATE-P).
``metrics``         the estimators of Algorithm 1's closing steps and of the
                    Section 3 definitions, in exact integer arithmetic with one
                    final rounding per value.
``dense_rounds``    the ball recurrence of Section 4 on a dense boolean
                    signature matrix, one boolean matrix product per round
                    (numpy), used to cross-check the BFS form on small graphs.
``brute_force_counts``  all-pairs distances by repeated boolean matrix
                    products, for tiny graphs.
``node_stats``      (module ``oracle.node_stats``) per-node reach counts and
                    distance sums to the seeds, from the BFS distances.
``progressive``     (module ``oracle.progressive``) seed groups added until a
                    Hoeffding half-width of the average distance meets a
                    target (Section 4 error bounds).
``propagate_s``     (module ``oracle.propagate_s``) Algorithm 2, PROPAGATE-S:
                    one seed at a time with one bit per node and the early
                    break, pure Python, for small graphs.

Parity pins for each function live in ``tests/test_oracle_*.py``.  The
paper's own algorithm returns the integer effective diameter; the
interpolated form (linear between hops) is a reading of the fractional values
its tables print, with no worked value to check against; its arithmetic is
pinned against numpy.interp, which inverts the piecewise-linear cumulative
pair count independently.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bfs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain C11 + pthreads)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-pthread",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_propagate.restype = ctypes.c_int
        lib.oracle_propagate.argtypes = [ctypes.c_int64, ctypes.c_int64, P, P, ctypes.c_int32,
                                         ctypes.c_int32, P, ctypes.c_int32, ctypes.c_int32,
                                         P, ctypes.c_int32, P, P, P, ctypes.c_int32, P, P, P]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def default_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def propagate(n, src, dst, seeds, undirected, transpose=False, sig_rounds=(),
              seed_counts=False, final_sig=False, dist=False, nthreads=None, cap=None):
    """Exact PROPAGATE-P outputs by one BFS per seed.

    Returns a dict with ``counts`` (int64 [D+1], c[0..D]), ``D``,
    optionally ``seed_counts`` (uint32 [D+1][s]), ``sigs`` (uint64
    [len(sig_rounds)][n][W]), ``final_sig`` (uint64 [n][W]) and ``dist``
    (int32 [s][n], d(u, x_i) or -1).
    Bit i of a signature is word i >> 6, bit i & 63 (least significant first).
    """
    lib = _load()
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    seeds = np.ascontiguousarray(seeds, dtype=np.int32)
    s = int(seeds.shape[0])
    W = (s + 63) // 64
    m = int(src.shape[0])
    if cap is None:
        cap = int(n) + 1
    cap = max(1, int(cap))
    counts = np.zeros(cap, dtype=np.int64)
    D = ctypes.c_int32(0)
    sc = np.zeros((cap, s), dtype=np.uint32) if seed_counts else None
    sr = np.ascontiguousarray(sig_rounds, dtype=np.int32)
    sg = np.zeros((len(sr), n, W), dtype=np.uint64) if len(sr) else None
    fs = np.zeros((n, W), dtype=np.uint64) if final_sig else None
    dd = np.zeros((s, n), dtype=np.int32) if dist else None
    nth = int(nthreads or default_threads())
    rc = lib.oracle_propagate(int(n), m, _ptr(src), _ptr(dst), int(bool(undirected)), int(bool(transpose)),
                              _ptr(seeds), s, nth, _ptr(counts), cap, ctypes.byref(D), _ptr(sc),
                              _ptr(sr) if len(sr) else None, len(sr), _ptr(sg), _ptr(fs), _ptr(dd))
    if rc != 0:
        raise RuntimeError(f"oracle_propagate failed with code {rc}")
    Dv = int(D.value)
    out = {"counts": counts[:Dv + 1].copy(), "D": Dv, "s": s, "n": int(n)}
    if sc is not None:
        out["seed_counts"] = sc[:Dv + 1].copy()
    if sg is not None:
        out["sigs"] = sg
    if fs is not None:
        out["final_sig"] = fs
    if dd is not None:
        out["dist"] = dd
    return out


# ---------------------------------------------------------------------------
# estimators
# ---------------------------------------------------------------------------

def metrics(counts, n: int, s: int, tau_num: int = 9, tau_den: int = 10) -> dict:
    """Distance metrics from per-round counts c[0..D], exact until one final rounding.

    Readings of the paper used here (Algorithm 1 closing steps; Section 3):
      * c[0] = s counts the seeds' own pairs; R[k] = c[0] + ... + c[k] is the
        number of (node, seed) pairs within distance k, so T = R[D] includes
        the s self-pairs.
      * diameter lower bound D = last round with new collisions.
      * effective diameter: least k with R[k] >= tau * R[D], tau = tau_num /
        tau_den compared exactly; the interpolated form places the crossing
        linearly between k-1 and k.
      * reachable pairs: (n / s) * R[D] (self-pairs included).
      * connectivity rate alpha: pairs u != v over n (n - 1), i.e.
        (T - s) / (s (n - 1)); 0 when n = 1.
      * average distance over pairs u != v: sum_r r c[r] / (T - s); the form
        that keeps the self-pairs in the denominator (as Algorithm 1's final
        division does) is ``avg_dist_paper`` = sum_r r c[r] / T.
    Every ratio is formed from exact Python integers and rounded to double
    once per operand conversion exactly as written below.
    """
    c = [int(x) for x in counts]
    if len(c) == 0:
        raise ValueError("counts must hold at least c[0]")
    if s <= 0 or n <= 0 or tau_den <= 0 or tau_num < 0 or tau_num > tau_den:
        raise ValueError("invalid metric arguments")
    # D: last round with new collisions
    D = 0
    for r, x in enumerate(c):
        if x > 0:
            D = r
    R = []
    acc = 0
    for x in c[:D + 1]:
        acc += x
        R.append(acc)
    T = R[D]
    P1 = T - s
    Sd = sum(r * c[r] for r in range(1, D + 1))
    # effective diameter, exact comparison
    k_star = D
    for k in range(D + 1):
        if tau_den * R[k] >= tau_num * T:
            k_star = k
            break
    if k_star == 0:
        eff_interp = 0.0
    else:
        num = tau_num * T - tau_den * R[k_star - 1]
        den = tau_den * (R[k_star] - R[k_star - 1])
        eff_interp = float(k_star - 1) + float(num) / float(den)
    return {
        "diameter": D,
        "eff_diam": float(k_star),
        "eff_diam_interp": eff_interp,
        "avg_dist": (float(Sd) / float(P1)) if P1 > 0 else 0.0,
        "avg_dist_paper": (float(Sd) / float(T)) if T > 0 else 0.0,
        "reachable_pairs": float(n * T) / float(s),
        "alpha": (float(P1) / float(s * (n - 1))) if n > 1 else 0.0,
        "R_final": T,
        "rounds_executed": D + 1,
    }


# ---------------------------------------------------------------------------
# cross-check implementations
# ---------------------------------------------------------------------------

def dense_rounds(n, src, dst, seeds, undirected, transpose=False, max_rounds=None):
    """The ball recurrence of Section 4 on a dense boolean signature matrix.

    Sig_0[u, i] = [u = x_i]; Sig_r = Sig_{r-1} OR (A Sig_{r-1} > 0) with
    A[u, v] = 1 for every arc u -> v (u keeps its own ball, as Algorithm 1's
    update does), and c[r] = the number of bits Sig_r has that Sig_{r-1}
    lacks, until a round adds none.  Hops are numbered from 1 with c[0] = s.
    Returns (counts, the signature matrices after each round, from round 0 up
    to and including the round that added nothing).
    """
    seeds = np.asarray(seeds, dtype=np.int64)
    s = seeds.shape[0]
    A = np.zeros((n, n), dtype=np.int64)
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    a, b = (dst, src) if transpose else (src, dst)
    A[a, b] = 1
    if undirected:
        A[b, a] = 1
    sig = np.zeros((n, s), dtype=bool)
    sig[seeds, np.arange(s)] = True
    counts = [s]
    history = [sig.copy()]
    cap = max_rounds if max_rounds is not None else n + 1
    for _ in range(cap):
        nxt = sig | ((A @ sig.astype(np.int64)) > 0)
        added = int(np.count_nonzero(nxt & ~sig))
        sig = nxt
        history.append(sig.copy())
        if added == 0:
            break
        counts.append(added)
    return np.asarray(counts, dtype=np.int64), history


def brute_force_counts(n, src, dst, seeds, undirected, transpose=False):
    """c[r] from all-pairs distances computed by boolean matrix powers.

    reach_k[u, v] = there is a walk u -> v of length <= k.  d(u, v) is the
    least k with reach_k[u, v]; c[r] counts pairs (u, x_i) at distance r.
    """
    A = np.zeros((n, n), dtype=bool)
    for u, v in zip(np.asarray(src).tolist(), np.asarray(dst).tolist()):
        A[u, v] = True
        if undirected:
            A[v, u] = True
    if transpose:
        A = A.T.copy()
    dist = np.full((n, n), -1, dtype=np.int64)
    reach = np.eye(n, dtype=bool)
    dist[reach] = 0
    k = 0
    while True:
        k += 1
        nxt = reach | ((reach.astype(np.int64) @ A.astype(np.int64)) > 0)
        newly = nxt & ~reach
        if not newly.any():
            break
        dist[newly] = k
        reach = nxt
    cols = dist[:, np.asarray(seeds, dtype=np.int64)]
    D = int(cols.max()) if cols.size else 0
    counts = np.array([int(np.count_nonzero(cols == r)) for r in range(D + 1)], dtype=np.int64)
    return counts, dist


def bits_from_matrix(sig_bool) -> np.ndarray:
    """Pack an [n][s] boolean matrix into [n][W] uint64 words (bit i -> word i>>6, bit i&63)."""
    n, s = sig_bool.shape
    W = (s + 63) // 64
    out = np.zeros((n, W), dtype=np.uint64)
    for i in range(s):
        out[:, i >> 6] |= sig_bool[:, i].astype(np.uint64) << np.uint64(i & 63)
    return out


def tau_fraction(tau_num: int, tau_den: int) -> Fraction:
    return Fraction(tau_num, tau_den)
