"""ctypes binding of libpp.so with the C interface's entry-point names.

Argument marshalling only: every step of the propagation runs in the HIP
library.  Loading fails loudly if the library has not been built; there is
no fallback.  Host arrays are numpy; device arrays may be torch tensors
(their data pointers are passed through) and streams are torch streams or
raw hipStream_t integers.
"""
from __future__ import annotations

import ctypes
import os
import sys
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpp.so")

PP_OK, PP_EINVAL, PP_ERANGE, PP_ENOMEM, PP_EDEVICE, PP_ENOTCONV, PP_ESTATE = 0, -1, -2, -3, -4, -5, -6
PP_UNDIRECTED, PP_INPUT_ON_DEVICE, PP_TRANSPOSE, PP_KEEP_ORDER = 1, 2, 4, 8
PP_BUILD_ON_HOST, PP_BUILD_ON_DEVICE, PP_HUBS_ONLY = 16, 32, 64
DEVICE_BUILD_MIN = 1 << 20
PP_SCHED_HEURISTIC, PP_SCHED_PULL, PP_SCHED_PUSH, PP_SCHED_FUZZ, PP_SCHED_MLP, PP_SCHED_PLAN = 0, 1, 2, 3, 4, 5
PP_GROUPS_BY_REACH, PP_ORDER_BY_REACH = -1, 1
MODE_PULL, MODE_PUSH, MODE_INIT, MODE_SPULL, MODE_PUSH_FLAT = 0, 1, 2, 3, 4   # entries of the per-round mode log
_NAMES = {0: "PP_OK", -1: "PP_EINVAL", -2: "PP_ERANGE", -3: "PP_ENOMEM", -4: "PP_EDEVICE",
          -5: "PP_ENOTCONV", -6: "PP_ESTATE"}


class PPError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("scheduler", ctypes.c_int32), ("seed_counts", ctypes.c_int32), ("max_rounds", ctypes.c_int32),
                ("rounds_per_sync", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("push_div", ctypes.c_int32),
                ("fuzz_seed", ctypes.c_uint64), ("time_kernels", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("pull_k", ctypes.c_int32), ("node_stats", ctypes.c_int32), ("sparse_pull", ctypes.c_int32),
                ("seed_groups", ctypes.c_int32), ("seed_order", ctypes.c_int32)]


class TuneEntry(ctypes.Structure):
    _fields_ = [("pull_k", ctypes.c_int32), ("push_div", ctypes.c_int32), ("rounds_per_sync", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("sparse_pull", ctypes.c_int32), ("ms", ctypes.c_float)]


class Progress(ctypes.Structure):
    _fields_ = [("seeds", ctypes.c_int32), ("groups", ctypes.c_int32), ("met", ctypes.c_int32), ("D", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("eps", ctypes.c_double), ("bound", ctypes.c_double)]


class Metrics(ctypes.Structure):
    _fields_ = [("diameter", ctypes.c_int32), ("rounds_executed", ctypes.c_int32), ("R_final", ctypes.c_int64),
                ("eff_diam", ctypes.c_double), ("eff_diam_interp", ctypes.c_double), ("avg_dist", ctypes.c_double),
                ("avg_dist_paper", ctypes.c_double), ("reachable_pairs", ctypes.c_double),
                ("alpha", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = ["pp_options_default", "pp_csr_build", "pp_graph_arcs", "pp_graph_nodes", "pp_graph_count",
           "pp_graph_get_csr",
           "pp_seeds_init", "pp_propagate_round", "pp_propagate_until_converged", "pp_estimate_metrics",
           "pp_get_signatures", "pp_get_seed_counts", "pp_run_round", "pp_run_words", "pp_get_round_log",
           "pp_run_snapshot", "pp_run_restore", "pp_run_free", "pp_graph_free", "pp_last_error",
           "pp_seeds_reset", "pp_get_kernel_times", "pp_run_set_mlp", "pp_get_round_features",
           "pp_time_round", "pp_mlp_forward", "pp_mlp_loss_grad", "pp_mlp_train", "pp_autotune", "pp_exact_counts",
           "pp_propagate_s", "pp_progressive_sample", "pp_get_node_stats", "pp_set_allocator",
           "pp_propagate_s_noalloc", "pp_run_groups", "pp_run_group_words", "pp_get_group_log",
           "pp_run_set_plan", "pp_get_round_times"]

MLP_IN, MLP_HID, MLP_OUT = 8, 32, 4
MLP_PARAMS = MLP_HID * MLP_IN + MLP_HID + MLP_HID * MLP_HID + MLP_HID + MLP_OUT * MLP_HID + MLP_OUT   # 1476

_lib = None


def lib():
    """The loaded library; raises if libpp.so is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2301_06499_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    sig = {
        "pp_options_default": (None, [P]),
        "pp_csr_build": (ctypes.c_int, [I64, I64, P, P, U32, P, I32, P, P]),
        "pp_graph_arcs": (I64, [P]), "pp_graph_nodes": (I64, [P]), "pp_graph_count": (I32, [P]),
        "pp_graph_get_csr": (ctypes.c_int, [P, P, P, P, P, P]),
        "pp_seeds_init": (ctypes.c_int, [P, P, I32, P, P, P]),
        "pp_propagate_round": (ctypes.c_int, [P, P, P]),
        "pp_propagate_until_converged": (ctypes.c_int, [P, I32, P, I32, P]),
        "pp_estimate_metrics": (ctypes.c_int, [P, I32, I64, I32, U32, U32, P]),
        "pp_get_signatures": (ctypes.c_int, [P, P, I32]),
        "pp_get_seed_counts": (ctypes.c_int, [P, P, I32]),
        "pp_run_round": (I32, [P]), "pp_run_words": (I32, [P]),
        "pp_run_groups": (I32, [P]), "pp_run_group_words": (I32, [P]),
        "pp_get_group_log": (ctypes.c_int, [P, I32, P, P, I32]),
        "pp_run_set_plan": (ctypes.c_int, [P, P, I32]),
        "pp_get_round_times": (ctypes.c_int, [P, P, I32]),
        "pp_get_round_log": (ctypes.c_int, [P, P, P, I32]),
        "pp_run_snapshot": (ctypes.c_int, [P, P]), "pp_run_restore": (ctypes.c_int, [P, P]),
        "pp_run_free": (None, [P]), "pp_graph_free": (None, [P]),
        "pp_last_error": (ctypes.c_char_p, []),
        "pp_seeds_reset": (ctypes.c_int, [P, P, I32]),
        "pp_get_kernel_times": (ctypes.c_int, [P, P, I32]),
        "pp_run_set_mlp": (ctypes.c_int, [P, P]),
        "pp_get_round_features": (ctypes.c_int, [P, P, I32]),
        "pp_time_round": (ctypes.c_int, [P, I32, P, P]),
        "pp_mlp_forward": (ctypes.c_int, [P, P, I64, P]),
        "pp_mlp_loss_grad": (ctypes.c_int, [P, P, P, I64, P, P]),
        "pp_mlp_train": (ctypes.c_int, [P, P, P, I64, I32, ctypes.c_float, P]),
        "pp_autotune": (ctypes.c_int, [P, P, I32, P, I32, P, P, I32, P]),
        "pp_exact_counts": (ctypes.c_int, [P, I32, P, P, I32, P]),
        "pp_propagate_s": (ctypes.c_int, [P, P, I32, I32, P, P, I32, P, P]),
        "pp_propagate_s_noalloc": (ctypes.c_int, [P, P, I32, I32, P, P, I32, P, P]),
        "pp_progressive_sample": (ctypes.c_int, [P, P, I32, I32, ctypes.c_double, ctypes.c_double, P, P, I32, P]),
        "pp_get_node_stats": (ctypes.c_int, [P, P, P]),
        "pp_set_allocator": (ctypes.c_int, [P, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def hip_runtime() -> str | None:
    """Path of the HIP runtime library mapped into this process (the one libpp.so
    calls): a process that loads PyTorch first binds the library to PyTorch's
    bundled copy, otherwise the system's.  None when none is mapped yet."""
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64" in line:
                    return line.split()[-1]
    except OSError:
        pass
    return None


def _check(rc: int):
    if rc != PP_OK:
        raise PPError(rc, lib().pp_last_error().decode())


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(int(stream.cuda_stream))


def _is_device(a) -> bool:
    return hasattr(a, "is_cuda") and a.is_cuda


def options(scheduler=PP_SCHED_HEURISTIC, seed_counts=False, max_rounds=0, rounds_per_sync=0,
            use_graph=True, push_div=0, fuzz_seed=0, time_kernels=False, persistent=False, pull_k=0,
            node_stats=False, sparse_pull=0, seed_groups=0, seed_order=0) -> Options:
    o = Options()
    lib().pp_options_default(ctypes.byref(o))
    o.scheduler = scheduler
    o.seed_counts = int(bool(seed_counts))
    o.max_rounds = int(max_rounds)
    o.rounds_per_sync = int(rounds_per_sync)
    o.use_graph = int(bool(use_graph))
    if push_div:
        o.push_div = int(push_div)
    o.fuzz_seed = int(fuzz_seed)
    o.time_kernels = int(bool(time_kernels))
    o.persistent = int(bool(persistent))
    o.pull_k = int(pull_k)
    o.node_stats = int(bool(node_stats))
    o.sparse_pull = int(sparse_pull)
    o.seed_groups = int(seed_groups)
    o.seed_order = int(seed_order)
    return o


class Graph:
    """Owns a pp_graph handle (device CSR, predecessor lists, tiling)."""

    def __init__(self, handle):
        self._h = handle

    @property
    def handle(self):
        return self._h

    @property
    def arcs(self) -> int:
        return int(lib().pp_graph_arcs(self._h))

    @property
    def nodes(self) -> int:
        return int(lib().pp_graph_nodes(self._h))

    @property
    def count(self) -> int:
        return int(lib().pp_graph_count(self._h))

    def free(self):
        if self._h:
            lib().pp_graph_free(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter shutdown the HIP runtime (and a profiler's hooks) may
        # already be going away: leave the memory to the process's end then
        # (the check is bound here: the module's globals may be gone by then)
        if _finalizing():
            return
        try:
            self.free()
        except Exception:
            pass


def pp_csr_build(n, src, dst, undirected=False, transpose=False, node_offsets=None, stream=None,
                 keep_order=False, build="auto", hubs_only=False) -> Graph:
    """Build the device graph from m arcs src[k] -> dst[k] (numpy int32 or device tensors).
    build: "auto" (the library's choice by size), "host" or "device".
    hubs_only: the high-degree nodes first, the others in input order (no
    breadth-first numbering; a faster build)."""
    if build not in ("auto", "host", "device"):
        raise ValueError("build must be 'auto', 'host' or 'device'")
    flags = ((PP_UNDIRECTED if undirected else 0) | (PP_TRANSPOSE if transpose else 0) |
             (PP_KEEP_ORDER if keep_order else 0) | (PP_HUBS_ONLY if hubs_only else 0) |
             {"auto": 0, "host": PP_BUILD_ON_HOST, "device": PP_BUILD_ON_DEVICE}[build])
    keep = []
    if _is_device(src):
        flags |= PP_INPUT_ON_DEVICE
        m = int(src.numel())
        ps, pd = ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr())
    else:
        s = np.ascontiguousarray(src, dtype=np.int32)
        d = np.ascontiguousarray(dst, dtype=np.int32)
        keep += [s, d]
        m = int(s.shape[0])
        ps, pd = _np_ptr(s), _np_ptr(d)
    if node_offsets is not None:
        off = np.ascontiguousarray(node_offsets, dtype=np.int64)
        keep.append(off)
        po, G = _np_ptr(off), int(off.shape[0] - 1)
    else:
        po, G = None, 1
    h = ctypes.c_void_p()
    _check(lib().pp_csr_build(int(n), m, ps, pd, flags, po, G, _stream_ptr(stream), ctypes.byref(h)))
    return Graph(h)


def pp_graph_get_csr(graph: Graph):
    """(rp, col, trp, tcol, perm) of the stored adjacency, host copies (storage order)."""
    n, m = graph.nodes, graph.arcs
    rp = np.zeros(n + 1, np.int64)
    col = np.zeros(max(m, 1), np.int32)
    trp = np.zeros(n + 1, np.int64)
    tcol = np.zeros(max(m, 1), np.int32)
    perm = np.zeros(n, np.int32)
    _check(lib().pp_graph_get_csr(graph.handle, _np_ptr(rp), _np_ptr(col), _np_ptr(trp), _np_ptr(tcol),
                                  _np_ptr(perm)))
    return rp, col[:m], trp, tcol[:m], perm


class Run:
    """Owns a pp_run handle (signatures, frontier, per-round logs)."""

    def __init__(self, handle, graph: Graph, s: int, opts: Options):
        self._h = handle
        self.graph = graph
        self.s = s
        self.opts = opts

    @property
    def handle(self):
        return self._h

    @property
    def round(self) -> int:
        return int(lib().pp_run_round(self._h))

    @property
    def words(self) -> int:
        return int(lib().pp_run_words(self._h))

    @property
    def groups(self) -> int:
        return int(lib().pp_run_groups(self._h))

    @property
    def group_words(self) -> int:
        return int(lib().pp_run_group_words(self._h))

    def free(self):
        if self._h:
            lib().pp_run_free(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter shutdown the HIP runtime (and a profiler's hooks) may
        # already be going away: leave the memory to the process's end then
        # (the check is bound here: the module's globals may be gone by then)
        if _finalizing():
            return
        try:
            self.free()
        except Exception:
            pass


def pp_seeds_init(graph: Graph, seeds, s=None, opts: Options | None = None, stream=None) -> Run:
    seeds = np.ascontiguousarray(seeds, dtype=np.int32)
    G = graph.count
    if s is None:
        s = int(seeds.size // G)
    h = ctypes.c_void_p()
    o = opts if opts is not None else options()
    _check(lib().pp_seeds_init(graph.handle, _np_ptr(seeds.reshape(-1)), int(s), ctypes.byref(o),
                               _stream_ptr(stream), ctypes.byref(h)))
    return Run(h, graph, int(s), o)


def pp_seeds_reset(run: Run, seeds):
    """Re-run the initialisation on an existing run (no allocation).

    ``seeds`` is a numpy int32 array (host) or an int32 device tensor.
    """
    if _is_device(seeds):
        _check(lib().pp_seeds_reset(run.handle, ctypes.c_void_p(seeds.data_ptr()), 1))
    else:
        a = np.ascontiguousarray(seeds, dtype=np.int32).reshape(-1)
        _check(lib().pp_seeds_reset(run.handle, _np_ptr(a), 0))


def pp_get_kernel_times(run: Run, cap: int):
    a = np.zeros(cap, dtype=np.float32)
    _check(lib().pp_get_kernel_times(run.handle, _np_ptr(a), int(cap)))
    return a


def pp_propagate_round(run: Run):
    """One round; returns (new bits per graph as int64 array, all_converged)."""
    G = run.graph.count
    nb = np.zeros(G, dtype=np.int64)
    conv = ctypes.c_int32(0)
    _check(lib().pp_propagate_round(run.handle, _np_ptr(nb), ctypes.byref(conv)))
    return nb, bool(conv.value)


def pp_propagate_until_converged(run: Run, max_rounds: int = 0, cap_rounds: int | None = None,
                                 raise_on_cap: bool = True):
    """Rounds to convergence; returns (counts [G][D_max+1] int64, D [G] int32)."""
    G = run.graph.count
    D = np.zeros(G, dtype=np.int32)
    rc = lib().pp_propagate_until_converged(run.handle, int(max_rounds), None, 0, _np_ptr(D))
    if rc not in (PP_OK, PP_ENOTCONV) or (rc == PP_ENOTCONV and raise_on_cap):
        _check(rc)
    # the run has stopped: a second call only copies the logs out
    cap = int(cap_rounds) if cap_rounds else max(int(D.max()), run.round) + 1
    counts = np.zeros((G, cap), dtype=np.int64)
    rc2 = lib().pp_propagate_until_converged(run.handle, int(max_rounds), _np_ptr(counts), cap, _np_ptr(D))
    if rc2 not in (PP_OK, PP_ENOTCONV):
        _check(rc2)
    return counts[:, :int(D.max()) + 1].copy(), D


def pp_estimate_metrics(counts, n: int, s: int, tau_num: int = 9, tau_den: int = 10) -> dict:
    c = np.ascontiguousarray(counts, dtype=np.int64)
    out = Metrics()
    _check(lib().pp_estimate_metrics(_np_ptr(c), int(c.shape[0]), int(n), int(s), int(tau_num), int(tau_den),
                                     ctypes.byref(out)))
    return out.as_dict()


def pp_get_signatures(run: Run, out=None):
    """Signatures [n][W] uint64: into a device tensor `out` if given, else a new numpy array."""
    n, W = run.graph.nodes, run.words
    if out is not None and _is_device(out):
        _check(lib().pp_get_signatures(run.handle, ctypes.c_void_p(out.data_ptr()), 1))
        return out
    a = np.zeros((n, W), dtype=np.uint64)
    _check(lib().pp_get_signatures(run.handle, _np_ptr(a), 0))
    return a


def pp_get_node_stats(run: Run):
    """Per-node (reached int32 [n], dist_sum int64 [n]) by input node id (needs options(node_stats=True))."""
    n = run.graph.nodes
    reached = np.zeros(n, dtype=np.int32)
    dist_sum = np.zeros(n, dtype=np.int64)
    _check(lib().pp_get_node_stats(run.handle, _np_ptr(reached), _np_ptr(dist_sum)))
    return reached, dist_sum


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
_allocators = []   # every callback pair ever set: blocks go back to the pair that gave them


def pp_set_allocator(alloc=None, release=None):
    """Device memory for the library from the caller.

    alloc(nbytes, stream) returns a device pointer (int; 0 when out of memory),
    release(ptr, stream) takes it back; stream is the raw hipStream_t as an int
    (0: the legacy default stream).  Both None: hipMalloc / hipFree again.
    """
    if alloc is None and release is None:
        _check(lib().pp_set_allocator(None, None, None))
        return
    if alloc is None or release is None:
        raise PPError(PP_EINVAL, "alloc and release: both or neither")
    a = _ALLOC_FN(lambda n, st, ctx: alloc(int(n), st or 0) or None)
    r = _RELEASE_FN(lambda p, st, ctx: release(p, st or 0))
    _allocators.append((a, r))
    _check(lib().pp_set_allocator(ctypes.cast(a, ctypes.c_void_p), ctypes.cast(r, ctypes.c_void_p), None))


def use_torch_allocator(torch):
    """Route the library's device memory through PyTorch's caching allocator."""
    dev = torch.cuda.current_device()
    pp_set_allocator(lambda n, st: torch.cuda.caching_allocator_alloc(n, dev, st),
                     lambda p, st: torch.cuda.caching_allocator_delete(p))


def pp_get_seed_counts(run: Run, cap_rounds: int):
    G = run.graph.count
    a = np.zeros((G, cap_rounds, run.s), dtype=np.uint32)
    _check(lib().pp_get_seed_counts(run.handle, _np_ptr(a), int(cap_rounds)))
    return a


def pp_get_round_log(run: Run, cap: int):
    mode = np.zeros(cap, dtype=np.int32)
    arcs = np.zeros(cap, dtype=np.int64)
    _check(lib().pp_get_round_log(run.handle, _np_ptr(mode), _np_ptr(arcs), int(cap)))
    return mode, arcs


def pp_get_group_log(run: Run, group: int, cap: int):
    """(mode [cap], arcs [cap]) of one seed group of the run."""
    mode = np.zeros(cap, dtype=np.int32)
    arcs = np.zeros(cap, dtype=np.int64)
    _check(lib().pp_get_group_log(run.handle, int(group), _np_ptr(mode), _np_ptr(arcs), int(cap)))
    return mode, arcs


def pp_run_snapshot(run: Run) -> Run:
    h = ctypes.c_void_p()
    _check(lib().pp_run_snapshot(run.handle, ctypes.byref(h)))
    return Run(h, run.graph, run.s, run.opts)


def pp_run_restore(run: Run, src: Run):
    _check(lib().pp_run_restore(run.handle, src.handle))


def _f32(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def pp_run_set_mlp(run: Run, params):
    """Cost-model weights of a PP_SCHED_MLP run ([MLP_PARAMS] float32), or None to clear them."""
    if params is None:
        _check(lib().pp_run_set_mlp(run.handle, None))
    else:
        _check(lib().pp_run_set_mlp(run.handle, _np_ptr(_f32(params, (MLP_PARAMS,)))))


def pp_run_set_plan(run: Run, plan):
    """Actions of a PP_SCHED_PLAN run (cost-model action indices per round; -1: the heuristic)."""
    a = np.ascontiguousarray(plan, dtype=np.int32).reshape(-1)
    _check(lib().pp_run_set_plan(run.handle, _np_ptr(a) if a.size else None, int(a.size)))


def pp_get_round_times(run: Run, cap: int):
    """Device-clock ms of each round of the last propagation (0 for rounds not run)."""
    a = np.zeros(cap, dtype=np.float32)
    _check(lib().pp_get_round_times(run.handle, _np_ptr(a), int(cap)))
    return a


def pp_get_round_features(run: Run, cap: int):
    a = np.zeros((cap, MLP_IN), dtype=np.float32)
    _check(lib().pp_get_round_features(run.handle, _np_ptr(a), int(cap)))
    return a


def pp_time_round(run: Run, mode: int):
    """Runs the next round with action `mode` (MODE_PULL / MODE_PUSH (direct slots) / MODE_PUSH_FLAT /
    MODE_SPULL); returns (features [8], ms).

    MODE_PUSH stands for the run's sparse direction (a sparse pull when the run
    was created with sparse_pull=1)."""
    f = np.zeros(MLP_IN, dtype=np.float32)
    ms = ctypes.c_float(0.0)
    _check(lib().pp_time_round(run.handle, int(mode), _np_ptr(f), ctypes.byref(ms)))
    return f, float(ms.value)


def pp_mlp_forward(params, x):
    p = _f32(params, (MLP_PARAMS,))
    x = _f32(x)
    n = int(x.shape[0])
    y = np.zeros((n, MLP_OUT), dtype=np.float32)
    _check(lib().pp_mlp_forward(_np_ptr(p), _np_ptr(x.reshape(n, MLP_IN)), n, _np_ptr(y)))
    return y


def pp_mlp_loss_grad(params, x, t):
    p = _f32(params, (MLP_PARAMS,))
    x = _f32(x)
    t = _f32(t)
    n = int(x.shape[0])
    if t.shape != (n, MLP_OUT) or x.shape != (n, MLP_IN):
        raise ValueError("x must be [n][8] and t [n][4]")
    g = np.zeros(MLP_PARAMS, dtype=np.float32)
    loss = ctypes.c_float(0.0)
    _check(lib().pp_mlp_loss_grad(_np_ptr(p), _np_ptr(x), _np_ptr(t), n, _np_ptr(g), ctypes.byref(loss)))
    return float(loss.value), g


def pp_mlp_train(params, x, t, steps: int, lr: float):
    """Full-batch Adam; returns (trained params, loss before each step)."""
    p = _f32(params, (MLP_PARAMS,)).copy()
    x = _f32(x)
    t = _f32(t)
    n = int(x.shape[0])
    if t.shape != (n, MLP_OUT) or x.shape != (n, MLP_IN):
        raise ValueError("x must be [n][8] and t [n][4]")
    log = np.zeros(max(int(steps), 1), dtype=np.float32)
    _check(lib().pp_mlp_train(_np_ptr(p), _np_ptr(x), _np_ptr(t), n, int(steps), float(lr), _np_ptr(log)))
    return p, log[:int(steps)]


def pp_autotune(graph: Graph, seeds, s=None, base: Options | None = None, reps: int = 3):
    """Options picked by measurement; returns (best Options, list of dicts for every candidate tried)."""
    seeds = np.ascontiguousarray(seeds, dtype=np.int32).reshape(-1)
    if s is None:
        s = int(seeds.size // graph.count)
    best = Options()
    cap = 32
    table = (TuneEntry * cap)()
    n = ctypes.c_int32(0)
    _check(lib().pp_autotune(graph.handle, _np_ptr(seeds), int(s), ctypes.byref(base) if base is not None else None,
                             int(reps), ctypes.byref(best), table, cap, ctypes.byref(n)))
    rows = [{k: getattr(table[i], k) for k, _ in TuneEntry._fields_} for i in range(min(n.value, cap))]
    return best, rows


def pp_exact_counts(graph: Graph, group: int = 512, opts: Options | None = None, cap_rounds: int | None = None):
    """Exact neighbourhood function increments c[0..D] (every node a seed); returns (counts, D)."""
    cap = int(cap_rounds) if cap_rounds else graph.nodes + 1
    c = np.zeros(cap, dtype=np.int64)
    D = ctypes.c_int32(0)
    _check(lib().pp_exact_counts(graph.handle, int(group), ctypes.byref(opts) if opts is not None else None,
                                 _np_ptr(c), cap, ctypes.byref(D)))
    return c[:D.value + 1].copy(), int(D.value)


def pp_progressive_sample(graph: Graph, pool, group: int, target: float, delta: float, opts: Options | None = None,
                          cap_rounds: int | None = None):
    """Progressive sampling; returns a dict: counts c[0..D] of the seeds used, and the Progress figures."""
    a = np.ascontiguousarray(pool, dtype=np.int32).reshape(-1)
    cap = int(cap_rounds) if cap_rounds else graph.nodes + 1
    c = np.zeros(cap, dtype=np.int64)
    out = Progress()
    _check(lib().pp_progressive_sample(graph.handle, _np_ptr(a), int(a.shape[0]), int(group), float(target),
                                       float(delta), ctypes.byref(opts) if opts is not None else None,
                                       _np_ptr(c), cap, ctypes.byref(out)))
    res = {k: getattr(out, k) for k, _ in Progress._fields_}
    res["met"] = bool(res["met"])
    res["counts"] = c[:out.D + 1].copy()
    return res


def pp_propagate_s(graph: Graph, seeds, concurrent: int = 0, cap_rounds: int | None = None, stream=None):
    """PROPAGATE-S (Algorithm 2); host seeds; returns (counts c[0..D] int64, D, arcs examined)."""
    a = np.ascontiguousarray(seeds, dtype=np.int32).reshape(-1)
    cap = int(cap_rounds) if cap_rounds else graph.nodes + 1
    c = np.zeros(cap, dtype=np.int64)
    D = ctypes.c_int32(0)
    ex = ctypes.c_int64(0)
    _check(lib().pp_propagate_s(graph.handle, _np_ptr(a), int(a.shape[0]), int(concurrent), _stream_ptr(stream),
                                _np_ptr(c), cap, ctypes.byref(D), ctypes.byref(ex)))
    return c[:D.value + 1].copy(), int(D.value), int(ex.value)


def pp_propagate_s_noalloc(graph: Graph, seeds, concurrent: int = 0, cap_rounds: int | None = None, stream=None):
    """PROPAGATE-S with its device buffers in the library's fixed region (no allocation);
    returns (counts c[0..D] int64, D, arcs examined) like pp_propagate_s."""
    a = np.ascontiguousarray(seeds, dtype=np.int32).reshape(-1)
    cap = int(cap_rounds) if cap_rounds else graph.nodes + 1
    c = np.zeros(cap, dtype=np.int64)
    D = ctypes.c_int32(0)
    ex = ctypes.c_int64(0)
    _check(lib().pp_propagate_s_noalloc(graph.handle, _np_ptr(a), int(a.shape[0]), int(concurrent),
                                        _stream_ptr(stream), _np_ptr(c), cap, ctypes.byref(D), ctypes.byref(ex)))
    return c[:D.value + 1].copy(), int(D.value), int(ex.value)


NOALLOC_BYTES = 64 << 20   # PP_NOALLOC_BYTES


def propagate(n, src, dst, seeds, undirected=False, transpose=False, opts=None, stream=None):
    """Convenience: build, initialise, run to convergence; returns (counts, D, run)."""
    g = pp_csr_build(n, src, dst, undirected=undirected, transpose=transpose, stream=stream)
    r = pp_seeds_init(g, seeds, opts=opts, stream=stream)
    counts, D = pp_propagate_until_converged(r)
    return counts[0], int(D[0]), r
