"""Autotuned run options with a JSON cache.

``pp_autotune`` (the library) times every candidate configuration -- pull
tile shape (arcs per lane, which also sets the high-degree split length),
push threshold, push or sparse pull for sparse rounds, per-round or
persistent engine -- and returns the fastest.
This module keys the result by the workload (nodes, stored arcs, graphs,
seeds, and a caller-chosen name) and keeps it in a JSON file so a workload
is tuned once per machine.
"""
from __future__ import annotations

import json
import os

from . import pp

TUNED_FIELDS = ("pull_k", "push_div", "rounds_per_sync", "persistent", "sparse_pull")


def default_cache_path() -> str:
    return os.environ.get("PP_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "pp_tune.json"))


def workload_key(graph: pp.Graph, s: int, name: str = "") -> str:
    return f"{name}|n={graph.nodes}|m={graph.arcs}|G={graph.count}|s={s}"


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def _store(path: str, data: dict) -> None:
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def apply(opts: pp.Options, tuned: dict) -> pp.Options:
    """A copy of opts with the tuned fields set."""
    out = pp.Options.from_buffer_copy(opts)
    for k in TUNED_FIELDS:
        if k in tuned:   # a record written before a field existed leaves it as given
            setattr(out, k, int(tuned[k]))
    return out


def tune(graph: pp.Graph, seeds, s: int | None = None, base: pp.Options | None = None, reps: int = 3,
         name: str = "", cache_path: str | None = None, retune: bool = False):
    """Tuned options for the workload: from the cache, or measured and stored.

    Returns (options, record) where record holds the tuned fields, the best
    time and every candidate's time (when measured now).
    """
    import numpy as np
    seeds = np.ascontiguousarray(seeds, dtype=np.int32).reshape(-1)
    if s is None:
        s = int(seeds.size // graph.count)
    base = base if base is not None else pp.options()
    path = cache_path or default_cache_path()
    key = workload_key(graph, s, name)
    cache = _load(path)
    if not retune and key in cache:
        return apply(base, cache[key]), dict(cache[key], cached=True)
    best, table = pp.pp_autotune(graph, seeds, s, base, reps)
    record = {k: int(getattr(best, k)) for k in TUNED_FIELDS}
    record["ms"] = min(r["ms"] for r in table)
    record["candidates"] = table
    cache[key] = record
    _store(path, cache)
    return apply(base, record), dict(record, cached=False)
