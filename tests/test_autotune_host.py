"""The autotuner's cache logic (no GPU): keys, reuse, re-tuning, option merge."""
import json

import pytest

from paper_2301_06499_amd import autotune, pp


class FakeGraph:
    nodes, arcs, count = 1000, 5000, 1


def test_cache_roundtrip(tmp_path, monkeypatch):
    calls = []

    def fake_autotune(graph, seeds, s, base, reps):
        calls.append(reps)
        best = pp.Options.from_buffer_copy(base)
        best.pull_k, best.push_div, best.rounds_per_sync, best.persistent = 2, 16, 0, 0
        return best, [{"pull_k": 4, "push_div": 8, "rounds_per_sync": 0, "persistent": 0, "ms": 2.0},
                      {"pull_k": 2, "push_div": 16, "rounds_per_sync": 0, "persistent": 0, "ms": 1.5}]

    monkeypatch.setattr(pp, "pp_autotune", fake_autotune)
    path = str(tmp_path / "tune.json")
    base = pp.options(max_rounds=100, seed_counts=True)
    o, rec = autotune.tune(FakeGraph(), [1, 2, 3], base=base, name="w", cache_path=path)
    assert not rec["cached"] and (o.pull_k, o.push_div) == (2, 16)
    assert (o.max_rounds, o.seed_counts) == (100, 1)          # the caller's other options are kept
    assert rec["ms"] == 1.5 and len(rec["candidates"]) == 2
    stored = json.load(open(path))
    assert list(stored) == [autotune.workload_key(FakeGraph(), 3, "w")]
    o2, rec2 = autotune.tune(FakeGraph(), [1, 2, 3], base=base, name="w", cache_path=path)
    assert rec2["cached"] and (o2.pull_k, o2.push_div) == (2, 16) and len(calls) == 1
    autotune.tune(FakeGraph(), [1, 2, 3], base=base, name="other", cache_path=path)
    assert len(calls) == 2 and len(json.load(open(path))) == 2
    autotune.tune(FakeGraph(), [1, 2, 3], base=base, name="w", cache_path=path, retune=True)
    assert len(calls) == 3


def test_unreadable_cache_is_ignored(tmp_path, monkeypatch):
    path = tmp_path / "bad.json"
    path.write_text("not json")
    monkeypatch.setattr(pp, "pp_autotune", lambda *a: (pp.options(pull_k=4, push_div=8), [{"ms": 1.0}]))
    o, rec = autotune.tune(FakeGraph(), [0], cache_path=str(path))
    assert not rec["cached"] and o.push_div == 8


def test_autotune_argument_errors():
    L = pp.lib()
    assert L.pp_autotune(None, None, 1, None, 1, None, None, 0, None) == pp.PP_EINVAL


def test_sparse_pull_is_tuned_and_old_records_still_apply(tmp_path):
    """A record carries the sparse direction; one written before that field existed
    leaves the caller's value as it was."""
    base = pp.options(sparse_pull=2, max_rounds=50)
    o = autotune.apply(base, {"pull_k": 4, "push_div": 16, "rounds_per_sync": 0, "persistent": 0, "sparse_pull": 1})
    assert (o.sparse_pull, o.push_div, o.max_rounds) == (1, 16, 50)
    old = {"pull_k": 2, "push_div": 8, "rounds_per_sync": 0, "persistent": 0}
    o = autotune.apply(base, old)
    assert (o.sparse_pull, o.pull_k) == (2, 2)
    assert "sparse_pull" in autotune.TUNED_FIELDS
