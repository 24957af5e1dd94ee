"""The C-ABI library loads, exports what include/pp.h declares, and checks
arguments before any device work (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2301_06499_amd import pp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "pp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pp_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    L = pp.lib()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(pp.EXPORTS)


def test_struct_layouts_match_header():
    assert ctypes.sizeof(pp.Options) == 64
    assert ctypes.sizeof(pp.TuneEntry) == 6 * 4
    assert ctypes.sizeof(pp.Progress) == 4 * 4 + 3 * 8
    assert ctypes.sizeof(pp.Metrics) == 4 + 4 + 8 + 6 * 8


def test_struct_offsets_match_a_c_compiler(tmp_path):
    """Every field of the binding's structures sits where a C compiler puts it."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"pp_options": pp.Options, "pp_tune_entry": pp.TuneEntry, "pp_progress": pp.Progress,
               "pp_metrics": pp.Metrics}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "pp.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    include = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.check_call([cc, "-I", include, str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        cname, f, v = line.split()
        got[(cname, f)] = int(v)
    for cname, cls in structs.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


def test_validation_before_device_work():
    s = np.array([0, 1], np.int32)
    d = np.array([1, 2], np.int32)
    for args, code in [((0, s, d), pp.PP_EINVAL),                 # n < 1
                       ((2, s, d), pp.PP_ERANGE),                 # id 2 >= n
                       ((3, np.array([0, -1], np.int32), d), pp.PP_ERANGE)]:
        with pytest.raises(pp.PPError) as e:
            pp.pp_csr_build(*args)
        assert e.value.code == code
    # an arc across two graphs of a batch
    with pytest.raises(pp.PPError) as e:
        pp.pp_csr_build(4, np.array([0, 1], np.int32), np.array([1, 2], np.int32), node_offsets=[0, 2, 4])
    assert e.value.code == pp.PP_ERANGE
    with pytest.raises(pp.PPError) as e:
        pp.pp_csr_build(4, s, d, node_offsets=[0, 3, 2, 4])
    assert e.value.code == pp.PP_EINVAL
    L = pp.lib()
    out = ctypes.c_void_p()
    assert L.pp_seeds_init(None, None, 1, None, None, ctypes.byref(out)) == pp.PP_EINVAL
    assert L.pp_propagate_round(None, None, None) == pp.PP_EINVAL
    assert L.pp_propagate_until_converged(None, 0, None, 0, None) == pp.PP_EINVAL
    assert L.pp_get_signatures(None, None, 0) == pp.PP_EINVAL
    assert L.pp_propagate_s(None, None, 1, 0, None, None, 1, None, None) == pp.PP_EINVAL
    fn = pp._ALLOC_FN(lambda n, st, ctx: None)
    assert L.pp_set_allocator(ctypes.cast(fn, ctypes.c_void_p), None, None) == pp.PP_EINVAL
    assert L.pp_set_allocator(None, None, None) == pp.PP_OK
    with pytest.raises(pp.PPError):
        pp.pp_set_allocator(lambda n, st: 0, None)
    assert L.pp_progressive_sample(None, None, 1, 1, 1.0, 0.05, None, None, 1, None) == pp.PP_EINVAL
    assert L.pp_get_node_stats(None, None, None) == pp.PP_EINVAL
    assert "NULL" in L.pp_last_error().decode()


@pytest.mark.parametrize("trial", range(40))
def test_metrics_match_oracle_bit_for_bit(trial):
    """pp_estimate_metrics (C, 128-bit) equals the oracle's (Python integers) exactly."""
    rng = np.random.default_rng(trial)
    s = int(rng.integers(1, 600))
    n = int(rng.integers(s, 10**8))
    L = int(rng.integers(1, 40))
    c = np.concatenate([[s], rng.integers(0, 10**9, L - 1)]).astype(np.int64)
    if trial % 5 == 0:
        c = np.concatenate([c, np.zeros(3, np.int64)])
    tn, td = (9, 10) if trial % 2 else (int(rng.integers(0, 50)), 50)
    a = pp.pp_estimate_metrics(c, n, s, tn, td)
    b = oracle.metrics(c, n, s, tn, td)
    for k, v in b.items():
        assert a[k] == v, (k, a[k], v)


def test_metrics_argument_errors():
    with pytest.raises(pp.PPError):
        pp.pp_estimate_metrics([1, 2], 4, 0)
    with pytest.raises(pp.PPError):
        pp.pp_estimate_metrics([1, 2], 4, 1, 11, 10)
    with pytest.raises(pp.PPError):
        pp.pp_estimate_metrics([1, -2], 4, 1)


def test_cost_model_layout_and_argument_errors():
    text = open(os.path.join(ROOT, "include", "pp.h")).read()
    assert int(re.search(r"#define PP_MLP_PARAMS (\d+)", text).group(1)) == pp.MLP_PARAMS == 1476
    L = pp.lib()
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    p = np.zeros(pp.MLP_PARAMS, np.float32)
    x = np.zeros((4, 8), np.float32)
    t = np.zeros((4, pp.MLP_OUT), np.float32)
    y = np.zeros((4, pp.MLP_OUT), np.float32)
    assert L.pp_run_set_mlp(None, None) == pp.PP_EINVAL
    assert L.pp_time_round(None, 0, None, None) == pp.PP_EINVAL
    assert L.pp_get_round_features(None, None, 1) == pp.PP_EINVAL
    assert L.pp_mlp_forward(None, ptr(x), 4, ptr(y)) == pp.PP_EINVAL
    assert L.pp_mlp_forward(ptr(p), ptr(x), 4, None) == pp.PP_EINVAL
    assert L.pp_mlp_forward(ptr(p), ptr(x), 0, ptr(y)) == pp.PP_EINVAL
    assert L.pp_mlp_loss_grad(ptr(p), ptr(x), None, 4, None, None) == pp.PP_EINVAL
    assert L.pp_mlp_train(ptr(p), ptr(x), ptr(t), 4, 10, 0.0, None) == pp.PP_EINVAL
    assert L.pp_mlp_train(ptr(p), ptr(x), ptr(t), 4, 10, float("nan"), None) == pp.PP_EINVAL
    assert L.pp_mlp_train(ptr(p), ptr(x), ptr(t), 4, -1, 0.01, None) == pp.PP_EINVAL
    assert "steps" in L.pp_last_error().decode()
    with pytest.raises(ValueError):
        pp.pp_mlp_loss_grad(p, x, np.zeros((3, 2), np.float32))
