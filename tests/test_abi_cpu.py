"""CPU-side checks of the C ABI: the library loads and exports what include/bt.h declares.

No compute call is made (there is no GPU here); only host-only helpers are called.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1912_03998_amd import bt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bt.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bt_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_binding_names():
    assert declared_functions() == sorted(bt.EXPORTED)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(bt.LIB_PATH):
        pytest.skip("libbt.so not built")
    L = C.CDLL(bt.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_host_only_helpers():
    if not os.path.exists(bt.LIB_PATH):
        pytest.skip("libbt.so not built")
    p = bt.bt_params_default()
    assert p.max_depth == 3 and p.t_min == 1e-3 and p.edge_delta == 1e-5
    assert p.air_m == 0.0 and p.e_min == 0.0 and not p.hit_out
    assert bt.lib().bt_status_str(0) == b"ok"
    assert bt.lib().bt_status_str(-1) == b"invalid argument"
    assert bt.lib().bt_last_error(None) == b"null context"


def test_null_context_calls_are_refused():
    """Entry points given no context return BT_EINVAL before touching any device."""
    if not os.path.exists(bt.LIB_PATH):
        pytest.skip("libbt.so not built")
    L = bt.lib()
    p = bt.bt_params_default()
    assert L.bt_set_partitions(None, 2) == -1
    assert L.bt_trace_all(None, None, None, C.byref(p)) == -1
    assert L.bt_trace(None, None, None, C.byref(p), None) == -1
    assert L.bt_accumulate_mics(None, None, None, C.byref(p), None) == -1


def _c_layout(struct, fields, tmp_path):
    """sizeof and offsetof of a bt.h struct, from a gcc-compiled probe."""
    src = tmp_path / "probe.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "bt.h"', "int main(void) {",
             f'  printf("%zu\\n", sizeof({struct}));']
    lines += [f'  printf("%zu\\n", offsetof({struct}, {f}));' for f in fields]
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    import subprocess
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    out = subprocess.check_output([str(exe)]).decode().split()
    return [int(x) for x in out]


@pytest.mark.parametrize("name", ["bt_params", "bt_stats", "bt_request", "bt_result", "bt_scenario",
                                  "bt_batch_opts", "bt_batch_stats", "bt_server_opts", "bt_serve_result"])
def test_struct_layouts_match_header(name, tmp_path):
    cls = getattr(bt, name)
    fields = [f[0] for f in cls._fields_]
    got = _c_layout(name, fields, tmp_path)
    want = [C.sizeof(cls)] + [getattr(cls, f).offset for f in fields]
    assert got == want


# ---------------------------------------------------------------------------------------
# host-only argument checks (no context, no device): the checks the calls make before
# they touch the GPU
# ---------------------------------------------------------------------------------------

def _lib_or_skip():
    if not os.path.exists(bt.LIB_PATH):
        pytest.skip("libbt.so not built")


def test_validate_mesh_errors():
    _lib_or_skip()
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [2, 2, 2]], np.float32)
    t = np.array([[0, 1, 2]], np.int32)
    a = np.array([0.1], np.float32)
    assert bt.bt_validate_mesh(v, t, a) == (0, "")
    assert bt.bt_validate_mesh(v, t, a, 4, 3)[0] == 0
    cases = [
        (v, np.array([[0, 1, 4]], np.int32), a, 1, 1, "out of range"),
        (v, np.array([[0, -1, 2]], np.int32), a, 1, 1, "out of range"),
        (np.where(np.arange(12).reshape(4, 3) == 4, np.nan, v).astype(np.float32), t, a, 1, 1, "not finite"),
        (np.where(np.arange(12).reshape(4, 3) == 0, np.inf, v).astype(np.float32), t, a, 1, 1, "not finite"),
        (v, t, np.array([1.5], np.float32), 1, 1, "absorption"),
        (v, t, np.array([-0.1], np.float32), 1, 1, "absorption"),
        (v, t, np.array([np.nan], np.float32), 1, 1, "absorption"),
        (np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0]], np.float32), t, a, 1, 1, "zero area"),
        (v, np.array([[0, 0, 2]], np.int32), a, 1, 1, "zero area"),
        (v, t, a, 0, 1, "tiles"),
        (v, t, a, 1, 65, "tiles"),
    ]
    for xyz, tri, alpha, tx, ty, why in cases:
        st, msg = bt.bt_validate_mesh(xyz, tri, alpha, tx, ty)
        assert st == -1 and why in msg, (why, st, msg)


def test_validate_sources_errors():
    _lib_or_skip()
    s, w = np.array([[0, 0, 1]], np.float32), np.array([1.0], np.float32)
    assert bt.bt_validate_sources(s, w, 3)[0] == 0
    assert bt.bt_validate_sources(s, w, 9)[0] == 0
    assert bt.bt_validate_sources(np.zeros((0, 3), np.float32), np.zeros(0, np.float32), 3)[0] == 0
    for src, pw, level, why in [(s, w, 10, "level"), (s, w, -1, "level"),
                                (np.array([[0, np.nan, 1]], np.float32), w, 3, "not finite"),
                                (s, np.array([-1.0], np.float32), 3, "power"),
                                (s, np.array([np.inf], np.float32), 3, "power"),
                                (np.zeros((410, 3), np.float32), np.ones(410, np.float32), 9, "too many beams")]:
        st, msg = bt.bt_validate_sources(src, pw, level)
        assert st == -1 and why in msg, (why, st, msg)
    wt = np.ones((1, 1280), np.float32)
    assert bt.bt_validate_sources(s, w, 3, wt)[0] == 0
    wt[0, 17] = -1.0
    st, msg = bt.bt_validate_sources(s, w, 3, wt)
    assert st == -1 and "weight 17" in msg


def test_validate_grid_errors():
    _lib_or_skip()
    assert bt.bt_validate_grid(0, 0, 1.5, 4, 4, 0, 500, 500, 1)[0] == 0
    assert bt.bt_validate_grid(0, 0, 2, 4, 4, 4, 625, 375, 58)[0] == 0
    for args, why in [((0, 0, 1.5, 4, 4, 0, 0, 500, 1), "bad microphone grid"),
                      ((0, 0, 1.5, 4, 4, 0, 65536, 65536, 1), "bad microphone grid"),
                      ((0, 0, 1.5, 0, 4, 0, 5, 5, 1), "geometry"),
                      ((float("nan"), 0, 1.5, 4, 4, 0, 5, 5, 1), "geometry"),
                      ((0, 0, 1.5, 4, 4, 0, 5, 5, 3), "geometry"),
                      ((0, 0, 1.5, 4, 4, 1, 1 << 24, 2, 2), "below 2^24")]:
        st, msg = bt.bt_validate_grid(*args)
        assert st == -1 and why in msg, (args, st, msg)


def test_validate_params_errors():
    _lib_or_skip()
    assert bt.bt_validate_params(bt.bt_params_default()) == (0, "")
    for kw, why in [({"max_depth": 32}, "max_depth"), ({"max_depth": -1}, "max_depth"),
                    ({"t_min": -1.0}, "t_min"), ({"t_min": float("inf")}, "t_min"),
                    ({"edge_delta": 2e-3}, "edge_delta"), ({"air_m": float("nan")}, "air_m"),
                    ({"e_min": -1.0}, "e_min"), ({"queue_rounds": 9}, "queue_rounds")]:
        st, msg = bt.bt_validate_params(bt.bt_params_default(**kw))
        assert st == -1 and why in msg, (kw, st, msg)
