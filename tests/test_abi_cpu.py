"""CPU-side checks of the C ABI: the library loads and exports what include/bt.h declares.

No compute call is made (there is no GPU here); only host-only helpers are called.
"""
import ctypes as C
import os
import re

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
