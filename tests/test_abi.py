"""The C-ABI library builds for gfx950, loads, and exports every entry point
that include/bfscut.h declares (no compute calls: this runs without a GPU)."""

import ctypes
import os
import re
import subprocess

import pytest

import paper_1507_01490_amd as bc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(bc_[a-z_0-9]+)\s*\(", txt))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("bc_graph_create", "bc_graph_destroy", "bc_topk", "bc_last_error", "bc_opts_default"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(bc.LIB_PATH):
        pytest.fail("libbfscut.so is not built (run python -m paper_1507_01490_amd.build)")
    lib = ctypes.CDLL(bc.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_opts_defaults_and_version():
    lib = bc.load_library()
    o = bc.Opts()
    lib.bc_opts_default(ctypes.byref(o))
    assert o.size == ctypes.sizeof(bc.Opts)
    assert o.width == 64 and o.mode == bc.MODE_PLAIN and o.order == bc.ORDER_AUTO and not o.mlp
    assert lib.bc_version().decode().startswith("bfscut")


def test_struct_layouts_match_header(tmp_path):
    """Size and every field offset of bc_opts / bc_stats as a C compiler
    lays them out from the header, against the binding's ctypes structs."""
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "bfscut.h"', 'int main(void) {']
    for cname, py in (("bc_opts", bc.Opts), ("bc_stats", bc.Stats)):
        lines.append(f'printf("{cname} __sizeof %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        c, f, v = line.split()
        got[(c, f)] = int(v)
    for cname, py in (("bc_opts", bc.Opts), ("bc_stats", bc.Stats)):
        assert got[(cname, "__sizeof")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_null_arguments_rejected_without_gpu_work():
    lib = bc.load_library()
    assert lib.bc_graph_create(0, 0, None, None, 0, None, None) == -1
    assert lib.bc_topk(None, 1, None, None, None, None, None, None) == -1
    assert b"NULL" in lib.bc_last_error()
