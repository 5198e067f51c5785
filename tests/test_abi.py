"""The C-ABI library builds for gfx950, loads, and exports every entry point
that include/bfscut.h declares (no compute calls: this runs without a GPU)."""

import ctypes
import os
import re

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
    assert o.width == 64 and o.mode == bc.MODE_PLAIN and o.order == bc.ORDER_AUTO
    assert lib.bc_version().decode().startswith("bfscut")


def test_struct_sizes_match_header():
    # bc_opts: 4 x int32, 2 pointers, 2 floats, 4 x int32 ; bc_stats: see header
    assert ctypes.sizeof(bc.Opts) == 4 * 4 + 2 * 8 + 2 * 4 + 6 * 4
    assert ctypes.sizeof(bc.Stats) == 8 + 7 * 8 + 4 * 8 + 5 * 8 + 2 * 8 + 5 * 8 + 3 * 8


def test_null_arguments_rejected_without_gpu_work():
    lib = bc.load_library()
    assert lib.bc_graph_create(0, 0, None, None, 0, None, None) == -1
    assert lib.bc_topk(None, 1, None, None, None, None, None, None) == -1
    assert b"NULL" in lib.bc_last_error()
