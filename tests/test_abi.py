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


def test_loading_the_library_imports_torch_first():
    """torch's own HIP runtime libraries must be loaded before the library's
    (the GPU test of the same name shows why); checked in a fresh process,
    where nothing else imported torch, without a device call."""
    import sys
    code = ("import sys, ctypes\n"
            "import paper_1507_01490_amd as bc\n"
            "bc.load_library()\n"
            "print('torch' in sys.modules)\n")
    env = dict(os.environ, PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
    out = subprocess.check_output([sys.executable, "-c", code], cwd=ROOT, env=env, text=True, timeout=300)
    assert out.strip().endswith("True")


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
    structs = (("bc_opts", bc.Opts), ("bc_stats", bc.Stats), ("bc_server_opts", bc.ServerOpts),
               ("bc_request_info", bc.RequestInfo), ("bc_server_stats", bc.ServerStats))
    for cname, py in structs:
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
    for cname, py in structs:
        assert got[(cname, "__sizeof")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_null_arguments_rejected_without_gpu_work():
    lib = bc.load_library()
    assert lib.bc_graph_create(0, 0, None, None, 0, None, None) == -1
    assert lib.bc_topk(None, 1, None, None, None, None, None, None) == -1
    assert b"NULL" in lib.bc_last_error()


def test_footprint_arithmetic():
    """The serving admission estimate (pure host arithmetic, no device call)."""
    n, m = 20000, 160000
    g, u, q_plain = bc.footprint(n, m, k=10, mode="plain")
    # undirected, below the renumbering size: CSR, packed arcs, per-node arrays
    # (degree, reach pair, seven cached orders, features and core numbers)
    assert g == 4 * (n + 1) + 12 * m + 56 * n
    assert u == 12 * m + 40 * n + (1 << 20)
    # from 100,000 nodes: the two renumbering maps, and the first build held
    # while the renumbered one is made
    nb, mb = 200000, 1600000
    gb, ub, _ = bc.footprint(nb, mb)
    assert gb == 4 * (nb + 1) + 12 * mb + 56 * nb + 8 * nb
    assert ub == 12 * mb + 40 * nb + (1 << 20) + gb + 16 * nb + 4 * mb
    per_slot = n * (8 * 4 + 12)
    _, _, q16 = bc.footprint(n, m, k=10, mode="batched", slots=16)
    _, _, q32 = bc.footprint(n, m, k=10, mode="batched", slots=32)
    assert q16 - q_plain == 16 * per_slot + 4 * 16
    assert q32 - q16 == 16 * per_slot + 4 * 16
    # W = 256 records are four times wider
    _, _, q256 = bc.footprint(n, m, k=10, mode="batched", slots=16, width=256)
    assert q256 - q16 == 17 * n * 8 * 12
    # slots never exceed the number of batches
    _, _, qs = bc.footprint(100, 400, k=1, mode="batched", slots=64)
    _, _, qp = bc.footprint(100, 400, k=1, mode="plain")
    assert qs - qp == 2 * 100 * 44 + 8
    gd, ud, _ = bc.footprint(n, m, directed=True)
    assert gd - g == 4 * (n + 1) + 4 * m
    assert ud == 12 * m + 40 * n + (1 << 20)
    # a learned order adds its features and core numbers (16 B), scores and the
    # score order (8 B) per node, and the perceptron's parameters
    _, _, ql = bc.footprint(n, m, k=10, mode="plain", order="learned")
    assert ql - q_plain == 24 * n + 4 * bc.MLP_PARAMS
    for big in (bc.footprint(2 * n, m), bc.footprint(n, 2 * m), bc.footprint(n, m, k=100)):
        assert big[0] + big[2] > g + q_plain
