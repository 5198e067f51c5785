"""CPU oracle for exact top-k closeness (ctypes wrapper over bfscut_oracle.c).

TEST INFRASTRUCTURE ONLY: the slow, obviously correct reference the GPU path
is checked against.  Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The GPU library
neither imports it nor shares code with it.

Besides the C functions, :func:`topk_by_definition` states the result
directly from its definition in exact Python integers: the k nodes with the
largest generalised closeness (r-1)^2 / ((n-1) f) (Section 1), ties broken by
smaller id.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bfscut_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-g", "-std=c11", "-Wall", "-Wextra", "-fPIC",
                               "-shared", "-pthread", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


class Stats(ctypes.Structure):
    _fields_ = [("m_vis", ctypes.c_uint64), ("n_cut", ctypes.c_uint64),
                ("n_done", ctypes.c_uint64), ("n_trivial", ctypes.c_uint64)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    lib.orc_canonicalize.argtypes = [i32, P, P, P, P]
    lib.orc_canonicalize.restype = i64
    lib.orc_bfs.argtypes = [i32, P, P, i32, P]
    lib.orc_bruteforce.argtypes = [i32, P, P, P, P, ctypes.c_int]
    lib.orc_reach_undirected.argtypes = [i32, P, P, P]
    lib.orc_scc.argtypes = [i32, P, P, P]
    lib.orc_scc.restype = i32
    lib.orc_alpha_omega.argtypes = [i32, P, P, P, P]
    lib.orc_alpha_omega_ex.argtypes = [i32, P, P, ctypes.c_int, P, P]
    lib.orc_topk_ex.argtypes = [i32, P, P, ctypes.c_int, i32, P, ctypes.c_int, ctypes.c_uint32, P, P, P, P, P,
                                ctypes.POINTER(Stats)]
    lib.orc_topk_ex.restype = i32
    lib.orc_topk.argtypes = [i32, P, P, ctypes.c_int, i32, P, ctypes.c_int, P, P, P, P, P,
                             ctypes.POINTER(Stats)]
    lib.orc_topk.restype = i32
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _csr(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    if col.shape[0] == 0:
        col = np.zeros(1, np.int32)
    return rp, col


def canonicalize(g):
    lib = _load()
    rp, col = _csr(g)
    out_rp = np.zeros(g.n + 1, np.int32)
    out_col = np.zeros(max(g.m, 1), np.int32)
    m = lib.orc_canonicalize(g.n, _p(rp), _p(col), _p(out_rp), _p(out_col))
    return out_rp, out_col[:m].copy()


def bfs(g, src: int) -> np.ndarray:
    lib = _load()
    rp, col = _csr(g)
    dist = np.zeros(max(g.n, 1), np.int32)
    lib.orc_bfs(g.n, _p(rp), _p(col), int(src), _p(dist))
    return dist[:g.n]


def bruteforce(g, nthreads: int = 1):
    """Textbook algorithm (one BFS per node): exact (r, f) of every node."""
    lib = _load()
    rp, col = _csr(g)
    r = np.zeros(max(g.n, 1), np.uint32)
    f = np.zeros(max(g.n, 1), np.uint64)
    lib.orc_bruteforce(g.n, _p(rp), _p(col), _p(r), _p(f), int(nthreads))
    return r[:g.n], f[:g.n]


def reach_undirected(g) -> np.ndarray:
    lib = _load()
    rp, col = _csr(g)
    r = np.zeros(max(g.n, 1), np.uint32)
    lib.orc_reach_undirected(g.n, _p(rp), _p(col), _p(r))
    return r[:g.n]


def scc(g):
    lib = _load()
    rp, col = _csr(g)
    comp = np.zeros(max(g.n, 1), np.int32)
    nc = lib.orc_scc(g.n, _p(rp), _p(col), _p(comp))
    return int(nc), comp[:g.n]


def alpha_omega(g, big_scc: bool = False):
    """alpha(v) <= r(v) <= omega(v) over the SCC DAG (Section 2.4); with
    big_scc, the largest-SCC refinement of the same section."""
    lib = _load()
    rp, col = _csr(g)
    a = np.zeros(max(g.n, 1), np.uint32)
    o = np.zeros(max(g.n, 1), np.uint32)
    lib.orc_alpha_omega_ex(g.n, _p(rp), _p(col), int(bool(big_scc)), _p(a), _p(o))
    return a[:g.n], o[:g.n]


FOOTNOTE = 0x1   # undirected: ~gamma_{d+1} with (degree - 1) for d >= 1 (Section 2.3 footnote)
BIG_SCC = 0x2    # directed: reach bounds with the largest-SCC refinement (Section 2.4)


def topk(g, k: int, order=None, nthreads: int = 1, trace: bool = False, footnote: bool = False,
         big_scc: bool = False):
    """Algorithm 1 with BFSCut.  Returns dict(ids, f, r, stats[, cut_level, mvis]).
    footnote / big_scc switch on the optional tighter bounds (same result)."""
    lib = _load()
    rp, col = _csr(g)
    kk = max(0, min(int(k), g.n))
    ids = np.zeros(max(kk, 1), np.int32)
    f = np.zeros(max(kk, 1), np.uint64)
    r = np.zeros(max(kk, 1), np.uint32)
    o = None if order is None else np.ascontiguousarray(order, dtype=np.int32)
    cl = np.zeros(max(g.n, 1), np.int32) if trace else None
    mv = np.zeros(max(g.n, 1), np.uint64) if trace else None
    st = Stats()
    flags = (FOOTNOTE if footnote else 0) | (BIG_SCC if big_scc else 0)
    cnt = lib.orc_topk_ex(g.n, _p(rp), _p(col), int(g.directed), int(k), _p(o), int(nthreads), flags,
                          _p(ids), _p(f), _p(r), _p(cl), _p(mv), ctypes.byref(st))
    if cnt < 0:
        raise MemoryError("oracle allocation failed")
    out = dict(ids=ids[:cnt].copy(), f=f[:cnt].copy(), r=r[:cnt].copy(),
               stats=dict(m_vis=st.m_vis, n_cut=st.n_cut, n_done=st.n_done,
                          n_trivial=st.n_trivial))
    if trace:
        out["cut_level"] = cl[:g.n].copy()
        out["mvis"] = mv[:g.n].copy()
    return out


def closeness_key(r: int, f: int) -> Fraction:
    """(r-1)^2 / f as an exact rational (the common 1/(n-1) dropped); 0 when r = 1."""
    r, f = int(r), int(f)
    return Fraction(0) if r <= 1 else Fraction((r - 1) ** 2, f)


def topk_by_definition(r, f, k: int):
    """The k nodes of largest closeness, ties by smaller id (the result the
    method must reach), from exact per-node reach and farness."""
    n = len(r)
    order = sorted(range(n), key=lambda v: (-closeness_key(r[v], f[v]), v))
    sel = order[:max(0, min(k, n))]
    return (np.array(sel, np.int32), np.array([int(f[v]) for v in sel], np.uint64),
            np.array([int(r[v]) for v in sel], np.uint32))
