"""Exact top-k closeness centrality on AMD MI355X (gfx950).

Thin ctypes binding over ``libbfscut.so`` (C ABI in ``include/bfscut.h``):
argument marshalling only, every step runs in the library's HIP kernels.
PyTorch is used, when given, only for device memory and streams.

Example::

    import paper_1507_01490_amd as bc
    from paper_1507_01490_amd import synth
    g = synth.barabasi_albert(100000, 5, seed=1)
    with bc.Graph(g.row_ptr, g.col, directed=False) as G:
        res = G.topk(10)
    res.ids, res.farness, res.reach      # decreasing closeness, ties by id
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

__all__ = ["Graph", "TopK", "Opts", "Stats", "BcError", "load_library", "closeness",
           "MODE_PLAIN", "MODE_BATCHED", "ORDER_DEGREE", "ORDER_GIVEN", "ORDER_SCORES", "ORDER_GROUPED",
           "ORDER_LEARNED", "ORDER_LEARNED_GROUPED", "MLP_PARAMS", "Server", "ServerOpts", "RequestInfo",
           "ServerStats", "footprint", "LIB_PATH", "MLP_PATH", "default_mlp", "mlp_forward", "mlp_loss_grad",
           "mlp_adam", "MultiLaunch", "topk_multi"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbfscut.so")
# trained parameters of the order perceptron (written by train_order.py)
MLP_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "order_mlp.npy")

BC_DIRECTED, BC_VALIDATE, BC_DEVICE_PTRS, BC_BIG_SCC, BC_KEEP_IDS = 0x1, 0x2, 0x4, 0x8, 0x10
BC_BOUND_FOOTNOTE, BC_BOUND_NO_TRIAL = 0x1, 0x2
ORDER_DEGREE, ORDER_GIVEN, ORDER_SCORES, ORDER_GROUPED, ORDER_LEARNED, ORDER_LEARNED_GROUPED, ORDER_AUTO = \
    0, 1, 2, 3, 4, 5, -1
ORDER_LOCALITY = 6
ORDER_LEARNED_LOCALITY = 7
MLP_PARAMS = 4481
MODE_PLAIN, MODE_BATCHED = 0, 1
_STATUS = {0: "BC_OK", -1: "BC_EINVAL", -2: "BC_EGRAPH", -3: "BC_ENOMEM", -4: "BC_EDEVICE",
           -5: "BC_EAGAIN", -6: "BC_ECANCELED"}


class BcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        self.status = status
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")


class Opts(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("mode", ctypes.c_int32), ("order", ctypes.c_int32),
                ("width", ctypes.c_int32), ("perm", ctypes.c_void_p), ("scores", ctypes.c_void_p),
                ("pull_alpha", ctypes.c_float), ("pull_beta", ctypes.c_float),
                ("slots", ctypes.c_int32), ("seed_batches", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("defer_arcs", ctypes.c_int32),
                ("lds_tables", ctypes.c_int32), ("defer_width", ctypes.c_int32), ("mlp", ctypes.c_void_p),
                ("graph_levels", ctypes.c_int32), ("seed_width", ctypes.c_int32), ("bounds", ctypes.c_uint32),
                ("first", ctypes.c_void_p), ("nfirst", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("batches", ctypes.c_uint32), ("m_vis", ctypes.c_uint64),
                ("node_arcs", ctypes.c_uint64), ("levels", ctypes.c_uint64),
                ("pull_levels", ctypes.c_uint64), ("n_cut", ctypes.c_uint64),
                ("n_done", ctypes.c_uint64), ("n_trivial", ctypes.c_uint64),
                ("preprocess_ms", ctypes.c_double), ("query_ms", ctypes.c_double),
                ("seed_ms", ctypes.c_double), ("persistent_ms", ctypes.c_double),
                ("frontier_entries", ctypes.c_uint64), ("discovered", ctypes.c_uint64),
                ("persistent_arcs", ctypes.c_uint64), ("persistent_entries", ctypes.c_uint64),
                ("persistent_discovered", ctypes.c_uint64), ("defer_ms", ctypes.c_double),
                ("n_deferred", ctypes.c_uint64), ("phase_ms", ctypes.c_double * 5),
                ("lds_levels", ctypes.c_uint64), ("record_levels", ctypes.c_uint64),
                ("spills", ctypes.c_uint64), ("record_ms", ctypes.c_double), ("record_arcs", ctypes.c_uint64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "size"}
        d["phase_ms"] = list(self.phase_ms)
        return d


class TuneReport(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("trials", ctypes.c_int32), ("default_ms", ctypes.c_double),
                ("best_ms", ctypes.c_double)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("lanes", ctypes.c_int32), ("slots", ctypes.c_int32),
                ("device", ctypes.c_int32), ("budget_bytes", ctypes.c_uint64), ("queue", ctypes.c_int32),
                ("queue_width", ctypes.c_int32), ("queue_slots", ctypes.c_int32)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("lane", ctypes.c_int32), ("uploaded", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("submit_ms", ctypes.c_double), ("start_ms", ctypes.c_double),
                ("finish_ms", ctypes.c_double), ("footprint_bytes", ctypes.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k not in ("size", "reserved")}


class ServerStats(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("graphs", ctypes.c_uint32), ("resident_graphs", ctypes.c_uint32),
                ("queued", ctypes.c_uint32), ("running", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("budget_bytes", ctypes.c_uint64), ("used_bytes", ctypes.c_uint64), ("peak_bytes", ctypes.c_uint64),
                ("uploads", ctypes.c_uint64), ("evictions", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("canceled", ctypes.c_uint64), ("queue_inflight", ctypes.c_uint64),
                ("queue_launches", ctypes.c_uint64), ("queue_batches", ctypes.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k not in ("size", "reserved")}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libbfscut.so.  Raises if it has not been built (there is no
    fallback: the library is the only implementation)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1507_01490_amd.build`")
    # torch carries HIP runtime libraries of its own.  Loaded after this
    # library has brought in the system's, they fail to find the GPU, and the
    # torch tensors this binding hands out (features, scores) cannot be made;
    # loaded first, both work side by side.  Importing torch touches no device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    lib.bc_last_error.restype = ctypes.c_char_p
    lib.bc_version.restype = ctypes.c_char_p
    lib.bc_opts_default.argtypes = [ctypes.POINTER(Opts)]
    lib.bc_graph_create.argtypes = [i32, i64, P, P, u32, P, ctypes.POINTER(P)]
    lib.bc_graph_destroy.argtypes = [P]
    lib.bc_graph_info.argtypes = [P, P, P, P, P]
    lib.bc_graph_reach.argtypes = [P, P, P]
    lib.bc_graph_csr.argtypes = [P, P, P]
    lib.bc_topk.argtypes = [P, i32, ctypes.POINTER(Opts), P, P, P, P, ctypes.POINTER(Stats)]
    f32 = ctypes.c_float
    lib.bc_farness_all.argtypes = [P, ctypes.POINTER(Opts), P, P, ctypes.POINTER(Stats)]
    lib.bc_topk_static.argtypes = [P, i32, P, P, P, P]
    lib.bc_source_order.argtypes = [P, i32, ctypes.POINTER(Opts), P]
    u64 = ctypes.c_uint64
    lib.bc_server_opts_default.argtypes = [ctypes.POINTER(ServerOpts)]
    lib.bc_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(P)]
    lib.bc_server_destroy.argtypes = [P]
    lib.bc_server_add_graph.argtypes = [P, i32, i64, P, P, u32, ctypes.POINTER(i32)]
    lib.bc_submit.argtypes = [P, i32, i32, ctypes.POINTER(Opts), ctypes.POINTER(u64)]
    lib.bc_wait.argtypes = [P, u64, i32]
    lib.bc_poll.argtypes = [P, u64, P, P, P, P, ctypes.POINTER(Stats), ctypes.POINTER(RequestInfo)]
    lib.bc_cancel.argtypes = [P, u64]
    lib.bc_progress.argtypes = [P, u64, ctypes.POINTER(u64), ctypes.POINTER(u64)]
    lib.bc_server_info.argtypes = [P, ctypes.POINTER(ServerStats)]
    lib.bc_autotune.argtypes = [P, i32, ctypes.POINTER(Opts), i32, ctypes.POINTER(Opts), ctypes.POINTER(TuneReport)]
    lib.bc_footprint.argtypes = [i32, i64, u32, i32, ctypes.POINTER(Opts), i32, ctypes.POINTER(u64),
                                 ctypes.POINTER(u64), ctypes.POINTER(u64)]
    lib.bc_multi_create.argtypes = [P, i32, P, ctypes.POINTER(Opts), i32, P, ctypes.POINTER(P)]
    lib.bc_multi_run.argtypes = [P, P, P, P, P, P]
    lib.bc_multi_destroy.argtypes = [P]
    lib.bc_topk_multi.argtypes = [P, i32, P, ctypes.POINTER(Opts), P, P, P, P, P]
    lib.bc_graph_features.argtypes = [P, P, P]
    lib.bc_mlp_forward.argtypes = [P, P, i64, P, P]
    lib.bc_mlp_loss_grad.argtypes = [P, P, P, P, i64, P, i64, P, ctypes.POINTER(ctypes.c_double), P]
    lib.bc_mlp_adam.argtypes = [P, P, P, P, i32, f32, f32, f32, f32, P]
    for name in ("bc_graph_create", "bc_graph_destroy", "bc_graph_info", "bc_graph_reach",
                 "bc_graph_csr", "bc_topk", "bc_farness_all", "bc_source_order", "bc_graph_features", "bc_server_create",
                 "bc_server_destroy", "bc_server_add_graph", "bc_submit", "bc_wait", "bc_poll", "bc_cancel",
                 "bc_server_info", "bc_footprint", "bc_autotune", "bc_mlp_forward", "bc_mlp_loss_grad",
                 "bc_mlp_adam", "bc_multi_create", "bc_multi_run", "bc_multi_destroy", "bc_topk_multi",
                 "bc_topk_static", "bc_progress"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        raise BcError(status, load_library().bc_last_error().decode(errors="replace"))


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _dptr(t, dtype, numel=None):
    """Device pointer of a contiguous torch CUDA tensor of `dtype` (None -> NULL)."""
    if t is None:
        return None
    if not (_is_torch(t) and t.is_cuda and t.is_contiguous() and t.dtype == dtype):
        raise TypeError(f"expected a contiguous CUDA tensor of {dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def default_mlp() -> np.ndarray:
    """The trained order perceptron shipped with the package (float32, MLP_PARAMS)."""
    if not os.path.exists(MLP_PATH):
        raise FileNotFoundError(f"{MLP_PATH} is missing: train it with `python -m paper_1507_01490_amd.train_order`")
    p = np.load(MLP_PATH, allow_pickle=False).astype(np.float32)
    if p.shape != (MLP_PARAMS,):
        raise ValueError(f"{MLP_PATH} holds {p.shape}, expected ({MLP_PARAMS},)")
    return p


def mlp_forward(params, x):
    """Scores y (float32 CUDA tensor, rows of x) of the order perceptron."""
    import torch
    n = x.shape[0]
    y = torch.empty(n, dtype=torch.float32, device=x.device)
    _check(load_library().bc_mlp_forward(_dptr(params, torch.float32, MLP_PARAMS), _dptr(x, torch.float32, 3 * n),
                                         n, _dptr(y, torch.float32), _stream()))
    return y


def mlp_loss_grad(params, x, t, w=None, idx=None):
    """(gradient tensor, loss) of sum w (y - t)^2 / sum w over rows idx (or all)."""
    import torch
    rows = x.shape[0]
    count = rows if idx is None else idx.numel()
    grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=x.device)
    loss = ctypes.c_double()
    _check(load_library().bc_mlp_loss_grad(
        _dptr(params, torch.float32, MLP_PARAMS), _dptr(x, torch.float32, 3 * rows), _dptr(t, torch.float32, rows),
        _dptr(w, torch.float32, rows), rows, _dptr(idx, torch.int32), count, _dptr(grad, torch.float32),
        ctypes.byref(loss), _stream()))
    return grad, loss.value


def mlp_adam(params, grad, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
             eps: float = 1e-8):
    """One Adam step on params (in place; m, v are the moment tensors)."""
    import torch
    f = torch.float32
    _check(load_library().bc_mlp_adam(_dptr(params, f, MLP_PARAMS), _dptr(grad, f, MLP_PARAMS),
                                      _dptr(m, f, MLP_PARAMS), _dptr(v, f, MLP_PARAMS), int(step), float(lr),
                                      float(beta1), float(beta2), float(eps), _stream()))


def _set_first(o: Opts, first, keep: list):
    """opts.first / nfirst from a sequence of node ids (None: none)."""
    if first is None or len(first) == 0:
        o.first, o.nfirst = None, 0
        return
    a = np.ascontiguousarray(first, dtype=np.int32)
    keep.append(a)
    o.first, o.nfirst = a.ctypes.data_as(ctypes.c_void_p), int(a.shape[0])


def make_opts(n: int, keep: list, mode="plain", width=64, order=None, scores=None, pull_alpha=3.0, pull_beta=24.0,
              slots=0, seed_batches=-1, defer_arcs=0, chunk=0, lds_tables=True, mlp=None, defer_width=0,
              graph_levels=None, seed_width=0, footnote=False, trial=True, first=None) -> Opts:
    """bc_opts for a graph of n nodes; host arrays the options point at are
    appended to `keep` (they must outlive the call that reads them)."""
    lib = load_library()
    o = Opts()
    lib.bc_opts_default(ctypes.byref(o))
    if isinstance(mode, str) and mode not in ("plain", "batched"):
        raise ValueError(f"unknown mode {mode!r}")
    o.mode = {"plain": MODE_PLAIN, "batched": MODE_BATCHED}[mode] if isinstance(mode, str) else int(mode)
    o.width = int(width)
    o.pull_alpha = float(pull_alpha)
    o.pull_beta = float(pull_beta)
    o.slots = int(slots)
    o.seed_batches = int(seed_batches)
    o.defer_arcs = int(defer_arcs)
    o.chunk = int(chunk)
    o.lds_tables = 1 if lds_tables == "spill" else (0 if lds_tables else -1)
    o.defer_width = int(defer_width)
    o.seed_width = int(seed_width)
    o.bounds = (BC_BOUND_FOOTNOTE if footnote else 0) | (0 if trial else BC_BOUND_NO_TRIAL)
    _set_first(o, first, keep)
    if graph_levels is not None:
        o.graph_levels = int(graph_levels)
    if isinstance(order, str) and order in ("learned", "learned_grouped", "learned_locality"):
        prm = np.ascontiguousarray(default_mlp() if mlp is None else mlp, dtype=np.float32)
        if prm.shape != (MLP_PARAMS,):
            raise ValueError(f"mlp must hold {MLP_PARAMS} floats")
        o.order = {"learned": ORDER_LEARNED, "learned_grouped": ORDER_LEARNED_GROUPED,
                   "learned_locality": ORDER_LEARNED_LOCALITY}[order]
        o.mlp = prm.ctypes.data
        keep.append(prm)
    elif isinstance(order, str):
        o.order = {"degree": ORDER_DEGREE, "grouped": ORDER_GROUPED, "locality": ORDER_LOCALITY,
                   "auto": ORDER_AUTO}[order]
    elif order is not None:
        perm = np.ascontiguousarray(order, dtype=np.int32)
        if perm.shape[0] != n:
            raise ValueError("order must hold n entries")
        o.order = ORDER_GIVEN
        o.perm = perm.ctypes.data
        keep.append(perm)
    elif scores is not None:
        sc = np.ascontiguousarray(scores, dtype=np.float32)
        if sc.shape[0] != n:
            raise ValueError("scores must hold n entries")
        o.order = ORDER_SCORES
        o.scores = sc.ctypes.data
        keep.append(sc)
    return o


def footprint(n: int, m: int, directed: bool = False, k: int = 10, slots: int = 64, **kw):
    """(graph_bytes, upload_bytes, query_bytes): the serving admission estimate."""
    keep = []
    o = make_opts(n, keep, **kw)
    g, u, q = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    _check(load_library().bc_footprint(int(n), int(m), BC_DIRECTED if directed else 0, int(k), ctypes.byref(o),
                                       int(slots), ctypes.byref(g), ctypes.byref(u), ctypes.byref(q)))
    return g.value, u.value, q.value


def closeness(r, f, n: int) -> np.ndarray:
    """(r-1)^2 / ((n-1) f) for display (0 when r = 1); ranking never uses it."""
    r = np.asarray(r, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        c = (r - 1.0) ** 2 / (max(n - 1, 1) * f)
    return np.where(r <= 1, 0.0, c)


@dataclass
class TopK:
    ids: np.ndarray
    farness: np.ndarray
    reach: np.ndarray
    stats: dict = field(default_factory=dict)


class Graph:
    """A CSR graph resident on the GPU with its pre-processed reach data.

    ``row_ptr``/``col`` are int32 numpy arrays (host) or int32 torch CUDA
    tensors (device); either way the library copies them.  big_scc: directed
    reach bounds with the largest-SCC refinement (BC_BIG_SCC); keep_ids: no
    breadth-first renumbering of an undirected graph on the device
    (BC_KEEP_IDS; results are in the caller's ids either way)."""

    def __init__(self, row_ptr, col, directed: bool = False, validate: bool = False, stream=None,
                 big_scc: bool = False, keep_ids: bool = False):
        lib = load_library()
        flags = (BC_DIRECTED if directed else 0) | (BC_VALIDATE if validate else 0) | (BC_BIG_SCC if big_scc else 0) \
            | (BC_KEEP_IDS if keep_ids else 0)
        if _is_torch(row_ptr):
            if not row_ptr.is_cuda:
                row_ptr, col = row_ptr.numpy(), col.numpy()
            else:
                flags |= BC_DEVICE_PTRS
        if flags & BC_DEVICE_PTRS:
            n = int(row_ptr.numel()) - 1
            m = int(col.numel())
            rp_p = ctypes.c_void_p(row_ptr.data_ptr())
            col_p = ctypes.c_void_p(col.data_ptr()) if m else None
            keep = (row_ptr, col)
        else:
            rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
            cl = np.ascontiguousarray(col, dtype=np.int32)
            n = int(rp.shape[0]) - 1
            m = int(cl.shape[0])
            rp_p, col_p = _ptr(rp), (_ptr(cl) if m else None)
            keep = (rp, cl)
        s = None
        if stream is not None:
            s = ctypes.c_void_p(int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream))
        h = ctypes.c_void_p()
        _check(lib.bc_graph_create(n, m, rp_p, col_p, flags, s, ctypes.byref(h)))
        del keep
        self._h = h
        self.directed = bool(directed)
        nn, mm, dd, pp = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_double()
        _check(lib.bc_graph_info(h, ctypes.byref(nn), ctypes.byref(mm), ctypes.byref(dd), ctypes.byref(pp)))
        self.n, self.m, self.preprocess_ms = nn.value, mm.value, pp.value

    # context manager / lifetime
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(load_library().bc_graph_destroy(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reach(self):
        """(lo, hi) per node: undirected r(v) twice; directed alpha(v), omega(v)."""
        lo = np.zeros(max(self.n, 1), np.uint32)
        hi = np.zeros(max(self.n, 1), np.uint32)
        _check(load_library().bc_graph_reach(self._h, _ptr(lo), _ptr(hi)))
        return lo[:self.n], hi[:self.n]

    def csr(self):
        rp = np.zeros(self.n + 1, np.int32)
        col = np.zeros(max(self.m, 1), np.int32)
        _check(load_library().bc_graph_csr(self._h, _ptr(rp), _ptr(col)))
        return rp, col[:self.m]

    def features(self):
        """(x, core): standardised order features (float32 CUDA tensor n x 3)
        and core numbers (int32 CUDA tensor, values of the uint32 array)."""
        import torch
        x = torch.empty((max(self.n, 1), 3), dtype=torch.float32, device="cuda")
        core = torch.empty(max(self.n, 1), dtype=torch.int32, device="cuda")
        _check(load_library().bc_graph_features(self._h, ctypes.c_void_p(x.data_ptr()),
                                                ctypes.c_void_p(core.data_ptr())))
        return x[:self.n], core[:self.n]

    def _opts(self, mode, width, order, scores, pull_alpha, pull_beta, slots, seed_batches, defer_arcs, chunk,
              lds_tables, mlp, keep):
        return make_opts(self.n, keep, mode=mode, width=width, order=order, scores=scores, pull_alpha=pull_alpha,
                         pull_beta=pull_beta, slots=slots, seed_batches=seed_batches, defer_arcs=defer_arcs,
                         chunk=chunk, lds_tables=lds_tables, mlp=mlp)

    def topk(self, k: int, mode: str | int = "plain", width: int = 64, order=None, scores=None,
             pull_alpha: float = 3.0, pull_beta: float = 24.0, slots: int = 0,
             seed_batches: int = -1, defer_arcs: int = 0, chunk: int = 0,
             lds_tables: bool = True, mlp=None, defer_width: int = 0, graph_levels=None,
             seed_width: int = 0, footnote: bool = False, trial: bool = True, first=None) -> TopK:
        """The k nodes of largest closeness: ids, exact farness, exact reach.

        order: None (automatic), "degree", "grouped", "locality" (breadth-first
        from an approximate centre), "learned" (the order
        perceptron `mlp`, default the trained one), "learned_grouped" (the
        k best-scored sources, then the grouped order), "learned_locality" (the
        k best-scored sources, then the locality order), or a
        permutation of range(n); scores: per-node floats (decreasing score
        first); footnote: the undirected footnote bound (BC_BOUND_FOOTNOTE); trial=False skips
        the over-counted bound test before exact level counts (BC_BOUND_NO_TRIAL); first: node ids
        taken before all others (a warm start, e.g. the previous top-k of a grown graph)."""
        keep = []
        o = self._opts(mode, width, order, scores, pull_alpha, pull_beta, slots, seed_batches, defer_arcs, chunk,
                       lds_tables, mlp, keep)
        o.defer_width = int(defer_width)
        o.seed_width = int(seed_width)
        o.bounds = (BC_BOUND_FOOTNOTE if footnote else 0) | (0 if trial else BC_BOUND_NO_TRIAL)
        _set_first(o, first, keep)
        if graph_levels is not None:
            o.graph_levels = int(graph_levels)
        kk = max(1, int(k))
        ids = np.zeros(kk, np.int32)
        far = np.zeros(kk, np.uint64)
        rea = np.zeros(kk, np.uint32)
        cnt = ctypes.c_int32()
        st = Stats()
        st.size = ctypes.sizeof(Stats)
        _check(load_library().bc_topk(self._h, int(k), ctypes.byref(o), _ptr(ids), _ptr(far), _ptr(rea),
                                      ctypes.byref(cnt), ctypes.byref(st)))
        c = cnt.value
        return TopK(ids[:c].copy(), far[:c].copy(), rea[:c].copy(), st.as_dict())

    def topk_static(self, k: int) -> TopK:
        """bc_topk_static: plain-mode top-k with every buffer in the library's
        static device array (no allocation; graphs up to ~900k nodes)."""
        kk = max(1, int(k))
        ids = np.zeros(kk, np.int32)
        far = np.zeros(kk, np.uint64)
        rea = np.zeros(kk, np.uint32)
        cnt = ctypes.c_int32()
        _check(load_library().bc_topk_static(self._h, int(k), _ptr(ids), _ptr(far), _ptr(rea), ctypes.byref(cnt)))
        c = cnt.value
        return TopK(ids[:c].copy(), far[:c].copy(), rea[:c].copy(), {})

    def source_order(self, k: int = 10, mode: str | int = "batched", width: int = 64, order=None, scores=None,
                     mlp=None, seed_batches: int = -1, seed_width: int = 0, first=None) -> np.ndarray:
        """The order (n node ids) in which topk with the same arguments takes its sources."""
        keep = []
        o = self._opts(mode, width, order, scores, 3.0, 24.0, 0, seed_batches, 0, 0, True, mlp, keep)
        o.seed_width = int(seed_width)
        _set_first(o, first, keep)
        out = np.zeros(max(1, self.n), np.int32)
        _check(load_library().bc_source_order(self._h, int(k), ctypes.byref(o), _ptr(out)))
        return out[:self.n].copy()

    def autotune(self, k: int, repeats: int = 1, **kw):
        """(best options as topk keyword arguments, report) for this graph and k."""
        keep = []
        o = self._opts(kw.pop("mode", "batched"), kw.pop("width", 64), kw.pop("order", None), None,
                       kw.pop("pull_alpha", 3.0), kw.pop("pull_beta", 24.0), kw.pop("slots", 0),
                       kw.pop("seed_batches", -1), kw.pop("defer_arcs", 0), 0, kw.pop("lds_tables", True), None, keep)
        if kw:
            raise TypeError(f"unexpected options {sorted(kw)}")
        best = Opts()
        rep = TuneReport()
        rep.size = ctypes.sizeof(TuneReport)
        _check(load_library().bc_autotune(self._h, int(k), ctypes.byref(o), int(repeats), ctypes.byref(best),
                                          ctypes.byref(rep)))
        order = {ORDER_DEGREE: "degree", ORDER_GROUPED: "grouped", ORDER_LOCALITY: "locality",
                 ORDER_AUTO: None}.get(best.order, None)
        tuned = dict(mode="batched", width=best.width, defer_arcs=best.defer_arcs, defer_width=best.defer_width,
                     pull_alpha=best.pull_alpha, slots=best.slots, order=order)
        return tuned, dict(trials=rep.trials, default_ms=rep.default_ms, best_ms=rep.best_ms)

    def farness_all(self, mode: str | int = "batched", width: int = 64, order=None, slots: int = 0,
                    seed_batches: int = -1, defer_arcs: int = 0, lds_tables: bool = True):
        """(farness, reach, stats) of every node, exactly (no cut)."""
        keep = []
        o = self._opts(mode, width, order, None, 3.0, 24.0, slots, seed_batches, defer_arcs, 0, lds_tables,
                       None, keep)
        far = np.zeros(max(self.n, 1), np.uint64)
        rea = np.zeros(max(self.n, 1), np.uint32)
        st = Stats()
        st.size = ctypes.sizeof(Stats)
        _check(load_library().bc_farness_all(self._h, ctypes.byref(o), _ptr(far), _ptr(rea), ctypes.byref(st)))
        return far[:self.n], rea[:self.n], st.as_dict()


class Server:
    """Serving queue over registered graphs (bc_server_*): submit returns a
    ticket at once; poll returns None until the result is ready."""

    def __init__(self, lanes: int = 4, slots: int = 64, budget_bytes: int = 0, device: int = -1, queue: bool = False,
                 queue_width: int = 64, queue_slots: int = 0):
        """queue=True: continuous batching through the device-visible queue of
        one running persistent kernel (bc_server_opts.queue)."""
        lib = load_library()
        o = ServerOpts()
        lib.bc_server_opts_default(ctypes.byref(o))
        o.lanes, o.slots, o.budget_bytes, o.device = int(lanes), int(slots), int(budget_bytes), int(device)
        o.queue, o.queue_width, o.queue_slots = int(bool(queue)), int(queue_width), int(queue_slots)
        h = ctypes.c_void_p()
        _check(lib.bc_server_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._n = {}
        self._k = {}

    def add_graph(self, row_ptr, col, directed: bool = False, validate: bool = False, big_scc: bool = False) -> int:
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        gid = ctypes.c_int32()
        flags = (BC_DIRECTED if directed else 0) | (BC_VALIDATE if validate else 0) | (BC_BIG_SCC if big_scc else 0)
        _check(load_library().bc_server_add_graph(self._h, int(rp.shape[0]) - 1, int(cl.shape[0]), _ptr(rp),
                                                  _ptr(cl) if cl.shape[0] else None, flags, ctypes.byref(gid)))
        self._n[gid.value] = int(rp.shape[0]) - 1
        return gid.value

    def submit(self, graph_id: int, k: int, **kw) -> int:
        keep = []
        o = make_opts(self._n.get(graph_id, 0), keep, **kw)
        t = ctypes.c_uint64()
        _check(load_library().bc_submit(self._h, int(graph_id), int(k), ctypes.byref(o), ctypes.byref(t)))
        self._k[t.value] = max(1, int(k))
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1) -> bool:
        st = load_library().bc_wait(self._h, ctypes.c_uint64(ticket), int(timeout_ms))
        if st == -5:
            return False
        _check(st)
        return True

    def poll(self, ticket: int):
        kk = self._k.get(ticket, 1)
        ids = np.zeros(kk, np.int32)
        far = np.zeros(kk, np.uint64)
        rea = np.zeros(kk, np.uint32)
        cnt = ctypes.c_int32()
        st = Stats()
        st.size = ctypes.sizeof(Stats)
        info = RequestInfo()
        info.size = ctypes.sizeof(RequestInfo)
        rc = load_library().bc_poll(self._h, ctypes.c_uint64(ticket), _ptr(ids), _ptr(far), _ptr(rea),
                                    ctypes.byref(cnt), ctypes.byref(st), ctypes.byref(info))
        if rc == -5:
            return None
        self._k.pop(ticket, None)
        _check(rc)
        c = cnt.value
        res = TopK(ids[:c].copy(), far[:c].copy(), rea[:c].copy(), st.as_dict())
        res.info = info.as_dict()
        return res

    def progress(self, ticket: int):
        """(finished batches, all batches) of a request in the device queue (0, 0 otherwise)."""
        d, t = ctypes.c_uint64(), ctypes.c_uint64()
        _check(load_library().bc_progress(self._h, ctypes.c_uint64(ticket), ctypes.byref(d), ctypes.byref(t)))
        return d.value, t.value

    def cancel(self, ticket: int):
        _check(load_library().bc_cancel(self._h, ctypes.c_uint64(ticket)))

    def info(self) -> dict:
        st = ServerStats()
        st.size = ctypes.sizeof(ServerStats)
        _check(load_library().bc_server_info(self._h, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(load_library().bc_server_destroy(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _multi_args(graphs, ks, keep, order=None, width=64, slots=0, footnote=False, mlp=None):
    graphs = list(graphs)
    ks = [int(k) for k in ks]
    if len(graphs) != len(ks) or not graphs:
        raise ValueError("one k per graph, at least one graph")
    o = make_opts(max(g.n for g in graphs), keep, mode="batched", width=width, slots=slots, footnote=footnote,
                  order=order if (order is None or isinstance(order, str)) else None, mlp=mlp)
    if order is not None and not isinstance(order, str):
        raise TypeError("job launches take an order rule (a string), not a permutation")
    hs = (ctypes.c_void_p * len(graphs))(*[g._h.value for g in graphs])
    kv = np.ascontiguousarray(ks, dtype=np.int32)
    keep += [hs, kv]
    return graphs, ks, o, hs, kv


def _multi_results(graphs, ks, ids, far, rea, cnt, sts):
    out, off = [], 0
    for i, k in enumerate(ks):
        c = int(cnt[i])
        out.append(TopK(ids[off:off + c].copy(), far[off:off + c].copy(), rea[off:off + c].copy(),
                        sts[i].as_dict()))
        off += k
    return out


class MultiLaunch:
    """Top-k queries over several graphs in one persistent launch
    (bc_multi_create / bc_multi_run): results are each graph's own top-k.
    capture=True records the launch as a HIP graph replayed by every run()."""

    def __init__(self, graphs, ks, capture: bool = True, stream=None, **kw):
        keep = []
        self._graphs, self._ks, o, hs, kv = _multi_args(graphs, ks, keep, **kw)
        s = None
        if stream is not None:
            s = ctypes.c_void_p(int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream))
        h = ctypes.c_void_p()
        _check(load_library().bc_multi_create(hs, len(self._graphs), _ptr(kv), ctypes.byref(o), int(bool(capture)), s,
                                              ctypes.byref(h)))
        self._h = h

    def run(self):
        """List of TopK, one per query, in the order given."""
        tot = sum(self._ks)
        ids = np.zeros(tot, np.int32)
        far = np.zeros(tot, np.uint64)
        rea = np.zeros(tot, np.uint32)
        cnt = np.zeros(len(self._ks), np.int32)
        sts = (Stats * len(self._ks))()
        for st in sts:
            st.size = ctypes.sizeof(Stats)
        _check(load_library().bc_multi_run(self._h, _ptr(ids), _ptr(far), _ptr(rea), _ptr(cnt),
                                           ctypes.cast(sts, ctypes.c_void_p)))
        return _multi_results(self._graphs, self._ks, ids, far, rea, cnt, sts)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(load_library().bc_multi_destroy(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def topk_multi(graphs, ks, **kw):
    """Top-k of several graphs in one persistent launch (bc_topk_multi)."""
    keep = []
    graphs, ks, o, hs, kv = _multi_args(graphs, ks, keep, **kw)
    tot = sum(ks)
    ids = np.zeros(tot, np.int32)
    far = np.zeros(tot, np.uint64)
    rea = np.zeros(tot, np.uint32)
    cnt = np.zeros(len(ks), np.int32)
    sts = (Stats * len(ks))()
    for st in sts:
        st.size = ctypes.sizeof(Stats)
    _check(load_library().bc_topk_multi(hs, len(graphs), _ptr(kv), ctypes.byref(o), _ptr(ids), _ptr(far), _ptr(rea),
                                        _ptr(cnt), ctypes.cast(sts, ctypes.c_void_p)))
    return _multi_results(graphs, ks, ids, far, rea, cnt, sts)
