"""Seeded synthetic graph generators.

These build the *inputs* of the top-k closeness method; they contain none of
its arithmetic (no distances, reach, farness or bounds).  Both the GPU path and
the CPU oracle read graphs made here and nothing else is shared between them.

Every generator draws from ``numpy.random.Generator(PCG64(seed))`` and returns a
:class:`Csr` (int32 ``row_ptr[n+1]``, int32 ``col[m]``).  Undirected graphs are
stored symmetrically (one arc per direction).  Unless a generator says
otherwise, rows are sorted, self-loops and duplicate arcs are removed.

Families (sizes are those of the workloads the method is benchmarked on):

* Barabasi-Albert preferential attachment (heavy-tailed social networks),
* R-MAT (directed web/social graphs with many strongly connected components),
* Erdos-Renyi G(n, M), 2-D grid plus random shortcuts,
* collaboration projection (actors x groups, Zipf group sizes),
* random geometric graph in the unit square (high hop diameter),
* closed-form graphs (paths, stars, cycles, complete, grids, bipartite, ...)
  used by the tests.
"""

from __future__ import annotations

import hashlib
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Csr", "from_edges", "raw_csr", "barabasi_albert", "rmat", "erdos_renyi",
    "grid_shortcuts", "collaboration", "collaboration_snapshots", "random_geometric", "path", "star",
    "cycle", "complete", "grid", "complete_bipartite", "directed_path",
    "directed_cycle", "out_star", "disjoint_union", "empty", "random_small",
]


@dataclass
class Csr:
    n: int
    row_ptr: np.ndarray  # int32 [n+1]
    col: np.ndarray      # int32 [m]
    directed: bool
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.col.shape[0])

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.ascontiguousarray(self.row_ptr, dtype=np.int32).tobytes())
        h.update(np.ascontiguousarray(self.col, dtype=np.int32).tobytes())
        return h.hexdigest()

    def edges(self):
        src = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))
        return src, self.col.astype(np.int64)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def from_edges(n: int, src, dst, directed: bool, name: str = "") -> Csr:
    """CSR with sorted rows and no self-loops or duplicate arcs.

    For ``directed=False`` every pair is stored in both directions."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    if not directed:
        src, dst = np.concatenate([src, dst]), np.concatenate([dst, src])
    keep = src != dst
    src, dst = src[keep], dst[keep]
    key = np.unique(src * np.int64(max(n, 1)) + dst)
    s = key // max(n, 1)
    d = key - s * max(n, 1)
    counts = np.bincount(s, minlength=n) if n else np.zeros(0, np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("graph too large for int32 CSR")
    return Csr(n, row_ptr.astype(np.int32), d.astype(np.int32), directed, name)


def raw_csr(n: int, src, dst, directed: bool, rng: np.random.Generator | None = None,
            name: str = "") -> Csr:
    """CSR that keeps duplicates and self-loops, with each row in a random
    order (for tests of input canonicalisation).  Undirected pairs are stored
    in both directions."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    if not directed:
        src, dst = np.concatenate([src, dst]), np.concatenate([dst, src])
    if rng is None:
        rng = _rng(0)
    perm = rng.permutation(src.shape[0])
    src, dst = src[perm], dst[perm]
    order = np.argsort(src, kind="stable")
    src, dst = src[order], dst[order]
    counts = np.bincount(src, minlength=n) if n else np.zeros(0, np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Csr(n, row_ptr.astype(np.int32), dst.astype(np.int32), directed, name)


# ---------------------------------------------------------------- families

def barabasi_albert(n: int, m: int, seed: int) -> Csr:
    """Undirected preferential attachment.

    Nodes 0..m form a clique K_{m+1}.  Every later node v attaches to m
    *distinct* earlier nodes, each drawn with probability proportional to its
    current degree, i.e. uniformly from the list of edge endpoints created so
    far.  The endpoint list is resolved in vectorised form: a target slot
    stores the index of the endpoint it copies, chains of copies are collapsed
    by pointer jumping, and rows with a repeated target redraw the repeated
    slots until all m targets of every node are distinct."""
    if n <= m:
        return complete(n)
    rng = _rng(seed)
    ci, cj = np.triu_indices(m + 1, k=1)
    n_seed = 2 * ci.shape[0]  # endpoint slots of the seed clique
    n_new = n - m - 1
    n_slots = n_seed + 2 * m * n_new
    val = np.empty(n_slots, dtype=np.int64)
    val[0:n_seed:2] = ci
    val[1:n_seed:2] = cj
    # node v's slots: [v, t_1, v, t_2, ..., v, t_m]
    v_of = np.repeat(np.arange(m + 1, n, dtype=np.int64), m)
    base = n_seed + 2 * m * (v_of - (m + 1))
    tslot = n_seed + 2 * np.arange(m * n_new, dtype=np.int64) + 1
    val[tslot - 1] = v_of
    # ptr[t]: endpoint slot copied by target slot t (t indexes target slots)
    ptr = np.minimum((rng.random(tslot.shape[0]) * base).astype(np.int64), base - 1)

    def is_target(s):
        return (s >= n_seed) & (((s - n_seed) & 1) == 1)

    while True:
        # collapse copy chains by pointer jumping over unresolved slots only
        p = ptr.copy()
        todo = np.nonzero(is_target(p))[0]
        while todo.shape[0]:
            p[todo] = p[(p[todo] - n_seed - 1) // 2]
            todo = todo[is_target(p[todo])]
        tv = val[p].reshape(n_new, m)
        srt = np.sort(tv, axis=1)
        dup_row = np.any(srt[:, 1:] == srt[:, :-1], axis=1)
        if not dup_row.any():
            break
        rows = np.nonzero(dup_row)[0]
        sub = tv[rows]
        # mark every repeat after its first occurrence in the row
        redo = np.zeros_like(sub, dtype=bool)
        for j in range(1, m):
            redo[:, j] = np.any(sub[:, :j] == sub[:, j:j + 1], axis=1)
        rr, jj = np.nonzero(redo)
        t = rows[rr] * m + jj
        ptr[t] = np.minimum((rng.random(t.shape[0]) * base[t]).astype(np.int64), base[t] - 1)
    src = np.concatenate([ci, v_of])
    dst = np.concatenate([cj, tv.reshape(-1)])
    return from_edges(n, src, dst, directed=False, name=f"ba_n{n}_m{m}_s{seed}")


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int,
         relabel: bool = True) -> Csr:
    """Directed R-MAT: ``edge_factor * 2**scale`` arcs, each placed by ``scale``
    independent quadrant choices with probabilities (a, b, c, 1-a-b-c);
    self-loops and duplicates removed, then node ids relabelled by a seeded
    random permutation so that hubs are not clustered at low ids."""
    n = 1 << scale
    rng = _rng(seed)
    n_samp = edge_factor * n
    src = np.zeros(n_samp, dtype=np.int64)
    dst = np.zeros(n_samp, dtype=np.int64)
    ab, abc = a + b, a + b + c
    for lvl in range(scale):
        u = rng.random(n_samp)
        sbit = u >= ab
        dbit = ((u >= a) & (u < ab)) | (u >= abc)
        src |= sbit.astype(np.int64) << lvl
        dst |= dbit.astype(np.int64) << lvl
        del u, sbit, dbit
    if relabel:
        perm = rng.permutation(n).astype(np.int64)
        src, dst = perm[src], perm[dst]
    return from_edges(n, src, dst, directed=True, name=f"rmat_s{scale}_e{edge_factor}_s{seed}")


def erdos_renyi(n: int, avg_deg: float, seed: int) -> Csr:
    """Undirected G(n, M) with M = round(n * avg_deg / 2) uniform pairs
    (self-loops and repeats dropped)."""
    rng = _rng(seed)
    M = int(round(n * avg_deg / 2))
    u = rng.integers(0, n, size=M)
    v = rng.integers(0, n, size=M)
    return from_edges(n, u, v, directed=False, name=f"er_n{n}_d{avg_deg}_s{seed}")


def grid_shortcuts(n: int, frac: float, seed: int) -> Csr:
    """Undirected 2-D grid with floor(sqrt(n)) columns in row-major order,
    truncated to n nodes, plus floor(frac * |grid edges|) uniform random
    shortcut pairs."""
    rng = _rng(seed)
    a = max(1, int(np.floor(np.sqrt(n))))
    ids = np.arange(n, dtype=np.int64)
    right = ids[((ids % a) != a - 1) & (ids + 1 < n)]
    down = ids[ids + a < n]
    src = np.concatenate([right, down])
    dst = np.concatenate([right + 1, down + a])
    n_sc = int(np.floor(frac * src.shape[0]))
    su = rng.integers(0, n, size=n_sc)
    sv = rng.integers(0, n, size=n_sc)
    return from_edges(n, np.concatenate([src, su]), np.concatenate([dst, sv]),
                      directed=False, name=f"grid_n{n}_f{frac}_s{seed}")


def collaboration(n_actors: int, n_groups: int, s: float, cap: int, seed: int) -> Csr:
    """Undirected projection of a random actor-group bipartite graph.

    Group sizes follow a Zipf law with exponent s truncated to 1..cap; the
    members of a group are distinct actors drawn uniformly; every group
    becomes a clique among its members."""
    sizes, offs, members = _collab_groups(n_actors, n_groups, s, cap, seed)
    return _collab_graph(n_actors, sizes, offs, members, n_groups, f"collab_a{n_actors}_g{n_groups}_s{seed}")


def collaboration_snapshots(n_actors: int, n_groups: int, s: float, cap: int, seed: int, count: int) -> list:
    """A growing collaboration graph: the groups of ``collaboration`` with the
    same arguments arrive in their drawing order, and snapshot t (t = 1 ..
    count) holds the first ceil(t n_groups / count) of them over all n_actors
    nodes (actors without a group yet are isolated).  Each snapshot's edges
    contain the previous one's; the last snapshot is ``collaboration(...)``."""
    sizes, offs, members = _collab_groups(n_actors, n_groups, s, cap, seed)
    out = []
    for t in range(1, count + 1):
        ng = -(-t * n_groups // count)
        out.append(_collab_graph(n_actors, sizes, offs, members, ng,
                                 f"collab_a{n_actors}_g{n_groups}_s{seed}_t{t}of{count}"))
    return out


def _collab_groups(n_actors: int, n_groups: int, s: float, cap: int, seed: int):
    """Group sizes (Zipf(s) on 1..cap), their offsets and distinct members."""
    rng = _rng(seed)
    ks = np.arange(1, cap + 1, dtype=np.float64)
    pmf = ks ** (-s)
    cdf = np.cumsum(pmf / pmf.sum())
    sizes = np.searchsorted(cdf, rng.random(n_groups), side="right") + 1
    sizes = np.minimum(sizes, cap).astype(np.int64)
    offs = np.zeros(n_groups + 1, dtype=np.int64)
    np.cumsum(sizes, out=offs[1:])
    members = rng.integers(0, n_actors, size=int(offs[-1]))
    gid = np.repeat(np.arange(n_groups, dtype=np.int64), sizes)
    # redraw repeated members inside a group until all are distinct
    while True:
        order = np.lexsort((members, gid))
        g2, m2 = gid[order], members[order]
        rep = np.zeros(m2.shape[0], dtype=bool)
        rep[1:] = (g2[1:] == g2[:-1]) & (m2[1:] == m2[:-1])
        if not rep.any():
            break
        idx = order[rep]
        members[idx] = rng.integers(0, n_actors, size=idx.shape[0])
    return sizes, offs, members


def _collab_graph(n_actors: int, sizes, offs, members, ng: int, name: str) -> Csr:
    """The projection of the first ng groups: a clique per group."""
    sizes = sizes[:ng]
    # clique pairs (i < j) inside every group, built group-size class by class
    src_l, dst_l = [], []
    for sz in np.unique(sizes):
        if sz < 2:
            continue
        gsel = np.nonzero(sizes == sz)[0]
        mem = members[offs[gsel][:, None] + np.arange(sz)[None, :]]
        ii, jj = np.triu_indices(int(sz), k=1)
        src_l.append(mem[:, ii].reshape(-1))
        dst_l.append(mem[:, jj].reshape(-1))
    src = np.concatenate(src_l) if src_l else np.zeros(0, np.int64)
    dst = np.concatenate(dst_l) if dst_l else np.zeros(0, np.int64)
    return from_edges(n_actors, src, dst, directed=False, name=name)


def random_geometric(n: int, avg_deg: float, seed: int) -> Csr:
    """Undirected random geometric graph: n uniform points in the unit square
    (no wrap-around), an edge between points at Euclidean distance <= rho with
    rho = sqrt(avg_deg / (pi n)); built with a cell grid of side >= rho."""
    rng = _rng(seed)
    xy = rng.random((n, 2))
    rho = float(np.sqrt(avg_deg / (np.pi * n)))
    g = max(1, int(np.floor(1.0 / rho)))
    cx = np.minimum((xy[:, 0] * g).astype(np.int64), g - 1)
    cy = np.minimum((xy[:, 1] * g).astype(np.int64), g - 1)
    cell = cy * g + cx
    order = np.argsort(cell, kind="stable")
    cell_s = cell[order]
    start = np.searchsorted(cell_s, np.arange(g * g + 1))
    cnt = np.diff(start)
    src_l, dst_l = [], []
    r2 = rho * rho
    for dx, dy in ((0, 0), (1, 0), (-1, 1), (0, 1), (1, 1)):
        ax = np.arange(g * g) % g
        ay = np.arange(g * g) // g
        bx, by = ax + dx, ay + dy
        ok = (bx >= 0) & (bx < g) & (by < g)
        A = np.nonzero(ok)[0]
        B = by[A] * g + bx[A]
        na, nb = cnt[A], cnt[B]
        npair = na * nb
        tot = int(npair.sum())
        if tot == 0:
            continue
        pa = np.repeat(A, npair)
        pb = np.repeat(B, npair)
        k = np.arange(tot) - np.repeat(np.cumsum(npair) - npair, npair)
        nbr = np.repeat(nb, npair)
        ia = start[pa] + k // nbr
        ib = start[pb] + k % nbr
        u, v = order[ia], order[ib]
        if dx == 0 and dy == 0:
            keep = u < v
            u, v = u[keep], v[keep]
        d2 = ((xy[u] - xy[v]) ** 2).sum(axis=1)
        keep = d2 <= r2
        src_l.append(u[keep])
        dst_l.append(v[keep])
    return from_edges(n, np.concatenate(src_l), np.concatenate(dst_l), directed=False,
                      name=f"rgg_n{n}_d{avg_deg}_s{seed}")


def random_small(n: int, p: float, directed: bool, seed: int) -> Csr:
    """Tiny G(n, p) graph for fuzz tests (disconnected and with many strongly
    connected components at small p)."""
    rng = _rng(seed)
    if n == 0:
        return empty(0, directed)
    mask = rng.random((n, n)) < p
    if not directed:
        mask = np.triu(mask, 1)
    u, v = np.nonzero(mask)
    return from_edges(n, u, v, directed=directed, name=f"small_n{n}_p{p}_s{seed}")


# ---------------------------------------------------------- closed forms

def empty(n: int, directed: bool = False) -> Csr:
    return Csr(n, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), directed, f"empty{n}")


def path(n: int) -> Csr:
    i = np.arange(max(n - 1, 0))
    return from_edges(n, i, i + 1, directed=False, name=f"path{n}")


def star(n: int) -> Csr:
    i = np.arange(1, n)
    return from_edges(n, np.zeros_like(i), i, directed=False, name=f"star{n}")


def cycle(n: int) -> Csr:
    i = np.arange(n)
    return from_edges(n, i, (i + 1) % n, directed=False, name=f"cycle{n}")


def circulant(n: int, gens) -> Csr:
    """Circulant graph: node i joined to (i + s) mod n for each s in gens.
    Vertex-transitive, so every node has the same farness and reach."""
    i = np.arange(n)
    src = np.concatenate([i for _ in gens])
    dst = np.concatenate([(i + s) % n for s in gens])
    return from_edges(n, src, dst, directed=False, name=f"circulant{n}")


def complete(n: int) -> Csr:
    i, j = np.triu_indices(n, k=1)
    return from_edges(n, i, j, directed=False, name=f"complete{n}")


def grid(a: int, b: int) -> Csr:
    """Full a x b grid, node (i, j) has id i * b + j."""
    ids = np.arange(a * b).reshape(a, b)
    src = np.concatenate([ids[:, :-1].ravel(), ids[:-1, :].ravel()])
    dst = np.concatenate([ids[:, 1:].ravel(), ids[1:, :].ravel()])
    return from_edges(a * b, src, dst, directed=False, name=f"grid{a}x{b}")


def complete_bipartite(a: int, b: int) -> Csr:
    """K_{a,b}: side A = 0..a-1, side B = a..a+b-1."""
    i, j = np.meshgrid(np.arange(a), np.arange(a, a + b), indexing="ij")
    return from_edges(a + b, i.ravel(), j.ravel(), directed=False, name=f"K{a},{b}")


def directed_path(n: int) -> Csr:
    i = np.arange(max(n - 1, 0))
    return from_edges(n, i, i + 1, directed=True, name=f"dpath{n}")


def directed_cycle(n: int) -> Csr:
    i = np.arange(n)
    return from_edges(n, i, (i + 1) % n, directed=True, name=f"dcycle{n}")


def out_star(n: int) -> Csr:
    i = np.arange(1, n)
    return from_edges(n, np.zeros_like(i), i, directed=True, name=f"ostar{n}")


def disjoint_union(*gs: Csr) -> Csr:
    directed = gs[0].directed
    off = 0
    src_l, dst_l = [], []
    for g in gs:
        s, d = g.edges()
        src_l.append(s + off)
        dst_l.append(d + off)
        off += g.n
    # stored arcs already hold both directions for undirected inputs
    c = from_edges(off, np.concatenate(src_l), np.concatenate(dst_l), directed=True,
                   name="+".join(g.name for g in gs))
    c.directed = directed
    return c
