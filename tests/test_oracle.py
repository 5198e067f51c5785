"""Pins of the CPU oracle against things other than itself.

* closed forms of reach and farness on paths, stars, cycles, complete graphs,
  grids, complete bipartite graphs, directed paths/cycles/out-stars and
  disjoint unions (values derived by hand, written below);
* exact visited-arc counts on stars and complete graphs derived by hand from
  Lemma 1 (the bound is tight at level 0 there, so a dropped or wrong term
  changes where the search stops);
* brute force checked against SciPy's shortest paths and NetworkX closeness;
* top-k from Algorithm 1 equal to the top-k of the definition on thousands of
  fuzzed graphs (directed, undirected, disconnected, many SCCs), for any
  processing order and thread count;
* SCCs against SciPy; alpha <= r <= omega against brute-force reach, with
  hand-derived values on small DAGs;
* per-source cut levels and visited arcs re-derived from SciPy distances.
"""

from fractions import Fraction

import networkx as nx
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components, shortest_path

import oracle
from paper_1507_01490_amd import synth


def scipy_dist(g):
    A = sp.csr_matrix((np.ones(g.m), g.col, g.row_ptr), shape=(g.n, g.n))
    return shortest_path(A, method="D", directed=True, unweighted=True)


def scipy_rf(g):
    D = scipy_dist(g)
    fin = np.isfinite(D)
    r = fin.sum(axis=1).astype(np.int64)
    f = np.where(fin, D, 0).sum(axis=1).astype(np.int64)
    return r, f


def path_far(L, i):
    return i * (i + 1) // 2 + (L - 1 - i) * (L - i) // 2


def check_topk_all_k(g, r_exp, f_exp):
    n = g.n
    for k in sorted({1, 2, 3, n // 2, n - 1, n, n + 3}):
        if k < 1:
            continue
        ids_d, f_d, r_d = oracle.topk_by_definition(r_exp, f_exp, k)
        for nth in (1, 3):
            got = oracle.topk(g, k, nthreads=nth)
            assert got["ids"].tolist() == ids_d.tolist(), (g.name, k, nth)
            assert got["f"].tolist() == f_d.tolist()
            assert got["r"].tolist() == r_d.tolist()


# ------------------------------------------------------------ closed forms

@pytest.mark.parametrize("n", [2, 3, 4, 7, 10, 31])
def test_path(n):
    g = synth.path(n)
    r, f = oracle.bruteforce(g)
    assert r.tolist() == [n] * n
    assert f.tolist() == [path_far(n, i) for i in range(n)]
    got = oracle.topk(g, 1)
    assert got["ids"].tolist() == [(n - 1) // 2]
    check_topk_all_k(g, r, f)


@pytest.mark.parametrize("n", [2, 3, 5, 17])
def test_star(n):
    g = synth.star(n)
    r, f = oracle.bruteforce(g)
    assert f.tolist() == [n - 1] + [2 * n - 3] * (n - 1)
    check_topk_all_k(g, r, f)


@pytest.mark.parametrize("n", [3, 4, 9, 10])
def test_cycle(n):
    g = synth.cycle(n)
    r, f = oracle.bruteforce(g)
    exp = (n * n - 1) // 4 if n % 2 else n * n // 4
    assert f.tolist() == [exp] * n
    for k in (1, 3, n):
        assert oracle.topk(g, k)["ids"].tolist() == list(range(min(k, n)))


@pytest.mark.parametrize("n", [1, 2, 5, 12])
def test_complete(n):
    g = synth.complete(n)
    r, f = oracle.bruteforce(g)
    assert f.tolist() == [n - 1] * n
    assert r.tolist() == [n] * n
    for k in (1, 4, n):
        assert oracle.topk(g, k)["ids"].tolist() == list(range(min(k, n)))


@pytest.mark.parametrize("a,b", [(1, 1), (1, 5), (3, 4), (6, 6), (2, 9)])
def test_grid(a, b):
    g = synth.grid(a, b)
    r, f = oracle.bruteforce(g)
    exp = [b * path_far(a, i) + a * path_far(b, j) for i in range(a) for j in range(b)]
    assert f.tolist() == exp
    check_topk_all_k(g, r, f)


@pytest.mark.parametrize("a,b", [(1, 3), (2, 5), (4, 4), (3, 7)])
def test_complete_bipartite(a, b):
    g = synth.complete_bipartite(a, b)
    r, f = oracle.bruteforce(g)
    assert f.tolist() == [b + 2 * (a - 1)] * a + [a + 2 * (b - 1)] * b
    check_topk_all_k(g, r, f)


@pytest.mark.parametrize("n", [1, 2, 6, 15])
def test_directed_path(n):
    g = synth.directed_path(n)
    r, f = oracle.bruteforce(g)
    assert r.tolist() == [n - i for i in range(n)]
    assert f.tolist() == [(n - i - 1) * (n - i) // 2 for i in range(n)]
    check_topk_all_k(g, r, f)


@pytest.mark.parametrize("n", [2, 5, 11])
def test_directed_cycle(n):
    g = synth.directed_cycle(n)
    r, f = oracle.bruteforce(g)
    assert r.tolist() == [n] * n and f.tolist() == [n * (n - 1) // 2] * n
    a, o = oracle.alpha_omega(g)
    assert a.tolist() == [n] * n and o.tolist() == [n] * n
    check_topk_all_k(g, r, f)


@pytest.mark.parametrize("n", [2, 6, 13])
def test_out_star(n):
    g = synth.out_star(n)
    r, f = oracle.bruteforce(g)
    assert r.tolist() == [n] + [1] * (n - 1)
    assert f.tolist() == [n - 1] + [0] * (n - 1)
    check_topk_all_k(g, r, f)


def test_disjoint_union():
    g = synth.disjoint_union(synth.path(5), synth.star(4), synth.complete(3), synth.empty(2))
    r, f = oracle.bruteforce(g)
    assert r.tolist() == [5] * 5 + [4] * 4 + [3] * 3 + [1, 1]
    assert f.tolist() == [path_far(5, i) for i in range(5)] + [3, 5, 5, 5] + [2, 2, 2] + [0, 0]
    check_topk_all_k(g, r, f)


def test_empty_and_isolated():
    for n in (1, 2, 5):
        g = synth.empty(n)
        got = oracle.topk(g, 3)
        assert got["ids"].tolist() == list(range(min(3, n)))
        assert got["r"].tolist() == [1] * min(3, n)
        assert got["f"].tolist() == [0] * min(3, n)
    assert oracle.topk(synth.empty(0), 3)["ids"].tolist() == []
    assert oracle.topk(synth.path(4), 0)["ids"].tolist() == []


# -------------------------------------- visited arcs derived by hand (Lemma 1)

@pytest.mark.parametrize("n", [4, 9, 40])
def test_star_visited_arcs(n):
    """Star, centre 0, degree order = centre then leaves by id.

    k=1: the centre's search scans n-1 arcs at level 0 and n-1 at level 1.
    Every leaf is cut at level 0: its bound f_0 - deg + 2 (n - 1) = 2n - 3
    equals its exact farness, larger than the centre's n - 1.
    k=2: leaf 1 completes (1 + (n-1) + (n-2) arcs); every later leaf ties
    with it at level 0 and loses the tie on id, so it is cut there."""
    g = synth.star(n)
    o1 = oracle.topk(g, 1, trace=True)
    assert o1["stats"]["m_vis"] == 2 * (n - 1)
    assert o1["cut_level"].tolist() == [-1] + [0] * (n - 1)
    o2 = oracle.topk(g, 2, trace=True)
    assert o2["stats"]["m_vis"] == 2 * (n - 1) + (2 * n - 2)
    assert o2["cut_level"].tolist() == [-1, -1] + [0] * (n - 2)
    assert o2["ids"].tolist() == [0, 1]


@pytest.mark.parametrize("n", [3, 6, 20])
def test_complete_visited_arcs(n):
    """K_n, k=1: node 0 scans (n-1) + (n-1)^2 arcs; each later node has the
    level-0 bound 0 - (n-1) + 2 (n-1) = n - 1, equal to node 0's farness, and
    is cut on the id tie-break without scanning an arc."""
    g = synth.complete(n)
    o = oracle.topk(g, 1, trace=True)
    assert o["stats"]["m_vis"] == (n - 1) + (n - 1) ** 2
    assert o["cut_level"].tolist() == [-1] + [0] * (n - 1)


def test_path_first_cut_by_hand():
    """Path 0-1-2-3-4, k=1.  Degree order: 1, 2, 3 (degree 2), then 0, 4.
    Node 1 completes (f=7, r=5) and becomes the threshold.  Node 2: its
    level bounds f_d - ~gamma_{d+1} + (d+2)(5 - n_d) are 0-2+8 = 6, 2-4+6 = 4
    and 6-2+0 = 4, all below 7, so it completes with f=6 and replaces node 1.
    Node 3: level-0 bound 0-2+8 = 6 equals 6 and id 3 > 2, cut at level 0.
    Nodes 0 and 4: level-0 bound 0-1+8 = 7 > 6, cut at level 0."""
    g = synth.path(5)
    o = oracle.topk(g, 1, trace=True)
    assert o["ids"].tolist() == [2] and o["f"].tolist() == [6]
    assert o["cut_level"].tolist() == [0, -1, -1, 0, 0]
    # node 1 scans 2 + 3 + 2 + 1 arcs (levels 0..3), node 2 scans 2 + 4 + 2
    assert o["mvis"].tolist() == [0, 8, 8, 0, 0]


# ------------------------------------------- independent library brute force

@pytest.mark.parametrize("seed", range(12))
def test_bruteforce_vs_scipy(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 70))
    directed = bool(seed % 2)
    g = synth.random_small(n, float(rng.uniform(0.01, 0.15)), directed, seed)
    r, f = oracle.bruteforce(g, nthreads=2)
    r2, f2 = scipy_rf(g)
    assert r.tolist() == r2.tolist() and f.tolist() == f2.tolist()


@pytest.mark.parametrize("seed", range(6))
def test_bruteforce_vs_networkx(seed):
    directed = bool(seed % 2)
    g = synth.random_small(40, 0.06, directed, 100 + seed)
    r, f = oracle.bruteforce(g)
    G = nx.DiGraph() if directed else nx.Graph()
    G.add_nodes_from(range(g.n))
    s, d = g.edges()
    G.add_edges_from(zip(s.tolist(), d.tolist()))
    # NetworkX measures incoming distances on digraphs, hence the reverse
    c = nx.closeness_centrality(G.reverse() if directed else G, wf_improved=True)
    for v in range(g.n):
        mine = 0.0 if r[v] <= 1 else (int(r[v]) - 1) ** 2 / ((g.n - 1) * int(f[v]))
        assert abs(mine - c[v]) <= 1e-12 * max(1.0, abs(c[v]))


def test_ba2000_bruteforce_vs_scipy():
    g = synth.barabasi_albert(2000, 5, 0)
    r, f = oracle.bruteforce(g, nthreads=8)
    r2, f2 = scipy_rf(g)
    assert r.tolist() == r2.tolist() and f.tolist() == f2.tolist()
    for k in (1, 10):
        ids_d, f_d, r_d = oracle.topk_by_definition(r, f, k)
        got = oracle.topk(g, k)
        assert got["ids"].tolist() == ids_d.tolist()
        assert got["f"].tolist() == f_d.tolist() and got["r"].tolist() == r_d.tolist()
        # the method prunes: far fewer arcs than the textbook n * m
        assert got["stats"]["m_vis"] < 0.2 * g.n * g.m


# ------------------------------------------------------------- fuzzing

@pytest.mark.parametrize("block", range(8))
def test_fuzz_topk_equals_definition(block):
    rng = np.random.default_rng(1000 + block)
    for it in range(60):
        n = int(rng.integers(1, 48))
        directed = bool(rng.integers(0, 2))
        p = float(rng.choice([0.02, 0.05, 0.1, 0.25]))
        g = synth.random_small(n, p, directed, int(rng.integers(0, 2**31)))
        r, f = scipy_rf(g)
        k = int(rng.integers(1, n + 2))
        ids_d, f_d, r_d = oracle.topk_by_definition(r, f, k)
        order = None
        if it % 3 == 1:
            order = rng.permutation(n).astype(np.int32)
        nth = 1 if it % 2 == 0 else 3
        got = oracle.topk(g, k, order=order, nthreads=nth)
        assert got["ids"].tolist() == ids_d.tolist(), (n, directed, p, k)
        assert got["f"].tolist() == f_d.tolist()
        assert got["r"].tolist() == r_d.tolist()


def test_canonicalisation():
    rng = np.random.default_rng(7)
    for directed in (False, True):
        n = 30
        s = rng.integers(0, n, 200)
        d = rng.integers(0, n, 200)
        s = np.concatenate([s, np.arange(5)])
        d = np.concatenate([d, np.arange(5)])      # self-loops
        s = np.concatenate([s, s[:40]])
        d = np.concatenate([d, d[:40]])            # repeats
        raw = synth.raw_csr(n, s, d, directed, rng)
        clean = synth.from_edges(n, s, d, directed)
        rp, col = oracle.canonicalize(raw)
        assert rp.tolist() == clean.row_ptr.tolist() and col.tolist() == clean.col.tolist()
        for k in (1, 5, 30):
            a = oracle.topk(raw, k)
            b = oracle.topk(clean, k)
            assert a["ids"].tolist() == b["ids"].tolist() and a["f"].tolist() == b["f"].tolist()


# ------------------------------------------------------------ SCC, alpha/omega

@pytest.mark.parametrize("seed", range(10))
def test_scc_vs_scipy(seed):
    g = synth.random_small(80, 0.02 + 0.004 * seed, True, 500 + seed)
    nc, comp = oracle.scc(g)
    A = sp.csr_matrix((np.ones(g.m), g.col, g.row_ptr), shape=(g.n, g.n))
    nc2, lab = connected_components(A, directed=True, connection="strong")
    assert nc == nc2
    # same partition
    pairs = set(zip(comp.tolist(), lab.tolist()))
    assert len(pairs) == nc
    # completion order is reverse topological: arcs go to smaller component ids
    s, d = g.edges()
    cs, cd = comp[s], comp[d]
    assert np.all((cs == cd) | (cs > cd))


@pytest.mark.parametrize("seed", range(10))
def test_alpha_omega_bracket_reach(seed):
    g = synth.random_small(70, 0.015 + 0.004 * seed, True, 900 + seed)
    r, _ = scipy_rf(g)
    a, o = oracle.alpha_omega(g)
    assert np.all(a <= r) and np.all(r <= o) and np.all(o <= g.n)
    assert np.all(a >= 1)
    # alpha = 1 exactly for nodes without out-arcs
    deg = np.diff(g.row_ptr)
    assert np.array_equal(a == 1, deg == 0)


def test_alpha_omega_by_hand():
    # diamond 0->1, 0->2, 1->3, 2->3 plus a tail 3->4 and an isolated 5
    g = synth.from_edges(6, [0, 0, 1, 2, 3], [1, 2, 3, 3, 4], directed=True)
    a, o = oracle.alpha_omega(g)
    # sinks: alpha = omega = 1; 3: 2; 1, 2: 3; 0: 1 + max(3, 3) = 4, 1 + 3 + 3 = 7 -> cap n = 6
    assert a.tolist() == [4, 3, 3, 2, 1, 1]
    assert o.tolist() == [6, 3, 3, 2, 1, 1]
    # a cycle 0<->1 feeding a path 1->2->3: SCC {0,1} of weight 2
    g = synth.from_edges(4, [0, 1, 1, 2], [1, 0, 2, 3], directed=True)
    a, o = oracle.alpha_omega(g)
    assert a.tolist() == [4, 4, 2, 1] and o.tolist() == [4, 4, 2, 1]
    # repeated DAG arcs between two SCCs count once: {0,1} -> {2} via 0->2 and
    # 1->2 gives omega = 2 + 1 = 3, not 4 (nodes 3, 4 keep the cap n = 5 away)
    g = synth.from_edges(5, [0, 1, 0, 1], [1, 0, 2, 2], directed=True)
    a, o = oracle.alpha_omega(g)
    assert a.tolist() == [3, 3, 1, 1, 1] and o.tolist() == [3, 3, 1, 1, 1]


# ---------------------------------- per-source trace from independent distances

def rederive_trace(g, r_true, order, k, footnote=False, big_scc=False):
    """Sequential Algorithm 1 replayed from SciPy distances: for each source
    in order, the level where the cut rule first fires (or -1), and the arcs
    scanned.  X = {r} (undirected) or {alpha, omega} (directed).  footnote:
    the undirected ~gamma_{d+1} for d >= 1 counts degree - 1 per node of
    Gamma_d (Section 2.3 footnote)."""
    D = scipy_dist(g)
    deg = np.diff(g.row_ptr).astype(np.int64)
    if g.directed:
        a, o = oracle.alpha_omega(g, big_scc=big_scc)
        X = [sorted({int(a[v]), int(o[v])}) for v in range(g.n)]
    else:
        X = [[int(r_true[v])] for v in range(g.n)]
    top = []  # list of (key, id, r, f)
    cut = {}
    mv = {}
    for v in order:
        v = int(v)
        if X[v][0] <= 1:
            cut[v], mv[v] = -2, 0
            top.append((Fraction(0), v))
            top.sort(key=lambda t: (-t[0], t[1]))
            top = top[:k]
            continue
        row = D[v]
        fin = np.isfinite(row)
        dist = row[fin].astype(np.int64)
        nodes = np.nonzero(fin)[0]
        ecc = int(dist.max())
        th = top[k - 1] if len(top) == k else None
        scanned = 0
        res = -1
        for d in range(ecc + 1):
            nd = int((dist <= d).sum())
            fd = int(dist[dist <= d].sum())
            arcs = int(deg[nodes[dist == d]].sum())
            gt = arcs
            if footnote and not g.directed and d >= 1:
                gt -= int((dist == d).sum())
            if th is not None:
                keyth, idth = th
                vals = [Fraction(fd - gt + (d + 2) * (x - nd), (x - 1) ** 2) for x in X[v]]
                inv = Fraction(1) / keyth if keyth != 0 else None
                if inv is not None and (all(q > inv for q in vals) or
                                        (all(q >= inv for q in vals) and v > idth)):
                    res = d
                    break
            scanned += arcs
        cut[v], mv[v] = res, scanned
        if res == -1:
            rr, ff = int(fin.sum()), int(dist.sum())
            top.append((oracle.closeness_key(rr, ff), v))
            top.sort(key=lambda t: (-t[0], t[1]))
            top = top[:k]
    return cut, mv


@pytest.mark.parametrize("seed", range(8))
def test_cut_levels_rederived(seed):
    rng = np.random.default_rng(77 + seed)
    directed = bool(seed % 2)
    if directed:
        g = synth.random_small(60, 0.05, True, 300 + seed)
    else:
        g = synth.barabasi_albert(120, 2, seed)
    r, f = scipy_rf(g)
    k = [1, 3, 10][seed % 3]
    order = rng.permutation(g.n).astype(np.int32) if seed % 4 == 3 else None
    got = oracle.topk(g, k, order=order, trace=True)
    if order is None:
        deg = np.diff(g.row_ptr)
        order = np.lexsort((np.arange(g.n), -deg))
    cut, mv = rederive_trace(g, r, order, k)
    assert got["cut_level"].tolist() == [cut[v] for v in range(g.n)]
    assert got["mvis"].tolist() == [mv[v] for v in range(g.n)]
    assert got["stats"]["m_vis"] == sum(mv.values())


# ---------------------------------------------------- the paper's invariants

@pytest.mark.parametrize("directed", [False, True])
def test_lemma_invariants(directed):
    """Lemma 1 / Lemma 2 and Table 1 relations at every level of every BFS:
    ~f_d(v, r) <= f(v), gamma_{d+1} <= ~gamma_{d+1}, n_d non-decreasing up to
    r(v), sum_d gamma_d = r(v), sum_d d gamma_d = f(v)."""
    g = synth.random_small(50, 0.06, directed, 4242) if directed else synth.barabasi_albert(150, 2, 9)
    D = scipy_dist(g)
    r, f = oracle.bruteforce(g)
    a, o = oracle.alpha_omega(g) if directed else (r, r)
    deg = np.diff(g.row_ptr).astype(np.int64)
    for v in range(g.n):
        row = D[v]
        fin = np.isfinite(row)
        dist = row[fin].astype(np.int64)
        nodes = np.nonzero(fin)[0]
        ecc = int(dist.max())
        prev = 0
        gam = [int((dist == d).sum()) for d in range(ecc + 2)]
        assert sum(gam) == r[v] and sum(d * x for d, x in enumerate(gam)) == f[v]
        for d in range(ecc + 1):
            nd = int((dist <= d).sum())
            fd = int(dist[dist <= d].sum())
            gt = int(deg[nodes[dist == d]].sum())
            assert gam[d + 1] <= gt
            assert nd >= prev
            prev = nd
            assert fd - gt + (d + 2) * (int(r[v]) - nd) <= int(f[v])
            if int(r[v]) > 1 and int(a[v]) > 1:
                lam = min(Fraction(fd - gt + (d + 2) * (int(x) - nd), (int(x) - 1) ** 2)
                          for x in (a[v], o[v]))
                assert lam <= Fraction(int(f[v]), (int(r[v]) - 1) ** 2)
        assert prev == r[v]


# ------------------------ the optional tighter bounds (Section 2.3 footnote, 2.4)

def test_footnote_path7_by_hand():
    """Path 0-...-6, k=1; order 1, 2, 3, 4, 5 (degree 2), then 0, 6.
    Node 1 (f=16), node 2 (f=13) and node 3 (f=12) complete in turn.
    Node 4 against f=12: with Table 1's ~gamma the level bounds are 10, 10,
    11, then 9 - 2 + 5 = 12 at d = 3 (tie, id 4 > 3: cut there, after 2 + 4
    + 3 arcs); with the footnote ~gamma_2 = 1 + 1, so d = 1 gives
    2 - 2 + 3 * 4 = 12 and the cut comes after 2 arcs.  Node 5: cut at d = 2
    (4 - 2 + 12 = 14) after 5 arcs, with the footnote at d = 1
    (2 - 1 + 12 = 13) after 2.  Nodes 0 and 6 are cut at d = 1 either way."""
    g = synth.path(7)
    plain = oracle.topk(g, 1, trace=True)
    foot = oracle.topk(g, 1, trace=True, footnote=True)
    for o in (plain, foot):
        assert o["ids"].tolist() == [3] and o["f"].tolist() == [12] and o["r"].tolist() == [7]
    assert plain["cut_level"].tolist() == [1, -1, -1, -1, 3, 2, 1]
    assert plain["mvis"].tolist() == [1, 12, 12, 12, 9, 5, 1]
    assert foot["cut_level"].tolist() == [1, -1, -1, -1, 1, 1, 1]
    assert foot["mvis"].tolist() == [1, 12, 12, 12, 2, 2, 1]


@pytest.mark.parametrize("seed", range(6))
def test_footnote_trace_rederived_and_never_later(seed):
    """The footnote bound replayed from SciPy distances gives the oracle's
    cut levels and arcs; the answer equals the definition; and since the
    bound is tighter at every level while the k-th record evolves the same
    way, no source is cut later or scans more arcs than with Table 1's."""
    rng = np.random.default_rng(500 + seed)
    g = synth.barabasi_albert(150, 2, 40 + seed) if seed % 2 else synth.random_small(90, 0.04, False, 60 + seed)
    r, f = scipy_rf(g)
    k = [1, 5, 20][seed % 3]
    order = rng.permutation(g.n).astype(np.int32) if seed % 3 == 2 else None
    foot = oracle.topk(g, k, order=order, trace=True, footnote=True)
    plain = oracle.topk(g, k, order=order, trace=True)
    ids, ff, rr = oracle.topk_by_definition(r, f, k)
    assert foot["ids"].tolist() == ids.tolist() and foot["f"].tolist() == ff.tolist()
    assert foot["r"].tolist() == rr.tolist()
    if order is None:
        deg = np.diff(g.row_ptr)
        order = np.lexsort((np.arange(g.n), -deg))
    cut, mv = rederive_trace(g, r, order, k, footnote=True)
    assert foot["cut_level"].tolist() == [cut[v] for v in range(g.n)]
    assert foot["mvis"].tolist() == [mv[v] for v in range(g.n)]
    assert np.all(foot["mvis"] <= plain["mvis"])
    assert foot["stats"]["m_vis"] <= plain["stats"]["m_vis"]


def test_footnote_lemma1_invariant():
    """Lemma 1 with the footnote ~gamma: gamma_{d+1} <= sum over Gamma_d of
    (deg - 1) for d >= 1, so f_d - ~gamma_{d+1} + (d+2)(r - n_d) <= f(v) at
    every level of every BFS."""
    for g in (synth.barabasi_albert(200, 3, 5), synth.random_small(80, 0.05, False, 7), synth.grid(6, 9)):
        D = scipy_dist(g)
        r, f = oracle.bruteforce(g)
        deg = np.diff(g.row_ptr).astype(np.int64)
        for v in range(g.n):
            row = D[v]
            fin = np.isfinite(row)
            dist = row[fin].astype(np.int64)
            nodes = np.nonzero(fin)[0]
            ecc = int(dist.max())
            for d in range(ecc + 1):
                lev = nodes[dist == d]
                gt = int(deg[lev].sum()) - (len(lev) if d >= 1 else 0)
                assert int((dist == d + 1).sum()) <= gt
                nd = int((dist <= d).sum())
                fd = int(dist[dist <= d].sum())
                assert fd - gt + (d + 2) * (int(r[v]) - nd) <= int(f[v])


def _largest_scc_nodes(g):
    A = sp.csr_matrix((np.ones(g.m), g.col, g.row_ptr), shape=(g.n, g.n))
    _, lab = connected_components(A, directed=True, connection="strong")
    sizes = np.bincount(lab)
    best = sizes.max()
    # among the largest components, the one holding the smallest node id
    first = min(int(np.nonzero(lab == c)[0][0]) for c in np.nonzero(sizes == best)[0])
    return np.nonzero(lab == lab[first])[0]


@pytest.mark.parametrize("seed", range(10))
def test_big_scc_bounds_bracket_reach_and_tighten(seed):
    """alpha <= r <= omega still holds with the largest-SCC refinement, it
    is never looser than the plain recurrence, and it is exact on the
    largest SCC (r from SciPy distances)."""
    g = synth.random_small(80, 0.012 + 0.004 * seed, True, 1300 + seed)
    r, _ = scipy_rf(g)
    a0, o0 = oracle.alpha_omega(g)
    a, o = oracle.alpha_omega(g, big_scc=True)
    assert np.all(a <= r) and np.all(r <= o) and np.all(o <= g.n)
    assert np.all(a >= a0) and np.all(o <= o0)
    big = _largest_scc_nodes(g)
    assert np.all(a[big] == r[big]) and np.all(o[big] == r[big])


def test_big_scc_by_hand():
    """Cycle T = {0,1,2} (the largest SCC) with 0->3, 1->4, 3->5, 4->5; node 6
    -> 0; 7, 8, 9 isolated (n = 10, no cap).  Plain recurrence: alpha(T) =
    3 + 2 = 5 and omega(T) = 3 + 2 + 2 = 7, while R(T) = 6; node 6 gets
    (6, 8).  Refined: T exact (6, 6), and node 6 gets alpha = 1 + 6 = 7 and
    omega = min(1 + 6, 6 + omega'(6) = 6 + 1) = 7, its exact reach."""
    g = synth.from_edges(10, [0, 1, 2, 0, 1, 3, 4, 6], [1, 2, 0, 3, 4, 5, 5, 0], directed=True)
    a0, o0 = oracle.alpha_omega(g)
    assert a0.tolist() == [5, 5, 5, 2, 2, 1, 6, 1, 1, 1]
    assert o0.tolist() == [7, 7, 7, 2, 2, 1, 8, 1, 1, 1]
    a, o = oracle.alpha_omega(g, big_scc=True)
    assert a.tolist() == [6, 6, 6, 2, 2, 1, 7, 1, 1, 1]
    assert o.tolist() == [6, 6, 6, 2, 2, 1, 7, 1, 1, 1]
    # second bound alone: T = cycle {0,1,2} -> 3 -> 4, node 5 -> 0 and 5 -> 3,
    # 6..8 isolated.  Plain omega(5) = 1 + 5 + 2 = 8; both successors lie in
    # R(T), so omega'(5) = 1 and omega(5) = 5 + 1 = 6 = r(5).
    g = synth.from_edges(9, [0, 1, 2, 2, 3, 5, 5], [1, 2, 0, 3, 4, 0, 3], directed=True)
    a0, o0 = oracle.alpha_omega(g)
    a, o = oracle.alpha_omega(g, big_scc=True)
    assert (int(a0[5]), int(o0[5])) == (6, 8)
    assert (int(a[5]), int(o[5])) == (6, 6)
    # two largest SCCs of equal size: the one holding node 0 is refined
    g = synth.from_edges(6, [0, 1, 2, 3, 0, 3], [1, 0, 3, 2, 4, 4], directed=True)
    a, o = oracle.alpha_omega(g, big_scc=True)
    assert a.tolist() == [3, 3, 3, 3, 1, 1]


@pytest.mark.parametrize("seed", range(6))
def test_big_scc_trace_rederived(seed):
    """Directed runs with the refined reach bounds: cut levels and arcs as
    replayed from SciPy distances with the refined alpha/omega, the answer
    of the definition, and never more arcs per source than the plain bounds."""
    g = synth.random_small(70, 0.03 + 0.01 * (seed % 3), True, 2100 + seed)
    r, f = scipy_rf(g)
    k = [1, 4, 10][seed % 3]
    got = oracle.topk(g, k, trace=True, big_scc=True)
    plain = oracle.topk(g, k, trace=True)
    ids, ff, rr = oracle.topk_by_definition(r, f, k)
    assert got["ids"].tolist() == ids.tolist() and got["f"].tolist() == ff.tolist()
    deg = np.diff(g.row_ptr)
    order = np.lexsort((np.arange(g.n), -deg))
    cut, mv = rederive_trace(g, r, order, k, big_scc=True)
    assert got["cut_level"].tolist() == [cut[v] for v in range(g.n)]
    assert got["mvis"].tolist() == [mv[v] for v in range(g.n)]
    assert got["stats"]["m_vis"] <= plain["stats"]["m_vis"]
