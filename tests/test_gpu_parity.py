"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bit-exact: same ids, same integer farness and reach, in the same order (the
key order with the id tie-break makes the answer unique).  Covered: closed
forms, fuzzed small graphs (directed / undirected / disconnected / many SCCs)
in every mode, width and order, the BA n=2000 workload against brute force,
reach data, canonicalisation of raw input, and error handling."""

import numpy as np
import pytest

import oracle
import paper_1507_01490_amd as bc
from paper_1507_01490_amd import synth

pytestmark = pytest.mark.gpu

VARIANTS = [
    dict(mode="plain", width=64),
    dict(mode="plain", width=64, pull_alpha=0.0),
    dict(mode="plain", width=128),
    dict(mode="plain", width=256),
    dict(mode="plain", width=64, pull_alpha=1e9, pull_beta=1e-9),  # bottom-up from level 1 on
    dict(mode="plain", width=256, pull_alpha=14.0),
    dict(mode="batched", width=64),
    dict(mode="batched", width=64, lds_tables=False),
    dict(mode="batched", width=64, lds_tables="spill"),              # every batch continues on the node records
    dict(mode="batched", width=64, seed_width=256),                  # wider seed batches
    dict(mode="batched", width=128, seed_width=256, seed_batches=2),
    dict(mode="batched", width=64, seed_batches=0, slots=7),
    dict(mode="batched", width=128, seed_batches=0),
    dict(mode="batched", width=256, slots=3),
    dict(mode="batched", width=64, defer_arcs=1),    # nearly every source re-run level-synchronously
    dict(mode="batched", width=128, defer_arcs=40, slots=5),
    dict(mode="batched", width=64, defer_arcs=1, defer_width=64),    # deferred sources re-run 64 at a time
    dict(mode="batched", width=256, defer_arcs=40, defer_width=128, slots=3),
    dict(mode="plain", width=64, graph_levels=4),                     # captured level steps
    dict(mode="batched", width=128, defer_arcs=40, graph_levels=3),
    dict(mode="plain", width=256, pull_alpha=1e9, pull_beta=1e-9, graph_levels=2),
    dict(mode="plain", width=64, graph_levels=-1),                    # one cooperative launch
    dict(mode="batched", width=64, defer_arcs=1, graph_levels=-1),
]


def gpu_topk(g, k, **kw):
    with bc.Graph(g.row_ptr, g.col, directed=g.directed) as G:
        return G.topk(k, **kw)


def assert_same(res, ref, ctx=""):
    assert res.ids.tolist() == ref["ids"].tolist(), ctx
    assert res.farness.tolist() == ref["f"].tolist(), ctx
    assert res.reach.tolist() == ref["r"].tolist(), ctx


CLOSED = [synth.path(9), synth.star(12), synth.cycle(10), synth.complete(7), synth.grid(5, 7),
          synth.complete_bipartite(3, 5), synth.directed_path(8), synth.directed_cycle(6),
          synth.out_star(9), synth.empty(5), synth.empty(1),
          synth.disjoint_union(synth.path(5), synth.star(4), synth.complete(3), synth.empty(2))]


@pytest.mark.parametrize("gi", range(len(CLOSED)))
def test_closed_forms(gi):
    g = CLOSED[gi]
    for k in sorted({1, 2, 3, g.n, g.n + 2}):
        ref = oracle.topk(g, k)
        for v in VARIANTS:
            assert_same(gpu_topk(g, k, **v), ref, (g.name, k, v))


@pytest.mark.parametrize("block", range(6))
def test_fuzz_small(block):
    rng = np.random.default_rng(4000 + block)
    for it in range(12):
        n = int(rng.integers(2, 400))
        directed = bool(rng.integers(0, 2))
        p = float(rng.choice([0.003, 0.01, 0.03, 0.08])) * (40.0 / max(n, 40)) * 4
        g = synth.random_small(n, min(p, 0.5), directed, int(rng.integers(0, 2**31)))
        k = int(rng.choice([1, 2, 10, 50, n]))
        ref = oracle.topk(g, k)
        v = VARIANTS[(block * 12 + it) % len(VARIANTS)]
        assert_same(gpu_topk(g, k, **v), ref, (n, directed, p, k, v))


def test_orders_do_not_change_the_answer():
    g = synth.barabasi_albert(3000, 3, 11)
    rng = np.random.default_rng(5)
    ref = oracle.topk(g, 10)
    with bc.Graph(g.row_ptr, g.col) as G:
        for v in VARIANTS:
            assert_same(G.topk(10, order=rng.permutation(g.n), **v), ref, v)
            assert_same(G.topk(10, scores=rng.random(g.n), **v), ref, v)
            assert_same(G.topk(10, order=np.arange(g.n)[::-1], **v), ref, v)
            assert_same(G.topk(10, order="grouped", **v), ref, v)
            assert_same(G.topk(10, order="degree", **v), ref, v)


@pytest.mark.parametrize("k", [1, 10])
def test_ba2000_against_bruteforce(k):
    g = synth.barabasi_albert(2000, 5, 0)
    r, f = oracle.bruteforce(g, nthreads=8)
    ids, ff, rr = oracle.topk_by_definition(r, f, k)
    for v in VARIANTS:
        res = gpu_topk(g, k, **v)
        assert res.ids.tolist() == ids.tolist() and res.farness.tolist() == ff.tolist()
        assert res.reach.tolist() == rr.tolist()


@pytest.mark.parametrize("kind", ["ba", "er", "grid", "rmat"])
def test_medium_graphs(kind):
    if kind == "ba":
        g = synth.barabasi_albert(30000, 4, 21)
    elif kind == "er":
        g = synth.erdos_renyi(30000, 8, 22)
    elif kind == "grid":
        g = synth.grid_shortcuts(30000, 0.01, 23)
    else:
        g = synth.rmat(14, 16, 0.57, 0.19, 0.19, 24)
    for k in (1, 10, 100):
        ref = oracle.topk(g, k, nthreads=8)
        with bc.Graph(g.row_ptr, g.col, directed=g.directed) as G:
            for v in VARIANTS:
                assert_same(G.topk(k, **v), ref, (kind, k, v))


LOOP_GRAPHS = [lambda: synth.barabasi_albert(3000, 4, 21), lambda: synth.grid_shortcuts(4000, 0.01, 22),
               lambda: synth.rmat(12, 8, 0.57, 0.19, 0.19, 23), lambda: synth.random_small(600, 0.005, True, 24),
               lambda: synth.disjoint_union(synth.path(40), synth.star(30), synth.empty(7))]


@pytest.mark.parametrize("gi", range(len(LOOP_GRAPHS)))
def test_level_loops_agree(gi):
    """The three drivers of the level-synchronous batches (one host round
    trip per level, one cooperative launch, captured level steps) run the same
    level steps: the same answer everywhere, and in plain mode, where each
    batch starts from the state the previous one left, the same counters."""
    g = LOOP_GRAPHS[gi]()
    print(f"[loops] graph {gi} n={g.n} m={g.m}", flush=True)
    with bc.Graph(g.row_ptr, g.col, directed=g.directed) as G:
        for k in (1, 10, 70):
            ref = oracle.topk(g, k)
            for kw in (dict(mode="plain", width=64), dict(mode="plain", width=256, pull_alpha=14.0),
                       dict(mode="batched", width=64, defer_arcs=1), dict(mode="batched", width=128, seed_width=256)):
                runs = [G.topk(k, graph_levels=gl, **kw) for gl in (0, -1, 3)]
                for r in runs:
                    assert_same(r, ref, (gi, k, kw))
                if kw["mode"] == "plain":
                    for key in ("m_vis", "levels", "pull_levels", "node_arcs", "batches", "n_cut", "n_done"):
                        vals = [int(r.stats[key]) for r in runs]
                        assert len(set(vals)) == 1, (gi, k, kw, key, vals)


def test_level_list_checks(monkeypatch):
    """With BC_CHECK_LISTS=1 the host-driven level loop copies the frontier
    and reset lists after every level and checks every id against n; the
    queries (plain mode, and the seed batches and deferred re-run of the
    batched mode) pass the check and still equal the oracle."""
    monkeypatch.setenv("BC_CHECK_LISTS", "1")
    for g in (synth.path(9), synth.star(12), synth.empty(5), synth.barabasi_albert(3000, 4, 31),
              synth.rmat(11, 8, 0.57, 0.19, 0.19, 32)):
        with bc.Graph(g.row_ptr, g.col, directed=g.directed) as G:
            for k in (1, 10):
                ref = oracle.topk(g, k)
                for kw in (dict(mode="plain", width=64), dict(mode="plain", width=256, pull_alpha=1e9, pull_beta=1e-9),
                           dict(mode="batched", width=64, defer_arcs=1)):
                    assert_same(G.topk(k, **kw), ref, (g.n, k, kw))


def test_reach_data_matches_oracle():
    for seed in range(4):
        g = synth.random_small(300, 0.006 + 0.002 * seed, True, 77 + seed)
        a, o = oracle.alpha_omega(g)
        with bc.Graph(g.row_ptr, g.col, directed=True) as G:
            lo, hi = G.reach()
        assert lo.tolist() == a.tolist() and hi.tolist() == o.tolist()
        u = synth.random_small(300, 0.004 + 0.002 * seed, False, 88 + seed)
        r = oracle.reach_undirected(u)
        with bc.Graph(u.row_ptr, u.col) as G:
            lo, hi = G.reach()
        assert lo.tolist() == r.tolist() and hi.tolist() == r.tolist()
    g = synth.rmat(15, 16, 0.57, 0.19, 0.19, 3)
    a, o = oracle.alpha_omega(g)
    with bc.Graph(g.row_ptr, g.col, directed=True) as G:
        lo, hi = G.reach()
    assert lo.tolist() == a.tolist() and hi.tolist() == o.tolist()


def test_canonicalisation_of_raw_input():
    rng = np.random.default_rng(3)
    for directed in (False, True):
        n = 500
        s = rng.integers(0, n, 3000)
        d = rng.integers(0, n, 3000)
        s = np.concatenate([s, np.arange(50), s[:300]])
        d = np.concatenate([d, np.arange(50), d[:300]])
        raw = synth.raw_csr(n, s, d, directed, rng)
        rp, col = oracle.canonicalize(raw)
        with bc.Graph(raw.row_ptr, raw.col, directed=directed) as G:
            grp, gcol = G.csr()
            assert grp.tolist() == rp.tolist() and gcol.tolist() == col.tolist()
            for k in (1, 7, 40):
                assert_same(G.topk(k), oracle.topk(raw, k), (directed, k))


def test_errors():
    g = synth.path(5)
    with pytest.raises(bc.BcError) as e:
        bc.Graph(np.array([0, 1, 1, 0, 2, 2], np.int32), np.array([1, 0], np.int32))
    assert e.value.status == -2
    with pytest.raises(bc.BcError) as e:
        bc.Graph(np.array([0, 1, 2], np.int32), np.array([1, 5], np.int32))
    assert e.value.status == -2
    with pytest.raises(bc.BcError) as e:   # asymmetric "undirected" input
        bc.Graph(np.array([0, 1, 1], np.int32), np.array([1], np.int32), validate=True)
    assert e.value.status == -2
    with bc.Graph(g.row_ptr, g.col) as G:
        with pytest.raises(bc.BcError) as e:
            G.topk(0)
        assert e.value.status == -1
        with pytest.raises(bc.BcError) as e:
            G.topk(3, width=96)
        assert e.value.status == -1
        with pytest.raises(bc.BcError) as e:
            G.topk(3, order=np.array([0, 0, 1, 2, 3]))
        assert e.value.status == -1
        with pytest.raises(bc.BcError) as e:
            G.topk(3, mode="plain", graph_levels=-2)
        assert e.value.status == -1
        assert_same(G.topk(3), oracle.topk(g, 3))  # still usable after errors
