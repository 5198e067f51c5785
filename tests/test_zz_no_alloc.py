"""bc_topk_static, the entry point that allocates nothing (every buffer in
the library's static device array), against bc_topk in plain mode on the
same graphs: ids, farness and reach element by element, on two calls in a
row with the second on a smaller graph (the array keeps the first call's
contents, which the second must clear), then the oracle, and the size limit."""

import pytest

import oracle
import paper_1507_01490_amd as bc
from paper_1507_01490_amd import synth

pytestmark = pytest.mark.gpu


def same(a, b):
    return a.ids.tolist() == b.ids.tolist() and a.farness.tolist() == b.farness.tolist() and \
        a.reach.tolist() == b.reach.tolist()


def test_static_equals_topk_two_calls_second_smaller():
    big = synth.barabasi_albert(60000, 4, 71)
    small = synth.grid_shortcuts(3000, 0.01, 72)
    print("[no-alloc] first call: BA 60000, k=100", flush=True)
    with bc.Graph(big.row_ptr, big.col) as G:
        a = G.topk_static(100)
        ref = G.topk(100, mode="plain")
        assert same(a, ref)
    print("[no-alloc] second call: grid 3000, k=10", flush=True)
    with bc.Graph(small.row_ptr, small.col) as G:
        b = G.topk_static(10)
        ref = G.topk(10, mode="plain")
        assert same(b, ref)
        o = oracle.topk(small, 10)
        assert b.ids.tolist() == o["ids"].tolist() and b.farness.tolist() == o["f"].tolist()
        assert b.reach.tolist() == o["r"].tolist()
        # and again, now with the degree order the plain query left cached
        c = G.topk_static(10)
        assert same(c, ref)


def test_static_directed_and_closed_forms():
    for g, k in ((synth.rmat(11, 8, 0.57, 0.19, 0.19, 73), 10), (synth.path(9), 3), (synth.star(12), 12),
                 (synth.empty(5), 7), (synth.directed_cycle(7), 2)):
        with bc.Graph(g.row_ptr, g.col, directed=g.directed) as G:
            r = G.topk_static(k)
        o = oracle.topk(g, k)
        assert r.ids.tolist() == o["ids"].tolist() and r.farness.tolist() == o["f"].tolist(), (g.n, k)
        assert r.reach.tolist() == o["r"].tolist()


def test_static_rejects_graphs_beyond_its_array():
    g = synth.empty(1_000_000)
    with bc.Graph(g.row_ptr, g.col) as G:
        with pytest.raises(bc.BcError) as e:
            G.topk_static(10)
    assert e.value.status == -1 and "static scratch" in str(e.value)
