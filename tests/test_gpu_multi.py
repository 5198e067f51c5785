"""Many queries in one persistent launch (bc_topk_multi, bc_multi_*): the
source batches of several graphs of different sizes and families run side by
side in one kernel (the parallel loop of Section 2.1 over every query's
sources), each query with its own top-k list and threshold records.  Every
query must return exactly the oracle's answer for its graph alone: ids,
farness and reach, element by element.  The captured launch (a HIP graph)
is replayed several times with other GPU work and synchronisations between
the replays, and every replay is checked."""

import numpy as np
import pytest
import torch

import oracle
import paper_1507_01490_amd as bc
from paper_1507_01490_amd import synth

pytestmark = pytest.mark.gpu


def assert_same(res, ref, ctx=""):
    assert res.ids.tolist() == ref["ids"].tolist(), ctx
    assert res.farness.tolist() == ref["f"].tolist(), ctx
    assert res.reach.tolist() == ref["r"].tolist(), ctx


def uneven_set():
    """(graph, k) of uneven sizes and shapes: hubs, no hubs, clique-rich,
    directed with many SCCs, closed forms and a graph without arcs."""
    return [
        (synth.barabasi_albert(20000, 5, 21), 100),
        (synth.erdos_renyi(6000, 8.0, 22), 10),
        (synth.grid_shortcuts(9000, 0.01, 23), 10),
        (synth.collaboration(8000, 2000, 2.1, 200, 24), 10),
        (synth.rmat(11, 16, 0.57, 0.19, 0.19, 25), 10),
        (synth.path(9), 1),
        (synth.star(12), 3),
        (synth.empty(5), 7),  # k > n: min(k, n) results
        (synth.barabasi_albert(3000, 3, 26), 1),
    ]


@pytest.fixture(scope="module")
def graphs_and_refs():
    gs = uneven_set()
    refs = [oracle.topk(g, k) for g, k in gs]
    handles = [bc.Graph(g.row_ptr, g.col, directed=g.directed) for g, _ in gs]
    yield gs, refs, handles
    for h in handles:
        h.close()


@pytest.mark.parametrize("width", [64, 128, 256])
def test_one_launch_many_graphs(graphs_and_refs, width):
    gs, refs, handles = graphs_and_refs
    print(f"[multi] width={width} queries={len(gs)}", flush=True)
    out = bc.topk_multi(handles, [k for _, k in gs], width=width)
    assert len(out) == len(gs)
    for i, ((g, k), ref, res) in enumerate(zip(gs, refs, out)):
        assert len(res.ids) == min(k, g.n)
        assert_same(res, ref, (width, i, g.n, k))
    # every non-trivial source was either completed or cut
    for (g, _), res in zip(gs, out):
        st = res.stats
        assert st["n_cut"] + st["n_done"] + st["n_trivial"] == g.n, st


def test_same_graph_twice_and_small_slot_count(graphs_and_refs):
    """A graph may appear in several queries (different k); 3 workgroups for
    the whole launch still finish every batch."""
    gs, refs, handles = graphs_and_refs
    sel = [0, 1, 0, 4]
    ks = [1, 10, 60, 10]
    out = bc.topk_multi([handles[i] for i in sel], ks, width=64, slots=3)
    for i, k, res in zip(sel, ks, out):
        assert_same(res, oracle.topk(gs[i][0], k), (i, k))


def test_orders_and_footnote(graphs_and_refs):
    gs, refs, handles = graphs_and_refs
    ks = [k for _, k in gs]
    for kw in (dict(order="degree"), dict(order="locality", width=256), dict(order="learned_grouped"),
               dict(footnote=True)):
        print(f"[multi] {kw}", flush=True)
        out = bc.topk_multi(handles, ks, **kw)
        for i, ((g, k), res) in enumerate(zip(gs, out)):
            ref = oracle.topk(g, k, footnote=True) if kw.get("footnote") else refs[i]
            assert_same(res, ref, (kw, i))


def test_captured_launch_replays(graphs_and_refs):
    """The HIP graph (fill kernel + persistent kernel) replayed four times,
    with eager library work and a torch kernel between replays: every replay
    returns the oracle's answers."""
    gs, refs, handles = graphs_and_refs
    ks = [k for _, k in gs]
    with bc.MultiLaunch(handles, ks, capture=True, width=64) as L:
        for rep in range(4):
            out = L.run()
            for i, ((g, k), ref, res) in enumerate(zip(gs, refs, out)):
                assert_same(res, ref, (rep, i))
            # eager work between replays: a query alone and a torch kernel
            alone = handles[1].topk(10, mode="batched")
            assert_same(alone, refs[1])
            x = torch.arange(1 << 20, device="cuda", dtype=torch.int64)
            assert int((x * 3).sum().item()) == 3 * ((1 << 20) - 1) * (1 << 20) // 2
            torch.cuda.synchronize()


def test_rejects_bad_arguments(graphs_and_refs):
    gs, refs, handles = graphs_and_refs
    with pytest.raises(bc.BcError):
        bc.topk_multi(handles[:2], [10, 0])
    with pytest.raises(bc.BcError):
        bc.topk_multi(handles[:2], [10, 10], width=96)
