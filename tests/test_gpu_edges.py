"""Degenerate inputs through every top-k entry point: a graph without nodes
gives an empty answer (the oracle's: no node, no closeness), and a graph of
isolated nodes gives k nodes of closeness 0 in id order (reading 1: r = 1
means c = 0), whether the query runs alone, in a multi-graph launch, without
allocation or through a server."""

import numpy as np
import pytest

import oracle
import paper_1507_01490_amd as bc
from paper_1507_01490_amd import synth

pytestmark = pytest.mark.gpu


def entry_points(g, k):
    """(name, result) of every entry point on graph g."""
    out = []
    with bc.Graph(g.row_ptr, g.col, directed=g.directed) as G:
        for kw in (dict(mode="plain", width=64), dict(mode="batched", width=64), dict(mode="batched", width=256),
                   dict(mode="plain", width=64, graph_levels=-1)):
            out.append((f"topk {kw}", G.topk(k, **kw)))
        out.append(("topk_static", G.topk_static(k)))
        out.append(("topk_multi", bc.topk_multi([G], [k])[0]))
    for queue in (False, True):
        with bc.Server(lanes=1, budget_bytes=1 << 28, queue=queue) as S:
            gid = S.add_graph(g.row_ptr, g.col, directed=g.directed)
            t = S.submit(gid, k, mode="batched")
            assert S.wait(t, 60000)
            out.append((f"server queue={queue}", S.poll(t)))
    return out


@pytest.mark.parametrize("directed", [False, True])
def test_graph_without_nodes(directed):
    g = synth.empty(0, directed=directed)
    print(f"[edges] n=0 directed={directed}", flush=True)
    assert oracle.topk(g, 3)["ids"].tolist() == []
    for name, res in entry_points(g, 3):
        assert len(res.ids) == 0 and len(res.farness) == 0 and len(res.reach) == 0, name


def test_isolated_nodes_k_above_n():
    g = synth.empty(7)
    ref = oracle.topk(g, 10)
    print("[edges] 7 isolated nodes, k = 10", flush=True)
    assert ref["ids"].tolist() == list(range(7))
    for name, res in entry_points(g, 10):
        assert res.ids.tolist() == ref["ids"].tolist(), name
        assert res.farness.tolist() == ref["f"].tolist() and res.reach.tolist() == ref["r"].tolist(), name
