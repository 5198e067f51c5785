"""Warm-started queries over a growing graph.  opts.first puts the previous
snapshot's top-k at the head of the source order (Algorithm 1 is exact for
any order, Section 2.1), so every snapshot's answer must equal the oracle's,
cold or warm, in every mode."""

import numpy as np
import pytest

import oracle
import paper_1507_01490_amd as bc
from paper_1507_01490_amd import synth

pytestmark = pytest.mark.gpu


def same(res, ref):
    return (res.ids.tolist() == ref["ids"].tolist() and res.farness.tolist() == ref["f"].tolist()
            and res.reach.tolist() == ref["r"].tolist())


@pytest.mark.parametrize("k", [1, 10, 70])
def test_warm_series_equals_oracle(k):
    snaps = synth.collaboration_snapshots(4000, 1000, 2.1, 200, 5, 6)
    prev = None
    for t, g in enumerate(snaps):
        print(f"[snapshots] k={k} t={t} n={g.n} m={g.m}", flush=True)
        ref = oracle.topk(g, k)
        with bc.Graph(g.row_ptr, g.col) as G:
            for kw in (dict(mode="batched"), dict(mode="plain"), dict(mode="batched", width=256)):
                assert same(G.topk(k, **kw), ref), (k, t, kw)
                if prev is not None:
                    assert same(G.topk(k, first=prev, **kw), ref), (k, t, kw, "warm")
        prev = ref["ids"]


def test_front_list_order_and_errors():
    g = synth.barabasi_albert(3000, 3, 21)
    first = np.array([2999, 5, 17, 1200], np.int32)
    with bc.Graph(g.row_ptr, g.col) as G:
        base = G.source_order(10, mode="batched")
        o = G.source_order(10, mode="batched", first=first)
        assert o[:4].tolist() == first.tolist()
        assert sorted(o.tolist()) == list(range(g.n))
        rest = [v for v in base.tolist() if v not in set(first.tolist())]
        assert o[4:].tolist() == rest
        for bad in (np.array([1, 1], np.int32), np.array([3000], np.int32), np.array([-1], np.int32)):
            with pytest.raises(bc.BcError) as e:
                G.topk(5, first=bad)
            assert e.value.status == -1
        assert same(G.topk(5, first=first, mode="batched"), oracle.topk(g, 5))
