"""Serving on the GPU: a mix of requests over many graphs, with a memory
budget small enough that requests queue and idle graphs are evicted and
uploaded again.  Every request's result must equal the same query run alone
(bc_topk on its own graph), and a subset is checked against the oracle.
Also: latency bookkeeping, cancellation, and a request that can never fit."""

import time

import numpy as np
import pytest

import oracle
import paper_1507_01490_amd as bc
from paper_1507_01490_amd import synth

pytestmark = pytest.mark.gpu


def mix_graphs():
    rng = np.random.default_rng(77)
    out = []
    for i in range(30):
        n = int(np.exp(rng.uniform(np.log(500), np.log(20000))))
        fam = i % 5
        if fam == 0:
            g = synth.erdos_renyi(n, 8, 500 + i)
        elif fam == 1:
            g = synth.barabasi_albert(n, 4, 500 + i)
        elif fam == 2:
            g = synth.grid_shortcuts(n, 0.01, 500 + i)
        elif fam == 3:
            g = synth.random_small(min(n, 3000), 4.0 / min(n, 3000), True, 500 + i)
        else:
            g = synth.rmat(11, 8, 0.57, 0.19, 0.19, 500 + i)
        out.append(g)
    out += [synth.star(40), synth.path(30), synth.empty(5), synth.directed_cycle(12)]
    return out


CHOICES = [dict(mode="plain"), dict(mode="batched"), dict(mode="batched", width=256),
           dict(mode="batched", order="learned_grouped"), dict(mode="plain", order="degree", width=128)]


def same(a, b):
    return a.ids.tolist() == b.ids.tolist() and a.farness.tolist() == b.farness.tolist() and \
        a.reach.tolist() == b.reach.tolist()


def test_mix_equals_alone_and_oracle():
    graphs = mix_graphs()
    rng = np.random.default_rng(5)
    reqs = []
    for i in range(140):
        gi = int(rng.integers(0, len(graphs)))
        k = int(rng.choice([1, 10, 100]))
        kw = CHOICES[int(rng.integers(0, len(CHOICES)))]
        reqs.append((gi, k, kw))
    # a budget of 1.25 x the largest single request (its graph, upload and
    # working memory): requests queue, and idle graphs must be evicted
    need = max(sum(bc.footprint(graphs[gi].n, graphs[gi].m, graphs[gi].directed, k, 16, **kw))
               for gi, k, kw in reqs)
    with bc.Server(lanes=4, slots=16, budget_bytes=int(1.25 * need)) as S:
        gids = [S.add_graph(g.row_ptr, g.col, directed=g.directed) for g in graphs]
        tickets = []
        for gi, k, kw in reqs:
            tickets.append(S.submit(gids[gi], k, **kw))
            if len(tickets) % 20 == 0:
                time.sleep(0.01)
        results = []
        for t in tickets:
            assert S.wait(t, 120000)
            r = S.poll(t)
            assert r is not None
            results.append(r)
        info = S.info()
    assert info["completed"] == len(reqs) and info["failed"] == 0
    assert info["peak_bytes"] <= info["budget_bytes"]
    assert info["evictions"] > 0 and info["uploads"] > info["evictions"]
    for r in results:
        i = r.info
        assert i["submit_ms"] <= i["start_ms"] <= i["finish_ms"] and 0 <= i["lane"] < 4
    # each result equals the same query alone, and the oracle on a subset
    alone = {}
    for (gi, k, kw), r in zip(reqs, results):
        key = (gi, k, tuple(sorted(kw.items())))
        if key not in alone:
            g = graphs[gi]
            with bc.Graph(g.row_ptr, g.col, directed=g.directed) as G:
                alone[key] = G.topk(k, **kw)
        assert same(r, alone[key]), (gi, k, kw)
    for gi in range(0, len(graphs), 3):
        g = graphs[gi]
        for (gj, k, kw), r in zip(reqs, results):
            if gj == gi:
                ref = oracle.topk(g, k, nthreads=8)
                assert r.ids.tolist() == ref["ids"].tolist() and r.farness.tolist() == ref["f"].tolist()
                break


def test_cancel_and_errors():
    big = synth.erdos_renyi(60000, 8, 9)
    small = synth.path(20)
    with bc.Server(lanes=1, slots=8, budget_bytes=256 << 20) as S:
        gb = S.add_graph(big.row_ptr, big.col)
        gs = S.add_graph(small.row_ptr, small.col)
        first = [S.submit(gb, 100, mode="plain") for _ in range(3)]
        late = S.submit(gs, 3)
        S.cancel(late)  # still queued behind the slow requests on the single lane
        with pytest.raises(bc.BcError) as e:
            S.poll(late)
        assert e.value.status == -6
        for t in first:
            assert S.wait(t, 120000)
            assert S.poll(t) is not None
        with pytest.raises(bc.BcError):
            S.submit(99, 3)
        with pytest.raises(bc.BcError):
            S.poll(123456)
        info = S.info()
        assert info["canceled"] == 1 and info["completed"] == 3
    # a request larger than the whole budget fails instead of waiting for ever
    with bc.Server(lanes=2, slots=8, budget_bytes=1 << 20) as S:
        g = S.add_graph(big.row_ptr, big.col)
        t = S.submit(g, 10, mode="batched")
        assert S.wait(t, 60000)
        with pytest.raises(bc.BcError) as e:
            S.poll(t)
        assert e.value.status == -3
