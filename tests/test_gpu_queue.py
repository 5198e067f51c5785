"""Continuous batching: the serving queue drained by one running persistent
kernel (bc_server_opts.queue).  Lanes only prepare requests; the kernel's
workgroups claim the next source batch of whichever queued request it
belongs to, so requests that arrive while others run start on free
workgroups and run beside them.  Every result must equal the same query
alone (bc_topk on its own graph), and the oracle's answer on a subset; the
requests' time on the GPU must overlap; the kernel must be launched again
when it has ended for lack of work and a request arrives."""

import time

import numpy as np
import pytest

import oracle
import paper_1507_01490_amd as bc
from paper_1507_01490_amd import synth

pytestmark = pytest.mark.gpu


def graphs_for_queue():
    rng = np.random.default_rng(91)
    out = []
    for i in range(24):
        n = int(np.exp(rng.uniform(np.log(500), np.log(30000))))
        fam = i % 4
        if fam == 0:
            out.append(synth.erdos_renyi(n, 8, 900 + i))
        elif fam == 1:
            out.append(synth.barabasi_albert(n, 4, 900 + i))
        elif fam == 2:
            out.append(synth.grid_shortcuts(n, 0.01, 900 + i))
        else:
            out.append(synth.rmat(11, 8, 0.57, 0.19, 0.19, 900 + i))
    out += [synth.star(40), synth.path(30), synth.empty(5), synth.directed_cycle(12)]
    return out


CHOICES = [dict(mode="batched"), dict(mode="batched", order="locality"), dict(mode="batched", order="degree"),
           dict(mode="batched", order="learned_grouped"), dict(mode="plain")]


def same(a, b):
    return a.ids.tolist() == b.ids.tolist() and a.farness.tolist() == b.farness.tolist() and \
        a.reach.tolist() == b.reach.tolist()


def max_overlap(results):
    ev = []
    for r in results:
        ev.append((r.info["start_ms"], 1))
        ev.append((r.info["finish_ms"], -1))
    cur = best = 0
    for _, d in sorted(ev, key=lambda x: (x[0], x[1])):
        cur += d
        best = max(best, cur)
    return best


@pytest.mark.parametrize("width", [64, 256])
def test_queue_mix_equals_alone_and_oracle(width):
    graphs = graphs_for_queue()
    rng = np.random.default_rng(8 + width)
    reqs = []
    for i in range(120):
        gi = int(rng.integers(0, len(graphs)))
        k = int(rng.choice([1, 10, 100]))
        kw = CHOICES[int(rng.integers(0, len(CHOICES)))]
        reqs.append((gi, k, kw))
    print(f"[queue] width={width} requests={len(reqs)}", flush=True)
    with bc.Server(lanes=3, slots=16, budget_bytes=4 << 30, queue=True, queue_width=width, queue_slots=64) as S:
        gids = [S.add_graph(g.row_ptr, g.col, directed=g.directed) for g in graphs]
        tickets = []
        for j, (gi, k, kw) in enumerate(reqs):
            tickets.append(S.submit(gids[gi], k, **kw))
            if j % 10 == 9:
                time.sleep(0.005)  # arrivals while earlier requests run
        results = []
        for j, t in enumerate(tickets):
            assert S.wait(t, 30000), (j, reqs[j])
            r = S.poll(t)
            assert r is not None
            results.append(r)
            if j % 30 == 29:
                print(f"[queue] {j + 1} finished", flush=True)
        info = S.info()
    assert info["completed"] == len(reqs) and info["failed"] == 0
    assert max_overlap(results) >= 2
    alone = {}
    for (gi, k, kw), r in zip(reqs, results):
        key = (gi, k, tuple(sorted(kw.items())))
        if key not in alone:
            g = graphs[gi]
            with bc.Graph(g.row_ptr, g.col, directed=g.directed) as G:
                alone[key] = G.topk(k, **kw)
        assert same(r, alone[key]), (gi, k, kw)
    checked = 0
    for gi in range(0, len(graphs), 3):
        for (gj, k, kw), r in zip(reqs, results):
            if gj == gi:
                ref = oracle.topk(graphs[gi], k, nthreads=8)
                assert r.ids.tolist() == ref["ids"].tolist() and r.farness.tolist() == ref["f"].tolist()
                assert r.reach.tolist() == ref["r"].tolist()
                checked += 1
                break
    assert checked >= 4


def test_queue_kernel_ends_and_restarts():
    """One request, then a pause long enough for the kernel to end with
    nothing to claim, then more requests: they are served by a new launch."""
    g1 = synth.barabasi_albert(5000, 4, 31)
    g2 = synth.erdos_renyi(4000, 8, 32)
    with bc.Server(lanes=2, budget_bytes=1 << 30, queue=True) as S:
        a = S.add_graph(g1.row_ptr, g1.col)
        b = S.add_graph(g2.row_ptr, g2.col)
        t = S.submit(a, 10, mode="batched")
        assert S.wait(t, 60000)
        r1 = S.poll(t)
        time.sleep(0.2)
        ts = [S.submit(b, k, mode="batched") for k in (1, 10, 100)]
        rs = []
        for t in ts:
            assert S.wait(t, 60000)
            rs.append(S.poll(t))
    ref = oracle.topk(g1, 10)
    assert r1.ids.tolist() == ref["ids"].tolist() and r1.farness.tolist() == ref["f"].tolist()
    for k, r in zip((1, 10, 100), rs):
        ref = oracle.topk(g2, k)
        assert r.ids.tolist() == ref["ids"].tolist() and r.farness.tolist() == ref["f"].tolist()
        assert r.reach.tolist() == ref["r"].tolist()


def test_queue_large_k_and_late_graph_use_lanes():
    """k above the queue's result capacity, and a graph registered after the
    queue was sized and larger than it, run as whole-request launches; the
    answers are still exact."""
    small = synth.barabasi_albert(3000, 4, 41)
    late = synth.erdos_renyi(9000, 8, 42)
    with bc.Server(lanes=2, budget_bytes=1 << 30, queue=True) as S:
        a = S.add_graph(small.row_ptr, small.col)
        t = S.submit(a, 10, mode="batched")  # makes the queue, sized for 3000 nodes
        assert S.wait(t, 60000)
        r0 = S.poll(t)
        b = S.add_graph(late.row_ptr, late.col)
        t1 = S.submit(a, 300, mode="batched")
        t2 = S.submit(b, 10, mode="batched")
        assert S.wait(t1, 60000) and S.wait(t2, 60000)
        r1, r2 = S.poll(t1), S.poll(t2)
    for g, k, r in ((small, 10, r0), (small, 300, r1), (late, 10, r2)):
        ref = oracle.topk(g, k)
        assert r.ids.tolist() == ref["ids"].tolist() and r.farness.tolist() == ref["f"].tolist()
