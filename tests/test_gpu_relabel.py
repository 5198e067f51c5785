"""Renumbering of undirected graphs on upload (breadth-first order, for the
locality of node records) is invisible to the caller: with and without it
(BC_KEEP_IDS) every query returns the same ids, farness and reach (ties are
broken by the caller's ids), and the per-node outputs (canonical CSR, reach
data, features, source orders) come back in the caller's numbering."""

import numpy as np
import pytest
import torch

import oracle
import paper_1507_01490_amd as bc
from paper_1507_01490_amd import synth

pytestmark = pytest.mark.gpu

# graphs of 100,000 nodes and more are renumbered
GRAPHS = [
    ("ba", lambda: synth.barabasi_albert(120000, 4, 81), (1, 10, 50)),
    ("grid", lambda: synth.grid_shortcuts(110000, 0.01, 82), (1, 10, 50)),
    ("collab", lambda: synth.collaboration(120000, 30000, 2.1, 200, 83), (10,)),
    # vertex-transitive, a few dozen levels deep: every node ties, so the
    # caller's ids decide
    ("circulant", lambda: synth.circulant(100000, (1, 47, 2209)), (10,)),
    ("union", lambda: synth.disjoint_union(synth.path(9), synth.star(12), synth.empty(99970), synth.complete(5)),
     (1, 10, 50)),
]


def same(a, b):
    return a.ids.tolist() == b.ids.tolist() and a.farness.tolist() == b.farness.tolist() and \
        a.reach.tolist() == b.reach.tolist()


@pytest.mark.parametrize("gi", range(len(GRAPHS)))
def test_renumbering_is_invisible(gi):
    name, make, ks = GRAPHS[gi]
    g = make()
    print(f"[relabel] {name} n={g.n}", flush=True)
    refs = {k: oracle.topk(g, k, nthreads=16) for k in set(ks) | {10}}
    with bc.Graph(g.row_ptr, g.col) as R, bc.Graph(g.row_ptr, g.col, keep_ids=True) as K:
        for k in ks:
            print(f"[relabel] {name} k={k}", flush=True)
            ref = refs[k]
            for kw in (dict(mode="plain"), dict(mode="batched"), dict(mode="batched", width=256),
                       dict(mode="batched", order="learned_grouped"), dict(mode="batched", order="locality")):
                a, b = R.topk(k, **kw), K.topk(k, **kw)
                assert same(a, b), (name, k, kw)
                assert a.ids.tolist() == ref["ids"].tolist() and a.farness.tolist() == ref["f"].tolist(), (name, kw)
            assert same(R.topk_static(k), K.topk_static(k))
            out = bc.topk_multi([R, K], [k, k])
            assert same(out[0], out[1]) and out[0].ids.tolist() == ref["ids"].tolist()
        # per-node outputs in the caller's numbering
        print(f"[relabel] {name} per-node outputs", flush=True)
        rp_r, col_r = R.csr()
        rp_k, col_k = K.csr()
        assert rp_r.tolist() == rp_k.tolist() and col_r.tolist() == col_k.tolist()
        lo_r, hi_r = R.reach()
        lo_k, hi_k = K.reach()
        assert lo_r.tolist() == lo_k.tolist() and hi_r.tolist() == hi_k.tolist()
        x_r, c_r = R.features()
        x_k, c_k = K.features()
        assert torch.equal(c_r, c_k)
        assert torch.allclose(x_r, x_k, rtol=0, atol=1e-5)
        f_r, r_r, _ = R.farness_all()
        f_k, r_k, _ = K.farness_all()
        assert f_r.tolist() == f_k.tolist() and r_r.tolist() == r_k.tolist()
        # orders given in the caller's ids come back as given; warm starts too
        perm = np.random.default_rng(gi).permutation(g.n).astype(np.int32)
        assert R.source_order(10, order=perm).tolist() == perm.tolist()
        first = perm[:5]
        assert R.source_order(10, mode="plain", order="degree", first=first)[:5].tolist() == first.tolist()
        a = R.topk(10, mode="batched", order=perm)
        b = R.topk(10, mode="batched", first=first)
        ref = refs[10]
        assert a.ids.tolist() == ref["ids"].tolist() and b.ids.tolist() == ref["ids"].tolist()
        sc = np.random.default_rng(7).random(g.n).astype(np.float32)
        assert R.topk(10, mode="plain", scores=sc).ids.tolist() == ref["ids"].tolist()


def test_server_on_renumbered_graphs():
    g = synth.barabasi_albert(150000, 4, 84)
    ref = oracle.topk(g, 10, nthreads=16)
    for queue in (False, True):
        with bc.Server(lanes=1, budget_bytes=1 << 30, queue=queue) as S:
            gid = S.add_graph(g.row_ptr, g.col)
            t = S.submit(gid, 10, mode="batched")
            assert S.wait(t, 60000)
            r = S.poll(t)
        assert r.ids.tolist() == ref["ids"].tolist() and r.farness.tolist() == ref["f"].tolist()
