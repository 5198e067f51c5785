"""GPU parity of the learned-order path and of the every-node farness.

* bc_farness_all: exact farness and reach of every node against brute force.
* Features: core numbers bit-exact against the oracle's peeling; the
  standardised features (fp64 on the device, stored as fp32) within a few
  fp32 ulps of the oracle's float64 values.
* Perceptron forward, loss gradient and Adam step against the float64
  oracle, with tolerances sized from the arithmetic: fp32 sums of at most
  64 (forward) or 128 (one gradient tile) terms, each entry bounded by the
  same computation with every factor replaced by its absolute value.
* The learned order never changes the answer (bit-exact against the
  oracle), and BC_ORDER_LEARNED equals sorting the device scores through
  the scores path (same processing, same m_vis)."""

import numpy as np
import pytest

import oracle
import paper_1507_01490_amd as bc
from oracle import mlp as omlp
from paper_1507_01490_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def rand_params(seed):
    rng = np.random.default_rng(seed)
    p = np.zeros(bc.MLP_PARAMS, np.float32)
    p[0:192] = rng.normal(0, np.sqrt(2 / 3), 192)
    p[192:256] = rng.normal(0, 0.2, 64)
    p[256:4352] = rng.normal(0, np.sqrt(2 / 64), 4096)
    p[4352:4416] = rng.normal(0, 0.2, 64)
    p[4416:4480] = rng.normal(0, np.sqrt(1 / 64), 64)
    p[4480] = 0.1
    return p


def cuda(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda().contiguous()


FEATURE_GRAPHS = [
    synth.erdos_renyi(4000, 8, 1), synth.barabasi_albert(30000, 5, 2), synth.grid_shortcuts(5000, 0.01, 3),
    synth.collaboration(8000, 2000, 2.1, 200, 4), synth.random_geometric(6000, 6.0, 5),
    synth.random_small(800, 0.01, True, 6), synth.rmat(13, 16, 0.57, 0.19, 0.19, 7),
    synth.star(300), synth.cycle(11), synth.empty(4), synth.complete(9),
]


@pytest.mark.parametrize("gi", range(len(FEATURE_GRAPHS)))
def test_features_vs_oracle(gi):
    g = FEATURE_GRAPHS[gi]
    with bc.Graph(g.row_ptr, g.col, directed=g.directed) as G:
        x, core = G.features()
        x = x.cpu().numpy().astype(np.float64)
        core = core.cpu().numpy().view(np.uint32)
    assert core.tolist() == omlp.core_number(g).tolist()
    ref = omlp.features(g)
    assert np.all(np.abs(x - ref) <= 4 * U32 * (1 + np.abs(ref))), np.abs(x - ref).max()


@pytest.mark.parametrize("seed", range(3))
def test_forward_vs_oracle(seed):
    rng = np.random.default_rng(seed)
    p = rand_params(10 + seed)
    x = rng.normal(size=(20011, 3)).astype(np.float32)
    y = bc.mlp_forward(cuda(p), cuda(x)).cpu().numpy().astype(np.float64)
    ref = omlp.forward(p.astype(np.float64), x.astype(np.float64))
    # magnitude bound: the same network with |weights| on |inputs|
    pa = np.abs(p.astype(np.float64))
    mag = omlp.forward(pa, np.abs(x.astype(np.float64)))
    assert np.all(np.abs(y - ref) <= 200 * U32 * mag + 1e-7)


@pytest.mark.parametrize("case", ["all", "idx", "weights", "ragged"])
def test_loss_grad_vs_oracle(case):
    rng = np.random.default_rng(["all", "idx", "weights", "ragged"].index(case) + 50)
    g = synth.barabasi_albert(5000, 4, 8) if case != "ragged" else synth.erdos_renyi(1000, 6, 9)
    with bc.Graph(g.row_ptr, g.col) as G:
        x, _ = G.features()
    xn = x.cpu().numpy().astype(np.float64)
    rows = xn.shape[0]
    t = rng.normal(size=rows).astype(np.float32)
    w = (rng.random(rows) < 0.7).astype(np.float32) if case in ("weights", "ragged") else None
    idx = rng.integers(0, rows, 3001).astype(np.int32) if case in ("idx", "ragged") else None
    p = rand_params(20)
    grad, loss = bc.mlp_loss_grad(cuda(p), x.contiguous(), cuda(t), None if w is None else cuda(w),
                                  None if idx is None else cuda(idx, torch.int32))
    lref, gref, mag = omlp.loss_grad(p.astype(np.float64), xn, t.astype(np.float64),
                                     None if w is None else w.astype(np.float64), idx)
    grad = grad.cpu().numpy().astype(np.float64)
    assert abs(loss - lref) <= 1e-5 * abs(lref) + 1e-9
    assert np.all(np.abs(grad - gref) <= 400 * U32 * mag + 1e-9), np.abs(grad - gref).max()


def test_loss_grad_edges():
    p = cuda(rand_params(1))
    x = cuda(np.zeros((5, 3), np.float32))
    t = cuda(np.zeros(5, np.float32))
    grad, loss = bc.mlp_loss_grad(p, x, t, None, cuda(np.zeros(0, np.int32), torch.int32))
    assert loss == 0.0 and float(grad.abs().max()) == 0.0
    with pytest.raises(bc.BcError) as e:
        bc.mlp_loss_grad(p, x, t, None, cuda(np.array([0, 5], np.int32), torch.int32))
    assert e.value.status == -1


def test_adam_vs_oracle():
    rng = np.random.default_rng(3)
    p = rng.normal(size=bc.MLP_PARAMS).astype(np.float32)
    pt, mt, vt = cuda(p), torch.zeros(bc.MLP_PARAMS, device="cuda"), torch.zeros(bc.MLP_PARAMS, device="cuda")
    pr, mr, vr = p.astype(np.float64), np.zeros(bc.MLP_PARAMS), np.zeros(bc.MLP_PARAMS)
    for step in range(1, 6):
        gr = rng.normal(size=bc.MLP_PARAMS).astype(np.float32)
        bc.mlp_adam(pt, cuda(gr), mt, vt, step, 1e-3)
        pr, mr, vr = omlp.adam_step(pr, gr.astype(np.float64), mr, vr, step, 1e-3)
        # each step moves p by at most ~lr; fp32 keeps p to 1 ulp and the
        # update to a few ulps of lr
        assert np.all(np.abs(pt.cpu().numpy() - pr) <= step * (4 * U32 * (1 + np.abs(pr)) + 1e-3 * 1e-5))
        assert np.allclose(mt.cpu().numpy(), mr, rtol=1e-5, atol=1e-6)
        assert np.allclose(vt.cpu().numpy(), vr, rtol=1e-5, atol=1e-7)


FARNESS_GRAPHS = [synth.path(9), synth.star(12), synth.directed_path(8), synth.out_star(9), synth.empty(3),
                  synth.disjoint_union(synth.path(5), synth.complete(3)), synth.barabasi_albert(2000, 5, 0),
                  synth.random_small(500, 0.008, True, 44), synth.random_small(700, 0.004, False, 45),
                  synth.rmat(11, 8, 0.57, 0.19, 0.19, 46)]


@pytest.mark.parametrize("gi", range(len(FARNESS_GRAPHS)))
def test_farness_all_vs_bruteforce(gi):
    g = FARNESS_GRAPHS[gi]
    r, f = oracle.bruteforce(g, nthreads=8)
    with bc.Graph(g.row_ptr, g.col, directed=g.directed) as G:
        for kw in (dict(mode="plain"), dict(mode="batched"), dict(mode="batched", width=256),
                   dict(mode="plain", width=128), dict(mode="batched", defer_arcs=1)):
            far, rea, st = G.farness_all(**kw)
            assert far.tolist() == f.tolist() and rea.tolist() == r.tolist(), kw
            assert st["n_cut"] == 0 and st["n_done"] + st["n_trivial"] == g.n


LEARNED_GRAPHS = [synth.barabasi_albert(20000, 4, 31), synth.random_geometric(8000, 6.0, 32),
                  synth.collaboration(12000, 3000, 2.1, 200, 33), synth.rmat(13, 16, 0.57, 0.19, 0.19, 34),
                  synth.grid_shortcuts(9000, 0.01, 35)]


@pytest.mark.parametrize("gi", range(len(LEARNED_GRAPHS)))
def test_learned_order_is_exact(gi):
    g = LEARNED_GRAPHS[gi]
    p = rand_params(40 + gi)
    with bc.Graph(g.row_ptr, g.col, directed=g.directed) as G:
        x, _ = G.features()
        scores = bc.mlp_forward(cuda(p), x.contiguous()).cpu().numpy()
        for k in (1, 10, 100):
            ref = oracle.topk(g, k, nthreads=8)
            for order in ("learned", "learned_grouped"):
                for kw in (dict(mode="plain"), dict(mode="batched"), dict(mode="batched", width=256),
                           dict(mode="batched", seed_batches=3)):
                    a = G.topk(k, order=order, mlp=p, **kw)
                    assert a.ids.tolist() == ref["ids"].tolist(), (k, order, kw)
                    assert a.farness.tolist() == ref["f"].tolist() and a.reach.tolist() == ref["r"].tolist()
            # the learned order is the scores order of the device scores
            a = G.topk(k, order="learned", mlp=p, mode="plain")
            b = G.topk(k, scores=scores, mode="plain")
            assert a.stats["m_vis"] == b.stats["m_vis"] and a.stats["batches"] == b.stats["batches"]


def _spearman(a, b):
    ra = np.argsort(np.argsort(a, kind="stable"), kind="stable").astype(np.float64)
    rb = np.argsort(np.argsort(b, kind="stable"), kind="stable").astype(np.float64)
    ra -= ra.mean()
    rb -= rb.mean()
    return float((ra * rb).sum() / np.sqrt((ra * ra).sum() * (rb * rb).sum()))


GAIN_GRAPHS = [("ba", synth.barabasi_albert(20000, 4, 9101)), ("er", synth.erdos_renyi(20000, 8, 9102)),
               ("grid", synth.grid_shortcuts(20000, 0.01, 9103))]


@pytest.mark.parametrize("gi", range(len(GAIN_GRAPHS)))
def test_learned_order_gain(gi):
    """The shipped perceptron ranks held-out graphs (seeds outside the
    training set) closer to their true closeness order than the degree does
    (Spearman correlation over the nodes with r > 1, exact closeness from
    bc_farness_all), and the answer stays exact."""
    fam, g = GAIN_GRAPHS[gi]
    p = bc.default_mlp()
    with bc.Graph(g.row_ptr, g.col) as G:
        far, rea, _ = G.farness_all()
        x, _ = G.features()
        y = bc.mlp_forward(cuda(p), x.contiguous()).cpu().numpy().astype(np.float64)
        r = rea.astype(np.float64)
        c = np.where(r > 1, (r - 1) ** 2 / np.maximum(far.astype(np.float64), 1), 0.0)
        ok = r > 1
        s_learned = _spearman(y[ok], c[ok])
        s_degree = _spearman(np.diff(g.row_ptr)[ok].astype(np.float64), c[ok])
        print(f"{fam}: spearman learned {s_learned:.4f} degree {s_degree:.4f}")
        assert s_learned > s_degree + 0.02, (fam, s_learned, s_degree)
        ref = oracle.topk(g, 100, nthreads=8)
        for order in ("learned", "learned_grouped"):
            a = G.topk(100, mode="batched", order=order)
            assert a.ids.tolist() == ref["ids"].tolist(), order
            assert a.farness.tolist() == ref["f"].tolist() and a.reach.tolist() == ref["r"].tolist(), order


def test_learned_grouped_falls_back_to_degree_order_on_directed_graphs():
    """The shipped perceptron is trained on undirected families; on a
    directed graph the learned-grouped order is the grouped degree order
    (the fallback), and the answer is the oracle's."""
    g = synth.rmat(12, 16, 0.57, 0.19, 0.19, 61)
    with bc.Graph(g.row_ptr, g.col, directed=True) as G:
        a = G.source_order(10, mode="batched", order="learned_grouped")
        b = G.source_order(10, mode="batched", order="grouped")
        assert a.tolist() == b.tolist()
        res = G.topk(10, mode="batched", order="learned_grouped")
    ref = oracle.topk(g, 10)
    assert res.ids.tolist() == ref["ids"].tolist() and res.farness.tolist() == ref["f"].tolist()
    u = synth.barabasi_albert(3000, 3, 62)
    with bc.Graph(u.row_ptr, u.col) as G:
        a = G.source_order(10, mode="batched", order="learned_grouped")
        b = G.source_order(10, mode="batched", order="grouped")
        assert a.tolist() != b.tolist()  # undirected: the learned head is used


@pytest.mark.parametrize("width", [64, 256])
def test_learned_locality_order(width):
    """BC_ORDER_LEARNED_LOCALITY: the k best-scored sources (the head of the
    pure learned order), then the locality order without them; exact."""
    g = synth.random_geometric(6000, 6.0, 71)
    k = 10
    with bc.Graph(g.row_ptr, g.col) as G:
        ll = G.source_order(k, mode="batched", width=width, order="learned_locality")
        lr = G.source_order(k, mode="batched", width=width, order="learned")
        loc = G.source_order(k, mode="batched", width=width, order="locality")
        assert sorted(ll.tolist()) == list(range(g.n))
        head = ll[:k].tolist()
        assert head == lr[:k].tolist()
        assert ll[k:].tolist() == [v for v in loc.tolist() if v not in set(head)]
        res = G.topk(k, mode="batched", width=width, order="learned_locality")
    ref = oracle.topk(g, k)
    assert res.ids.tolist() == ref["ids"].tolist() and res.farness.tolist() == ref["f"].tolist()
