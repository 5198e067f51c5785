"""Pins of the learned-order oracle (oracle/mlp.py) against independent code:
networkx k-cores, the core definition by repeated pruning, scipy sparse
products, torch.nn / torch autograd / torch.optim.Adam in float64, and
central finite differences."""

import itertools

import networkx as nx
import numpy as np
import pytest
import scipy.sparse as sp
import torch

from oracle import mlp
from paper_1507_01490_amd import synth


def _init(seed):
    rng = np.random.default_rng(seed)
    p = np.zeros(mlp.N_PARAMS)
    p[mlp.OFF_W1:mlp.OFF_B1] = rng.normal(0, np.sqrt(2 / 3), 192)
    p[mlp.OFF_B1:mlp.OFF_W2] = rng.normal(0, 0.1, 64)
    p[mlp.OFF_W2:mlp.OFF_B2] = rng.normal(0, np.sqrt(2 / 64), 4096)
    p[mlp.OFF_B2:mlp.OFF_W3] = rng.normal(0, 0.1, 64)
    p[mlp.OFF_W3:mlp.OFF_B3] = rng.normal(0, np.sqrt(1 / 64), 64)
    p[mlp.OFF_B3] = 0.3
    return p


def _core_by_pruning(g):
    """core(v) = max c such that v survives repeated deletion of the nodes
    with fewer than c out-neighbours left (the definition, one c at a time)."""
    n = g.n
    succ = [set(g.col[g.row_ptr[v]:g.row_ptr[v + 1]].tolist()) for v in range(n)]
    core = np.zeros(n, np.int64)
    for c in itertools.count(1):
        alive = set(range(n))
        changed = True
        while changed:
            changed = False
            for v in list(alive):
                if len(succ[v] & alive) < c:
                    alive.discard(v)
                    changed = True
        if not alive:
            return core
        for v in alive:
            core[v] = c


@pytest.mark.parametrize("seed", range(6))
def test_core_number_vs_networkx(seed):
    for g in (synth.random_small(200, 0.03, False, 900 + seed), synth.barabasi_albert(500, 3 + seed % 3, seed),
              synth.grid_shortcuts(400, 0.05, seed)):
        G = nx.Graph()
        G.add_nodes_from(range(g.n))
        G.add_edges_from(zip(*(a.tolist() for a in g.edges())))
        ref = nx.core_number(G)
        assert mlp.core_number(g).tolist() == [ref[v] for v in range(g.n)]


@pytest.mark.parametrize("seed", range(8))
def test_core_number_by_definition_directed(seed):
    g = synth.random_small(40, 0.08 + 0.02 * (seed % 4), True, 700 + seed)
    assert mlp.core_number(g).tolist() == _core_by_pruning(g).tolist()


def test_core_number_closed_forms():
    assert mlp.core_number(synth.complete(6)).tolist() == [5] * 6
    assert mlp.core_number(synth.path(7)).tolist() == [1] * 7
    assert mlp.core_number(synth.star(9)).tolist() == [1] * 9
    assert mlp.core_number(synth.directed_cycle(5)).tolist() == [1] * 5
    assert mlp.core_number(synth.directed_path(5)).tolist() == [0] * 5
    assert mlp.core_number(synth.empty(3)).tolist() == [0] * 3
    # K4 with a pendant path: the clique is the 3-core, the path the 1-core
    s, d = synth.disjoint_union(synth.complete(4), synth.path(3)).edges()
    g2 = synth.from_edges(7, np.r_[s, 3], np.r_[d, 4], False)
    assert mlp.core_number(g2).tolist() == [3, 3, 3, 3, 1, 1, 1]


@pytest.mark.parametrize("directed", [False, True])
def test_two_hop_sum_vs_sparse_product(directed):
    g = synth.random_small(300, 0.02, directed, 31)
    A = sp.csr_matrix((np.ones(g.m), g.col, g.row_ptr), shape=(g.n, g.n))
    deg = np.asarray(A.sum(axis=1)).ravel()
    assert mlp.two_hop_degree_sum(g).tolist() == (A @ deg).astype(np.int64).tolist()


def test_standardise_invariants():
    g = synth.erdos_renyi(3000, 6, 5)
    x = mlp.features(g)
    assert np.allclose(x.mean(axis=0), 0, atol=1e-12)
    assert np.allclose(x.std(axis=0), 1, atol=1e-12)
    # constant columns become 0: every node of a cycle looks alike, and every
    # node of a Barabasi-Albert graph with m = 4 has core number 4
    assert np.all(mlp.features(synth.cycle(9)) == 0)
    assert np.all(mlp.features(synth.barabasi_albert(3000, 4, 5))[:, 2] == 0)
    # the raw columns are monotone images of degree, 2-hop sum and core
    raw = mlp.raw_features(g)
    assert np.allclose(np.expm1(raw[:, 0]), np.diff(g.row_ptr))


def _torch_net(p):
    W1, b1, W2, b2, w3, b3 = mlp.unpack(p)
    net = torch.nn.Sequential(torch.nn.Linear(3, 64), torch.nn.ReLU(), torch.nn.Linear(64, 64), torch.nn.ReLU(),
                              torch.nn.Linear(64, 1)).double()
    with torch.no_grad():
        net[0].weight.copy_(torch.from_numpy(W1))
        net[0].bias.copy_(torch.from_numpy(b1))
        net[2].weight.copy_(torch.from_numpy(W2))
        net[2].bias.copy_(torch.from_numpy(b2))
        net[4].weight.copy_(torch.from_numpy(w3[None, :]))
        net[4].bias.copy_(torch.tensor([b3]))
    return net


def _flat_grad(net):
    return np.concatenate([net[0].weight.grad.numpy().ravel(), net[0].bias.grad.numpy(),
                           net[2].weight.grad.numpy().ravel(), net[2].bias.grad.numpy(),
                           net[4].weight.grad.numpy().ravel(), net[4].bias.grad.numpy()])


@pytest.mark.parametrize("seed", range(3))
def test_forward_and_grad_vs_torch(seed):
    rng = np.random.default_rng(seed)
    p = _init(seed)
    x = rng.normal(size=(500, 3))
    t = rng.normal(size=500)
    w = (rng.random(500) < 0.8).astype(np.float64)
    idx = rng.integers(0, 500, 300)
    net = _torch_net(p)
    y = net(torch.from_numpy(x)).detach().numpy()[:, 0]
    assert np.allclose(mlp.forward(p, x), y, rtol=1e-12, atol=1e-12)
    loss, grad, mag = mlp.loss_grad(p, x, t, w, idx)
    xt = torch.from_numpy(x[idx])
    tt = torch.from_numpy(t[idx])
    wt = torch.from_numpy(w[idx])
    lt = (wt * (net(xt)[:, 0] - tt) ** 2).sum() / wt.sum()
    lt.backward()
    assert abs(loss - lt.item()) < 1e-12
    assert np.allclose(grad, _flat_grad(net), rtol=1e-10, atol=1e-12)
    assert np.all(mag >= np.abs(grad) - 1e-12)


def test_grad_vs_finite_differences():
    rng = np.random.default_rng(9)
    p = _init(9)
    x = rng.normal(size=(64, 3))
    t = rng.normal(size=64)
    _, grad, _ = mlp.loss_grad(p, x, t)
    h = 1e-6
    for j in list(range(0, mlp.N_PARAMS, 97)) + [mlp.OFF_B3, mlp.OFF_W3 + 5, mlp.OFF_B1 + 7]:
        e = np.zeros(mlp.N_PARAMS)
        e[j] = h
        fd = (mlp.loss_grad(p + e, x, t)[0] - mlp.loss_grad(p - e, x, t)[0]) / (2 * h)
        assert abs(fd - grad[j]) <= 1e-6 * (1 + abs(grad[j])), j


def test_adam_vs_torch():
    rng = np.random.default_rng(4)
    p0 = rng.normal(size=50)
    pt = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for step in range(1, 8):
        g = rng.normal(size=50)
        pt.grad = torch.from_numpy(g.copy())
        opt.step()
        p, m, v = mlp.adam_step(p, g, m, v, step, 3e-3)
        assert np.allclose(p, pt.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_label_definition():
    r = np.array([1, 5, 5, 3, 1])
    f = np.array([0, 4, 8, 2, 0])
    t, w = mlp.closeness_label(r, f)
    assert w.tolist() == [0, 1, 1, 1, 0]
    raw = np.log(np.array([16 / 4, 16 / 8, 4 / 2]))
    z = (raw - raw.mean()) / raw.std()
    assert np.allclose(t[[1, 2, 3]], z) and t[0] == 0 and t[4] == 0
