"""CPU oracle of the learned source order (features, MLP, loss gradient, Adam).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: the plain float64
reference the GPU kernels of the learned order are checked against.  Only the
test suite may import it; the GPU library shares no code with it.

Algorithm 1 may process the sources in any order and returns the same top-k
(the order only changes how soon the k-th best value is known, Section 2.1);
the paper uses decreasing degree.  The learned order replaces the degree by
the score of a small multilayer perceptron over three per-node features:

  x0(v) = log(1 + outdeg(v))
  x1(v) = log(1 + sum of outdeg(u) over the out-neighbours u of v)
  x2(v) = log(1 + core(v))

where core(v) is the largest c such that v lies in a subgraph in which every
node has at least c out-neighbours inside the subgraph (the k-core number for
an undirected graph).  Each column is standardised over the nodes of the
graph: (x - mean) / std with the population std; a column whose integers
are all equal becomes 0.

Network (fp32 on the device, float64 here), parameters in one flat vector:
  W1[64][3] @0, b1[64] @192, W2[64][64] @256, b2[64] @4352, w3[64] @4416, b3 @4480
  h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = w3 . h2 + b3
Loss over the samples i (node idx[i], or i itself):
  L = sum_i w_i (y_i - t_i)^2 / sum_i w_i
Adam (Kingma and Ba, 2015) with bias correction.

None of this is in the paper.  tests/test_oracle_mlp.py pins it against
independent code (networkx k-cores, torch.nn layers, torch autograd and
torch.optim.Adam in float64, scipy sparse products), central finite
differences, and the core definition written out on tiny inputs.
"""

from __future__ import annotations

import heapq

import numpy as np

HIDDEN = 64
N_IN = 3
OFF_W1 = 0
OFF_B1 = OFF_W1 + HIDDEN * N_IN
OFF_W2 = OFF_B1 + HIDDEN
OFF_B2 = OFF_W2 + HIDDEN * HIDDEN
OFF_W3 = OFF_B2 + HIDDEN
OFF_B3 = OFF_W3 + HIDDEN
N_PARAMS = OFF_B3 + 1  # 4481


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    assert p.shape == (N_PARAMS,)
    return (p[OFF_W1:OFF_B1].reshape(HIDDEN, N_IN), p[OFF_B1:OFF_W2], p[OFF_W2:OFF_B2].reshape(HIDDEN, HIDDEN),
            p[OFF_B2:OFF_W3], p[OFF_W3:OFF_B3], p[OFF_B3])


def out_degree(g) -> np.ndarray:
    return np.diff(g.row_ptr.astype(np.int64))


def two_hop_degree_sum(g) -> np.ndarray:
    """sum of outdeg(u) over the out-arcs v -> u (one term per arc)."""
    deg = out_degree(g)
    rows = np.repeat(np.arange(g.n), deg)
    s = np.zeros(g.n, np.int64)
    np.add.at(s, rows, deg[g.col.astype(np.int64)])
    return s


def core_number(g) -> np.ndarray:
    """Out-core number by peeling: repeatedly remove a node of smallest
    remaining out-degree; core(v) is the largest such smallest degree seen up
    to v's removal.  Removing v lowers the out-degree of its in-neighbours."""
    n = g.n
    deg = out_degree(g).copy()
    rp = g.row_ptr.astype(np.int64)
    col = g.col.astype(np.int64)
    # in-neighbour lists
    src = np.repeat(np.arange(n), np.diff(rp))
    order = np.argsort(col, kind="stable")
    in_src = src[order]
    in_rp = np.zeros(n + 1, np.int64)
    np.add.at(in_rp, col + 1, 1)
    in_rp = np.cumsum(in_rp)
    removed = np.zeros(n, bool)
    heap = [(int(deg[v]), v) for v in range(n)]
    heapq.heapify(heap)
    core = np.zeros(n, np.int64)
    level = 0
    while heap:
        d, v = heapq.heappop(heap)
        if removed[v] or d != deg[v]:
            continue
        removed[v] = True
        level = max(level, d)
        core[v] = level
        for u in in_src[in_rp[v]:in_rp[v + 1]]:
            if not removed[u]:
                deg[u] -= 1
                heapq.heappush(heap, (int(deg[u]), int(u)))
    return core


def raw_features(g) -> np.ndarray:
    deg = out_degree(g)
    return np.stack([np.log1p(deg.astype(np.float64)), np.log1p(two_hop_degree_sum(g).astype(np.float64)),
                     np.log1p(core_number(g).astype(np.float64))], axis=1)


def standardise(x: np.ndarray, constant=None) -> np.ndarray:
    """(x - mean) / std per column (population std).  A column flagged in
    `constant` (decided on the integers the features are computed from, all
    equal) becomes 0; its floating std would be a rounding residue."""
    x = np.asarray(x, dtype=np.float64)
    if x.shape[0] == 0:
        return x.copy()
    if constant is None:
        constant = [bool(np.all(x[:, j] == x[0, j])) for j in range(x.shape[1])]
    mu = x.mean(axis=0)
    sd = np.sqrt(((x - mu) ** 2).mean(axis=0))
    out = np.zeros_like(x)
    for j in range(x.shape[1]):
        if not constant[j]:
            out[:, j] = (x[:, j] - mu[j]) / sd[j]
    return out


def features(g) -> np.ndarray:
    """Standardised (n, 3) features of the learned order."""
    ints = [out_degree(g), two_hop_degree_sum(g), core_number(g)]
    raw = np.stack([np.log1p(a.astype(np.float64)) for a in ints], axis=1)
    return standardise(raw, [len(a) == 0 or bool(a.min() == a.max()) for a in ints])


def forward(p, x, return_hidden: bool = False):
    W1, b1, W2, b2, w3, b3 = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    h1 = np.maximum(x @ W1.T + b1, 0.0)
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    y = h2 @ w3 + b3
    return (y, h1, h2) if return_hidden else y


def loss_grad(p, x, t, w=None, idx=None):
    """Loss and its gradient (flat, N_PARAMS), by backpropagation.  Also
    returns the same backpropagation with every factor replaced by its
    absolute value: a bound on the magnitude of the terms summed into each
    gradient entry (used to size floating-point tolerances)."""
    x = np.asarray(x, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    if idx is not None:
        idx = np.asarray(idx, dtype=np.int64)
        x, t = x[idx], t[idx]
        w = None if w is None else np.asarray(w, dtype=np.float64)[idx]
    w = np.ones(len(t)) if w is None else np.asarray(w, dtype=np.float64)
    W1, b1, W2, b2, w3, b3 = unpack(p)
    y, h1, h2 = forward(p, x, return_hidden=True)
    sw = w.sum()
    if sw == 0:
        return 0.0, np.zeros(N_PARAMS), np.zeros(N_PARAMS)
    r = y - t
    loss = float((w * r * r).sum() / sw)

    def backprop(dy, W2m, w3v, h1m, h2m, xm):
        a1 = (h1m > 0).astype(np.float64)
        a2 = (h2m > 0).astype(np.float64)
        g = np.zeros(N_PARAMS)
        g[OFF_W3:OFF_B3] = h2m.T @ dy
        g[OFF_B3] = dy.sum()
        d2 = np.outer(dy, w3v) * a2                    # (N, 64)
        g[OFF_W2:OFF_B2] = (d2.T @ h1m).reshape(-1)
        g[OFF_B2:OFF_W3] = d2.sum(axis=0)
        d1 = (d2 @ W2m) * a1                           # (N, 64)
        g[OFF_W1:OFF_B1] = (d1.T @ xm).reshape(-1)
        g[OFF_B1:OFF_W2] = d1.sum(axis=0)
        return g

    dy = 2.0 * w * r / sw
    grad = backprop(dy, W2, w3, h1, h2, x)
    mag = backprop(np.abs(dy), np.abs(W2), np.abs(w3), h1, h2, np.abs(x))
    return loss, grad, mag


def adam_step(p, g, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (returns new p, m, v); step counts from 1."""
    p = np.asarray(p, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def closeness_label(r, f):
    """Training target: log((r-1)^2 / f) standardised over the nodes with
    r > 1 (weight 1); nodes with r = 1 (closeness 0) get weight 0."""
    r = np.asarray(r, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    w = (r > 1).astype(np.float64)
    t = np.zeros(len(r))
    ok = w > 0
    if ok.any():
        t[ok] = np.log((r[ok] - 1) ** 2 / f[ok])
        mu = t[ok].mean()
        sd = np.sqrt(((t[ok] - mu) ** 2).mean())
        t[ok] = (t[ok] - mu) / sd if sd > 0 else 0.0
    return t, w
