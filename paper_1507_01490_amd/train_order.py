"""Train the order perceptron on the GPU and write ``order_mlp.npy``.

Training data: seeded synthetic graphs of the serving and large-graph
families (Erdos-Renyi average degree 8, Barabasi-Albert m = 4, 2-D grid with
1 % shortcuts, collaboration projection, random geometric average degree 6),
n log-uniform in [1e3, 2e4].  Label of node v: log((r-1)^2 / f), the log of
its closeness up to the common factor 1/(n-1), standardised per graph over
the nodes with r > 1; nodes with r = 1 get weight 0.  Exact r and f of every
node come from the library itself (bc_farness_all: one search per node, no
cut).

Features, forward pass, loss gradient and Adam all run in the library's HIP
kernels (bc_graph_features, bc_mlp_loss_grad, bc_mlp_adam); this script only
generates graphs and schedules the steps.

    python -m paper_1507_01490_amd.train_order [--graphs 40] [--steps 20000] [--batch 32768]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import paper_1507_01490_amd as bc  # noqa: E402
from paper_1507_01490_amd import synth  # noqa: E402

FAMILIES = ("er", "ba", "grid", "collab", "rgg")


def family_graph(fam: str, n: int, seed: int) -> synth.Csr:
    if fam == "er":
        return synth.erdos_renyi(n, 8.0, seed)
    if fam == "ba":
        return synth.barabasi_albert(n, 4, seed)
    if fam == "grid":
        return synth.grid_shortcuts(n, 0.01, seed)
    if fam == "collab":
        # actors : groups = 4 : 1 as in the large collaboration workload
        return synth.collaboration(n, max(1, n // 4), 2.1, 200, seed)
    if fam == "rgg":
        return synth.random_geometric(n, 6.0, seed)
    raise KeyError(fam)


def graph_set(count_per_family: int, seed0: int, lo: float = 1e3, hi: float = 2e4):
    rng = np.random.Generator(np.random.PCG64(seed0))
    out = []
    for i in range(count_per_family):
        for j, fam in enumerate(FAMILIES):
            n = int(np.exp(rng.uniform(np.log(lo), np.log(hi))))
            out.append((fam, family_graph(fam, n, seed0 + 1000 * j + i)))
    return out


def labels_of(G: "bc.Graph"):
    """(t, w, r, f) of every node from its exact reach and farness."""
    far, rea, _ = G.farness_all()
    r = rea.astype(np.float64)
    f = far.astype(np.float64)
    w = (r > 1).astype(np.float32)
    t = np.zeros(G.n, np.float64)
    ok = w > 0
    if ok.any():
        t[ok] = np.log((r[ok] - 1.0) ** 2 / f[ok])
        mu, sd = t[ok].mean(), t[ok].std()
        t[ok] = (t[ok] - mu) / sd if sd > 0 else 0.0
    return t.astype(np.float32), w, r, f


def init_params(seed: int) -> np.ndarray:
    """He-normal weights, zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = np.zeros(bc.MLP_PARAMS, np.float32)
    p[0:192] = rng.normal(0, np.sqrt(2 / 3), 192)
    p[256:4352] = rng.normal(0, np.sqrt(2 / 64), 4096)
    p[4416:4480] = rng.normal(0, np.sqrt(1 / 64), 64)
    return p


def spearman(a, b) -> float:
    ra = np.argsort(np.argsort(a, kind="stable"), kind="stable").astype(np.float64)
    rb = np.argsort(np.argsort(b, kind="stable"), kind="stable").astype(np.float64)
    ra -= ra.mean()
    rb -= rb.mean()
    d = np.sqrt((ra * ra).sum() * (rb * rb).sum())
    return float((ra * rb).sum() / d) if d > 0 else 0.0


def prepare(graphs, log=print):
    import torch
    xs, ts, ws, meta = [], [], [], []
    for fam, g in graphs:
        with bc.Graph(g.row_ptr, g.col, directed=g.directed) as G:
            x, _ = G.features()
            t, w, r, f = labels_of(G)
        xs.append(x.clone())
        ts.append(torch.from_numpy(t))
        ws.append(torch.from_numpy(w))
        meta.append(dict(family=fam, n=g.n, m=g.m, r=r, f=f, deg=np.diff(g.row_ptr)))
    X = torch.cat(xs).contiguous()
    T = torch.cat(ts).cuda().contiguous()
    W = torch.cat(ws).cuda().contiguous()
    return X, T, W, xs, meta


def evaluate(params_t, xs, meta):
    """Spearman rank correlation with the true closeness, learned scores vs
    out-degree, per family (mean over the graphs of the family)."""
    out = {}
    for x, mt in zip(xs, meta):
        y = bc.mlp_forward(params_t, x).cpu().numpy().astype(np.float64)
        r, f = mt["r"], mt["f"]
        c = np.where(r > 1, (r - 1) ** 2 / np.maximum(f, 1), 0.0)
        ok = r > 1
        if ok.sum() < 3:
            continue
        d = out.setdefault(mt["family"], dict(learned=[], degree=[]))
        d["learned"].append(spearman(y[ok], c[ok]))
        d["degree"].append(spearman(mt["deg"][ok].astype(np.float64), c[ok]))
    return {k: {kk: round(float(np.mean(vv)), 4) for kk, vv in v.items()} for k, v in out.items()}


def train(X, T, W, steps: int, batch: int, lr: float, seed: int, log=print):
    import torch
    params = torch.from_numpy(init_params(seed)).cuda()
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    rows = X.shape[0]
    for step in range(1, steps + 1):
        idx = torch.randint(0, rows, (batch,), device="cuda", dtype=torch.int32, generator=gen)
        grad, loss = bc.mlp_loss_grad(params, X, T, W, idx)
        lr_t = lr * (0.05 + 0.95 * 0.5 * (1 + np.cos(np.pi * step / steps)))
        bc.mlp_adam(params, grad, m, v, step, lr_t)
        if step % max(1, steps // 10) == 0 or step == 1:
            log(f"[train] step {step}/{steps} loss {loss:.4f} lr {lr_t:.2e}")
    return params


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--graphs", type=int, default=40, help="training graphs per family")
    ap.add_argument("--holdout", type=int, default=6, help="held-out graphs per family")
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--batch", type=int, default=32768)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--seed", type=int, default=100)
    ap.add_argument("--out", default=bc.MLP_PATH)
    args = ap.parse_args()

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    t0 = time.time()
    train_set = graph_set(args.graphs, args.seed)
    hold_set = graph_set(args.holdout, args.seed + 800)
    log(f"[train] generated {len(train_set)} + {len(hold_set)} graphs in {time.time() - t0:.1f}s")
    t0 = time.time()
    X, T, W, xs, meta = prepare(train_set, log)
    _, _, _, hxs, hmeta = prepare(hold_set, log)
    log(f"[train] features and exact labels of {X.shape[0]} nodes in {time.time() - t0:.1f}s")
    t0 = time.time()
    params = train(X, T, W, args.steps, args.batch, args.lr, args.seed, log)
    log(f"[train] {args.steps} Adam steps in {time.time() - t0:.1f}s")
    p = params.cpu().numpy().astype(np.float32)
    np.save(args.out, p, allow_pickle=False)
    summary = dict(samples=int(X.shape[0]), graphs=len(train_set), steps=args.steps,
                   holdout_spearman=evaluate(params, hxs, hmeta), out=os.path.basename(args.out))
    print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    main()
