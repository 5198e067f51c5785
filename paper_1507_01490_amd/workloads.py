"""Named synthetic workloads (graph family, size, seed and the k values they
are queried with).  Inputs only: no part of the method lives here.

  ba2k    undirected Barabasi-Albert, n = 2,000, m = 5, seed 0; k = 1, 10
  ba1m    undirected Barabasi-Albert, n = 1,000,000, m = 5, seed 1; k = 1, 10, 100
  rmat21  directed R-MAT scale 21, edge factor 16, (0.57, 0.19, 0.19, 0.05),
          self-loops and repeats removed, seed 2; k = 10
  collab  undirected collaboration projection: 2,000,000 actors, 500,000
          groups, Zipf(2.1) sizes capped at 200, seed 4; k = 10
  rgg     undirected random geometric graph, n = 4,000,000, average degree 6,
          seed 5; k = 10
"""

from __future__ import annotations

from . import synth

DESCRIPTION = {
    "ba2k": "undirected Barabasi-Albert n=2000 m=5 seed=0",
    "ba1m": "undirected Barabasi-Albert n=1000000 m=5 seed=1",
    "rmat21": "directed R-MAT scale=21 edge_factor=16 (0.57,0.19,0.19,0.05) dedup seed=2",
    "collab": "undirected collaboration projection actors=2000000 groups=500000 zipf=2.1 cap=200 seed=4",
    "rgg": "undirected random geometric graph n=4000000 avg_deg=6 seed=5",
}

KS = {"ba2k": (1, 10), "ba1m": (1, 10, 100), "rmat21": (10,), "collab": (10,), "rgg": (10,)}


def build(name: str) -> synth.Csr:
    if name == "ba2k":
        return synth.barabasi_albert(2000, 5, 0)
    if name == "ba1m":
        return synth.barabasi_albert(1_000_000, 5, 1)
    if name == "rmat21":
        return synth.rmat(21, 16, 0.57, 0.19, 0.19, 2)
    if name == "collab":
        return synth.collaboration(2_000_000, 500_000, 2.1, 200, 4)
    if name == "rgg":
        return synth.random_geometric(4_000_000, 6.0, 5)
    raise KeyError(name)
