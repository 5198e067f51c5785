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
  rgg18   the same random geometric family at n = 2^18 (the size the oracle
          and the GPU finish in minutes; n = 4M needs ~2e13 visited arcs)
  rgg20   the same random geometric family at n = 2^20 (the largest size the
          multi-threaded oracle finishes in about an hour)
  collab500k  the collaboration family at a quarter of the full size: 500,000
          actors, 125,000 groups, same size law, seed 4 (the oracle finishes it;
          the full 2M-actor graph needs ~2e13 visited arcs)
  serve512  serving mix: 512 graphs, n log-uniform in [1e3, 2e5], one third
          each Erdos-Renyi (average degree 8), Barabasi-Albert (m = 4) and
          2-D grid with 1 % random shortcuts; one request per graph with k
          uniform in {1, 10, 100}; seed 3
"""

from __future__ import annotations

from . import synth

DESCRIPTION = {
    "rgg18": "undirected random geometric graph n=262144 avg_deg=6 seed=5",
    "ba2k": "undirected Barabasi-Albert n=2000 m=5 seed=0",
    "ba1m": "undirected Barabasi-Albert n=1000000 m=5 seed=1",
    "rmat21": "directed R-MAT scale=21 edge_factor=16 (0.57,0.19,0.19,0.05) dedup seed=2",
    "collab": "undirected collaboration projection actors=2000000 groups=500000 zipf=2.1 cap=200 seed=4",
    "rgg": "undirected random geometric graph n=4000000 avg_deg=6 seed=5",
    "rgg20": "undirected random geometric graph n=1048576 avg_deg=6 seed=5",
    "collab500k": "undirected collaboration projection actors=500000 groups=125000 zipf=2.1 cap=200 seed=4",
}

KS = {"ba2k": (1, 10), "ba1m": (1, 10, 100), "rmat21": (10,), "collab": (10,), "rgg": (10,), "rgg18": (10,),
      "rgg20": (10,), "collab500k": (10,)}
DESCRIPTION["serve512"] = ("serving mix: 512 graphs n~logU[1e3,2e5] (ER deg 8 / BA m=4 / grid+1% shortcuts), "
                           "k~U{1,10,100}, seed=3")


def cpu_sample(name: str):
    """(graph, description) of the bounded sample the CPU oracle is timed on
    when the full workload takes it much longer than ~30 s: the same
    generator at a smaller size.  None when the full workload is the sample."""
    # sized for roughly 10-20 s of the 16-thread oracle
    if name == "rmat21":
        return (synth.rmat(20, 16, 0.57, 0.19, 0.19, 2),
                "directed R-MAT scale=20 edge_factor=16 (0.57,0.19,0.19,0.05) dedup seed=2, same generator")
    if name == "collab":
        return (synth.collaboration(250_000, 62_500, 2.1, 200, 4),
                "collaboration projection actors=250000 groups=62500 zipf=2.1 cap=200 seed=4, same generator")
    return None


def _serve_one(args):
    i, fam, n, seed = args
    if fam == 0:
        return synth.erdos_renyi(n, 8.0, seed)
    if fam == 1:
        return synth.barabasi_albert(n, 4, seed)
    return synth.grid_shortcuts(n, 0.01, seed)


def serve_mix(count: int = 512, seed: int = 3, workers: int = 16, max_n: float = 2e5):
    """[(graph, k)] of the serving workload, generated in a process pool
    (count graphs, n log-uniform in [1e3, max_n])."""
    import concurrent.futures as cf
    import os

    import numpy as np
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.exp(rng.uniform(np.log(1e3), np.log(max_n), count)).astype(np.int64)
    ks = rng.choice([1, 10, 100], count)
    jobs = [(i, i % 3, int(sizes[i]), seed * 100000 + i) for i in range(count)]
    nw = max(1, min(workers, os.cpu_count() or 1))
    with cf.ProcessPoolExecutor(max_workers=nw) as ex:
        graphs = list(ex.map(_serve_one, jobs, chunksize=8))
    return [(g, int(k)) for g, k in zip(graphs, ks)]


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
    if name == "rgg18":
        return synth.random_geometric(1 << 18, 6.0, 5)
    if name == "rgg20":
        return synth.random_geometric(1 << 20, 6.0, 5)
    if name == "collab500k":
        return synth.collaboration(500_000, 125_000, 2.1, 200, 4)
    raise KeyError(name)
