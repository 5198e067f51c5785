"""Write the stored expected results of the full-size workloads.

Every value here comes from the CPU oracle (``oracle/``) run on graphs from
the seeded generators; nothing is taken from the GPU path.  For each
workload the file records the SHA-256 of the canonical CSR (so a test can
check it rebuilt the same graph), the oracle's top-k (ids, farness, reach)
and the visited-arc count m_vis of the sequential run in decreasing-degree
order (Algorithm 1 with one thread), which the benchmark uses as the fixed
work numerator of its throughput.

Usage: python tests/golden/make_golden.py [ba1m] [rmat21] [collab] [rgg]
"""

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1507_01490_amd import workloads  # noqa: E402


def run(name: str, ks, threads: int):
    g = workloads.build(name)
    out = dict(workload=name, description=workloads.DESCRIPTION[name], n=g.n, m=g.m,
               directed=bool(g.directed), sha256=g.sha256(), results={})
    for k in ks:
        t0 = time.time()
        seq = oracle.topk(g, k, nthreads=1)
        t1 = time.time()
        out["results"][str(k)] = dict(ids=seq["ids"].tolist(), farness=[int(x) for x in seq["f"]],
                                      reach=[int(x) for x in seq["r"]], m_vis_seq=int(seq["stats"]["m_vis"]),
                                      n_done_seq=int(seq["stats"]["n_done"]), oracle_seq_s=round(t1 - t0, 2))
        if threads > 1:
            par = oracle.topk(g, k, nthreads=threads)
            assert par["ids"].tolist() == seq["ids"].tolist()
            assert par["f"].tolist() == seq["f"].tolist()
        print(name, k, f"{t1 - t0:.1f}s", seq["stats"], flush=True)
    path = os.path.join(HERE, f"{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    targets = sys.argv[1:] or ["ba1m"]
    for t in targets:
        run(t, workloads.KS[t], threads=8)
