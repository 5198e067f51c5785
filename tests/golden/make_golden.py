"""Write the stored expected results of the full-size workloads.

Every value here comes from the CPU oracle (``oracle/``) run on graphs from
the seeded generators; nothing is taken from the GPU path.  For each
workload the file records the SHA-256 of the canonical CSR (so a test can
check it rebuilt the same graph), the oracle's top-k (ids, farness, reach)
and the visited-arc count m_vis of the sequential run in decreasing-degree
order (Algorithm 1 with one thread), which the benchmark uses as the fixed
work numerator of its throughput.

Workloads too large for a single-threaded run (``PARALLEL_ONLY``) are run
with the oracle's parallel loop only (Section 2.1: threads share the k-th
best value; the answer is the same as the sequential one).  Their files
record ``m_vis_par`` (the arcs of that run, which depends on the thread
timing) instead of ``m_vis_seq``.

Usage: python tests/golden/make_golden.py [--threads T] [ba1m] [rmat21] [collab500k] [rgg20] ...
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

PARALLEL_ONLY = {"collab500k", "rgg20"}


def run(name: str, ks, threads: int):
    g = workloads.build(name)
    out = dict(workload=name, description=workloads.DESCRIPTION[name], n=g.n, m=g.m,
               directed=bool(g.directed), sha256=g.sha256(), results={})
    for k in ks:
        if name in PARALLEL_ONLY:
            t0 = time.time()
            par = oracle.topk(g, k, nthreads=threads)
            t1 = time.time()
            out["results"][str(k)] = dict(ids=par["ids"].tolist(), farness=[int(x) for x in par["f"]],
                                          reach=[int(x) for x in par["r"]], m_vis_par=int(par["stats"]["m_vis"]),
                                          n_done_par=int(par["stats"]["n_done"]), threads=threads,
                                          oracle_par_s=round(t1 - t0, 2))
            print(name, k, f"{t1 - t0:.1f}s with {threads} threads", par["stats"], flush=True)
            continue
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
    args = sys.argv[1:]
    threads = 8
    if "--threads" in args:
        i = args.index("--threads")
        threads = int(args[i + 1])
        del args[i:i + 2]
    for t in args or ["ba1m"]:
        run(t, workloads.KS[t], threads=threads)
