"""The full-size high-diameter workload: a random geometric graph with
n = 4,000,000 nodes, average degree 6, seed 5 (unit square, no wrap), k = 10.
The oracle's complete answer would take days on the host, so the check is
by sampling what it can compute one node at a time: each returned node's
exact reach and farness by one breadth-first search, the keys in decreasing
order, and a seeded sample of other nodes, each of which must rank below the
returned k-th node.  The query runs through the serving queue (W = 256, the
locality order) so that its progress, read from the counter the kernel
raises, is printed while it runs."""

import time

import numpy as np
import pytest

import oracle
import paper_1507_01490_amd as bc
from paper_1507_01490_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(1500)
def test_rgg_4m_sampled(capsys):
    def say(msg):
        # past pytest's capture: the run takes minutes and must not look silent
        with capsys.disabled():
            print(msg, flush=True)

    t0 = time.time()
    g = workloads.build("rgg")
    say(f"[rgg4m] built n={g.n} m={g.m} in {time.time() - t0:.0f} s")
    with bc.Server(lanes=1, budget_bytes=240 << 30, queue=True, queue_width=256) as S:
        gid = S.add_graph(g.row_ptr, g.col)
        t = S.submit(gid, 10, mode="batched", order="locality")
        t1 = time.time()
        while not S.wait(t, 20000):
            done, total = S.progress(t)
            say(f"[rgg4m] {done}/{total} batches after {time.time() - t1:.0f} s")
            assert time.time() - t1 < 1200, "query did not finish in 20 minutes"
        res = S.poll(t)
    say(f"[rgg4m] query {time.time() - t1:.1f} s, m_vis {res.stats['m_vis']}")
    assert len(res.ids) == 10

    def exact(v):
        d = oracle.bfs(g, int(v)).astype(np.int64)
        reached = d >= 0
        return int(reached.sum()), int(d[reached].sum())

    for v, f, r in zip(res.ids, res.farness, res.reach):
        assert exact(v) == (int(r), int(f)), v
    keys = [oracle.closeness_key(r, f) for r, f in zip(res.reach, res.farness)]
    for i in range(9):
        assert keys[i] > keys[i + 1] or (keys[i] == keys[i + 1] and res.ids[i] < res.ids[i + 1])
    kth_key, kth_id = keys[-1], int(res.ids[-1])
    rng = np.random.default_rng(13)
    top = set(res.ids.tolist())
    sample = [int(v) for v in rng.choice(g.n, 40, replace=False) if int(v) not in top][:32]
    for v in sample:
        r, f = exact(v)
        kv = oracle.closeness_key(r, f)
        assert kv < kth_key or (kv == kth_key and v > kth_id), v
    say(f"[rgg4m] checked {len(res.ids)} returned and {len(sample)} sampled nodes")
