"""The growing collaboration graph (a series of snapshots, the shape of the
paper's actor-graph case study on synthetic data): each snapshot contains the
previous one, the node set is fixed, and the last snapshot is the full
collaboration graph of the same seed."""

import numpy as np

import oracle
from paper_1507_01490_amd import synth


def edges(g):
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    return set(zip(src.tolist(), g.col.tolist()))


def test_snapshots_grow_and_end_at_the_full_graph():
    snaps = synth.collaboration_snapshots(3000, 800, 2.1, 200, 4, 5)
    full = synth.collaboration(3000, 800, 2.1, 200, 4)
    assert len(snaps) == 5 and all(s.n == 3000 for s in snaps)
    assert snaps[-1].sha256() == full.sha256()
    prev = set()
    for s in snaps:
        e = edges(s)
        assert prev <= e and len(e) == s.m
        prev = e
    assert snaps[0].m < snaps[-1].m


def test_oracle_answer_per_snapshot_matches_definition():
    """Each snapshot's top-k from the oracle equals the definition (brute
    force), so the GPU series test can compare against the oracle."""
    for s in synth.collaboration_snapshots(600, 200, 2.1, 40, 9, 3):
        r, f = oracle.bruteforce(s)
        ids, ff, rr = oracle.topk_by_definition(r, f, 10)
        got = oracle.topk(s, 10)
        assert got["ids"].tolist() == ids.tolist() and got["f"].tolist() == ff.tolist()
