"""CPU replay of the index arithmetic of the bottom-up step's neighbour scan
(the level-synchronous pull kernel), before it runs on a GPU.

The kernel gives each thread one node w = base + tid of a grid-stride loop
over workgroups of 256 threads (waves of 64 lanes).  A node with unseen live
bits and at most kPullWave in-arcs walks its list alone, stopping once every
unseen bit is found; a node with more is scanned by its whole wave, lane l
reading arc eb + l of each 64-arc round while eb + l < the row end.  The
replay below executes exactly those loops, lane by lane, and asserts that
every row-pointer, column and record index stays in bounds, and that the
bits found equal the plain definition: the OR over all in-neighbours u of
cur[u] & unseen[w]."""

import numpy as np
import pytest

from paper_1507_01490_amd import synth

BLK = 256        # threads per workgroup of the level kernels
LANES = 64       # lanes per wave
PULL_WAVE = 32   # in-arcs above which a node's list is scanned by its wave


def transpose(g):
    """In-arc CSR (irp, icol) of g: for undirected graphs the CSR itself."""
    if not g.directed:
        return g.row_ptr.astype(np.int64), g.col.astype(np.int64)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    order = np.argsort(g.col, kind="stable")
    irp = np.zeros(g.n + 1, np.int64)
    np.add.at(irp, g.col + 1, 1)
    return np.cumsum(irp), src[order].astype(np.int64)


def replay(n, irp, icol, seen, cur, act, grid):
    """The kernel's loops for one pull level; returns (acc per node, arcs read)."""
    ww = seen.shape[1]
    m = len(icol)
    acc_out = np.zeros((n, ww), np.uint64)
    scanned = 0
    stride = grid * BLK
    assert len(irp) == n + 1
    for blk in range(grid):
        base = blk * BLK
        while base < n:
            for wave in range(BLK // LANES):
                lanes = range(wave * LANES, (wave + 1) * LANES)
                unv = np.zeros((LANES, ww), np.uint64)
                acc = np.zeros((LANES, ww), np.uint64)
                e0 = [0] * LANES
                e1 = [0] * LANES
                anyb = [False] * LANES
                for li, tid in enumerate(lanes):
                    w = base + tid
                    if w < n:
                        unv[li] = act & ~seen[w]
                        anyb[li] = bool(np.any(unv[li]))
                        if anyb[li]:
                            assert 0 <= w and w + 1 <= n
                            e0[li], e1[li] = int(irp[w]), int(irp[w + 1])
                heavy = [anyb[li] and e1[li] - e0[li] > PULL_WAVE for li in range(LANES)]
                for li in range(LANES):            # light nodes: one thread each
                    if anyb[li] and not heavy[li]:
                        for e in range(e0[li], e1[li]):
                            assert 0 <= e < m
                            u = int(icol[e])
                            assert 0 <= u < n
                            scanned += 1
                            acc[li] |= cur[u] & unv[li]
                            if np.array_equal(acc[li], unv[li]):
                                break
                for l in [li for li in range(LANES) if heavy[li]]:   # heavy: the wave
                    h0, h1 = e0[l], e1[l]
                    hu = unv[l].copy()
                    ha = np.zeros(ww, np.uint64)
                    eb = h0
                    while eb < h1:
                        part = np.zeros(ww, np.uint64)
                        for lane in range(LANES):
                            e = eb + lane
                            if e < h1:
                                assert h0 <= e < h1 <= m
                                u = int(icol[e])
                                assert 0 <= u < n
                                part |= cur[u] & hu
                        scanned += min(LANES, h1 - eb)
                        ha |= part
                        if np.array_equal(ha, hu):
                            break
                        eb += LANES
                    acc[l] = ha
                for li, tid in enumerate(lanes):
                    w = base + tid
                    if w < n and anyb[li]:
                        acc_out[w] = acc[li]
            base += stride
    return acc_out, scanned


def definition(n, irp, icol, seen, cur, act):
    out = np.zeros_like(seen)
    for w in range(n):
        unv = act & ~seen[w]
        for e in range(int(irp[w]), int(irp[w + 1])):
            out[w] |= cur[int(icol[e])] & unv
    return out


GRAPHS = [lambda: synth.path(9), lambda: synth.star(12), lambda: synth.empty(5), lambda: synth.star(200),
          lambda: synth.complete(70), lambda: synth.barabasi_albert(1500, 4, 3),
          lambda: synth.rmat(10, 8, 0.57, 0.19, 0.19, 4),
          lambda: synth.disjoint_union(synth.star(100), synth.path(40), synth.empty(3))]


@pytest.mark.parametrize("gi", range(len(GRAPHS)))
@pytest.mark.parametrize("ww", [1, 4])
def test_pull_scan_indices_and_result(gi, ww):
    g = GRAPHS[gi]()
    irp, icol = transpose(g)
    rng = np.random.default_rng(100 * gi + ww)
    words = rng.integers(0, 2**63, size=(g.n, ww), dtype=np.uint64)
    seen = words & rng.integers(0, 2**63, size=(g.n, ww), dtype=np.uint64)   # about a quarter of bits seen
    cur = rng.integers(0, 2**63, size=(g.n, ww), dtype=np.uint64) & ~seen
    cur &= rng.integers(0, 2**63, size=(g.n, ww), dtype=np.uint64)
    act = rng.integers(0, 2**63, size=ww, dtype=np.uint64) | np.uint64(1)
    for grid in (1, 3):
        acc, scanned = replay(g.n, irp, icol, seen, cur, act, grid)
        assert np.array_equal(acc, definition(g.n, irp, icol, seen, cur, act))
        assert scanned <= len(icol)
