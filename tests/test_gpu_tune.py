"""The autotuner of the batched-mode knobs: every trial must return the
same top-k (it checks this itself), the setting it picks is never slower
than the base setting it measured, and that setting still gives the
oracle's answer."""

import pytest

import oracle
import paper_1507_01490_amd as bc
from paper_1507_01490_amd import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("which", ["ba", "rmat", "grid"])
def test_autotune_keeps_the_answer(which):
    g = {"ba": lambda: synth.barabasi_albert(20000, 4, 61),
         "rmat": lambda: synth.rmat(13, 16, 0.57, 0.19, 0.19, 62),
         "grid": lambda: synth.grid_shortcuts(8000, 0.01, 63)}[which]()
    ref = oracle.topk(g, 10, nthreads=8)
    with bc.Graph(g.row_ptr, g.col, directed=g.directed) as G:
        tuned, rep = G.autotune(10)
        assert rep["trials"] >= 12
        assert rep["best_ms"] <= rep["default_ms"]
        res = G.topk(10, **tuned)
    assert res.ids.tolist() == ref["ids"].tolist()
    assert res.farness.tolist() == ref["f"].tolist() and res.reach.tolist() == ref["r"].tolist()
