"""Full-size workloads against the oracle's stored answers.

tests/golden/<workload>.json holds the exact top-k of the CPU oracle
(written by tests/golden/make_golden.py, which calls only oracle/), with the
SHA-256 of the generated graph.  The GPU path must return the same ids,
farness and reach for every k, in each batched configuration the bench
uses and with the learned order."""

import json
import os

import pytest

import paper_1507_01490_amd as bc
from paper_1507_01490_amd import workloads

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
NAMES = [n for n in ("ba1m", "rmat21") if os.path.exists(os.path.join(HERE, "golden", f"{n}.json"))]


@pytest.mark.parametrize("name", NAMES)
def test_full_size_against_oracle(name):
    gold = json.load(open(os.path.join(HERE, "golden", f"{name}.json")))
    g = workloads.build(name)
    assert g.sha256() == gold["sha256"], "generator output changed"
    with bc.Graph(g.row_ptr, g.col, directed=g.directed) as G:
        for k, ref in gold["results"].items():
            k = int(k)
            for kw in (dict(mode="batched"), dict(mode="batched", width=256),
                       dict(mode="batched", order="learned_grouped")):
                res = G.topk(k, **kw)
                assert res.ids.tolist() == ref["ids"], (name, k, kw)
                assert [int(x) for x in res.farness] == ref["farness"], (name, k, kw)
                assert [int(x) for x in res.reach] == ref["reach"], (name, k, kw)
