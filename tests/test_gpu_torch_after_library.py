"""The binding hands out torch tensors (features, perceptron scores) after
the library has run: torch's own GPU start-up must work when the library was
used first, in a fresh process where nothing imported torch beforehand."""

import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import paper_1507_01490_amd as bc
from paper_1507_01490_amd import synth
g = synth.barabasi_albert(3000, 3, 5)
with bc.Server(lanes=1, budget_bytes=1 << 28) as S:
    gid = S.add_graph(g.row_ptr, g.col)
    t = S.submit(gid, 10, mode="batched")
    assert S.wait(t, 60000)
    ids = S.poll(t).ids.tolist()
with bc.Graph(g.row_ptr, g.col) as G:
    assert G.topk(10, mode="plain").ids.tolist() == ids
    x, core = G.features()
    assert x.shape == (g.n, 3) and x.is_cuda
import torch
assert float(torch.ones(4, device="cuda").sum()) == 4.0
print("ok", flush=True)
"""


def test_torch_gpu_after_library_use():
    env = dict(os.environ, PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-2000:] + r.stderr[-2000:]
