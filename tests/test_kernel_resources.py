"""Register budget of the level kernels, read from the gfx950 compiler's
resource report (no GPU needed).  The persistent W = 64 kernel runs 1024
threads per workgroup and so has 128 VGPRs per lane; values it keeps in
scratch are re-read every level, and spilled loop state once cost more HBM
traffic than the graph itself.  These bounds keep that from coming back."""

import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def resources(tmp_path_factory):
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    from paper_1507_01490_amd import build as b
    out = tmp_path_factory.mktemp("ru") / "topk.o"
    src = os.path.join(b.CSRC, "topk.hip")
    flags = [f for f in b.FLAGS if f != "-Wall"]
    r = subprocess.run([HIPCC, *flags, "--cuda-device-only", "-c", src, "-o", str(out),
                        "-Rpass-analysis=kernel-resource-usage"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    kern = {}
    name = None
    for line in r.stderr.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            kern[name] = {}
            continue
        m = re.search(r"remark:\s+([A-Za-z ]+?)(?: \[bytes/lane\])?: (\d+)", line)
        if m and name:
            kern[name][m.group(1).strip()] = int(m.group(2))
    return kern


def _find(kern, frag):
    hits = {k: v for k, v in kern.items() if frag in k}
    assert hits, f"no kernel matching {frag}"
    return hits


def test_persistent_lds_kernel_spills_little(resources):
    (name, r), = _find(resources, "k_batched_lds").items()
    assert r["VGPRs"] <= 128
    assert r["VGPRs Spill"] <= 32, r
    assert r["ScratchSize"] <= 320, r


def test_other_level_kernels_do_not_spill(resources):
    for frag in ("k_batchedILi", "k_plain_expand", "k_plain_pull", "k_plain_count", "k_plain_build"):
        for name, r in _find(resources, frag).items():
            assert r["VGPRs Spill"] == 0 and r["ScratchSize"] == 0, (name, r)
