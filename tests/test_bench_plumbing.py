"""Host-side plumbing of bench.py's roofline object (no GPU): the per-unit
algorithmic bytes, and the measured-traffic figure that is reported only
while the committed profile was taken on the current device code."""

import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_algorithmic_bytes_per_unit():
    # W = 64: 16 B per arc, 20 B per frontier entry, 48 B per discovered entry
    assert bench.algorithmic_bytes(1, 0, 0, 64) == 16
    assert bench.algorithmic_bytes(0, 1, 0, 64) == 20
    assert bench.algorithmic_bytes(0, 0, 1, 64) == 48
    # W = 256 (no trial cut: no per-arc degree): masks of 32 B
    assert bench.algorithmic_bytes(1, 1, 1, 256, trial=False) == (4 + 32) + (12 + 32) + (8 + 5 * 32)
    assert bench.algorithmic_bytes(1, 0, 0, 64, trial=False) == 12
    assert bench.algorithmic_bytes(10, 20, 30, 64) == 10 * 16 + 20 * 20 + 30 * 48


def test_traffic_follows_the_device_code_hash():
    path = os.path.join(ROOT, "profiles", "k_batched_lds_ba1m.md")
    info = json.loads(re.search(r"```json\n(.*?)\n```", open(path).read(), re.S).group(1))
    h = bench.device_source_hash()
    assert len(h) == 16
    got = bench.measured_traffic("k_batched_lds<1>", "ba1m")
    if info["device_source_sha256_16"] == h:
        assert got == info["traffic_bytes_per_launch"] and got > 0
    else:
        assert got is None
    assert bench.measured_traffic("k_batched_lds<1>", "no_such_workload") is None
