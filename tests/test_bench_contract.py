"""Host logic of bench.py (no GPU): the one-GPU refusal and the gating of
the committed HBM-traffic figure to the kernel source, image shape and
image-pass variant it was counted on."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_only_for_the_counted_kernel_shape_and_variant():
    with open(os.path.join(ROOT, "profiles", "image_pass_256_traffic.json")) as f:
        t = json.load(f)
    h = bench._src_hash()
    shape = tuple(t["image_shape"])
    if t["kernel_src_sha256_16"] == h:
        assert bench._traffic(h, shape, t["variant"]) == t["hbm_bytes_per_launch"]
    else:  # counters taken on another kernel source: no traffic is reported
        assert bench._traffic(h, shape, t["variant"]) is None
    assert bench._traffic(h, (512, 512, 1536), t["variant"]) is None
    assert bench._traffic(h, shape, "march32fit") is None
    assert bench._traffic("0" * 16, shape, t["variant"]) is None
