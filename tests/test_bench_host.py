"""Host logic of bench.py (no GPU): the one-GPU refusal, the algorithmic
byte counts behind roofline.achieved, and when counter traffic is reported."""
import argparse
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 2" in r.stderr
    assert r.stdout == ""


def test_product_bytes_per_launch():
    # benchmark workload: 10^6 spheres, 1.526e8 ordered pairs, 16-bit
    # halo-local indices; per particle 16 (position) + 12 (source) + 4
    # (count) + 12 (result) + 12 (Lanczos basis) bytes
    n, pairs = 1_000_000, 152_650_438
    assert bench.stage_bytes("spmv", n, 256, pairs, lanczos=True, index_bytes=2) == 56 * n + 2 * pairs
    assert bench.stage_bytes("spmv", n, 256, pairs, lanczos=False, index_bytes=2) == 44 * n + 2 * pairs
    assert abs(bench.stage_bytes("spmv", n, 256, pairs, lanczos=True, index_bytes=2) / 1e6 - 361.3) < 0.1


def test_grid_stage_bytes():
    # one 3-component FP32 grid of 256^3 nodes is 201.3 MB
    g = 3 * 256**3 * 4
    assert bench.stage_bytes("fft", 10, 256, 0, False) == 2 * g
    assert bench.stage_bytes("spread", 10, 256, 0, False) == 280 + g
    assert bench.stage_bytes("interp", 10, 256, 0, False) == g + 280
    assert bench.stage_bytes("nbr", 10, 256, 7, False) == 200 + 28
    assert bench.stage_bytes("lanczos", 10, 256, 7, False) is None


def test_traffic_only_on_the_profiled_workload():
    a = argparse.Namespace(**bench.TRAFFIC_WORKLOAD)
    t = bench.measured_traffic("spmv", a)
    assert t is None or t > bench.stage_bytes("spmv", a.n, a.grid, 0, lanczos=True)
    for k, v in [("n", 4_000_000), ("phi", 0.4), ("grid", 512), ("rc", 10.0)]:
        b = argparse.Namespace(**{**bench.TRAFFIC_WORKLOAD, k: v})
        assert bench.measured_traffic("spmv", b) is None
    assert bench.measured_traffic("fft", a) is None
