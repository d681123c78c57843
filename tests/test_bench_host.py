"""Host logic of bench.py (no GPU): the one-GPU refusal, the algorithmic
work behind each roofline entry, the work-model constants, and when counter
traffic is reported."""
import argparse
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 2" in r.stderr
    assert r.stdout == ""


def test_product_roofline_is_alu_bound_at_35_flop_per_pair():
    # benchmark workload: 10^6 spheres, 1.526e8 ordered pairs, 0.30 ms per launch
    n, pairs = 1_000_000, 152_650_438
    r = bench.stage_roofline("spmv", n, 256, pairs, 0.30)
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == 157.3
    assert r["algorithmic_flops_per_launch"] == 35 * pairs
    assert r["achieved"] == pytest.approx(35 * pairs / 0.30e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 157.3)
    # the HBM view counts positions, v and w once: 40 MB at 10^6 spheres
    assert r["hbm_view"]["algorithmic_bytes_per_launch"] == 40 * n


def test_grid_stage_rooflines():
    # one 3-component FP32 grid of 256^3 nodes is 201.3 MB
    g = 3 * 256**3 * 4
    ms = 0.1
    assert bench.stage_roofline("fft", 10, 256, 0, ms)["algorithmic_bytes_per_launch"] == 2 * g
    assert bench.stage_roofline("xfused", 10, 256, 0, ms)["algorithmic_bytes_per_launch"] == 2 * g
    assert bench.stage_roofline("spread", 10, 256, 0, ms)["algorithmic_bytes_per_launch"] == 280 + g
    assert bench.stage_roofline("interp", 10, 256, 0, ms)["algorithmic_bytes_per_launch"] == g + 280
    assert bench.stage_roofline("nbr", 10, 256, 7, ms)["algorithmic_bytes_per_launch"] == 200 + 14
    r = bench.stage_roofline("interp", 10, 256, 0, ms)
    assert r["bound"] == "hbm" and r["achieved"] == pytest.approx((g + 280) / 1e-4 / 1e9)
    assert bench.stage_roofline("lanczos", 10, 256, 7, ms) is None
    assert bench.stage_roofline("spmv", 10, 256, 7, 0.0) is None


def test_measured_constants():
    import types

    res = {"breakdown_ms": {"spmv": 1.8, "spread": 0.6, "interp": 0.4, "fft": 0.4, "xfused": 0.2, "bin": 0.2,
                            "lanczos": 0.1, "noise": 0.02, "other": 0.05},
           "launches": {"spmv": 6}, "neighbor_pairs": 1.5e8}
    p = types.SimpleNamespace(grid=256, support=8)
    c = bench.measured_constants(res, 1_000_000, p)
    # rounded to two significant digits
    assert c["c_pair"] == pytest.approx(0.3e-3 / 1.5e8, rel=0.01)
    assert c["c_node"] == pytest.approx(1.0e-3 / (2e6 * 512), rel=0.01)
    assert c["c_fft"] == pytest.approx(0.6e-3 / (256**3 * 24), rel=0.01)
    assert c["c_particle"] == pytest.approx(0.37e-3 / 1e6, rel=0.01)
    assert c["c_node"] == float(f"{c['c_node']:.2g}")


def test_traffic_only_on_the_profiled_workload():
    import types

    w = bench.TRAFFIC_WORKLOAD
    a = argparse.Namespace(**w)
    p = types.SimpleNamespace(grid=w["grid"], support=w["support"], xi=w["xi"], rcut=w["rc"])
    t = bench.measured_traffic("spmv", a, p)
    assert t is None or t > 40 * w["n"]
    for k, v in [("n", 4_000_000), ("phi", 0.4)]:
        b = argparse.Namespace(**{**w, k: v})
        assert bench.measured_traffic("spmv", b, p) is None
    q = types.SimpleNamespace(grid=w["grid"], support=w["support"], xi=0.56, rcut=4.69)
    assert bench.measured_traffic("spmv", a, q) is None
    assert bench.measured_traffic("fft", a, p) is None
