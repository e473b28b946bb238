"""Host-side logic of bench.py (no GPU): the one-GPU guard, the measured
traffic lookup keyed by the kernel sources, and the algorithmic byte
counts the roofline divides by."""
import os
import json
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_before_touching_a_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_measured_traffic_only_for_the_profiled_kernels():
    # no summary for an unknown workload, none for another kernel name
    assert bench.measured_traffic("no_such_workload", "density_relaxation") is None
    assert bench.measured_traffic("dambreak2d_51k", "no_such_kernel") is None
    # a committed summary counts only while it carries the hash of the
    # committed kernel sources
    h = bench.kernel_source_hash()
    for w in ("dambreak2d_51k", "dambreak3d_2M", "ensemble64", "sloshing2d_51k"):
        path = os.path.join(ROOT, "profiles", f"{w}_hot_kernels.md")
        if not os.path.exists(path):
            continue
        text = open(path).read()
        blob = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
        t = bench.measured_traffic(w, blob["kernel"])
        if blob["source_hash"] == h:
            assert t is not None and t > 0
        else:
            assert t is None


def test_algorithmic_bytes_are_the_state_of_the_method():
    # state only: 2D FP32 36 and 68 bytes per particle, 3D FP32 48 and 96
    assert bench.algorithmic_bytes(2, 1, 1) == (36, 68)
    assert bench.algorithmic_bytes(3, 1, 1) == (48, 96)
    a1, b1 = bench.algorithmic_bytes(2, 1, 1000)
    a2, b2 = bench.algorithmic_bytes(2, 1, 2000)
    assert a2 == 2 * a1 and b2 == 2 * b1
    # FP64 fields move more bytes than FP32 (positions are FP64 in both)
    assert bench.algorithmic_bytes(2, 0, 1) == (72, 104)
    # the stored configuration is counted apart: 4 bytes per directed pair plus per-particle counts
    assert bench.configuration_bytes(10, 5, 2) == 4 * 15 + 8 * 2


def test_roofline_takes_the_larger_bound():
    # 1 GB in 1 ms with no flops: HBM-bound at 1000 GB/s of 8000
    r = bench.roofline(1e9, 0.0, 1.0, 1)
    assert r["bound"] == "hbm" and abs(r["frac"] - 0.125) < 1e-12 and abs(r["achieved"] - 1000.0) < 1e-9
    # 157.3 GF in 2 ms with few bytes: ALU-bound at half the FP32 peak
    r = bench.roofline(1.0, 157.3e9, 2.0, 1)
    assert r["bound"] == "alu" and abs(r["frac"] - 0.5) < 1e-12 and r["unit"] == "TFLOP/s"
    assert abs(r["hbm_frac"] - 1.0 / 8e12 / 2e-3) < 1e-15
