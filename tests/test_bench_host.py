"""Host-side logic of bench.py (no GPU): the one-GPU guard, the measured
traffic lookup keyed by the kernel sources, and the algorithmic byte
counts the roofline divides by."""
import os
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
    # the committed summaries carry the hash of the committed kernel sources
    for w in ("dambreak2d_51k", "dambreak3d_2M", "ensemble64", "sloshing2d_51k"):
        t = bench.measured_traffic(w, "density_relaxation")
        assert t is not None and t > 0


def test_algorithmic_bytes_scale_with_particles_and_pairs():
    a1, b1 = bench.algorithmic_bytes(2, 1, 1000, 10000, 500)
    a2, b2 = bench.algorithmic_bytes(2, 1, 2000, 20000, 1000)
    assert a2 == 2 * a1 and b2 == 2 * b1
    # 4 bytes per directed pair (one list entry), the rest per particle
    a3, b3 = bench.algorithmic_bytes(2, 1, 1000, 10001, 500)
    assert a3 - a1 == 4 and b3 - b1 == 4
    # FP64 fields move more bytes than FP32, 3D more than 2D
    assert bench.algorithmic_bytes(2, 0, 1000, 0, 0)[0] > bench.algorithmic_bytes(2, 1, 1000, 0, 0)[0]
    assert bench.algorithmic_bytes(3, 1, 1000, 0, 0)[1] > bench.algorithmic_bytes(2, 1, 1000, 0, 0)[1]
