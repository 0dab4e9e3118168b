"""The benchmark's contract on the CPU: one GPU only, the roofline constants, and the HBM traffic
figure tied to the level-kernel sources it was measured on."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_roofline_constants():
    # 157.3 TFLOP/s of FP32 vector FMA counted as two flops: 256 CUs x 128 lanes x 2.4 GHz
    assert abs(bench.VALU_PEAK_OPS - 78.6432e12) < 1e3
    assert bench.OPS_PER_CELL_UPDATE == 121.0
    assert bench.COARSE_SHARE == 1.0 / 16.0


def test_traffic_counters_match_the_level_kernel_sources():
    """`roofline.traffic` is reported only while the level-kernel sources hash to the value its
    counters were taken on.  A failure here means those sources changed: re-take the counters
    (the profile named in TRAFFIC), or, for an edit that leaves the generated code unchanged,
    show that and update the hash."""
    assert bench.TRAFFIC["sha256"] == bench.kernel_source_sha256()
    assert os.path.exists(os.path.join(ROOT, bench.TRAFFIC["profile"]))
