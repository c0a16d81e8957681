"""Host-side pieces of bench.py: variant codes, the HBM view, and the one-GPU
guard (no GPU is touched)."""
import subprocess
import sys
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_variant_codes():
    assert bench.variant_name(16) == "vec16"
    assert bench.variant_name(128 | 64) == "mfma64"
    assert bench.variant_name(128 | 1) == "mfma-packed"
    assert bench.variant_name(256 | 128 | 16) == "mfma16/persistent"
    assert bench.variant_launches(64, 128 | 16) == 4
    assert bench.variant_launches(64, 128 | 64) == 1
    assert bench.variant_launches(3, 128 | 1) == 1
    assert bench.variant_launches(20, 8) == 3


def test_hbm_view():
    v = bench.hbm_view(8e9, 1000.0)  # 8 GB in one second
    assert abs(v["achieved_GBps"] - 8.0) < 1e-9
    assert abs(v["frac"] - 1e-3) < 1e-12


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)


def test_hbm_roofline():
    r = bench.roofline_hbm("k_accumulate_mfma", 16e9, 4.0, 8)  # 16 GB in 4 ms over 8 launches
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert abs(r["achieved"] - 4000.0) < 1e-9 and abs(r["frac"] - 0.5) < 1e-12
    assert abs(r["kernel_ms"] - 0.5) < 1e-12 and abs(r["bytes_per_launch"] - 2e9) < 1


def test_segment_subset():
    from paper_2604_17155_amd import synthetic as syn

    class S:
        def __init__(self, n):
            self.N = n
    scenes = [S(n) for n in (50, 10, 400, 30, 20, 70)]
    sub = bench.segment_subset(scenes)
    assert sub[0] == 1 and sub[1] == 2 and len(sub) == 4 and len(set(sub)) == 4
    assert sub == bench.segment_subset(scenes)  # fixed seed
