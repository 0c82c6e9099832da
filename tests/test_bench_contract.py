"""The benchmark's output contract, on the CPU: the one-GPU refusal, the
peaks its roofline objects are priced against, and the roofline objects
built from the committed counters of the benchmark's own workload."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2608_04085_amd import profiling  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_published_peaks():
    # MI355X: HBM 8 TB/s; FP64 vector 256 CUs x 4 SIMDs x 16 lanes x 2 x 2.4 GHz;
    # one wave64 VALU instruction per 4 cycles per SIMD
    assert bench.HBM_PEAK_GBS == 8000.0
    assert abs(bench.FP64_PEAK_TFLOPS - 256 * 4 * 16 * 2 * 2.4e9 / 1e12) < 0.05
    assert bench.VALU_ISSUE_PEAK == 614.4e9
    assert (bench.FWD_BYTES_PER_CELL, bench.ADJ_BYTES_PER_CELL) == (64.0, 96.0)


def test_roofline_objects_from_the_committed_counters():
    # the default tiles at 8 x 512x1024; a launch time in the measured range
    cells, tiles = 8 * 512 * 1024, "16x15/16x15"
    key = "cnop_8x512x1024"
    adj = bench.roofline("adjoint", 404.0, cells, profiling.traffic_for(key, "adjoint", tiles),
                         profiling.counters_for(key, ["adj_a", "adj_b"], tiles))
    stp = bench.roofline("step", 149.0, cells, profiling.traffic_for(key, "step_march", tiles),
                         profiling.counters_for(key, ["step_march"], tiles))
    for r, flops, nbytes in ((adj, bench.ADJ_FLOPS_PER_CELL, 96), (stp, bench.FWD_FLOPS_PER_CELL, 64)):
        assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == bench.FP64_PEAK_TFLOPS
        assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-4
        assert r["algorithmic_flops_per_launch"] == flops * cells
        assert r["hbm"]["algorithmic_bytes_per_launch"] == nbytes * cells
        # HBM bytes from the counters: at least the algorithmic ones
        assert r["traffic"] is not None and r["traffic"] >= 0.99 * nbytes * cells
        v = r["valu_issue"]
        assert v is not None and 0.0 < v["frac"] < 1.0 and v["per_64_cells"] > 0
    # the adjoint pair moves several times its algorithmic bytes (Z between the kernels)
    assert adj["traffic"] > 2.5 * 96 * cells
    # counters of other tile variants are not used
    assert profiling.counters_for(key, ["adj_a"], "32x16/32x8") is None
    assert bench.roofline("step", 149.0, cells, None, None)["valu_issue"] is None
