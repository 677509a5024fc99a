"""Host-side checks of bench.py: the one-GPU guard, the effective peak of a
mixed FP64/FP32 operation count, and that the recorded per-bin counter
figures belong to the kernel sources in the tree (else the roofline fields
would be reported as null)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr


def test_mixed_peak_is_the_time_floor_of_the_operation_mix():
    import bench
    # all FP64 -> the FP64 peak; all FP32 -> the FP32 peak; a mix lies between
    assert bench._peak_tflops("fp64") == pytest.approx(bench.PEAK_VALU_TFLOPS, rel=1e-3)
    f = bench.FLOP_PER_BIN["mixed"]
    f32 = bench.FLOP32_PER_BIN["mixed"]
    expect = f / ((f - f32) / bench.PEAK_VALU_TFLOPS + f32 / bench.PEAK_F32_TFLOPS)
    assert bench._peak_tflops("mixed") == pytest.approx(expect)
    assert bench.PEAK_VALU_TFLOPS < bench._peak_tflops("mixed") < bench.PEAK_F32_TFLOPS


def test_counter_figures_match_the_kernel_sources():
    import bench
    assert bench._kernel_sha() == bench.COUNTERS_SRC_SHA
