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
    p64, p32 = bench.PEAK_VALU_TFLOPS, bench.PEAK_F32_TFLOPS
    assert bench.floor_peak(1.0, 0.0, p64, p32) == pytest.approx(p64)
    assert bench.floor_peak(0.0, 1.0, p64, p32) == pytest.approx(p32)
    f64, f32 = bench.ALG_MIXED["deg6"]
    expect = (f64 + f32) / (f64 / p64 + f32 / p32)
    assert bench.floor_peak(f64, f32, p64, p32) == pytest.approx(expect)
    assert p64 < bench.floor_peak(f64, f32, p64, p32) < p32


def test_algorithmic_flops_follow_the_bin_mix():
    """Per-bin algorithmic counts of the interpolating loop: 63 + 4 (D - 1)
    FLOPs with the phase and sine at every bin, 46 + 4 (D - 1) (plus s^8 at
    D = 9) with the difference recurrence, at transfer degree D; the launch
    total is the bin-weighted sum of its kinds (exact-loop bins are not the
    main kernel's work)."""
    import bench
    for d in (5, 7, 9):
        assert bench.ALG_FP64[f"deg{d}"] == 63 + 4 * (d - 1)
        assert bench.ALG_FP64[f"rec{d}"] == 46 + 4 * (d - 1) + (d == 9)
    mix = [10, 20, 30, 1, 2, 3, 1000]
    f64, f32 = bench.alg_flops("fp64", mix)
    assert f32 == 0.0
    assert f64 == 10 * 79 + 20 * 87 + 30 * 95 + 1 * 62 + 2 * 70 + 3 * 79
    m64, m32 = bench.alg_flops("mixed", [40, 0, 60, 0, 0, 0, 1000])
    assert (m64, m32) == (100 * 24, 40 * 27 + 60 * 37)
    assert bench.bin_mix_dict(True, [40, 0, 60, 0, 0, 0, 1000]) == {
        "deg4": 40, "deg6": 60, "exact": 1000}
    assert list(bench.bin_mix_dict(False, mix).values()) == mix


def test_counter_figures_match_the_kernel_sources():
    import bench
    assert bench._kernel_sha() == bench.COUNTERS_SRC_SHA
