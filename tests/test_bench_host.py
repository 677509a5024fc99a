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
    FLOPs with the phase and sine at every bin, 38 + 2 D with the difference
    recurrence and binomial moments, at transfer degree D; per lane run the
    coefficients (12 + 16 D), and with the recurrence its set-up (223) and the
    moments' change to power form (4 D^2 + 3 D + 2); the mixed loop's phase
    differences (10 or 5 FP64) and moments (8 + 2 D FP32) per bin, its set-up
    (224 FP64, or 194 where it forms four differences), coefficients and
    change to power form (4 D^2 + 3 D FP32) per run.  The launch total is the
    bin- and run-weighted sum of its kinds (exact-loop bins are not the main
    kernel's work)."""
    import bench
    for d in (5, 7, 9):
        assert bench.ALG_FP64[f"deg{d}"] == 63 + 4 * (d - 1)
        assert bench.ALG_FP64[f"rec{d}"] == 38 + 2 * d
        assert bench.RUN_FP64[f"deg{d}"] == 12 + 16 * d
        assert bench.RUN_FP64[f"rec{d}"] == 223 + (4 * d * d + 3 * d + 2) + 12 + 16 * d
    for d in (4, 6):
        for k, setup in ((f"deg{d}", 224), (f"deg{d}_d4", 194)):
            assert bench.RUN_MIXED[k] == (setup + 12 + 16 * d, 4 * d * d + 3 * d)
            assert bench.ALG_MIXED[k] == (10.0 if k == f"deg{d}" else 5.0, 8 + 2 * d)
    mix = [10, 20, 30, 1, 2, 3, 1000, 4, 5, 6, 7, 8, 9, 11]
    f64, f32 = bench.alg_flops("fp64", mix)
    assert f32 == 0.0
    bins = 10 * 79 + 20 * 87 + 30 * 95 + 1 * 48 + 2 * 52 + 3 * 56
    assert bench.alg_flops("fp64", mix, runs=False) == (bins, 0.0)
    assert f64 == bins + 4 * 92 + 5 * 124 + 6 * 156 + 7 * 432 + 8 * 566 + 9 * 732
    mmix = [40, 0, 60, 20, 0, 30, 1000, 3, 0, 5, 2, 0, 4, 7]
    m64, m32 = bench.alg_flops("mixed", mmix)
    b64, b32 = 100 * 10 + 50 * 5, 60 * 16 + 90 * 20
    assert bench.alg_flops("mixed", mmix, runs=False) == (b64, b32)
    assert (m64, m32) == (b64 + 3 * 300 + 5 * 332 + 2 * 270 + 4 * 302,
                          b32 + 5 * 76 + 9 * 162)
    assert bench.bin_mix_dict(True, mmix) == (
        {"deg4": 40, "deg6": 60, "deg4_d4": 20, "deg6_d4": 30, "exact": 1000},
        {"deg4": 3, "deg6": 5, "deg4_d4": 2, "deg6_d4": 4, "exact": 7})
    b, r = bench.bin_mix_dict(False, mix)
    assert list(b.values()) == mix[:7] and list(r.values()) == mix[7:]


def test_counter_figures_match_the_kernel_sources():
    import bench
    assert bench._kernel_sha() == bench.COUNTERS_SRC_SHA
