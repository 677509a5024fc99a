"""Host-side checks of the C-ABI library (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fstat.h")).read()
    return sorted(set(re.findall(r"^(?:int|void|const char \*)\s*([a-z_]+)\(", src, re.M)))


def test_header_declares_the_boundary():
    assert _declared() == sorted(["fstat_plan_create", "fstat_plan_set_orbit", "fstat_eval",
                                  "fstat_eval_noalloc",
                                  "fstat_extrinsic", "fstat_waveform",
                                  "fstat_search", "fstat_search_boxes",
                                  "pso_stage", "fstat_profile_read", "fstat_interp_stats",
                                  "fstat_autotune",
                                  "fstat_mlp_grad", "fstat_mlp_forward",
                                  "fstat_surrogate_train", "fstat_surrogate_stats",
                                  "fstat_surrogate_params",
                                  "fstat_calibrate", "fstat_plan_destroy",
                                  "fstat_last_error"])


def test_library_loads_and_exports_every_declared_symbol():
    from paper_2407_10797_amd import fstat
    if not os.path.exists(fstat.LIB_PATH):
        pytest.skip("libfstat.so not built")
    lib = ctypes.CDLL(fstat.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(fstat.EXPORTS) == set(_declared())


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2407_10797_amd import fstat
    monkeypatch.setattr(fstat, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(fstat, "_lib", None)
    with pytest.raises(ImportError):
        fstat.lib()


def test_struct_layouts_match_header():
    from paper_2407_10797_amd import fstat
    assert ctypes.sizeof(fstat.fstat_data_desc) == 64
    assert ctypes.sizeof(fstat.fstat_opts) == 24
    assert ctypes.sizeof(fstat.pso_stage_desc) == 88
    assert ctypes.sizeof(fstat.pso_result) == 32
    assert ctypes.sizeof(fstat.fstat_surrogate_desc) == 56


def test_last_error_is_empty_string_initially():
    from paper_2407_10797_amd import fstat
    if not os.path.exists(fstat.LIB_PATH):
        pytest.skip("libfstat.so not built")
    assert isinstance(fstat.fstat_last_error(), str)
