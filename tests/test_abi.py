"""The C-ABI library loads, exports every declared symbol, and validates its
arguments on the host before touching the GPU (no compute calls here)."""

import ctypes
import re

import numpy as np
import pytest

import paper_2307_12988_amd as cg
from paper_2307_12988_amd import _lib

CODES = {"CG_OK": 0, "CG_ERR_INVALID_ARG": -1, "CG_ERR_UNSUPPORTED": -2, "CG_ERR_BAD_REF": -3,
         "CG_ERR_NULL": -4, "CG_ERR_OOM": -5, "CG_ERR_HIP": -6, "CG_ERR_WORKSPACE": -7,
         "CG_ERR_STATE": -8}


@pytest.fixture(scope="module")
def lib():
    return cg.load()


def test_exports_every_declared_symbol(lib):
    names = cg.header_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
        assert n in _lib.SIGNATURES, f"binding lacks {n}"
    assert set(_lib.SIGNATURES) == set(names)


def test_status_codes_match_header(lib):
    text = open(_lib.HEADER).read()
    for name, val in CODES.items():
        m = re.search(rf"#define {name}\s+\(?(-?\d+)\)?", text)
        assert m and int(m.group(1)) == val, name
        assert lib.cg_status_string(val) not in (None, b"unknown status")
    assert lib.cg_status_string(12345) == b"unknown status"
    assert lib.cg_version().startswith(b"combgpu")


def _create(lib, n, fs, bins, ref):
    h = ctypes.c_void_p(1234)
    b = np.ascontiguousarray(bins, dtype=np.int32)
    r = np.ascontiguousarray(ref, dtype=np.float32)
    st = lib.cg_create_plan(n, fs, b.ctypes.data_as(_lib._pi32), len(b),
                            r.ctypes.data_as(_lib._pf32), ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("n,fs,bins,ref,code", [
    (1000, 1e9, [1, 2], [1, 1], CODES["CG_ERR_UNSUPPORTED"]),       # not a power of two
    (256, 1e9, [1, 2], [1, 1], CODES["CG_ERR_UNSUPPORTED"]),        # too short
    (16384, 1e9, [1, 2], [1, 1], CODES["CG_ERR_UNSUPPORTED"]),      # too long
    (1024, 1e9, [1, 1], [1, 1], CODES["CG_ERR_INVALID_ARG"]),       # duplicate bin
    (1024, 1e9, [1, 513], [1, 1], CODES["CG_ERR_INVALID_ARG"]),     # above Nyquist
    (1024, 1e9, [-1, 3], [1, 1], CODES["CG_ERR_INVALID_ARG"]),      # negative bin
    (1024, 0.0, [1, 2], [1, 1], CODES["CG_ERR_INVALID_ARG"]),       # fs <= 0
    (1024, float("inf"), [1, 2], [1, 1], CODES["CG_ERR_INVALID_ARG"]),
    (1024, 1e9, [1, 2], [1, 0], CODES["CG_ERR_BAD_REF"]),           # ref <= 0
    (1024, 1e9, [1, 2], [1, float("nan")], CODES["CG_ERR_BAD_REF"]),
    (1024, 1e9, [1, 2], [float("inf"), 1], CODES["CG_ERR_BAD_REF"]),
    (512, 1e9, list(range(0, 258)), [1] * 258, CODES["CG_ERR_UNSUPPORTED"]),  # K > N/2+1
    (8192, 1e9, list(range(441)), [1] * 441, CODES["CG_ERR_UNSUPPORTED"]),    # K > 440
])
def test_create_plan_rejects(lib, n, fs, bins, ref, code):
    st, h = _create(lib, n, fs, bins, ref)
    assert st == code
    assert h.value is None
    assert len(lib.cg_last_error_detail()) > 0


def test_null_arguments(lib):
    h = ctypes.c_void_p()
    r = np.ones(2, dtype=np.float32)
    assert lib.cg_create_plan(1024, 1e9, None, 2, r.ctypes.data_as(_lib._pf32),
                              ctypes.byref(h)) == CODES["CG_ERR_NULL"]
    b = np.array([1, 2], dtype=np.int32)
    assert lib.cg_create_plan(1024, 1e9, b.ctypes.data_as(_lib._pi32), 2, None,
                              ctypes.byref(h)) == CODES["CG_ERR_NULL"]
    assert lib.cg_create_plan(1024, 1e9, b.ctypes.data_as(_lib._pi32), 2,
                              r.ctypes.data_as(_lib._pf32), None) == CODES["CG_ERR_NULL"]
    assert lib.cg_create_plan(1024, 1e9, b.ctypes.data_as(_lib._pi32), 0,
                              r.ctypes.data_as(_lib._pf32), ctypes.byref(h)) == \
        CODES["CG_ERR_INVALID_ARG"]
    assert lib.cg_destroy_plan(None) == 0
    assert lib.cg_process_batch(None, None, 0, None, None) == CODES["CG_ERR_NULL"]
    assert lib.cg_process_batch_ex(None, None, 0, None, None, None, None, None, None, 0, None, 0,
                                   None) == CODES["CG_ERR_NULL"]
    assert lib.cg_teeth(None, None, 0, None, None, 0, None) == CODES["CG_ERR_NULL"]
    assert lib.cg_fit_spectra(None, None, None, 0, 20, None, None, None, None, None) == \
        CODES["CG_ERR_NULL"]
    assert lib.cg_init_spectra(None, None, 0, None, None, None) == CODES["CG_ERR_NULL"]
    assert lib.cg_reference_from_frames(None, None, 1, None, None) == CODES["CG_ERR_NULL"]
    assert lib.cg_set_reference(None, None) == CODES["CG_ERR_NULL"]
    assert lib.cg_plan_info(None, None, None, None) == CODES["CG_ERR_NULL"]
    assert lib.cg_set_tuning(None, 1, 0) == CODES["CG_ERR_NULL"]
    assert lib.cg_init_spectra_listed(None, None, 0, None, None, None) == CODES["CG_ERR_NULL"]
    assert lib.cg_median_filter(None, None, 0, None, None) == CODES["CG_ERR_NULL"]
    assert lib.cg_start_points(None, None, 0, None, None) == CODES["CG_ERR_NULL"]
    sz = ctypes.c_size_t()
    assert lib.cg_workspace_bytes(None, 10, ctypes.byref(sz)) == CODES["CG_ERR_NULL"]


def test_python_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load()
