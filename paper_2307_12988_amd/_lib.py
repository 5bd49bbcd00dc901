"""ctypes loader for libcombgpu.so: declares every entry point of combgpu.h.

Loading fails loudly when the library has not been built; there is no other
implementation to fall back to.
"""

from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcombgpu.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "combgpu.h")

_c = ctypes
_vp = _c.c_void_p
_i32 = _c.c_int32
_i64 = _c.c_int64
_u32 = _c.c_uint32
_sz = _c.c_size_t
_dbl = _c.c_double
_pi32 = _c.POINTER(_c.c_int32)
_pf32 = _c.POINTER(_c.c_float)

# name -> (restype, argtypes); device pointers are passed as void*
SIGNATURES = {
    "cg_create_plan": (_i32, [_i32, _dbl, _pi32, _i32, _pf32, _c.POINTER(_vp)]),
    "cg_create_plan_ex": (_i32, [_i32, _dbl, _pi32, _i32, _pf32, _i32, _c.POINTER(_vp)]),
    "cg_plan_sample_bytes": (_i32, [_vp, _pi32]),
    "cg_destroy_plan": (_i32, [_vp]),
    "cg_set_reference": (_i32, [_vp, _pf32]),
    "cg_plan_info": (_i32, [_vp, _pi32, _pi32, _c.POINTER(_dbl)]),
    "cg_workspace_bytes": (_i32, [_vp, _i64, _c.POINTER(_sz)]),
    "cg_process_batch": (_i32, [_vp, _vp, _i64, _vp, _vp]),
    "cg_process_batch_ex": (_i32, [_vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _u32, _vp, _sz,
                                   _vp]),
    "cg_process_batch_static": (_i32, [_vp, _vp, _i64, _vp, _vp, _vp, _vp, _u32, _vp]),
    "cg_teeth": (_i32, [_vp, _vp, _i64, _vp, _vp, _u32, _vp]),
    "cg_reference_from_frames": (_i32, [_vp, _vp, _i64, _vp, _vp]),
    "cg_init_spectra": (_i32, [_vp, _vp, _i64, _vp, _vp, _vp]),
    "cg_init_spectra_listed": (_i32, [_vp, _vp, _i64, _vp, _vp, _vp]),
    "cg_start_centres": (_i32, [_vp, _vp, _i64, _vp, _vp]),
    "cg_median_filter": (_i32, [_vp, _vp, _i64, _vp, _vp]),
    "cg_start_points": (_i32, [_vp, _vp, _i64, _vp, _vp]),
    "cg_fit_spectra": (_i32, [_vp, _vp, _vp, _i64, _i32, _vp, _vp, _vp, _vp, _vp]),
    "cg_set_tuning": (_i32, [_vp, _i32, _i32]),
    "cg_get_tuning": (_i32, [_vp, _i32, _pi32]),
    "cg_set_mlp": (_i32, [_vp, _pf32, _pf32, _pf32, _c.c_float]),
    "cg_set_fano": (_i32, [_vp, _dbl, _dbl, _dbl, _dbl]),
    "cg_fit_fano": (_i32, [_vp, _vp, _vp, _i64, _i32, _vp, _vp, _vp, _vp, _vp]),
    "cg_set_polish_iters": (_i32, [_vp, _i32]),
    "cg_mlp_infer": (_i32, [_vp, _vp, _i64, _vp, _vp]),
    "cg_mlp_trainer_create": (_i32, [_i32, _pf32, _c.POINTER(_vp)]),
    "cg_mlp_trainer_destroy": (_i32, [_vp]),
    "cg_mlp_train_step": (_i32, [_vp, _vp, _vp, _vp, _vp, _c.c_float, _c.c_float, _c.c_float,
                                 _c.c_float, _vp, _vp]),
    "cg_mlp_gradients": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "cg_mlp_get_params": (_i32, [_vp, _pf32]),
    "cg_pipeline_create": (_i32, [_i32, _vp, _vp, _i32, _i32, _u32, _dbl, _c.POINTER(_vp)]),
    "cg_pipeline_create_ex": (_i32, [_i32, _vp, _vp, _i32, _i32, _u32, _i32, _dbl,
                                     _c.POINTER(_vp)]),
    "cg_pipeline_destroy": (_i32, [_vp]),
    "cg_pipeline_acquire": (_i32, [_vp, _i32, _pi32, _c.POINTER(_vp)]),
    "cg_pipeline_publish": (_i32, [_vp, _i32, _i32, _i32, _i64]),
    "cg_pipeline_put": (_i32, [_vp, _i32, _vp, _i32, _i64, _pi32]),
    "cg_pipeline_read": (_i32, [_vp, _i32, _pf32, _pi32, _i32, _pi32, _c.POINTER(_i64)]),
    "cg_pipeline_drain": (_i32, [_vp, _i32]),
    "cg_pipeline_stats": (_i32, [_vp, _c.POINTER(_dbl), _i32]),
    "cg_autotune": (_i32, [_vp, _vp, _i64, _u32, _vp, _sz, _pi32, _pf32]),
    "cg_psd_band": (_i32, [_i32, _dbl, _dbl, _dbl, _pi32, _pi32]),
    "cg_psd_workspace_bytes": (_i32, [_i64, _i32, _i32, _c.POINTER(_sz)]),
    "cg_psd_welch": (_i32, [_vp, _i64, _dbl, _i32, _i32, _i32, _vp, _vp, _sz, _vp]),
    "cg_resonance_fit": (_i32, [_vp, _i32, _dbl, _dbl, _i32, _dbl, _vp, _vp]),
    "cg_status_string": (_c.c_char_p, [_i32]),
    "cg_last_error_detail": (_c.c_char_p, []),
    "cg_version": (_c.c_char_p, []),
}

_lib = None


class CombGpuError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        msg = f"{where}: status {status}"
        if _lib is not None:
            msg += f" ({_lib.cg_status_string(status).decode()})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)


def header_functions(path: str = HEADER):
    """Names of the functions combgpu.h declares."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cg_[a-z0-9_]+)\s*\(", text)))


def load():
    """Load and declare the library (cached)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2307_12988_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int, where: str):
    if status != 0:
        detail = _lib.cg_last_error_detail().decode() if _lib is not None else ""
        raise CombGpuError(status, where, detail)
