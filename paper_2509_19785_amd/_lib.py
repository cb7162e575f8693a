"""ctypes binding of libtsnet.so: one Python function per C entry point, same names.

Argument marshalling only: every computation happens in the HIP library.
Device buffers are passed as integer addresses (``tensor.data_ptr()``), streams
as ``torch.cuda.Stream.cuda_stream`` integers (0 = default stream).
Importing this module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libtsnet.so")

TSNET_OK = 0
TSNET_EINVAL = -1
TSNET_EHIP = -2
TSNET_ENOMEM = -3
TSNET_EGRID = -4
TSNET_TIE_HASH = 0
TSNET_TIE_ID = 1
TSNET_STATUS_NONFINITE = 0x1
TSNET_STATUS_GRID_CAPPED = 0x2
TSNET_STATUS_ROW_LOW = 0x4
TSNET_STATUS_ROW_HIGH = 0x8
TSNET_STATUS_ROW_EMPTY = 0x10
TSNET_STATUS_WORKSPACE = 0x20

# every entry point declared in include/tsnet.h
EXPORTS = (
    "tsnet_default_params", "tsnet_default_step_params", "tsnet_ctx_create", "tsnet_ctx_destroy",
    "tsnet_build_P", "tsnet_P_from_host", "tsnet_P_info", "tsnet_P_export", "tsnet_P_free",
    "tsnet_grad", "tsnet_grad_terms", "tsnet_step", "tsnet_cost", "tsnet_grad_direct_f64",
    "tsnet_grid_info", "tsnet_status", "tsnet_set_timing", "tsnet_stage_count",
    "tsnet_stage_name", "tsnet_stage_times", "tsnet_last_error",
    "tsnet_default_pmds_params", "tsnet_pmds", "tsnet_np", "tsnet_stress", "tsnet_run",
    "tsnet_grad_direct_f64_static", "tsnet_workspace_bytes",
)


class tsnet_params(ctypes.Structure):
    _fields_ = [
        ("lambda_kl", ctypes.c_double), ("lambda_c", ctypes.c_double),
        ("lambda_r", ctypes.c_double), ("eps_r", ctypes.c_double),
        ("interval_width", ctypes.c_double), ("min_intervals", ctypes.c_int32),
        ("max_intervals", ctypes.c_int32), ("nodes_per_interval", ctypes.c_int32),
        ("attract_layout", ctypes.c_int32), ("repulsion", ctypes.c_int32),
        ("entropy", ctypes.c_int32), ("theta", ctypes.c_double),
        ("far_trim", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class tsnet_stage(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("reserved", ctypes.c_int32), ("params", tsnet_params)]


class tsnet_step_params(ctypes.Structure):
    _fields_ = [
        ("eta", ctypes.c_double), ("momentum_early", ctypes.c_double),
        ("momentum_late", ctypes.c_double), ("min_gain", ctypes.c_double),
        ("gain_up", ctypes.c_double), ("gain_down", ctypes.c_double),
        ("momentum_switch_iter", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class tsnet_pmds_params(ctypes.Structure):
    _fields_ = [
        ("pivots", ctypes.c_int32), ("seed", ctypes.c_uint64), ("scale", ctypes.c_double),
    ]


class TsnetError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tsnet error {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2509_19785_amd.build` "
            "(the GPU path has no fallback)")
    return ctypes.CDLL(LIB_PATH)


lib = _load()

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_dbl = ctypes.c_double
_P = ctypes.POINTER

_SIGS = {
    "tsnet_default_params": (None, [_P(tsnet_params)]),
    "tsnet_default_step_params": (None, [_P(tsnet_step_params)]),
    "tsnet_default_pmds_params": (None, [_P(tsnet_pmds_params)]),
    "tsnet_pmds": (_i32, [_vp, _vp, _vp, _i32, _i64, _vp, _i32, _P(tsnet_pmds_params), _vp, _vp,
                          _vp, _vp, _vp]),
    "tsnet_run": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _i32, _P(tsnet_step_params), _vp]),
    "tsnet_np": (_i32, [_vp, _vp, _vp, _i32, _i64, _vp, _i32, _vp, _vp, _i32, _vp, _vp, _vp, _vp]),
    "tsnet_stress": (_i32, [_vp, _vp, _vp, _i32, _i64, _vp, _i32, _vp, _vp, _i32, _vp, _vp, _vp]),
    "tsnet_ctx_create": (_i32, [_P(_vp), _i32]),
    "tsnet_ctx_destroy": (_i32, [_vp]),
    "tsnet_build_P": (_i32, [_vp, _vp, _vp, _i32, _i64, _vp, _i32, _dbl, _i32, _u64, _i32,
                             _P(_vp), _vp]),
    "tsnet_P_from_host": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _i32, _P(_vp)]),
    "tsnet_P_info": (_i32, [_vp, _P(_i64), _P(_i64), _P(_i32), _P(_i32)]),
    "tsnet_P_export": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "tsnet_P_free": (_i32, [_vp]),
    "tsnet_grad": (_i32, [_vp, _vp, _vp, _P(tsnet_params), _vp, _vp, _vp]),
    "tsnet_grad_terms": (_i32, [_vp, _vp, _vp, _P(tsnet_params), _vp, _vp, _vp, _vp, _vp, _vp,
                                _vp]),
    "tsnet_step": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _P(tsnet_step_params), _i32, _vp]),
    "tsnet_cost": (_i32, [_vp, _vp, _vp, _P(tsnet_params), _vp, _vp]),
    "tsnet_grad_direct_f64": (_i32, [_vp, _vp, _vp, _P(tsnet_params), _vp, _vp, _vp, _i32, _vp,
                                     _vp]),
    "tsnet_grad_direct_f64_static": (_i32, [_vp, _vp, _vp, _P(tsnet_params), _vp, _vp, _vp, _i32, _vp,
                                     _vp]),
    "tsnet_grid_info": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "tsnet_workspace_bytes": (_i32, [_vp, _P(ctypes.c_size_t)]),
    "tsnet_status": (_i32, [_vp, _P(ctypes.c_uint32)]),
    "tsnet_set_timing": (_i32, [_vp, ctypes.c_uint32]),
    "tsnet_stage_count": (_i32, []),
    "tsnet_stage_name": (ctypes.c_char_p, [_i32]),
    "tsnet_stage_times": (_i32, [_vp, _vp, _vp]),
    "tsnet_last_error": (ctypes.c_char_p, []),
}

for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def check(rc: int) -> None:
    if rc != TSNET_OK:
        raise TsnetError(rc, lib.tsnet_last_error().decode())


def _thin(name):
    fn = getattr(lib, name)

    def call(*args):
        return fn(*args)

    call.__name__ = name
    call.__doc__ = f"Direct call of the C function {name} (see include/tsnet.h)."
    return call


# module-level functions with the C names
for _name in EXPORTS:
    globals()[_name] = _thin(_name)
