"""ctypes declarations of libgpr's C ABI (include/gpr.h). Marshalling only."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgpr.so")

GPR_OK, GPR_ENOTPD, GPR_EINVAL, GPR_ENOMEM, GPR_EHIP, GPR_ENODEV, GPR_ENOTSUP = 0, 1, -1, -2, -3, -4, -5
GPR_FP64, GPR_MIXED_FP32, GPR_MIXED_BF16 = 0, 1, 2
GPR_EXEC_STREAMS, GPR_EXEC_PERSISTENT, GPR_EXEC_AUTO = 0, 1, 2
GPR_RIGHT_LOOKING, GPR_LEFT_LOOKING = 0, 1
GPR_STATE_EMPTY, GPR_STATE_K, GPR_STATE_L = 0, 1, 2


class Hyper(ctypes.Structure):
    _fields_ = [("lengthscale", ctypes.c_double),
                ("vertical_variance", ctypes.c_double),
                ("noise_variance", ctypes.c_double)]


class IRStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32),
                ("rel_residual", ctypes.c_double),
                ("fallback_precision", ctypes.c_int32),
                ("method", ctypes.c_int32)]


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)

# name -> (restype, argtypes)
SIGNATURES = {
    "gpr_abi_version": (ctypes.c_int, []),
    "gpr_source_hash": (ctypes.c_char_p, []),
    "gpr_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "gpr_ctx_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "gpr_ctx_destroy": (ctypes.c_int, [_vp]),
    "gpr_ctx_set_variant": (ctypes.c_int, [_vp, ctypes.c_int]),
    "gpr_assemble": (ctypes.c_int, [_vp, _vp, _i64, _i32, Hyper, _i32, ctypes.POINTER(_vp), _vp]),
    "gpr_cholesky": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _vp]),
    "gpr_cholesky_dense": (ctypes.c_int, [_vp, _vp, _i64, _i32, ctypes.c_int, _vp, _vp]),
    "gpr_predict": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i64, _vp, _i64, _i32, Hyper, _vp, _vp,
                                   ctypes.POINTER(IRStats), _vp]),
    "gpr_fit_predict": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp, _i64, _i32, Hyper, _i32,
                                       ctypes.c_int, ctypes.POINTER(_vp), _vp, _vp, _vp,
                                       ctypes.POINTER(IRStats), _vp]),
    "gpr_predict_var": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i64, _vp, _i64, _i32, Hyper, _vp,
                                       _vp, _vp, ctypes.POINTER(IRStats), _vp]),
    "gpr_fit_predict_var": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp, _i64, _i32, Hyper, _i32,
                                           ctypes.c_int, ctypes.POINTER(_vp), _vp, _vp, _vp,
                                           _vp, ctypes.POINTER(IRStats), _vp]),
    "gpr_solve": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "gpr_solve_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "gpr_nlml_grad": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i32, Hyper, _i32, ctypes.c_int, _vp,
                                     _vp, _vp, _vp]),
    "gpr_fit_hyper": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i32, _i32,
                                     ctypes.POINTER(ctypes.c_double), _i32, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double), _i32p, _vp]),
    "gpr_profile_enable": (ctypes.c_int, [_vp, ctypes.c_int]),
    "gpr_profile_read": (ctypes.c_int, [_vp, ctypes.c_int, _i64p, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double), ctypes.c_int]),
    "gpr_tiled_info": (ctypes.c_int, [_vp, _i64p, _i32p, _i32p]),
    "gpr_tiled_to_dense": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "gpr_tiled_free": (ctypes.c_int, [_vp]),
    "gpr_sync": (ctypes.c_int, [_vp, _vp, _i64p]),
    "gpr_schedule_describe": (ctypes.c_int, [_i32, _i32, _i32, _i32p, _i64, _i64p, _i32p, _i64,
                                             _i64p]),
    "gpr_schedule_describe_variant": (ctypes.c_int, [_i32, _i32, _i32, _i32, _i32p, _i64, _i64p,
                                                     _i32p, _i64, _i64p]),
    "gpr_adjoint_describe": (ctypes.c_int, [_i32, _i32, _i32p, _i64, _i64p, _i32p, _i64, _i64p,
                                            _i32p, _i64, _i64p]),
    "gpr_persist_describe": (ctypes.c_int, [_i32, _i32, _i32, _i32, _i32, _i32, _i32p, _i64p,
                                            _i64, _i64p]),
    "gpr_solve_plan_describe": (ctypes.c_int, [_i32, _i32, _i32p, _i32p, _i64, _i64p, _i32p,
                                               _i64, _i64p]),
}

_LIB = None


def load():
    """Loads the built library; raises if it has not been built, or was built
    from sources other than the ones in this tree (no fallback)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"libgpr.so not found at {LIB_PATH}; build it with "
                "`python -m paper_2602_19683_amd.build` (or __graft_entry__.build())")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        from .build import source_hash
        built, here = lib.gpr_source_hash().decode(), source_hash()
        if built != here:
            raise ImportError(
                f"libgpr.so was built from other sources (hash {built}, tree {here}); "
                "rebuild it with `python -m paper_2602_19683_amd.build`")
        _LIB = lib
    return _LIB


def library_hash() -> str:
    """Source hash compiled into the loaded library."""
    return load().gpr_source_hash().decode()
