"""ctypes binding of libmclbm.so (argument marshalling only).

Every call maps one-to-one onto an ``extern "C"`` entry point of
include/mclbm.h. The library must have been built (``build.py``); there is no
fallback: loading fails loudly when it is missing.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmclbm.so")

OK, ERR_ARG, ERR_OOM, ERR_HIP, ERR_STATE, ERR_UNSTABLE, ERR_UNSUPPORTED = range(7)
STATUS_NAMES = {0: "OK", 1: "ERR_ARG", 2: "ERR_OOM", 3: "ERR_HIP", 4: "ERR_STATE", 5: "ERR_UNSTABLE",
                6: "ERR_UNSUPPORTED"}
FP64, FP32_SHIFTED = 0, 1
D3Q27, D3Q19 = 27, 19
GAMMA_CLOSED_FORM, GAMMA_EXACT = 0, 1


class SampleDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("u0", ctypes.c_double), ("re", ctypes.c_double), ("amp", ctypes.c_double),
                ("project", ctypes.c_int32), ("stride", ctypes.c_int32)]


class MclbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_c = ctypes
_vp = _c.c_void_p
_i32 = _c.c_int32
_i64 = _c.c_int64
_u64 = _c.c_uint64
_sz = _c.c_size_t
_dp = _c.POINTER(_c.c_double)
_ip = _c.POINTER(_c.c_int32)
_descp = _c.POINTER(SampleDesc)
_ctxp = _c.c_void_p

# name: (restype, argtypes)
SIGNATURES = {
    "mclbm_omega": (_c.c_double, [_i32, _c.c_double, _c.c_double]),
    "mclbm_workspace_bytes": (_sz, [_i32, _descp, _i32, _i32]),
    "mclbm_create": (_i32, [_c.POINTER(_ctxp), _i32, _descp, _i32, _i32, _vp, _sz, _vp]),
    "mclbm_destroy": (_i32, [_ctxp]),
    "mclbm_init": (_i32, [_ctxp, _u64, _dp]),
    "mclbm_get_y": (_i32, [_ctxp, _dp]),
    "mclbm_set_viscosity": (_i32, [_ctxp, _dp]),
    "mclbm_step": (_i32, [_ctxp, _i64, _i32, _vp, _i64]),
    "mclbm_moments": (_i32, [_ctxp, _i32, _vp, _vp]),
    "mclbm_reduce": (_i32, [_ctxp, _vp]),
    "mclbm_check": (_i32, [_ctxp, _ip]),
    "mclbm_get_state": (_i32, [_ctxp, _i32, _vp]),
    "mclbm_set_state": (_i32, [_ctxp, _i32, _vp]),
    "mclbm_get_cells": (_i32, [_ctxp, _i32, _vp, _i32, _vp]),
    "mclbm_poison": (_i32, [_ctxp, _i32, _i64, _i32]),
    "mclbm_checkpoint_bytes": (_sz, [_ctxp]),
    "mclbm_checkpoint": (_i32, [_ctxp, _vp, _sz]),
    "mclbm_restore": (_i32, [_ctxp, _vp, _sz]),
    "mclbm_ckpt_bytes": (_sz, [_ctxp, _i64, _i32]),
    "mclbm_backward_work_bytes": (_sz, [_ctxp, _i32]),
    "mclbm_forward_ckpt": (_i32, [_ctxp, _i64, _i32, _vp, _sz]),
    "mclbm_backward": (_i32, [_ctxp, _i64, _i32, _vp, _sz, _vp, _sz, _vp, _vp]),
    "mclbm_step_vjp_work_bytes": (_sz, [_ctxp]),
    "mclbm_step_vjp": (_i32, [_ctxp, _vp, _vp, _vp, _sz]),
    "mclbm_observables_work_bytes": (_sz, [_ctxp, _i32]),
    "mclbm_observables": (_i32, [_ctxp, _i32, _vp, _vp, _vp, _sz]),
    "mclbm_observables_range_work_bytes": (_sz, [_ctxp, _i32, _i32]),
    "mclbm_observables_range": (_i32, [_ctxp, _i32, _i32, _vp, _vp, _vp, _sz]),
    "mclbm_velocity_bytes": (_sz, [_ctxp]),
    "mclbm_capture_velocity": (_i32, [_ctxp, _vp, _sz]),
    "mclbm_observables_velocity_range": (_i32, [_ctxp, _i32, _i32, _vp, _vp, _vp, _vp, _sz]),
    "mclbm_point_values": (_i32, [_ctxp, _i32, _i32, _vp]),
    "mclbm_w1_work_bytes": (_sz, [_i32]),
    "mclbm_w1_1pt": (_i32, [_vp, _vp, _i32, _i32, _vp, _vp, _sz, _vp]),
    "mclbm_ensemble_moments": (_i32, [_vp, _i32, _i32, _i64, _vp, _vp, _vp]),
    "mclbm_compensate": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp, _vp, _vp]),
    "mclbm_sample_error_work_bytes": (_sz, [_i32]),
    "mclbm_sample_error": (_i32, [_vp, _vp, _i32, _i32, _vp, _vp, _sz, _vp]),
    "mclbm_sample_error_noalloc": (_i32, [_vp, _vp, _i32, _i32, _vp, _vp]),
    "mclbm_eoc_slope": (_i32, [_vp, _vp, _i32, _vp]),
    "mclbm_set_launch": (_i32, [_ctxp, _i32, _i32, _i32, _i32]),
    "mclbm_get_launch": (_i32, [_ctxp, _ip, _ip, _ip, _ip]),
    "mclbm_autotune": (_i32, [_ctxp, _i32, _vp, _sz, _ip, _ip, _ip, _ip]),
    "mclbm_dissipation": (_i32, [_ctxp, _vp, _i32, _i64, _i32, _vp, _vp]),
    "mclbm_dissipation_spectra": (_i32, [_ctxp, _i32, _i32, _vp, _i32, _i64, _i32, _vp, _vp]),
    "mclbm_set_stabiliser": (_i32, [_ctxp, _i32]),
    "mclbm_use_graphs": (_i32, [_ctxp, _i32]),
    "mclbm_ticks": (_i64, [_ctxp]),
    "mclbm_steps": (_i64, [_ctxp, _i32]),
    "mclbm_time_launches": (_i32, [_ctxp, _i32]),
    "mclbm_launch_time": (_i32, [_ctxp, _dp, _c.POINTER(_i64)]),
    "mclbm_stream_copy": (_i32, [_vp, _vp, _sz, _vp]),
    "mclbm_last_error": (_c.c_char_p, []),
}

_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                              "(python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def check(status):
    if status != OK:
        raise MclbmError(status, lib().mclbm_last_error().decode())
    return status
