"""ctypes declarations of the libecc C ABI (include/ecc.h). Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libecc.so")

ECC_OK = 0
STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported", 3: "out of memory", 4: "HIP error",
          5: "plan mismatch", 6: "internal error"}
GROUP_ROTATION, GROUP_SCALE, GROUP_ROTATION_SCALE = 0, 1, 2
CORRELATION, CONVOLUTION = 0, 1
PREC_FP32, PREC_MFMA_FP16_HILO, PREC_MFMA_BF16_HILO = 0, 1, 2
STRATEGY_AUTO, STRATEGY_TWO_PASS, STRATEGY_TILED, STRATEGY_DIRECT = 0, 1, 2, 3
# ecc_ws_call: the calls whose workspace ecc_workspace_size reports
(WS_EXTENDED_CORRELATION, WS_EXTENDED_CONVOLUTION, WS_SCALE_SMOOTH, WS_MATCH_ROTATIONS,
 WS_BACKWARD_CONVOLUTION, WS_BACKWARD_CORRELATION, WS_NORMALIZED_CONVOLUTION, WS_JOINT_CONVOLUTION) = range(8)


class GroupParams(C.Structure):
    _fields_ = [
        ("angular_samples", C.c_int),
        ("sigma0", C.c_double),
        ("scale_min", C.c_double),
        ("scale_max", C.c_double),
        ("scale_components", C.c_int),
        ("scale_period_factor", C.c_double),
    ]


class Instance(C.Structure):
    """ecc_instance: one image of a batch (device pointers, strides in elements)."""
    _fields_ = [
        ("op", C.c_int),
        ("plan", C.c_void_p),
        ("ny", C.c_int),
        ("nx", C.c_int),
        ("signal", C.c_void_p),
        ("ld_signal", C.c_int),
        ("field", C.c_void_p),
        ("ld_field", C.c_int),
        ("out", C.c_void_p),
        ("ld_out", C.c_int),
    ]


BATCH_AUTOTUNE, BATCH_PERSISTENT = 1, 2


class EccError(RuntimeError):
    def __init__(self, status, text):
        super().__init__(f"libecc: {STATUS.get(status, status)}: {text}")
        self.status = status


_P = C.c_void_p
_I = C.c_int
_F = C.POINTER(C.c_float)

# name -> argument types (all return int status except where noted)
PROTOS = {
    "ecc_create": [_I, C.POINTER(_P)],
    "ecc_destroy": [_P],
    "ecc_fft_size": [_P, _I, _I, C.POINTER(_I)],
    "ecc_set_autotune": [_P, _I],
    "ecc_autotune_export": [_P, C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)],
    "ecc_autotune_import": [_P, C.c_char_p],
    "ecc_set_stage_events": [_P, C.POINTER(_P), _I],
    "ecc_set_strategy": [_P, _I],
    "ecc_describe": [_P, _I, _P, _I, _I, C.POINTER(_I), C.POINTER(_I), C.POINTER(_I)],
    "ecc_batch_plan_create": [_P, C.POINTER(Instance), _I, _I, C.POINTER(_P)],
    "ecc_batch_update": [_P, C.POINTER(Instance), _I],
    "ecc_batch_execute": [_P, _P],
    "ecc_batch_info": [_P, C.POINTER(_I), C.POINTER(_I), C.POINTER(_I)],
    "ecc_batch_plan_destroy": [_P],
    "ecc_filter_plan_create": [_P, _I, _P, _I, _I, C.POINTER(GroupParams), _P, C.POINTER(_P)],
    "ecc_filter_plan_from_components": [_P, _I, _P, _I, _I, C.POINTER(GroupParams), _P, C.POINTER(_P)],
    "ecc_filter_plan_get_components": [_P, _P, _P],
    "ecc_filter_plan_info": [_P, C.POINTER(_I), C.POINTER(_I), C.POINTER(_I)],
    "ecc_filter_plan_component_count": [_P, C.POINTER(_I)],
    "ecc_filter_plan_destroy": [_P],
    "ecc_extended": [_P, _I, _P, _I, _I, _I, _P, _I, _P, _I, _P, _I, _I, _P],
    "ecc_scale_smooth": [_P, _P, _I, _I, _P, _I, _P, _I, _P, _I, _I, _P],
    "ecc_normalized_convolution": [_P, _P, _I, _I, _I, _P, _I, _P, _I, _P, _I, _I, _P],
    "ecc_joint_convolution": [_P, _P, _I, _I, _I, _P, _I, _P, _I, _P, _I, _P, _I, _I, _P],
    "ecc_match_rotations": [_P, _P, _I, _I, _P, _I, _I, _P, _P, _I, _I, _P],
    "ecc_match_rotations_noalloc": [_P, _P, _I, _I, _P, _I, _I, _P, _P, _I, _I, _P],
    "ecc_extended_backward": [_P, _I, _P, _I, _I, _I, _P, _P, _P, _P, _P, _P, _P, _P],
    "ecc_backward_saved_size": [_P, _P, _I, _I, _I, C.POINTER(C.c_size_t)],
    "ecc_extended_save": [_P, _P, _I, _I, _I, _P, _P, _P, _P, _P],
    "ecc_gradient_field": [_P, _I, _I, _I, _P, _I, _P, _P, _I, _P],
    "ecc_voting_filter": [_P, _I, _P, _P, _P],
    "ecc_find_peaks": [_P, _I, _I, _P, _I, _I, C.c_float, _I, _I, _P, _P, _P, _P, _P],
    "ecc_volume_plan_create": [_P, _P, _I, _I, _P, C.POINTER(_P)],
    "ecc_volume_plan_destroy": [_P],
    "ecc_volume_plan_info": [_P, C.POINTER(_I), C.POINTER(_I)],
    "ecc_volume_plan_components": [_P, _P, _P, _P, _P],
    "ecc_extended_3d": [_P, _I, _P, _I, _I, _I, _P, _P, _P, _P, _P, _P],
    "ecc_volume_workspace_size": [_P, _P, _I, _I, _I, C.POINTER(C.c_size_t)],
    "ecc_workspace_size": [_P, _I, _P, _I, _I, _I, C.POINTER(C.c_size_t)],
    "ecc_workspace_reserve": [_P, C.c_size_t],
    "ecc_workspace_allocated": [_P, C.POINTER(C.c_size_t)],
}
EXTRA = {
    "ecc_status_string": ([_I], C.c_char_p),
    "ecc_last_error": ([_P], C.c_char_p),
}


def load(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise RuntimeError(
            f"libecc.so not found at {path}: build it first (python -m paper_2006_13188_amd.build)")
    lib = C.CDLL(path)
    for name, args in PROTOS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    for name, (args, res) in EXTRA.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


def exported_symbols():
    return list(PROTOS) + list(EXTRA)
