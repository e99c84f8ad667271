"""ctypes binding of ``libqt_hip.so`` (include/qtensor_hip.h, include/qtensor_planner.h).

Argument marshalling only: every step of the contraction runs in the HIP
library.  ``load()`` raises if the library has not been built -- there is
no fallback.
"""
from __future__ import annotations

import ctypes
from ctypes import POINTER, c_double, c_int32, c_int64, c_uint64, c_void_p
from pathlib import Path

LIB_PATH = Path(__file__).resolve().parent / "libqt_hip.so"

# qt_status
QT_OK = 0
QT_EINVAL = -1
QT_ENOMEM = -2
QT_EPLAN = -3
QT_EHIP = -4
QT_EUNSUPPORTED = -5
QT_EFAULT_INJECTED = -6
STATUS_NAMES = {
    0: "QT_OK", -1: "QT_EINVAL", -2: "QT_ENOMEM", -3: "QT_EPLAN", -4: "QT_EHIP",
    -5: "QT_EUNSUPPORTED", -6: "QT_EFAULT_INJECTED",
}

# qt_precision
QT_C128 = 0
QT_C64_SCALED = 1
QT_C64_SCALED_MFMA_FP32 = 2
QT_C64_SCALED_MFMA_BF16X3 = 3

# qt_tkind
QT_T_VEC_PLUS = 0
QT_T_ZZ = 1
QT_T_RX = 2
QT_T_BRA_BIT = 3
QT_T_ZZ_DAG = 4
QT_T_RX_DAG = 5
QT_T_OBS_CUT = 6
QT_T_DENSE = 7

# qt_order_algo
QT_ORDER_MIN_DEGREE = 0
QT_ORDER_MIN_FILL = 1
QT_ORDER_RGREEDY = 2


class qt_tensor_desc(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("rank", c_int32), ("layer", c_int32),
                ("vars", POINTER(c_int32)), ("dense", POINTER(c_double))]


class qt_network_desc(ctypes.Structure):
    _fields_ = [("n_vars", c_int32), ("n_tensors", c_int32), ("p", c_int32),
                ("tensors", POINTER(qt_tensor_desc))]


class qt_plan_desc(ctypes.Structure):
    _fields_ = [("order", POINTER(c_int32)), ("n_order", c_int32), ("n_groups", c_int32),
                ("group_step", POINTER(c_int32)), ("group_len", POINTER(c_int32)),
                ("slice_vars", POINTER(c_int32)), ("precision", c_int32), ("slice_batch", c_int64),
                ("flags", c_int32), ("n_open", c_int32), ("open_vars", POINTER(c_int32)),
                ("gemm_min_rank", c_int32)]


QT_NOALLOC_SCRATCH_BYTES = 64 << 20

QT_PLAN_PLAIN = 1
QT_PLAN_FOLD_PREFIX = 2
QT_PLAN_GRAPH = 4


class qt_amp(ctypes.Structure):
    _fields_ = [("re", c_double), ("im", c_double), ("log2_scale", c_double)]


class qt_plan_info(ctypes.Structure):
    _fields_ = [("n_steps", c_int32), ("n_prefix_steps", c_int32), ("width", c_int32),
                ("prefix_width", c_int32), ("slice_width", c_int32), ("n_slice_vars", c_int32),
                ("n_slices", c_int64), ("slice_batch", c_int64), ("prefix_bytes", c_double),
                ("slice_bytes", c_double), ("prefix_flops", c_double), ("slice_flops", c_double),
                ("workspace_bytes", c_int64), ("element_bytes", c_int32), ("n_launches", c_int32),
                ("n_open", c_int32), ("n_groups", c_int32)]


QT_MAX_SLICE_GROUPS = 16


class qt_slicing_opts(ctypes.Structure):
    _fields_ = [("algo", c_int32), ("n_slice_vars", c_int32), ("max_candidates", c_int32),
                ("threads", c_int32), ("tau", c_double), ("repeats", c_int32), ("seed", c_uint64),
                ("group_size", c_int32), ("exclude", POINTER(c_int32)), ("n_exclude", c_int32)]


class qt_slicing_result(ctypes.Structure):
    _fields_ = [("step", c_int32), ("width", c_int32), ("prefix_width", c_int32),
                ("slice_width", c_int32), ("unsliced_width", c_int32), ("peak_step", c_int32),
                ("cost", c_double), ("n_groups", c_int32), ("group_step", c_int32 * QT_MAX_SLICE_GROUPS),
                ("group_len", c_int32 * QT_MAX_SLICE_GROUPS)]


class qt_kernel_stats(ctypes.Structure):
    _fields_ = [("launches", c_int64), ("ms", c_double), ("bytes", c_double), ("flops", c_double)]


class qt_op_stats(ctypes.Structure):
    _fields_ = [("kclass", c_int32), ("op", c_int32), ("launches", c_int64), ("ms", c_double),
                ("bytes", c_double), ("flops", c_double)]


QT_KCLASS_NAMES = {0: "step_stream", 1: "step_small", 2: "lds", 3: "gemm", 4: "other"}
QT_KCLASS_COUNT = 8

# name -> (restype, argtypes); every symbol declared in include/*.h
class qt_tuning(ctypes.Structure):
    _fields_ = [("lds_waves", c_int32), ("lds_max_rank", c_int32), ("multi_waves", c_int32), ("grad_waves", c_int32),
                ("step_tiles", c_int32), ("gemm_tiles", c_int32), ("multi_lds_cap", c_int32),
                ("grad_lds_cap", c_int32)]


SIGNATURES = {
    "qt_load_network": (c_int32, [POINTER(qt_network_desc), POINTER(c_void_p)]),
    "qt_load_plan": (c_int32, [c_void_p, POINTER(qt_plan_desc), POINTER(c_void_p)]),
    "qt_contract_amplitude": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "qt_contract_batch": (c_int32, [POINTER(c_void_p), c_int32, c_int32, c_void_p, c_void_p,
                                    c_int64, c_int64, c_void_p, c_void_p, c_void_p]),
    "qt_contract_batch_noalloc": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_int64, c_int64, c_void_p,
                                            c_void_p, c_void_p]),
    "qt_energy_grad": (c_int32, [POINTER(c_void_p), c_int32, c_int32, c_void_p, c_void_p,
                                 c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "qt_energy_grad_weighted": (c_int32, [POINTER(c_void_p), c_void_p, c_int32, c_int32, c_void_p, c_void_p,
                                          c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "qt_plan_get_info": (c_int32, [c_void_p, POINTER(qt_plan_info)]),
    "qt_plan_set_tuning": (c_int32, [c_void_p, POINTER(qt_tuning)]),
    "qt_plan_get_tuning": (c_int32, [c_void_p, POINTER(qt_tuning)]),
    "qt_profile_enable": (c_int32, [c_void_p, c_int32]),
    "qt_profile_read": (c_int32, [c_void_p, POINTER(qt_kernel_stats), c_int32]),
    "qt_profile_read_ops": (c_int32, [c_void_p, POINTER(qt_op_stats), c_int32, POINTER(c_int32), c_int32]),
    "qt_plan_describe": (c_int32, [c_void_p, ctypes.c_char_p, c_int64, POINTER(c_int64)]),
    "qt_free_plan": (None, [c_void_p]),
    "qt_free_network": (None, [c_void_p]),
    "qt_last_error": (ctypes.c_char_p, []),
    "qt_order_greedy": (c_int32, [c_void_p, c_int32, POINTER(c_int32), c_int32, c_double, c_int32,
                                  c_uint64, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32)]),
    "qt_plan_slicing": (c_int32, [c_void_p, POINTER(qt_slicing_opts), POINTER(c_int32),
                                  POINTER(c_int32), POINTER(c_int32), POINTER(qt_slicing_result),
                                  POINTER(c_int32)]),
}

_LIB = None


class QTError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def load():
    """Load the built library; raises ImportError when it is missing."""
    global _LIB
    if _LIB is None:
        if not LIB_PATH.exists():
            raise ImportError(f"{LIB_PATH} is not built: run python -m paper_2012_02430_amd.build")
        # torch ships its own HIP runtime under the same soname as the
        # system one this library links; loading torch first makes the
        # library bind to that copy, so the process holds one HIP runtime
        # and device pointers and streams are shared with torch.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(str(LIB_PATH))
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def check(status: int) -> None:
    if status != QT_OK:
        raise QTError(status, load().qt_last_error().decode(errors="replace"))


def int32_array(values):
    values = [int(v) for v in values]
    return (c_int32 * max(1, len(values)))(*values)


def double_array(values):
    values = [float(v) for v in values]
    return (c_double * max(1, len(values)))(*values)
