"""ctypes binding of libnufftradon.so (argument marshalling only).

Every computation runs in the HIP library; this module only loads it and
declares the C signatures of ``include/nufftradon.h``.  Loading fails loudly
when the library has not been built.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int32, c_int64, c_size_t, c_uint64, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnufftradon.so")

NR_OK = 0
NR_INVALID_ARG = 1
NR_UNSUPPORTED_SIZE = 2
NR_WORKSPACE_TOO_SMALL = 3
NR_HIP_ERROR = 4
NR_NONFINITE = 5
NR_INTERNAL = 6


class NrSlice(ctypes.Structure):
    _fields_ = [("n", c_int32), ("n_det", c_int32), ("n_angles", c_int32),
                ("vol_off", c_int64), ("sino_off", c_int64), ("angle_off", c_int64), ("center", c_double)]


NR_FBP_RAMP = 0
NR_FBP_BUTTERWORTH = 1
NR_STREAM_FWD = 1
NR_STREAM_ADJ = 2
NR_STREAM_FBP = 3


class NrFbp(ctypes.Structure):
    _fields_ = [("filter", c_int32), ("order", c_int32), ("cutoff", c_double)]


class NrNufft(ctypes.Structure):
    _fields_ = [("sigma", c_double), ("width", c_int32), ("beta", c_double)]


class NrPrior(ctypes.Structure):
    _fields_ = [("p", c_float), ("sigma", c_float), ("c", c_float), ("lam", c_float),
                ("w_face", c_float), ("w_edge", c_float), ("w_corner", c_float)]


class NrMbir(ctypes.Structure):
    _fields_ = [("inv_L", c_float), ("restart", c_int32), ("nonneg", c_int32), ("monotone", c_int32)]


NR_MBIR_STATE_DOUBLES = 16
NR_WEIGHTS_INV_DISTANCE = 0
NR_WEIGHTS_GAUSSIAN = 1


class NrError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: status {status}: {message}")
        self.status = status


# name -> (restype, argtypes)
SIGNATURES = {
    "nr_status_str": (c_char_p, [c_int32]),
    "nr_last_error": (c_char_p, []),
    "nr_version": (c_char_p, []),
    "nr_plan_create": (c_int32, [POINTER(NrSlice), c_int32, POINTER(c_double), POINTER(NrNufft),
                                 POINTER(c_void_p)]),
    "nr_plan_workspace_bytes": (c_int32, [c_void_p, POINTER(c_size_t)]),
    "nr_plan_bind": (c_int32, [c_void_p, c_void_p, c_size_t, c_void_p]),
    "nr_plan_destroy": (c_int32, [c_void_p]),
    "nr_plan_tune": (c_int32, [c_void_p, c_char_p, c_int64]),
    "nr_plan_profile": (c_int32, [c_void_p, c_int32]),
    "nr_plan_profile_read": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_int64), c_int32]),
    "radon_fwd": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "radon_adj": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "radon_fbp": (c_int32, [c_void_p, POINTER(NrFbp), c_void_p, c_void_p, c_void_p]),
    "radon_stream": (c_int32, [c_void_p, c_int32, POINTER(NrFbp), c_void_p, c_void_p, c_int64,
                               POINTER(c_void_p), POINTER(c_void_p), c_void_p]),
    "radon_residual": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "radon_normal": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "qggmrf_grad": (c_int32, [c_void_p, c_int32, c_int32, POINTER(NrPrior), c_float, c_void_p, c_void_p,
                              c_void_p]),
    "mbir_step": (c_int32, [c_void_p, POINTER(NrPrior), POINTER(NrMbir), c_void_p, c_void_p, c_void_p,
                            c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "mbir_step_noalloc": (c_int32, [c_void_p, POINTER(NrPrior), POINTER(NrMbir), c_void_p, c_void_p, c_void_p,
                                    c_void_p, c_void_p, c_void_p, c_void_p]),
    "mbir_update": (c_int32, [POINTER(NrMbir), c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_void_p,
                              c_void_p]),
    "mbir_stream_work_bytes": (c_int32, [c_void_p, POINTER(c_size_t)]),
    "mbir_stream_iterate": (c_int32, [c_void_p, POINTER(NrPrior), POINTER(NrMbir), c_int64, c_void_p, c_void_p,
                                      c_void_p, c_void_p, c_void_p, c_size_t, c_void_p, c_void_p]),
    "mbir_state_init": (c_int32, [c_void_p, c_void_p]),
    "nr_prior_init": (c_int32, [POINTER(NrPrior), c_float, c_float, c_float, c_float, c_int32]),
    "nr_prior_lipschitz": (c_int32, [POINTER(NrPrior), POINTER(c_double)]),
    "nr_mbir_params": (c_int32, [c_double, POINTER(NrPrior), c_int32, c_int32, c_int32, POINTER(NrMbir)]),
    "nr_power_lipschitz": (c_int32, [c_void_p, c_int32, c_uint64, c_double, c_void_p, c_void_p, c_void_p, c_void_p,
                                     POINTER(c_double), c_void_p]),
    "nr_autotune": (c_int32, [c_void_p, c_void_p, c_size_t, c_char_p, c_void_p]),
    "nr_autotune_scratch_bytes": (c_int32, [c_void_p, POINTER(c_size_t)]),
    "nr_plan_get_tune": (c_int32, [c_void_p, c_char_p, POINTER(c_int64)]),
    "nr_graph_capture_radon": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, POINTER(c_void_p)]),
    "nr_graph_capture_mbir": (c_int32, [c_void_p, POINTER(NrPrior), POINTER(NrMbir), c_void_p, c_void_p, c_void_p,
                                        c_void_p, c_void_p, c_void_p, c_void_p, c_int32, POINTER(c_void_p)]),
    "nr_graph_launch": (c_int32, [c_void_p, c_void_p]),
    "nr_graph_destroy": (c_int32, [c_void_p]),
    "nr_kb_eval": (c_int32, [c_int32, c_double, c_int32, POINTER(c_double), POINTER(c_double),
                             POINTER(c_double), POINTER(c_double), POINTER(c_double)]),
    "nr_plan_info": (c_int32, [c_void_p, c_int32, POINTER(c_int64), c_int32]),
    "nr_plan_check": (c_int32, [c_void_p, c_void_p]),
}

_LIB = None


def lib() -> ctypes.CDLL:
    """The loaded library (raises if it is missing: there is no fallback path)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2304_12934_amd.build` (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def check(status: int, where: str) -> None:
    if status != NR_OK:
        msg = lib().nr_last_error().decode(errors="replace")
        raise NrError(status, where, msg)
