"""ctypes binding of the C ABI in include/lof.h (argument marshalling only).

Every step of the flagging path runs in the HIP library ``liblof.so``; this module
only loads it, mirrors its structs and passes device pointers (torch tensors'
``data_ptr()``) and HIP stream handles through.  It raises if the library has not
been built: there is no other implementation to fall back to.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblof.so")

LOF_OK, LOF_ERR_INVALID, LOF_ERR_NOMEM, LOF_ERR_DEVICE, LOF_ERR_CAPACITY = 0, -1, -2, -3, -4
LOF_CI8, LOF_C64, LOF_F32, LOF_C64_AMP = 0, 1, 2, 3
LOF_OPT_AUTOCOMMIT = 0x1
LOF_OPT_LITERAL_HISTORY_TIE = 0x2
LOF_OPT_GRAPH = 0x4
LOF_OPT_PHASE_TIMING = 0x8
LOF_OPT_SIR_PROSE = 0x10
LOF_OPT_INTEGRATED = 0x20
LOF_OPT_ROBUST_SIGMA = 0x40
LOF_OPT_PREFLAGGED = 0x80
# phases of lof_phase_times, in launch order
PHASES = ("stats", "sumthreshold_time", "sumthreshold_freq", "sir_time", "sir_freq", "history_write")
LOF_N_PHASES = len(PHASES)
LOF_MAX_LEVELS = 16
LOF_TUNE_BUCKETS = 5

EXPORTED = ("lof_default_params", "lof_create", "lof_flag_blocks", "lof_history_update",
            "lof_history_export", "lof_get_tuning", "lof_set_tuning", "lof_autotune", "lof_phase_times",
            "lof_destroy", "lof_last_error", "lof_flag_blocks_static")


class LofParams(ctypes.Structure):
    _fields_ = [
        ("start_threshold", ctypes.c_double),
        ("p", ctypes.c_double),
        ("sensitivity", ctypes.c_double),
        ("n_levels", ctypes.c_int32),
        ("n_levels_freq", ctypes.c_int32),
        ("sir_eta_num", ctypes.c_int32),
        ("sir_eta_den", ctypes.c_int32),
        ("history_sensitivity", ctypes.c_double),
        ("history_len", ctypes.c_int32),
        ("history_min", ctypes.c_int32),
        ("max_streams", ctypes.c_int32),
        ("max_channels", ctypes.c_int32),
        ("max_blocks_per_call", ctypes.c_int32),
        ("call_slots", ctypes.c_int32),
        ("max_samples_per_call", ctypes.c_int64),
        ("options", ctypes.c_uint32),
        ("partial_time", ctypes.c_int32),
        ("partial_freq", ctypes.c_int32),
        ("history_winsor", ctypes.c_int32),
    ]


class LofBlock(ctypes.Structure):
    _fields_ = [
        ("data", ctypes.c_void_p),
        ("flags", ctypes.c_void_p),
        ("data_row_stride", ctypes.c_int64),
        ("flag_row_stride", ctypes.c_int64),
        ("n_channels", ctypes.c_int32),
        ("n_times", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("stream_id", ctypes.c_int32),
    ]


class LofBlockStats(ctypes.Structure):
    _fields_ = [
        ("median", ctypes.c_double),
        ("stddev", ctypes.c_double),
        ("threshold", ctypes.c_double * LOF_MAX_LEVELS),
        ("n_flagged", ctypes.c_int64),
        ("history_flagged_rows", ctypes.c_int32),
        ("_pad", ctypes.c_int32),
    ]


class LofTuning(ctypes.Structure):
    _fields_ = [
        ("time_lanes", (ctypes.c_int32 * LOF_TUNE_BUCKETS) * 2),
        ("persistent", ctypes.c_int32),
        ("fuse_post", ctypes.c_int32),
    ]


STATS_BYTES = ctypes.sizeof(LofBlockStats)

_lib = None


def lib_exists() -> bool:
    return os.path.exists(LIB_PATH)


def load() -> ctypes.CDLL:
    """Load liblof.so (raises FileNotFoundError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FileNotFoundError(f"{LIB_PATH} is missing: build it with paper_1701_08197_amd.build.build()")
    # torch ships its own HIP runtime; load it first so that liblof binds to the
    # same libamdhip64 (two HIP runtimes in one process do not share the device)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    L.lof_default_params.argtypes = [ctypes.POINTER(LofParams)]
    L.lof_default_params.restype = ctypes.c_int
    L.lof_create.argtypes = [ctypes.POINTER(LofParams), ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]
    L.lof_create.restype = ctypes.c_int
    L.lof_flag_blocks.argtypes = [ctypes.c_void_p, ctypes.POINTER(LofBlock), ctypes.c_int32,
                                  ctypes.c_void_p, ctypes.c_void_p]
    L.lof_flag_blocks.restype = ctypes.c_int
    L.lof_history_update.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                     ctypes.c_void_p]
    L.lof_history_update.restype = ctypes.c_int
    L.lof_history_export.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]
    L.lof_history_export.restype = ctypes.c_int
    L.lof_get_tuning.argtypes = [ctypes.c_void_p, ctypes.POINTER(LofTuning)]
    L.lof_get_tuning.restype = ctypes.c_int
    L.lof_set_tuning.argtypes = [ctypes.c_void_p, ctypes.POINTER(LofTuning)]
    L.lof_set_tuning.restype = ctypes.c_int
    L.lof_autotune.argtypes = [ctypes.c_void_p, ctypes.POINTER(LofBlock), ctypes.c_int32, ctypes.c_void_p,
                               ctypes.c_int32, ctypes.POINTER(LofTuning)]
    L.lof_autotune.restype = ctypes.c_int
    L.lof_destroy.argtypes = [ctypes.c_void_p]
    L.lof_destroy.restype = ctypes.c_int
    L.lof_phase_times.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]
    L.lof_phase_times.restype = ctypes.c_int
    L.lof_flag_blocks_static.argtypes = [ctypes.POINTER(LofParams), ctypes.c_int, ctypes.POINTER(LofBlock),
                                         ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    L.lof_flag_blocks_static.restype = ctypes.c_int
    L.lof_last_error.argtypes = [ctypes.c_void_p]
    L.lof_last_error.restype = ctypes.c_char_p
    _lib = L
    return L
