"""ctypes binding of libdedisp (include/dedisp.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# DEDISP_LIB may name another build of the same library (the host-sanitized one)
LIB_PATH = os.environ.get("DEDISP_LIB") or os.path.join(_HERE, "libdedisp.so")

OK, ERR_INVALID_ARG, ERR_SHAPE, ERR_OVERFLOW, ERR_OOM, ERR_DEVICE, ERR_UNSUPPORTED = range(7)
U8, F32, I32 = 0, 1, 2
RULE_SMEAR, RULE_ALLNONZERO, RULE_GREEDY, RULE_EXPLICIT, RULE_FIXED = range(5)
W_UNIT, W_CHANNEL, W_TAP = range(3)

RULES = {"smear": RULE_SMEAR, "allnonzero": RULE_ALLNONZERO, "greedy": RULE_GREEDY,
         "explicit": RULE_EXPLICIT, "fixed": RULE_FIXED}
WMODES = {"unit": W_UNIT, "channel": W_CHANNEL, "tap": W_TAP}

# Every entry point declared in include/dedisp.h.
EXPORTS = [
    "dedisp_profile_init", "dedisp_plan_create", "dedisp_plan_destroy", "dedisp_plan_tables",
    "dedisp_plan_info", "dedisp_plan_out_len", "dedisp_dedisperse", "dedisp_work_bytes",
    "dedisp_detect", "dedisp_merge_candidates", "dedisp_check_search_tables", "dedisp_search", "dedisp_search_noalloc",
    "dedisp_dedisperse_backward",
    "dedisp_backward_sparse",
    "dedisp_dedisperse_gather", "dedisp_trial_dms", "dedisp_batch_create", "dedisp_batch_destroy",
    "dedisp_batch_work_bytes", "dedisp_batch_run", "dedisp_batch_info", "dedisp_autotune",
    "dedisp_set_tile", "dedisp_last_search_tile", "dedisp_set_kernel_events", "dedisp_status_string", "dedisp_last_error",
]


class Profile(ctypes.Structure):
    _fields_ = [
        ("rule", ctypes.c_int32),
        ("k_dm", ctypes.c_double),
        ("width_s", ctypes.c_double),
        ("scatter_s_1ghz", ctypes.c_double),
        ("scatter_index", ctypes.c_double),
        ("spectral_index", ctypes.c_double),
        ("nu0_ghz", ctypes.c_double),
        ("start", ctypes.c_void_p),
        ("ntap", ctypes.c_void_p),
        ("ktaps", ctypes.c_int32),
        ("wmode", ctypes.c_int32),
        ("weights", ctypes.c_void_p),
    ]


class DedispError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libdedisp status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libdedisp.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libdedisp.so not built at {LIB_PATH}; run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, sz, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_double
    sig = {
        "dedisp_profile_init": [P],
        "dedisp_plan_create": [P, i32, P, d, d, i32, P, P],
        "dedisp_plan_destroy": [P],
        "dedisp_plan_tables": [P, P, P],
        "dedisp_plan_info": [P, P, P, P, P, P],
        "dedisp_plan_out_len": [P, i64, P],
        "dedisp_dedisperse": [P, P, i32, i64, i64, i64, i32, P, i32, i64, i64, P, P],
        "dedisp_work_bytes": [P, i64, i32, P],
        "dedisp_detect": [P, P, i32, i64, i64, P, i32, P, P, P, P, P, P, sz, P],
        "dedisp_search": [P, P, i32, i64, i64, P, i32, P, P, P, P, P, P, sz, P],
        "dedisp_search_noalloc": [P, P, i32, i64, i64, P, i32, P, P, P, P, P, P],
        "dedisp_merge_candidates": [i32, P, P, P, i64, P, P, P, P],
        "dedisp_check_search_tables": [P, i32, P],
        "dedisp_dedisperse_backward": [P, P, i64, i64, i64, i32, P, i32, i64, i64, i64, P, P, P, P],
        "dedisp_backward_sparse": [P, i32, P, P, P, P, P, i32, i64, i64, i64, i32, P, P],
        "dedisp_dedisperse_gather": [P, i32, P, P, P, P, i32, i64, i64, i64, i32, P, P, P],
        "dedisp_trial_dms": [d, d, d, i32, P, d, d, d, i32, d, i32, P, P],
        "dedisp_batch_create": [P, i32, P, P, P, i32],
        "dedisp_batch_destroy": [P],
        "dedisp_batch_work_bytes": [P, P],
        "dedisp_batch_run": [P, P, P, P, P, P, P, P, P, sz, i32, P],
        "dedisp_batch_info": [P, P, P],
        "dedisp_autotune": [P, P, i64, i64, P, i32, P, P, P, sz, P, P],
        "dedisp_set_tile": [P, i32],
        "dedisp_set_kernel_events": [P, P, P, i32],
        "dedisp_last_search_tile": [P, P],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.dedisp_status_string.argtypes = [ctypes.c_int]
    L.dedisp_status_string.restype = ctypes.c_char_p
    L.dedisp_last_error.argtypes = []
    L.dedisp_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def check(status: int) -> None:
    if status != OK:
        msg = lib().dedisp_last_error().decode(errors="replace")
        raise DedispError(status, msg)
