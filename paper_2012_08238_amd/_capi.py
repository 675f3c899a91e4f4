"""ctypes declarations of the C ABI in ``include/sfft.h`` (marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsfft_mi355x.so")

SFFT_OK = 0
SFFT_E_INVALID = -1
SFFT_E_NOMEM = -2
SFFT_E_DEVICE = -3
SFFT_E_UNSUPPORTED = -4
SFFT_E_BUSY = -5
SFFT_E_NOTFOUND = -6

SFFT_FLAG_NO_RESIDUAL = 0x1
SFFT_FLAG_FOLD_GATHER = 0x2
SFFT_FLAG_FOLD_STRIP = 0x4
SFFT_FLAG_XCD_ORDER = 0x8
SFFT_FLAG_MEAN_ESTIMATE = 0x10
SFFT_FLAG_ITERATE = 0x20
SFFT_FLAG_PHASE_LOCATION = 0x40
SFFT_FLAG_FFT_TWO_PASS = 0x80
SFFT_FLAG_VOTE_BY_LOOP = 0x100
SFFT_FLAG_VOTE_BY_PAIR = 0x200
SFFT_FLAG_FUSED = 0x400


class Params(C.Structure):
    _fields_ = [("N", C.c_int64), ("K", C.c_int32), ("B", C.c_int32), ("L", C.c_int32),
                ("d", C.c_int32), ("w", C.c_int64), ("seed", C.c_uint64),
                ("vote_threshold", C.c_int32), ("n_resid", C.c_int32), ("gauss_c", C.c_double),
                ("flags", C.c_uint32), ("strip_cols", C.c_int32),
                ("sigma", C.POINTER(C.c_uint32)), ("tau", C.POINTER(C.c_uint32)),
                ("comb_b", C.c_int32), ("comb_loops", C.c_int32), ("comb_keep", C.c_int32),
                ("est_loops", C.c_int32), ("est_B", C.c_int32), ("est_w", C.c_int64)]


class PlanDesc(C.Structure):
    _fields_ = [("N", C.c_int64), ("w", C.c_int64), ("K", C.c_int32), ("B", C.c_int32),
                ("L", C.c_int32), ("d", C.c_int32), ("T", C.c_int32), ("n_resid", C.c_int32),
                ("fold_mode", C.c_int32), ("strip_cols", C.c_int32), ("cand_cap", C.c_int64),
                ("table_bytes", C.c_size_t), ("workspace_bytes", C.c_size_t),
                ("sampled_fraction_expected", C.c_double),
                ("sub_reach_lo", C.c_int32), ("sub_reach_hi", C.c_int32), ("sub_tail_bound", C.c_double),
                ("vote_pairs", C.c_int32), ("vote_pair", C.c_uint16 * 32)]


class Trace(C.Structure):
    _fields_ = [("uhat", C.POINTER(C.c_float)), ("jbits", C.POINTER(C.c_uint32)),
                ("jlist", C.POINTER(C.c_uint32)), ("cand", C.POINTER(C.c_uint32)),
                ("cand_count", C.c_int64), ("cbits", C.POINTER(C.c_uint32)),
                ("rec_idx", C.POINTER(C.c_uint32)), ("rec_val", C.POINTER(C.c_float)), ("rec_count", C.c_int64)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("rejected", C.c_uint64),
                ("failed", C.c_uint64), ("batches", C.c_uint64), ("max_batch", C.c_uint64),
                ("max_waves_in_flight", C.c_uint64),
                ("p50_latency_s", C.c_double), ("p99_latency_s", C.c_double), ("mean_latency_s", C.c_double),
                ("hbm_in_use", C.c_size_t), ("hbm_peak", C.c_size_t), ("hbm_budget", C.c_size_t),
                ("plan_cache_hits", C.c_uint64), ("plan_cache_misses", C.c_uint64),
                ("plan_cache_evictions", C.c_uint64)]


# (name, restype, argtypes) of every exported entry point
SIGNATURES = [
    ("sfft_params_init", C.c_int, [C.POINTER(Params), C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int64]),
    ("sfft_plan", C.c_int, [C.POINTER(C.c_void_p), C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int64]),
    ("sfft_plan_ex", C.c_int, [C.POINTER(C.c_void_p), C.POINTER(Params)]),
    ("sfft_destroy", C.c_int, [C.c_void_p]),
    ("sfft_plan_get_perms", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("sfft_plan_describe", C.c_int, [C.c_void_p, C.POINTER(PlanDesc)]),
    ("sfft_params_describe", C.c_int, [C.POINTER(Params), C.POINTER(PlanDesc)]),
    ("sfft_host_tables", C.c_int, [C.POINTER(Params), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p]),
    ("sfft_execute", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("sfft_execute_ex", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("sfft_execute_noalloc", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("sfft_plan_read_trace", C.c_int, [C.c_void_p, C.POINTER(Trace)]),
    ("sfft_batch_create", C.c_int, [C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_int32]),
    ("sfft_batch_create_ex", C.c_int, [C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_int32, C.c_int32]),
    ("sfft_batch_run", C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                 C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_void_p]),
    ("sfft_batch_run_timed", C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                       C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_void_p,
                                       C.c_void_p, C.c_void_p]),
    ("sfft_batch_destroy", C.c_int, [C.c_void_p]),
    ("sfft_execute_batch", C.c_int, [C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                     C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_int32, C.c_void_p]),
    ("sfft_server_create", C.c_int, [C.POINTER(C.c_void_p), C.c_size_t, C.c_int32, C.c_int32]),
    ("sfft_server_prepare", C.c_int, [C.c_void_p, C.POINTER(Params)]),
    ("sfft_server_submit", C.c_int, [C.c_void_p, C.POINTER(Params), C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.POINTER(C.c_uint64)]),
    ("sfft_server_submit_batch", C.c_int, [C.c_void_p, C.POINTER(Params), C.c_int32, C.POINTER(C.c_void_p),
                                           C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                           C.POINTER(C.c_uint64)]),
    ("sfft_server_poll", C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                   C.POINTER(C.c_int32)]),
    ("sfft_server_wait", C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    ("sfft_server_stats_get", C.c_int, [C.c_void_p, C.POINTER(ServerStats)]),
    ("sfft_server_destroy", C.c_int, [C.c_void_p]),
    ("sfft_status_string", C.c_char_p, [C.c_int]),
    ("sfft_last_error", C.c_char_p, []),
    ("sfft_version", C.c_char_p, []),
]

_lib = None


def load(path: str | None = None) -> C.CDLL:
    """Load the HIP library; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"HIP library {p} is missing: run __graft_entry__.build() "
                           "(or python paper_2012_08238_amd/build.py) first")
    lib = C.CDLL(p)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


class SfftError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


def check(status: int, where: str) -> None:
    if status != SFFT_OK:
        lib = load()
        raise SfftError(status, where, (lib.sfft_last_error() or b"").decode())
