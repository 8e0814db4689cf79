"""ctypes declarations of the C ABI in include/chain_rk4.h.

Loading fails loudly when the HIP library has not been built: there is no
fallback implementation of any part of the path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchainrk4.so")

CHAIN_QUARTIC, CHAIN_HARMONIC, CHAIN_ROESSLER = 0, 1, 2
CHAIN_QUARTIC_NNN, CHAIN_HARMONIC_NNN = 3, 4
CHAIN_FP64, CHAIN_FP32_KAHAN, CHAIN_FP32_KAHAN64, CHAIN_FP32 = 0, 1, 2, 3
CHAIN_FUSED, CHAIN_NAIVE = 0, 1
CHAIN_FLAG_GRAPH, CHAIN_FLAG_NO_RESIDENT, CHAIN_FLAG_RESIDENT = 1, 2, 4
CHAIN_FLAG_EXCHANGE = 8
CHAIN_BATCH_FENCES, CHAIN_BATCH_RESIDENT_RINGS, CHAIN_BATCH_WIDE_ONLY = 1, 2, 4
CHAIN_SCHEME_RK4, CHAIN_SCHEME_TABLEAU = 0, 1
CHAIN_MAX_STAGES = 8

CHAIN_OK = 0
CHAIN_EINVAL = -1
CHAIN_ENOMEM = -2
CHAIN_EHIP = -3
CHAIN_ENONFINITE = -4
CHAIN_EDEVICE = -5
CHAIN_ETIMEOUT = -6


class Desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("model", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("dt", ctypes.c_double), ("method", ctypes.c_int32),
                ("sites_per_lane", ctypes.c_int32), ("kdepth", ctypes.c_int32),
                ("waves_per_cluster", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("scheme", ctypes.c_int32)]


class Plan(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("sites_per_lane", ctypes.c_int32),
                ("kdepth", ctypes.c_int32), ("resident", ctypes.c_int32),
                ("waves_per_cluster", ctypes.c_int32), ("exchange", ctypes.c_int32),
                ("tile", ctypes.c_int64), ("halo", ctypes.c_int64), ("waves", ctypes.c_int64),
                ("overlap_factor", ctypes.c_double)]


class Tableau(ctypes.Structure):
    _fields_ = [("stages", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("a", (ctypes.c_double * CHAIN_MAX_STAGES) * CHAIN_MAX_STAGES),
                ("b", ctypes.c_double * CHAIN_MAX_STAGES)]


class BatchDesc(ctypes.Structure):
    _fields_ = [("max_steps", ctypes.c_int64), ("max_clusters", ctypes.c_int64),
                ("sites_per_lane", ctypes.c_int32), ("kdepth", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("spin_limit", ctypes.c_int32), ("max_chains", ctypes.c_int32)]


class BatchPlan(ctypes.Structure):
    _fields_ = [("sites_per_lane", ctypes.c_int32), ("kdepth", ctypes.c_int32),
                ("waves_per_cluster", ctypes.c_int32), ("grid_blocks", ctypes.c_int32),
                ("halo", ctypes.c_int64), ("tile_max", ctypes.c_int64),
                ("total_clusters", ctypes.c_int64), ("resident_chains", ctypes.c_int64),
                ("tile_narrow", ctypes.c_int64), ("narrow_clusters", ctypes.c_int64)]


class ChainError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: status {status}: {detail}")


_lib = None

VP = ctypes.c_void_p
H = ctypes.c_void_p  # opaque handle


def _declare(lib):
    D = ctypes.POINTER(Desc)
    sig = {
        "chain_rk4_workspace_bytes": (ctypes.c_size_t, [D]),
        "chain_rk4_create": (ctypes.c_int, [D, VP, VP, VP, ctypes.c_size_t, VP,
                                            ctypes.POINTER(H)]),
        "chain_rk4_create3": (ctypes.c_int, [D, VP, VP, VP, VP, ctypes.c_size_t, VP,
                                             ctypes.POINTER(H)]),
        "chain_rk4_step": (ctypes.c_int, [H, ctypes.c_int64]),
        "chain_rk4_set_tableau": (ctypes.c_int, [H, ctypes.POINTER(Tableau)]),
        "chain_rk4_tableau_reach": (ctypes.c_int64, [ctypes.c_int32, ctypes.POINTER(Tableau)]),
        "chain_rk4_energy": (ctypes.c_int, [H, ctypes.POINTER(ctypes.c_double)]),
        "chain_rk4_energy_noalloc": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32,
                                                    ctypes.c_int64, VP, VP, VP, VP, VP,
                                                    ctypes.POINTER(ctypes.c_double)]),
        "chain_rk4_set_stream": (ctypes.c_int, [H, VP]),
        "chain_rk4_get_plan": (ctypes.c_int, [H, ctypes.POINTER(Plan)]),
        "chain_rk4_plan_for": (ctypes.c_int, [D, ctypes.POINTER(Tableau), ctypes.POINTER(Plan)]),
        "chain_rk4_get_carries": (ctypes.c_int, [H, ctypes.POINTER(VP), ctypes.POINTER(VP)]),
        "chain_rk4_destroy": (ctypes.c_int, [H]),
        "chain_rk4_check": (ctypes.c_int, [H]),
        "chain_rk4_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "chain_rk4_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(H), ctypes.c_int,
                                                              ctypes.POINTER(BatchDesc)]),
        "chain_rk4_batch_create": (ctypes.c_int, [ctypes.POINTER(H), ctypes.c_int,
                                                  ctypes.POINTER(BatchDesc), VP, ctypes.c_size_t,
                                                  VP, ctypes.POINTER(VP)]),
        "chain_rk4_batch_step": (ctypes.c_int, [VP, ctypes.POINTER(ctypes.c_int64)]),
        "chain_rk4_batch_rebind": (ctypes.c_int, [VP, ctypes.POINTER(H), ctypes.c_int]),
        "chain_rk4_batch_clusters": (ctypes.c_int64, [ctypes.c_int64, ctypes.c_int32,
                                                      ctypes.c_int32]),
        "chain_rk4_batch_check": (ctypes.c_int, [VP]),
        "chain_rk4_batch_last_launch": (ctypes.c_int, [VP, ctypes.POINTER(ctypes.c_int64)]),
        "chain_rk4_batch_check_launch": (ctypes.c_int, [VP, ctypes.c_int64]),
        "chain_rk4_batch_layout": (ctypes.c_int64, [ctypes.c_int64, ctypes.POINTER(BatchDesc),
                                                    ctypes.POINTER(ctypes.c_int64),
                                                    ctypes.POINTER(ctypes.c_int64),
                                                    ctypes.POINTER(ctypes.c_int32), ctypes.c_int64]),
        "chain_rk4_batch_plan_for": (ctypes.c_int, [ctypes.POINTER(BatchDesc),
                                                    ctypes.POINTER(BatchPlan)]),
        "chain_rk4_batch_energy": (ctypes.c_int, [VP, ctypes.POINTER(ctypes.c_double)]),
        "chain_rk4_batch_get_plan": (ctypes.c_int, [VP, ctypes.POINTER(BatchPlan)]),
        "chain_rk4_batch_destroy": (ctypes.c_int, [VP]),
        "chain_rk4_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def lib():
    """The loaded HIP library (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1412_0544_amd.build`")
        _lib = _declare(ctypes.CDLL(LIB_PATH))
    return _lib


def check(status: int, where: str) -> None:
    if status != CHAIN_OK:
        L = lib()
        detail = (L.chain_rk4_last_error() or b"").decode() or L.chain_rk4_strerror(status).decode()
        raise ChainError(status, where, detail)
