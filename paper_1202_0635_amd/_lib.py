"""ctypes declarations of libswmc (include/sw.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libswmc.so")

SW_OK, SW_EINVAL, SW_ENOMEM, SW_EDEVICE, SW_ESTATE, SW_EBUDGET, SW_EBUSY = 0, -1, -2, -3, -4, -5, -6
SW_POTTS, SW_CLOCK = 0, 1
SW_MEASURE, SW_VERIFY, SW_PROFILE, SW_NO_GRAPH, SW_HASH = 1, 2, 4, 8, 16


class SwLattice(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32),
        ("q", ctypes.c_int32),
        ("model", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("T", ctypes.c_double),
        ("J", ctypes.c_double),
        ("seed", ctypes.c_uint64),
    ]


class SwObs(ctypes.Structure):
    _fields_ = [
        ("sweeps_done", ctypes.c_uint64),
        ("samples", ctypes.c_uint64),
        ("hist", ctypes.c_int64 * 32),
        ("pair_hist", ctypes.c_int64 * 32),
        ("e_per_site", ctypes.c_double),
        ("m2", ctypes.c_double),
        ("mean_e", ctypes.c_double),
        ("mean_m2", ctypes.c_double),
        ("mean_m4", ctypes.c_double),
        ("binder_u", ctypes.c_double),
        ("corr_hist", (ctypes.c_int64 * 32) * 2),
        ("g_quarter", ctypes.c_double),
        ("g_half", ctypes.c_double),
        ("mean_g_quarter", ctypes.c_double),
        ("mean_g_half", ctypes.c_double),
        ("corr_ratio", ctypes.c_double),
        ("absm", ctypes.c_double),
        ("hash_spins", ctypes.c_uint64),
        ("hash_labels", ctypes.c_uint64),
    ]


class SwRequest(ctypes.Structure):
    _fields_ = [("lattice", SwLattice), ("sweeps", ctypes.c_int64), ("tag", ctypes.c_uint64),
                ("t_arrival", ctypes.c_double)]


class SwResult(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("obs", SwObs), ("spin_hash", ctypes.c_uint64), ("t_arrival", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class SwServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("waiting", ctypes.c_int64), ("active", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("rejected", ctypes.c_int64), ("steps", ctypes.c_int64),
                ("spin_updates", ctypes.c_int64), ("budget_bytes", ctypes.c_uint64), ("used_bytes", ctypes.c_uint64)]


class SwError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {detail} (status {status})")
        self.status = status


_lib = None

# name -> (restype, argtypes); every exported symbol of include/sw.h
SIGNATURES = {
    "sw_state_bytes": (ctypes.c_size_t, [ctypes.POINTER(SwLattice)]),
    "sw_init": (ctypes.c_int, [ctypes.POINTER(SwLattice), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                               ctypes.POINTER(ctypes.c_void_p)]),
    "sw_sweep": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32]),
    "sw_measure": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SwObs)]),
    "sw_read_hashes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                      ctypes.POINTER(ctypes.c_size_t)]),
    "sw_read_spins": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "sw_read_labels": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "sw_read_bonds": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "sw_write_spins": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint64]),
    "sw_device_spins": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "sw_cutoff_table": (ctypes.c_int, [ctypes.POINTER(SwLattice), ctypes.c_void_p, ctypes.c_size_t]),
    "sw_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_char_p),
                                       ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                       ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "sw_set_tile_waves": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "sw_set_labeler": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "sw_labeler_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]),
    "sw_tune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "sw_free": (None, [ctypes.c_void_p]),
    "sw_sweep_static": (ctypes.c_int, [ctypes.POINTER(SwLattice), ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sw_batch_bytes": (ctypes.c_size_t, [ctypes.POINTER(SwLattice), ctypes.c_int32]),
    "sw_batch_init": (ctypes.c_int, [ctypes.POINTER(SwLattice), ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t,
                                     ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "sw_batch_sweep": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32]),
    "sw_batch_measure": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(SwObs)]),
    "sw_batch_read_spins": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t]),
    "sw_batch_read_labels": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t]),
    "sw_batch_read_hashes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t,
                                            ctypes.POINTER(ctypes.c_size_t)]),
    "sw_batch_size": (ctypes.c_int32, [ctypes.c_void_p]),
    "sw_batch_set_schedule": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "sw_batch_set_tile_waves": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "sw_batch_tune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32)]),
    "sw_batch_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_char_p),
                                             ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                             ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "sw_batch_free": (None, [ctypes.c_void_p]),
    "sw_server_create": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "sw_server_now": (ctypes.c_double, [ctypes.c_void_p]),
    "sw_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SwRequest)]),
    "sw_server_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "sw_server_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SwResult), ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_int32)]),
    "sw_server_stats_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SwServerStats)]),
    "sw_server_destroy": (None, [ctypes.c_void_p]),
    "sw_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "sw_last_error": (ctypes.c_char_p, []),
}


def lib() -> ctypes.CDLL:
    """Load the in-tree HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -m paper_1202_0635_amd.build, or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status: int, where: str) -> None:
    if status != SW_OK:
        detail = lib().sw_last_error().decode(errors="replace")
        raise SwError(status, where, detail or lib().sw_strerror(status).decode())
