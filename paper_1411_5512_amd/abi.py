"""ctypes binding of the C ABI in include/ea.h (argument marshalling only).

Every step of the simulation runs in the gfx950 library ``libea.so``; this
module loads it, declares the signatures and converts between numpy arrays and
pointers.  There is no fallback: if the library is missing or cannot be
loaded, :func:`lib` raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libea.so")

EA_OK, EA_ERR_ARG, EA_ERR_NOMEM, EA_ERR_DEVICE, EA_ERR_STATE, EA_ERR_BUSY = 0, -1, -2, -3, -4, -5


class EAError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"ea status {status}: {message}")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32),
        ("p", ctypes.c_double),
        ("T", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("sample", ctypes.c_uint32),
        ("n_tw_slots", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
        ("dev_buf", ctypes.c_void_p),
        ("dev_buf_bytes", ctypes.c_size_t),
        ("words_per_row", ctypes.c_int32),
    ]


class MscConfig(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32),
        ("n_samples", ctypes.c_int32),
        ("p", ctypes.c_double),
        ("T", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("sample0", ctypes.c_uint32),
        ("shared", ctypes.c_uint32),
        ("n_tw_slots", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
        ("dev_buf", ctypes.c_void_p),
        ("dev_buf_bytes", ctypes.c_size_t),
    ]


class Obs(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_uint64),
        ("unsat", ctypes.c_int64 * 2),
        ("mag", ctypes.c_int64 * 2),
        ("overlap", ctypes.c_int64),
        ("n_tw", ctypes.c_int32),
        ("tw", ctypes.POINTER(ctypes.c_uint64)),
        ("autocorr", ctypes.POINTER(ctypes.c_int64)),
        ("rmax", ctypes.c_int32),
        ("c4", ctypes.POINTER(ctypes.c_int64)),
    ]


class Job(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32),
        ("p", ctypes.c_double),
        ("T", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("sample", ctypes.c_uint32),
        ("n_sweeps", ctypes.c_uint64),
        ("meas_t", ctypes.POINTER(ctypes.c_uint64)),
        ("n_meas", ctypes.c_int32),
        ("tw", ctypes.POINTER(ctypes.c_uint64)),
        ("n_tw", ctypes.c_int32),
    ]


class BatchOpts(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_void_p), ("autotune", ctypes.c_int32), ("split", ctypes.c_int32)]


class TuneChoice(ctypes.Structure):
    _fields_ = [
        ("words_per_row", ctypes.c_int32),
        ("threads", ctypes.c_int32),
        ("select", ctypes.c_int32),
        ("ms", ctypes.c_double),
        ("parity_ok", ctypes.c_int32),
    ]


class ServerOpts(ctypes.Structure):
    _fields_ = [
        ("hbm_budget", ctypes.c_size_t),
        ("max_resident", ctypes.c_int32),
        ("max_pending", ctypes.c_int32),
        ("epoch_site_sweeps", ctypes.c_uint64),
        ("stream", ctypes.c_void_p),
    ]


class ServerReport(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_uint64),
        ("admitted", ctypes.c_uint64),
        ("completed", ctypes.c_uint64),
        ("epochs", ctypes.c_uint64),
        ("resident", ctypes.c_int32),
        ("pending", ctypes.c_int32),
        ("p50_latency_s", ctypes.c_double),
        ("p99_latency_s", ctypes.c_double),
        ("mean_latency_s", ctypes.c_double),
        ("max_latency_s", ctypes.c_double),
        ("flips", ctypes.c_double),
        ("busy_s", ctypes.c_double),
        ("wall_s", ctypes.c_double),
        ("ps_per_flip", ctypes.c_double),
        ("hbm_in_use", ctypes.c_size_t),
        ("hbm_peak", ctypes.c_size_t),
        ("streamed_small", ctypes.c_uint64),
        ("moved", ctypes.c_uint64),
    ]


# name -> (restype, argtypes)
_SIGS = {
    "ea_last_error": (ctypes.c_char_p, []),
    "ea_version": (ctypes.c_char_p, []),
    "ea_footprint": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "ea_thresholds": (ctypes.c_int, [ctypes.c_double, ctypes.POINTER(ctypes.c_uint32)]),
    "ea_set_debug": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32]),
    "ea_get_debug": (ctypes.c_int, [ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32)]),
    "ea_set_shell_route": (ctypes.c_int, [ctypes.c_int32]),
    "ea_get_shell_route": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int32)]),
    "ea_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                 ctypes.POINTER(ctypes.c_void_p)]),
    "ea_create_ex": (ctypes.c_int, [ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_void_p)]),
    "ea_destroy": (None, [ctypes.c_void_p]),
    "ea_msc_footprint": (ctypes.c_int, [ctypes.POINTER(MscConfig), ctypes.POINTER(ctypes.c_size_t)]),
    "ea_msc_create": (ctypes.c_int, [ctypes.POINTER(MscConfig), ctypes.POINTER(ctypes.c_void_p)]),
    "ea_msc_destroy": (None, [ctypes.c_void_p]),
    "ea_msc_sweep": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "ea_msc_snapshot": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "ea_msc_measure": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Obs)]),
    "ea_msc_get_spins": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int8)]),
    "ea_msc_set_spins": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int8)]),
    "ea_msc_get_bonds": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int8)]),
    "ea_msc_time": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "ea_msc_set_time": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "ea_msc_sync": (ctypes.c_int, [ctypes.c_void_p]),
    "ea_reset": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32]),
    "ea_sweep": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "ea_sweep_group": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.c_uint64]),
    "ea_snapshot": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "ea_measure": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Obs)]),
    "ea_time": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "ea_set_time": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "ea_sync": (ctypes.c_int, [ctypes.c_void_p]),
    "ea_set_slab_plan": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]),
    "ea_get_slab_plan": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32)]),
    "ea_get_spins": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int8)]),
    "ea_set_spins": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int8)]),
    "ea_get_bonds": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int8)]),
    "ea_set_bonds": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int8)]),
    "ea_batch_create": (ctypes.c_int, [ctypes.POINTER(Job), ctypes.c_int32, ctypes.POINTER(BatchOpts),
                                       ctypes.POINTER(ctypes.c_void_p)]),
    "ea_batch_destroy": (None, [ctypes.c_void_p]),
    "ea_batch_reset": (ctypes.c_int, [ctypes.c_void_p]),
    "ea_batch_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "ea_c4_shells": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
    "ea_c4_shells_into": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "ea_batch_c4_shells": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_int64)]),
    "ea_msc_c4_shells": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int64)]),
    "ea_tune_plain": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(TuneChoice), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "ea_footprint_ex": (ctypes.c_int, [ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_size_t)]),
    "ea_words_per_row": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "ea_tune": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(TuneChoice),
                               ctypes.POINTER(TuneChoice), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "ea_batch_capture": (ctypes.c_int, [ctypes.c_void_p]),
    "ea_batch_replay": (ctypes.c_int, [ctypes.c_void_p]),
    "ea_batch_time": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)]),
    "ea_batch_result": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Obs)]),
    "ea_batch_get_spins": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_int8)]),
    "ea_batch_parts": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "ea_server_create": (ctypes.c_int, [ctypes.POINTER(ServerOpts), ctypes.POINTER(ctypes.c_void_p)]),
    "ea_server_destroy": (None, [ctypes.c_void_p]),
    "ea_server_footprint": (ctypes.c_int, [ctypes.POINTER(Job), ctypes.POINTER(ctypes.c_size_t)]),
    "ea_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Job), ctypes.POINTER(ctypes.c_uint64)]),
    "ea_server_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "ea_server_start": (ctypes.c_int, [ctypes.c_void_p]),
    "ea_server_stop": (ctypes.c_int, [ctypes.c_void_p]),
    "ea_server_drain": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double]),
    "ea_server_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32)]),
    "ea_server_result": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.POINTER(Obs)]),
    "ea_server_latency": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]),
    "ea_server_release": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "ea_server_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ServerReport)]),
}

_lib = None


def lib():
    """Load libea.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                              "python paper_1411_5512_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int):
    if status != EA_OK:
        msg = lib().ea_last_error().decode(errors="replace")
        raise EAError(status, msg)


def ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def exported_names():
    return list(_SIGS)
