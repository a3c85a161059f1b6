"""ctypes declarations of the C ABI in include/potts.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpotts.so")

POTTS_QMAX = 256
ERRORS = {0: "ok", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ERANGE", -5: "EIO"}


class PottsError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{ERRORS.get(code, code)}: {message}")
        self.code = code


class PottsObs(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_int64),
        ("e_sat", ctypes.c_int64),
        ("nmax", ctypes.c_int64),
        ("q", ctypes.c_int32),
        ("L", ctypes.c_int32),
        ("hist", ctypes.c_int64 * POTTS_QMAX),
    ]


class PottsSummary(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("e", ctypes.c_double),
        ("C", ctypes.c_double),
        ("V_L", ctypes.c_double),
        ("m", ctypes.c_double),
        ("chi", ctypes.c_double),
    ]


class PottsJob(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32),
        ("q", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("start", ctypes.c_int32),
        ("_pad", ctypes.c_int32),
        ("beta", ctypes.c_double),
        ("nsweeps", ctypes.c_int64),
    ]


class PottsJobResult(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_int64),
        ("e_sat", ctypes.c_int64),
        ("nmax", ctypes.c_int64),
        ("stats", PottsSummary),
    ]


class PottsBatchOpts(ctypes.Structure):
    _fields_ = [
        ("graph", ctypes.c_int32),
        ("tune", ctypes.c_int32),
        ("window", ctypes.c_int32),
        ("strip_rows", ctypes.c_int32),
        ("hip_stream", ctypes.c_void_p),
        ("tune_cache", ctypes.c_char_p),
    ]


class PottsServerCfg(ctypes.Structure):
    _fields_ = [
        ("hbm_budget", ctypes.c_int64),
        ("max_slots", ctypes.c_int32),
        ("quantum", ctypes.c_int32),
        ("hip_stream", ctypes.c_void_p),
        ("tune", ctypes.c_int32),
        ("_pad", ctypes.c_int32),
        ("tune_cache", ctypes.c_char_p),
    ]


class PottsRequest(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32),
        ("q", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("start", ctypes.c_int32),
        ("npoints", ctypes.c_int32),
        ("betas", ctypes.POINTER(ctypes.c_double)),
        ("sweeps", ctypes.POINTER(ctypes.c_int64)),
        ("keep_spins", ctypes.c_int32),
        ("_pad", ctypes.c_int32),
        ("checkpoint", ctypes.c_char_p),
        ("resume_from", ctypes.c_char_p),
    ]


class PottsServed(ctypes.Structure):
    _fields_ = [
        ("ticket", ctypes.c_int64),
        ("L", ctypes.c_int32),
        ("q", ctypes.c_int32),
        ("npoints", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("sweeps", ctypes.c_int64),
        ("t_submit", ctypes.c_double),
        ("t_admit", ctypes.c_double),
        ("t_done", ctypes.c_double),
        ("e_sat", ctypes.c_int64),
        ("nmax", ctypes.c_int64),
    ]


class PottsNnnObs(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_int64),
        ("e1", ctypes.c_int64),
        ("e2", ctypes.c_int64),
        ("nmax", ctypes.c_int64),
        ("q", ctypes.c_int32),
        ("L", ctypes.c_int32),
        ("hist", ctypes.c_int64 * POTTS_QMAX),
    ]


_lib = None

# (name, restype, argtypes) for every exported symbol declared in include/potts.h
_VP = ctypes.c_void_p
_U32P = ctypes.POINTER(ctypes.c_uint32)
_I64P = ctypes.POINTER(ctypes.c_int64)
_U8P = ctypes.POINTER(ctypes.c_uint8)
SIGNATURES = [
    ("potts_init", ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(_VP)]),
    ("potts_init_ex", ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int, _VP, _VP,
                                     ctypes.c_size_t, _VP, ctypes.c_int64, ctypes.POINTER(_VP)]),
    ("potts_sweep", ctypes.c_int, [_VP, ctypes.c_double, ctypes.c_int64]),
    ("potts_sweep_thr", ctypes.c_int, [_VP, _U32P, ctypes.c_int64]),
    ("potts_sweep_heatbath", ctypes.c_int, [_VP, ctypes.c_double, ctypes.c_int64]),
    ("potts_sweep_heatbath_thr", ctypes.c_int, [_VP, _U32P, ctypes.c_int64]),
    ("potts_threshold_table", ctypes.c_int, [ctypes.c_double, _U32P]),
    ("potts_tune_occupancy", ctypes.c_int, [_VP, ctypes.c_int32]),
    ("potts_tune_graph", ctypes.c_int, [_VP, ctypes.c_int32]),
    ("potts_tune_tiles", ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    ("potts_tune_band", ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32]),
    ("potts_tune", ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    ("potts_slab_half_sweep", ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                             ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, _U32P, _VP,
                                             ctypes.c_int64, _VP]),
    ("potts_slab_records", ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                          ctypes.c_int64, _VP, _VP]),
    ("potts_sweep_static", ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64,
                                          _U32P, ctypes.c_int64, _VP, _VP]),
    ("potts_observables", ctypes.c_int, [_VP, ctypes.POINTER(PottsObs)]),
    ("potts_measure", ctypes.c_int, [_VP, ctypes.POINTER(PottsObs)]),
    ("potts_records", ctypes.c_int, [_VP, ctypes.c_int64, ctypes.c_int64, _I64P]),
    ("potts_stats", ctypes.c_int, [_VP, ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                                   ctypes.POINTER(PottsSummary)]),
    ("potts_reweight", ctypes.c_int, [_VP, ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                                      ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                      ctypes.POINTER(PottsSummary)]),
    ("potts_reserve_records", ctypes.c_int, [_VP, ctypes.c_int64]),
    ("potts_ramp", ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_int64, ctypes.POINTER(PottsSummary)]),
    ("potts_get_spins", ctypes.c_int, [_VP, _U8P]),
    ("potts_set_spins", ctypes.c_int, [_VP, _U8P, ctypes.c_int64]),
    ("potts_device_spins", _VP, [_VP]),
    ("potts_time", ctypes.c_int64, [_VP]),
    ("potts_stream", _VP, [_VP]),
    ("potts_save", ctypes.c_int, [_VP, ctypes.c_char_p]),
    ("potts_load", ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(_VP)]),
    ("potts_batch_create", ctypes.c_int, [ctypes.POINTER(PottsJob), ctypes.c_int32,
                                          ctypes.POINTER(PottsBatchOpts), ctypes.POINTER(_VP)]),
    ("potts_batch_run", ctypes.c_int, [_VP]),
    ("potts_batch_results", ctypes.c_int, [_VP, ctypes.POINTER(PottsJobResult)]),
    ("potts_batch_records", ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, _I64P]),
    ("potts_batch_spins", ctypes.c_int, [_VP, ctypes.c_int32, _U8P]),
    ("potts_batch_elapsed_ms", ctypes.c_double, [_VP]),
    ("potts_batch_tuning", ctypes.c_char_p, [_VP]),
    ("potts_batch_free", None, [_VP]),
    ("potts_kernel_digest", ctypes.c_char_p, []),
    ("potts_server_start", ctypes.c_int, [ctypes.POINTER(PottsServerCfg), ctypes.POINTER(_VP)]),
    ("potts_server_submit", ctypes.c_int, [_VP, ctypes.POINTER(PottsRequest), ctypes.POINTER(ctypes.c_int64)]),
    ("potts_server_wait", ctypes.c_int, [_VP, _I64P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    ("potts_server_collect", ctypes.c_int, [_VP, ctypes.c_int64, ctypes.POINTER(PottsServed),
                                            ctypes.POINTER(PottsSummary), _U8P]),
    ("potts_server_inject_fault", ctypes.c_int, [_VP, ctypes.c_int64, ctypes.c_int64]),
    ("potts_server_drain", ctypes.c_int, [_VP, ctypes.c_int32]),
    ("potts_server_now", ctypes.c_double, [_VP]),
    ("potts_server_iterations", ctypes.c_int64, [_VP]),
    ("potts_server_tuning", ctypes.c_int, [_VP, ctypes.c_char_p, ctypes.c_int32]),
    ("potts_server_stop", ctypes.c_int, [_VP]),
    ("potts_free", None, [_VP]),
    ("potts_nnn_init", ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int,
                                      ctypes.POINTER(_VP)]),
    ("potts_nnn_table", ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_uint64)]),
    ("potts_nnn_sweep", ctypes.c_int, [_VP, ctypes.c_double, ctypes.c_double, ctypes.c_int64]),
    ("potts_nnn_sweep_thr", ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int64]),
    ("potts_nnn_records", ctypes.c_int, [_VP, ctypes.c_int64, ctypes.c_int64, _I64P]),
    ("potts_nnn_observables", ctypes.c_int, [_VP, ctypes.POINTER(PottsNnnObs)]),
    ("potts_nnn_get_spins", ctypes.c_int, [_VP, _U8P]),
    ("potts_nnn_tune", ctypes.c_int, [_VP, ctypes.c_int32]),
    ("potts_nnn_time", ctypes.c_int64, [_VP]),
    ("potts_nnn_stream", _VP, [_VP]),
    ("potts_nnn_free", None, [_VP]),
    ("potts3d_init", ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int,
                                    ctypes.POINTER(_VP)]),
    ("potts3d_threshold_table", ctypes.c_int, [ctypes.c_double, _U32P]),
    ("potts3d_sweep", ctypes.c_int, [_VP, ctypes.c_double, ctypes.c_int64]),
    ("potts3d_sweep_thr", ctypes.c_int, [_VP, _U32P, ctypes.c_int64]),
    ("potts3d_records", ctypes.c_int, [_VP, ctypes.c_int64, ctypes.c_int64, _I64P]),
    ("potts3d_observables", ctypes.c_int, [_VP, ctypes.POINTER(PottsObs)]),
    ("potts3d_stats", ctypes.c_int, [_VP, ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                                     ctypes.POINTER(PottsSummary)]),
    ("potts3d_get_spins", ctypes.c_int, [_VP, _U8P]),
    ("potts3d_tune", ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32]),
    ("potts3d_time", ctypes.c_int64, [_VP]),
    ("potts3d_stream", _VP, [_VP]),
    ("potts3d_free", None, [_VP]),
    ("potts_strerror", ctypes.c_char_p, [ctypes.c_int]),
    ("potts_last_error", ctypes.c_char_p, []),
]


def load():
    """Loads libpotts.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "or python paper_1101_0876_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int) -> None:
    if rc != 0:
        msg = load().potts_last_error()
        raise PottsError(rc, msg.decode() if msg else "")
