"""CPU oracle for the checkerboard Metropolis sweep of the 2D q-state Potts model.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product library
(``paper_1101_0876_amd``) never imports it and shares no code with it.

The arithmetic lives in ``potts_oracle.c`` (plain serial C, built by
``oracle/build.py``); this module only marshals arguments through ctypes.
Derived FP64 statistics are in ``oracle/stats.py`` (exact rational arithmetic).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

ORDERED = 0
RANDOM = 1


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from oracle.build import build
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
    lib.oracle_philox4x32_10.restype = None
    lib.oracle_threshold_table.argtypes = [ctypes.c_double, u32p]
    lib.oracle_threshold_table.restype = ctypes.c_int
    lib.oracle_init.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_int, u8p]
    lib.oracle_init.restype = ctypes.c_int
    lib.oracle_site_update.argtypes = [ctypes.c_int, ctypes.c_int, u8p, ctypes.c_uint32,
                                       ctypes.c_uint32, u32p]
    lib.oracle_site_update.restype = ctypes.c_int
    lib.oracle_half_sweep.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                      ctypes.c_int, u32p, u8p, i64p]
    lib.oracle_half_sweep.restype = ctypes.c_int
    lib.oracle_observables.argtypes = [ctypes.c_int, ctypes.c_int, u8p, i64p, i64p]
    lib.oracle_observables.restype = ctypes.c_int
    lib.oracle_sweeps.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                  ctypes.c_int64, u32p, u8p, i64p]
    lib.oracle_sweeps.restype = ctypes.c_int
    lib.oracle_window.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_int,
                                  ctypes.c_int64, u32p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_int, u8p]
    lib.oracle_window.restype = ctypes.c_int
    lib.oracle_heatbath_site.argtypes = [ctypes.c_int, u8p, ctypes.c_uint32, u32p]
    lib.oracle_heatbath_site.restype = ctypes.c_int
    lib.oracle_heatbath_half_sweep.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                               ctypes.c_int, u32p, u8p]
    lib.oracle_heatbath_half_sweep.restype = ctypes.c_int
    lib.oracle_heatbath_sweeps.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                           ctypes.c_int64, u32p, u8p, i64p]
    lib.oracle_heatbath_sweeps.restype = ctypes.c_int
    lib.oracle_threshold_table6.argtypes = [ctypes.c_double, u32p]
    lib.oracle_threshold_table6.restype = ctypes.c_int
    lib.oracle3d_init.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_int, u8p]
    lib.oracle3d_init.restype = ctypes.c_int
    lib.oracle3d_site_update.argtypes = [ctypes.c_int, ctypes.c_int, u8p, ctypes.c_uint32, ctypes.c_uint32, u32p]
    lib.oracle3d_site_update.restype = ctypes.c_int
    lib.oracle3d_half_sweep.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                        u32p, u8p]
    lib.oracle3d_half_sweep.restype = ctypes.c_int
    lib.oracle3d_observables.argtypes = [ctypes.c_int, ctypes.c_int, u8p, i64p, i64p]
    lib.oracle3d_observables.restype = ctypes.c_int
    lib.oracle3d_sweeps.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                    u32p, u8p, i64p]
    lib.oracle3d_sweeps.restype = ctypes.c_int
    lib.oracle3d_window.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_int, ctypes.c_int64,
                                    u32p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, u8p]
    lib.oracle3d_window.restype = ctypes.c_int
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.oracle_nnn_table.argtypes = [ctypes.c_double, ctypes.c_double, u64p]
    lib.oracle_nnn_table.restype = ctypes.c_int
    lib.oracle_nnn_site_update.argtypes = [ctypes.c_int, ctypes.c_int, u8p, u8p, ctypes.c_uint32, ctypes.c_uint32,
                                           u64p]
    lib.oracle_nnn_site_update.restype = ctypes.c_int
    lib.oracle_nnn_colour_pass.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                           ctypes.c_int, u64p, u8p]
    lib.oracle_nnn_colour_pass.restype = ctypes.c_int
    lib.oracle_nnn_observables.argtypes = [ctypes.c_int, ctypes.c_int, u8p, i64p, i64p, i64p]
    lib.oracle_nnn_observables.restype = ctypes.c_int
    lib.oracle_nnn_sweeps.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                      ctypes.c_int64, u64p, u8p, i64p]
    lib.oracle_nnn_sweeps.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def philox4x32_10(ctr, key) -> np.ndarray:
    """One Philox4x32-10 block (Salmon et al., SC'11) for counter ctr[4], key key[2]."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().oracle_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32),
                                 _ptr(out, ctypes.c_uint32))
    return out


def threshold_table(beta: float) -> np.ndarray:
    """thr[d-1] = min(floor(exp(-beta*d) * 2^32), 2^32-1), d = 1..4."""
    thr = np.zeros(4, dtype=np.uint32)
    _check(_load().oracle_threshold_table(float(beta), _ptr(thr, ctypes.c_uint32)), "threshold_table")
    return thr


def init(L: int, q: int, seed: int, start: int) -> np.ndarray:
    spins = np.zeros(L * L, dtype=np.uint8)
    _check(_load().oracle_init(L, q, seed, start, _ptr(spins, ctypes.c_uint8)), "init")
    return spins.reshape(L, L)


def site_update(q: int, s: int, nb, w_prop: int, w_acc: int, thr) -> int:
    nbs = np.ascontiguousarray(nb, dtype=np.uint8)
    t = np.ascontiguousarray(thr, dtype=np.uint32)
    return int(_load().oracle_site_update(q, s, _ptr(nbs, ctypes.c_uint8), w_prop, w_acc,
                                          _ptr(t, ctypes.c_uint32)))


def half_sweep(spins: np.ndarray, q: int, seed: int, t: int, colour: int, thr, order=None) -> None:
    """In-place update of every site of one colour (row-major or the given visiting order)."""
    assert spins.dtype == np.uint8 and spins.flags.c_contiguous
    L = spins.shape[0]
    t_arr = np.ascontiguousarray(thr, dtype=np.uint32)
    o = None if order is None else np.ascontiguousarray(order, dtype=np.int64)
    optr = None if o is None else _ptr(o, ctypes.c_int64)
    _check(_load().oracle_half_sweep(L, q, seed, t, colour, _ptr(t_arr, ctypes.c_uint32),
                                     _ptr(spins, ctypes.c_uint8), optr), "half_sweep")


def observables(spins: np.ndarray, q: int):
    """(e_sat, hist) of a configuration by direct definition."""
    assert spins.dtype == np.uint8 and spins.flags.c_contiguous
    L = spins.shape[0]
    e = np.zeros(1, dtype=np.int64)
    hist = np.zeros(q, dtype=np.int64)
    _check(_load().oracle_observables(L, q, _ptr(spins, ctypes.c_uint8), _ptr(e, ctypes.c_int64),
                                      _ptr(hist, ctypes.c_int64)), "observables")
    return int(e[0]), hist


def sweeps(spins: np.ndarray, q: int, seed: int, t0: int, n: int, thr, record: bool = True):
    """n sweeps in place from sweep index t0; returns records shaped (n, 1+q) or None."""
    assert spins.dtype == np.uint8 and spins.flags.c_contiguous
    L = spins.shape[0]
    t_arr = np.ascontiguousarray(thr, dtype=np.uint32)
    rec = np.zeros((n, 1 + q), dtype=np.int64) if record else None
    rptr = _ptr(rec, ctypes.c_int64) if record else None
    _check(_load().oracle_sweeps(L, q, seed, t0, n, _ptr(t_arr, ctypes.c_uint32),
                                 _ptr(spins, ctypes.c_uint8), rptr), "sweeps")
    return rec


def heatbath_site(q: int, nb, w: int, thr) -> int:
    """Heat-bath draw for one site: nb = (up, down, left, right), w its word."""
    nbs = np.ascontiguousarray(nb, dtype=np.uint8)
    t = np.ascontiguousarray(thr, dtype=np.uint32)
    return int(_load().oracle_heatbath_site(q, _ptr(nbs, ctypes.c_uint8), w, _ptr(t, ctypes.c_uint32)))


def heatbath_half_sweep(spins: np.ndarray, q: int, seed: int, t: int, colour: int, thr) -> None:
    """In-place heat-bath update of every site of one colour."""
    assert spins.dtype == np.uint8 and spins.flags.c_contiguous
    L = spins.shape[0]
    t_arr = np.ascontiguousarray(thr, dtype=np.uint32)
    _check(_load().oracle_heatbath_half_sweep(L, q, seed, t, colour, _ptr(t_arr, ctypes.c_uint32),
                                              _ptr(spins, ctypes.c_uint8)), "heatbath_half_sweep")


def heatbath_sweeps(spins: np.ndarray, q: int, seed: int, t0: int, n: int, thr, record: bool = True):
    """n heat-bath sweeps in place from sweep index t0; records shaped (n, 1+q) or None."""
    assert spins.dtype == np.uint8 and spins.flags.c_contiguous
    L = spins.shape[0]
    t_arr = np.ascontiguousarray(thr, dtype=np.uint32)
    rec = np.zeros((n, 1 + q), dtype=np.int64) if record else None
    rptr = _ptr(rec, ctypes.c_int64) if record else None
    _check(_load().oracle_heatbath_sweeps(L, q, seed, t0, n, _ptr(t_arr, ctypes.c_uint32),
                                          _ptr(spins, ctypes.c_uint8), rptr), "heatbath_sweeps")
    return rec


# -- simple-cubic lattice ---------------------------------------------------------
def threshold_table6(beta: float) -> np.ndarray:
    """thr[d-1] = min(floor(exp(-beta*d) * 2^32), 2^32-1), d = 1..6 (cubic lattice)."""
    thr = np.zeros(6, dtype=np.uint32)
    _check(_load().oracle_threshold_table6(float(beta), _ptr(thr, ctypes.c_uint32)), "threshold_table6")
    return thr


def init3d(L: int, q: int, seed: int, start: int) -> np.ndarray:
    spins = np.zeros((L, L, L), dtype=np.uint8)  # [z, y, x]
    _check(_load().oracle3d_init(L, q, seed, start, _ptr(spins, ctypes.c_uint8)), "init3d")
    return spins


def site_update3d(q: int, s: int, nb, w_prop: int, w_acc: int, thr) -> int:
    nbs = np.ascontiguousarray(nb, dtype=np.uint8)
    t = np.ascontiguousarray(thr, dtype=np.uint32)
    return int(_load().oracle3d_site_update(q, s, _ptr(nbs, ctypes.c_uint8), w_prop, w_acc,
                                            _ptr(t, ctypes.c_uint32)))


def half_sweep3d(spins: np.ndarray, q: int, seed: int, t: int, colour: int, thr) -> None:
    assert spins.dtype == np.uint8 and spins.flags.c_contiguous
    t_arr = np.ascontiguousarray(thr, dtype=np.uint32)
    _check(_load().oracle3d_half_sweep(spins.shape[0], q, seed, t, colour, _ptr(t_arr, ctypes.c_uint32),
                                       _ptr(spins, ctypes.c_uint8)), "half_sweep3d")


def observables3d(spins: np.ndarray, q: int):
    e = np.zeros(1, dtype=np.int64)
    hist = np.zeros(q, dtype=np.int64)
    _check(_load().oracle3d_observables(spins.shape[0], q, _ptr(spins, ctypes.c_uint8), _ptr(e, ctypes.c_int64),
                                        _ptr(hist, ctypes.c_int64)), "observables3d")
    return int(e[0]), hist


def sweeps3d(spins: np.ndarray, q: int, seed: int, t0: int, n: int, thr, record: bool = True):
    assert spins.dtype == np.uint8 and spins.flags.c_contiguous
    t_arr = np.ascontiguousarray(thr, dtype=np.uint32)
    rec = np.zeros((n, 1 + q), dtype=np.int64) if record else None
    rptr = _ptr(rec, ctypes.c_int64) if record else None
    _check(_load().oracle3d_sweeps(spins.shape[0], q, seed, t0, n, _ptr(t_arr, ctypes.c_uint32),
                                   _ptr(spins, ctypes.c_uint8), rptr), "sweeps3d")
    return rec


def window3d(L: int, q: int, seed: int, start: int, nsweeps: int, thr, x0: int, y0: int, z0: int, d: int):
    """d^3 window ([z, y, x], corner (x0, y0, z0), periodic) of the cubic chain after
    nsweeps sweeps; only sites at distance >= 2*nsweeps from every face are exact."""
    out = np.zeros(d * d * d, dtype=np.uint8)
    t_arr = np.ascontiguousarray(thr, dtype=np.uint32)
    _check(_load().oracle3d_window(L, q, seed, start, nsweeps, _ptr(t_arr, ctypes.c_uint32), x0, y0, z0, d,
                                   _ptr(out, ctypes.c_uint8)), "window3d")
    return out.reshape(d, d, d)


# -- first and second neighbours ----------------------------------------------------
def nnn_table(beta: float, j2: float) -> np.ndarray:
    """81 acceptance entries, index (d1 + 4) * 9 + (d2 + 4): 2^32 when
    d1 + j2 d2 <= 0, else min(floor(exp(-beta (d1 + j2 d2)) 2^32), 2^32 - 1)."""
    thr = np.zeros(81, dtype=np.uint64)
    _check(_load().oracle_nnn_table(float(beta), float(j2), _ptr(thr, ctypes.c_uint64)), "nnn_table")
    return thr


def nnn_site_update(q: int, s: int, nb1, nb2, w_prop: int, w_acc: int, thr) -> int:
    a = np.ascontiguousarray(nb1, dtype=np.uint8)
    b = np.ascontiguousarray(nb2, dtype=np.uint8)
    t = np.ascontiguousarray(thr, dtype=np.uint64)
    return int(_load().oracle_nnn_site_update(q, s, _ptr(a, ctypes.c_uint8), _ptr(b, ctypes.c_uint8), w_prop,
                                              w_acc, _ptr(t, ctypes.c_uint64)))


def nnn_colour_pass(spins: np.ndarray, q: int, seed: int, t: int, colour: int, thr) -> None:
    assert spins.dtype == np.uint8 and spins.flags.c_contiguous
    t_arr = np.ascontiguousarray(thr, dtype=np.uint64)
    _check(_load().oracle_nnn_colour_pass(spins.shape[0], q, seed, t, colour, _ptr(t_arr, ctypes.c_uint64),
                                          _ptr(spins, ctypes.c_uint8)), "nnn_colour_pass")


def nnn_observables(spins: np.ndarray, q: int):
    e1 = np.zeros(1, dtype=np.int64)
    e2 = np.zeros(1, dtype=np.int64)
    hist = np.zeros(q, dtype=np.int64)
    _check(_load().oracle_nnn_observables(spins.shape[0], q, _ptr(spins, ctypes.c_uint8), _ptr(e1, ctypes.c_int64),
                                          _ptr(e2, ctypes.c_int64), _ptr(hist, ctypes.c_int64)), "nnn_observables")
    return int(e1[0]), int(e2[0]), hist


def nnn_sweeps(spins: np.ndarray, q: int, seed: int, t0: int, n: int, thr, record: bool = True):
    """n sweeps (nine colour passes each); records {e1, e2, hist[q]} per sweep."""
    assert spins.dtype == np.uint8 and spins.flags.c_contiguous
    t_arr = np.ascontiguousarray(thr, dtype=np.uint64)
    rec = np.zeros((n, 2 + q), dtype=np.int64) if record else None
    rptr = _ptr(rec, ctypes.c_int64) if record else None
    _check(_load().oracle_nnn_sweeps(spins.shape[0], q, seed, t0, n, _ptr(t_arr, ctypes.c_uint64),
                                     _ptr(spins, ctypes.c_uint8), rptr), "nnn_sweeps")
    return rec


def run(L: int, q: int, seed: int, start: int, beta: float, n: int):
    """init + n sweeps at one beta; returns (spins, records)."""
    spins = init(L, q, seed, start)
    rec = sweeps(spins, q, seed, 0, n, threshold_table(beta))
    return spins, rec


def window(L: int, q: int, seed: int, start: int, nsweeps: int, thr, x0: int, y0: int, h: int, w: int):
    """h x w window (top-left (x0, y0), periodic) after nsweeps sweeps from the initial
    condition; only sites at distance >= 2*nsweeps from the window edge are exact."""
    out = np.zeros(h * w, dtype=np.uint8)
    t_arr = np.ascontiguousarray(thr, dtype=np.uint32)
    _check(_load().oracle_window(L, q, seed, start, nsweeps, _ptr(t_arr, ctypes.c_uint32), x0, y0,
                                 h, w, _ptr(out, ctypes.c_uint8)), "window")
    return out.reshape(h, w)
