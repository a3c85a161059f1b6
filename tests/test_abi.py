"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every
function include/potts.h declares, validates arguments before touching the
device, and builds the same threshold table as the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

from tests.conftest import ROOT
from tests.inputs import beta_c

HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def declared_functions():
    names = []
    for path in HEADERS:
        text = open(path).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(potts(?:3d)?_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    import paper_1101_0876_amd as p

    return p.load()


def test_header_declares_the_core_calls():
    names = declared_functions()
    for core in ("potts_init", "potts_sweep", "potts_observables", "potts_free", "potts_strerror",
                 "potts3d_init", "potts3d_sweep", "potts3d_free"):
        assert core in names


def test_every_declared_symbol_is_exported(lib):
    from paper_1101_0876_amd._native import SIGNATURES

    bound = {name for name, _, _ in SIGNATURES}
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in bound, f"{name} has no Python binding"


@pytest.mark.parametrize("beta", [0.0, 0.3, beta_c(2), beta_c(6), 1.02 * np.log(4.0), beta_c(15), 3.0, 40.0])
def test_threshold_table_matches_oracle(oracle_lib, beta):
    import paper_1101_0876_amd as p

    assert np.array_equal(p.threshold_table(beta), oracle_lib.threshold_table(beta))


@pytest.mark.parametrize("L,q", [(0, 3), (3, 3), (6, 3), (8, 1), (8, 257), (-4, 2)])
def test_init_rejects_bad_shapes_without_device(lib, L, q):
    h = ctypes.c_void_p()
    rc = lib.potts_init(L, q, 1, 1, ctypes.byref(h))
    assert rc == -1 and not h.value
    assert lib.potts_last_error()


def test_init_rejects_bad_start_and_null(lib):
    h = ctypes.c_void_p()
    assert lib.potts_init(8, 3, 1, 7, ctypes.byref(h)) == -1
    assert lib.potts_init(8, 3, 1, 1, None) == -1


def test_bad_beta_and_null_state(lib):
    thr = (ctypes.c_uint32 * 4)()
    assert lib.potts_threshold_table(-1.0, thr) == -1
    assert lib.potts_threshold_table(float("nan"), thr) == -1
    assert lib.potts_threshold_table(float("inf"), thr) == -1
    assert lib.potts_sweep(None, 1.0, 1) == -1
    assert lib.potts_observables(None, None) == -1
    lib.potts_free(None)


def test_tuning_calls_reject_a_null_state(lib):
    # checked before any device query, so this holds without a GPU
    assert lib.potts_tune(None, 7, 0, 0) == -1
    assert lib.potts_tune_band(None, 8, 256) == -1
    assert lib.potts_tune_tiles(None, 0, 0, 0) == -1
    assert lib.potts_tune_graph(None, 0) == -1
    assert lib.potts_tune_occupancy(None, 0) == -1


@pytest.mark.parametrize("bad", [dict(L=20), dict(L=8), dict(L=65552), dict(q=1), dict(q=257), dict(h=0),
                                 dict(h=3), dict(y0=1), dict(y0=-2), dict(y0=240, h=32), dict(colour=2),
                                 dict(t=-1), dict(slab=None), dict(thr=None), dict(ring=None),
                                 dict(ring=None, colour=0), dict(L=65536, h=65534, y0=0),
                                 dict(slots=3), dict(slots=1)])
def test_slab_half_sweep_rejects_bad_arguments(lib, bad):
    """Every check happens on the host, before anything reaches the device (the
    pointers below are never dereferenced)."""
    a = dict(slab=ctypes.c_void_p(0x1000), L=256, h=32, y0=64, q=5, seed=1, t=0, colour=1,
             thr=(ctypes.c_uint32 * 4)(1, 2, 3, 4), ring=ctypes.c_void_p(0x2000), slots=4, stream=None)
    a.update(bad)
    rc = lib.potts_slab_half_sweep(a["slab"], a["L"], a["h"], a["y0"], a["q"], a["seed"], a["t"], a["colour"],
                                   a["thr"], a["ring"], a["slots"], a["stream"])
    assert rc == -1
    assert lib.potts_last_error()


def test_reweight_rejects_null_without_device(lib):
    betas = (ctypes.c_double * 1)(1.0)
    assert lib.potts_reweight(None, 0, 1, 1.0, betas, 1, None) == -1


@pytest.mark.parametrize("beta", [0.0, 0.2, 0.4433, 0.5505, 1.0, 3.0, 40.0])
def test_cubic_threshold_table_matches_oracle(oracle_lib, beta):
    import paper_1101_0876_amd as p

    assert np.array_equal(p.threshold_table6(beta), oracle_lib.threshold_table6(beta))


@pytest.mark.parametrize("L,q,start", [(0, 3, 1), (2, 3, 1), (6, 3, 1), (8, 1, 1), (8, 257, 1), (8, 3, 5),
                                       (2584, 3, 1)])
def test_cubic_init_rejects_bad_shapes_without_device(lib, L, q, start):
    h = ctypes.c_void_p()
    rc = lib.potts3d_init(L, q, 1, start, ctypes.byref(h))
    assert rc in (-1, -4) and not h.value
    assert lib.potts_last_error()


def test_cubic_null_state(lib):
    thr = (ctypes.c_uint32 * 6)()
    assert lib.potts3d_threshold_table(-1.0, thr) == -1
    assert lib.potts3d_threshold_table(float("inf"), thr) == -1
    assert lib.potts3d_threshold_table(0.5, None) == -1
    assert lib.potts3d_sweep(None, 1.0, 1) == -1
    assert lib.potts3d_sweep_thr(None, thr, 1) == -1
    assert lib.potts3d_observables(None, None) == -1
    assert lib.potts3d_records(None, 0, 1, None) == -1
    assert lib.potts3d_time(None) == -1
    lib.potts3d_free(None)


@pytest.mark.parametrize("beta,j2", [(0.0, 0.5), (0.3, 0.5), (0.7, -0.4), (1.1, 1.0), (2.0, 0.25), (40.0, 0.1)])
def test_nnn_table_matches_oracle(oracle_lib, beta, j2):
    import paper_1101_0876_amd as p

    assert np.array_equal(p.nnn_table(beta, j2), oracle_lib.nnn_table(beta, j2))


@pytest.mark.parametrize("L,q,start", [(0, 3, 1), (8, 3, 1), (18, 3, 1), (24, 1, 1), (24, 257, 1), (24, 3, 4),
                                       (131076, 3, 1)])
def test_nnn_init_rejects_bad_shapes_without_device(lib, L, q, start):
    h = ctypes.c_void_p()
    rc = lib.potts_nnn_init(L, q, 1, start, ctypes.byref(h))
    assert rc in (-1, -4) and not h.value
    assert lib.potts_last_error()


def test_nnn_null_state(lib):
    thr = (ctypes.c_uint64 * 81)()
    assert lib.potts_nnn_table(-1.0, 0.5, thr) == -1
    assert lib.potts_nnn_table(0.5, float("nan"), thr) == -1
    assert lib.potts_nnn_table(0.5, 0.5, None) == -1
    assert lib.potts_nnn_sweep(None, 1.0, 0.5, 1) == -1
    assert lib.potts_nnn_sweep_thr(None, thr, 1) == -1
    assert lib.potts_nnn_observables(None, None) == -1
    assert lib.potts_nnn_records(None, 0, 1, None) == -1
    assert lib.potts_nnn_time(None) == -1
    assert lib.potts_nnn_stream(None) is None
    lib.potts_nnn_free(None)


def test_strerror(lib):
    for code in (0, -1, -2, -3, -4, -5, -99):
        assert lib.potts_strerror(code)


def test_product_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_1101_0876_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "potts_oracle" not in text and "liboracle" not in text, f


def test_slab_records_validates_without_device(lib):
    buf = ctypes.c_void_p(8)  # never dereferenced: every call below fails validation first
    assert lib.potts_slab_records(None, 2, 8, 3, 0, 1, buf, None) == -1
    assert lib.potts_slab_records(buf, 2, 8, 3, 0, 1, None, None) == -1
    assert lib.potts_slab_records(buf, 0, 8, 3, 0, 1, buf, None) == -1
    assert lib.potts_slab_records(buf, 2, 6, 3, 0, 1, buf, None) == -1
    assert lib.potts_slab_records(buf, 2, 8, 1, 0, 1, buf, None) == -1
    assert lib.potts_slab_records(buf, 2, 8, 3, -1, 1, buf, None) == -1
    assert lib.potts_slab_records(buf, 2, 8, 3, 0, 9, buf, None) == -1


def test_init_ex_needs_both_buffers_or_neither(lib):
    h = ctypes.c_void_p()
    assert lib.potts_init_ex(64, 3, 1, 1, ctypes.c_void_p(8), None, 4096, None, 0, ctypes.byref(h)) == -1
    assert lib.potts_init_ex(64, 3, 1, 1, None, ctypes.c_void_p(8), 4096, None, 0, ctypes.byref(h)) == -1
    assert lib.potts_init_ex(64, 3, 1, 1, ctypes.c_void_p(8), ctypes.c_void_p(8), 100, None, 0,
                             ctypes.byref(h)) == -1
    assert not h.value
    assert lib.potts_stream(None) is None
