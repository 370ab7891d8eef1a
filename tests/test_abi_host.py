"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/wetsand_mi.h declares, and rejects bad arguments
with the documented status before touching the GPU."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wetsand_mi.h")
LIB = os.path.join(ROOT, "paper_2404_12134_amd", "libwetsand_mi.so")

WTS_OK, WTS_E_ARG, WTS_E_SHAPE, WTS_E_DTYPE, WTS_E_WORKSPACE = 0, -1, -2, -3, -4
WTS_E_HIP, WTS_E_UNSUPPORTED = -6, -8


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(wts_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2404_12134_amd import build
        build.build()
    L = ctypes.CDLL(LIB)
    L.wts_last_error.restype = ctypes.c_char_p
    return L


def test_header_declares_the_entry_points():
    names = declared()
    for n in ["wts_plan_create", "wts_plan_destroy", "wts_workspace_bytes", "wts_last_error",
              "wts_dtw_align", "wts_dba_iterate", "wts_softdtw_forward", "wts_softdtw_backward",
              "wts_anomaly_score", "wts_medoid", "wts_init_barycenter", "wts_subdtw",
              "wts_softdtw_grad_cycles"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared():
        assert hasattr(lib, name), name


def test_binding_names_match_header():
    from paper_2404_12134_amd import wetsand
    assert sorted(wetsand.exported_symbols()) == declared()


def _create(lib, n=2, d=1, dtype=0, offsets=(0, 3, 5), L=4, opts=None):
    h = ctypes.c_void_p()
    off = np.asarray(offsets, dtype=np.int64)
    rc = lib.wts_plan_create(ctypes.byref(h), 0, n, d, dtype, off.ctypes.data_as(ctypes.c_void_p),
                             ctypes.c_int64(L), opts)
    return rc, h


def test_plan_create_rejects_bad_shapes_before_any_gpu_call(lib):
    assert lib.wts_plan_create(None, 0, 1, 1, 0, None, ctypes.c_int64(1), None) == WTS_E_ARG
    assert _create(lib, n=0, offsets=(0,))[0] == WTS_E_SHAPE
    assert _create(lib, d=0)[0] == WTS_E_SHAPE
    assert _create(lib, d=9)[0] == WTS_E_UNSUPPORTED
    assert _create(lib, dtype=7)[0] == WTS_E_DTYPE
    assert _create(lib, offsets=(1, 3, 5))[0] == WTS_E_SHAPE          # offsets[0] != 0
    assert _create(lib, offsets=(0, 3, 3))[0] == WTS_E_SHAPE          # empty cycle
    assert _create(lib, L=-1)[0] == WTS_E_SHAPE
    assert b"length" in lib.wts_last_error() or len(lib.wts_last_error()) > 0
    from paper_2404_12134_amd.wetsand import _Opts
    for rho in (1, 3, 6, 8):   # rows per lane: 2, 4 or 5 only
        assert _create(lib, opts=ctypes.byref(_Opts(0, rho, 0, 0)))[0] == WTS_E_UNSUPPORTED
    assert _create(lib, opts=ctypes.byref(_Opts(0, 4, -1, 0)))[0] == WTS_E_ARG
    for band in (-0.5, float("nan"), float("inf")):   # Sakoe-Chiba bandwidth
        assert _create(lib, opts=ctypes.byref(_Opts(0, 4, 0, 0, band)))[0] == WTS_E_ARG
    assert _create(lib, opts=ctypes.byref(_Opts(0, 4, 0, 7)))[0] == WTS_E_ARG


def test_null_plan_is_rejected(lib):
    P = ctypes.c_void_p
    assert lib.wts_dtw_align(None, P(1), P(1), P(1), P(1), None, P(256), ctypes.c_size_t(1), None) == WTS_E_ARG
    assert lib.wts_dba_iterate(None, P(1), P(1), None, P(2), P(1), None, P(256), ctypes.c_size_t(1), None) == WTS_E_ARG
    assert lib.wts_anomaly_score(None, P(1), P(1), P(1), None, None, P(256), ctypes.c_size_t(1), None) == WTS_E_ARG
    assert lib.wts_medoid(None, P(1), None, None, P(1), P(256), ctypes.c_size_t(1), None) == WTS_E_ARG
    assert lib.wts_softdtw_grad_cycles(None, P(1), P(1), ctypes.c_double(1.0), None, P(1), P(256),
                                       ctypes.c_size_t(1), None) == WTS_E_ARG
    assert lib.wts_subdtw(None, P(1), P(1), P(1), P(1), P(1), P(256), ctypes.c_size_t(1), None) == WTS_E_ARG
    assert lib.wts_workspace_bytes(None, 0) == 0
    lib.wts_plan_destroy(None)   # no-op


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2404_12134_amd import wetsand
    monkeypatch.setattr(wetsand, "_lib", None)
    monkeypatch.setattr(wetsand, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        wetsand.load()
