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
WTS_E_CAPACITY, WTS_E_HIP, WTS_E_NONFINITE, WTS_E_UNSUPPORTED, WTS_E_DEVICE = -5, -6, -7, -8, -9


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
              "wts_softdtw_grad_cycles", "wts_plan_status", "wts_barycenter_objective"]:
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
    # sizes beyond the build's fixed limits: 2^24 samples per series
    assert _create(lib, L=(1 << 24) + 1)[0] == WTS_E_CAPACITY
    assert _create(lib, offsets=(0, 3, 3 + (1 << 24) + 1))[0] == WTS_E_CAPACITY
    assert b"length" in lib.wts_last_error() or len(lib.wts_last_error()) > 0
    from paper_2404_12134_amd.wetsand import _Opts
    for rho in (1, 3, 6, 8):   # rows per lane: 2, 4 or 5 only
        assert _create(lib, opts=ctypes.byref(_Opts(0, rho, 0, 0)))[0] == WTS_E_UNSUPPORTED
    assert _create(lib, opts=ctypes.byref(_Opts(0, 4, -1, 0)))[0] == WTS_E_ARG
    for band in (-0.5, float("nan"), float("inf")):   # Sakoe-Chiba bandwidth
        assert _create(lib, opts=ctypes.byref(_Opts(0, 4, 0, 0, band=band)))[0] == WTS_E_ARG
    assert _create(lib, opts=ctypes.byref(_Opts(0, 4, 0, 7)))[0] == WTS_E_ARG   # validate: 0 or 1
    for wk in (-1, 3):                                                            # walk: 0, 1 or 2
        assert _create(lib, opts=ctypes.byref(_Opts(0, 4, 0, 0, walk=wk)))[0] == WTS_E_ARG
    for de in (-1, 2):                                                            # dense_e: 0 or 1
        assert _create(lib, opts=ctypes.byref(_Opts(0, 4, 0, 0, dense_e=de)))[0] == WTS_E_ARG
    assert _create(lib, opts=ctypes.byref(_Opts(0, 4, 0, -1)))[0] == WTS_E_ARG
    # decision: 0 (float64) or 1 (float32), the latter on float32 cycles with the squared cost
    for dec in (-1, 2):
        assert _create(lib, opts=ctypes.byref(_Opts(0, 4, 0, 0, dec)))[0] == WTS_E_ARG
    assert _create(lib, dtype=1, opts=ctypes.byref(_Opts(0, 4, 0, 0, 1)))[0] == WTS_E_UNSUPPORTED
    assert _create(lib, opts=ctypes.byref(_Opts(1, 4, 0, 0, 1)))[0] == WTS_E_UNSUPPORTED


def test_null_plan_is_rejected(lib):
    P = ctypes.c_void_p
    assert lib.wts_dtw_align(None, P(1), P(1), P(1), P(1), None, P(256), ctypes.c_size_t(1), None) == WTS_E_ARG
    assert lib.wts_dba_iterate(None, P(1), P(1), None, P(2), P(1), None, P(256), ctypes.c_size_t(1), None) == WTS_E_ARG
    assert lib.wts_anomaly_score(None, P(1), P(1), P(1), None, None, P(256), ctypes.c_size_t(1), None) == WTS_E_ARG
    assert lib.wts_medoid(None, P(1), None, None, P(1), P(256), ctypes.c_size_t(1), None) == WTS_E_ARG
    assert lib.wts_softdtw_grad_cycles(None, P(1), P(1), ctypes.c_double(1.0), None, P(1), P(256),
                                       ctypes.c_size_t(1), None) == WTS_E_ARG
    assert lib.wts_subdtw(None, P(1), P(1), P(1), P(1), P(1), P(256), ctypes.c_size_t(1), None) == WTS_E_ARG
    D = ctypes.c_double
    assert lib.wts_softdtw_forward(None, P(1), P(1), D(1.0), P(1), P(256), ctypes.c_size_t(1),
                                   None) == WTS_E_ARG
    assert lib.wts_softdtw_backward(None, P(1), P(1), D(1.0), P(256), ctypes.c_size_t(1), None,
                                    P(1), None, 0, P(256), ctypes.c_size_t(1), None) == WTS_E_ARG
    assert lib.wts_plan_status(None, None) == WTS_E_ARG
    assert lib.wts_workspace_bytes(None, 0) == 0
    lib.wts_plan_destroy(None)   # no-op


def test_objective_rejects_bad_arguments_before_any_gpu_call(lib):
    P = ctypes.c_void_p
    assert lib.wts_barycenter_objective(None, None, 1, 0, P(8), None) == WTS_E_ARG
    assert lib.wts_barycenter_objective(P(8), None, 1, 0, None, None) == WTS_E_ARG
    assert lib.wts_barycenter_objective(P(8), None, 0, 0, P(8), None) == WTS_E_SHAPE
    assert lib.wts_barycenter_objective(P(8), None, 1, 2, P(8), None) == WTS_E_ARG
    assert lib.wts_precond_step(None, P(8), P(8), ctypes.c_int64(1), 1, ctypes.c_double(0.5),
                                None) == WTS_E_ARG


def test_status_codes_of_header_and_binding_agree():
    """The binding's status constants are the header's enum values."""
    from paper_2404_12134_amd import wetsand
    src = open(HEADER).read()
    body = src[src.index("typedef enum {"):src.index("} wts_status;")]
    codes = {m.group(1): int(m.group(2)) for m in re.finditer(r"WTS_(\w+)\s*=\s*(-?\d+)", body)}
    assert codes == {"OK": 0, "E_ARG": -1, "E_SHAPE": -2, "E_DTYPE": -3, "E_WORKSPACE": -4,
                     "E_CAPACITY": -5, "E_HIP": -6, "E_NONFINITE": -7, "E_UNSUPPORTED": -8,
                     "E_DEVICE": -9}
    for name, v in codes.items():
        assert getattr(wetsand, name) == v, name


def test_binding_checks_tensor_arguments_before_passing_pointers():
    """A wrong dtype, shape, device or a non-contiguous tensor is refused with
    ValueError before any pointer reaches the library (the ABI trusts sizes)."""
    import types
    import torch
    from paper_2404_12134_amd import wetsand as w
    plan = types.SimpleNamespace(device=0, L=5, d=3, n=2, dtype="f32",
                                 offsets=np.array([0, 4, 9], dtype=np.int64))
    with pytest.raises(ValueError, match="float64"):
        w._bary_arg(plan, torch.zeros((5, 3), dtype=torch.float32))
    with pytest.raises(ValueError, match="cuda"):
        w._bary_arg(plan, torch.zeros((5, 3), dtype=torch.float64))
    with pytest.raises(ValueError, match="float32"):
        w._cycles_arg(plan, torch.zeros((9, 3), dtype=torch.float64))
    with pytest.raises(ValueError, match="float64"):
        w._vec_arg(plan, torch.zeros(2, dtype=torch.float32), "weights")
    with pytest.raises(TypeError):
        w._bary_arg(plan, np.zeros((5, 3)))
    # shape, size and contiguity (checked with the device test relaxed to the CPU)
    cpu = torch.device("cpu")
    with pytest.raises(ValueError, match="shape"):
        w._need(torch.zeros((3, 5), dtype=torch.float64), "bary", torch.float64, cpu, shape=(5, 3))
    with pytest.raises(ValueError, match="contiguous"):
        w._need(torch.zeros((3, 5), dtype=torch.float64).t(), "bary", torch.float64, cpu,
                shape=(5, 3))
    with pytest.raises(ValueError, match="hold 27 values"):
        w._need(torch.zeros((8, 3), dtype=torch.float32), "cycles", torch.float32, cpu, numel=27)
    with pytest.raises(ValueError, match="at least"):
        w._need(torch.zeros(10, dtype=torch.uint8), "ckpt", torch.uint8, cpu, min_numel=11)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2404_12134_amd import wetsand
    monkeypatch.setattr(wetsand, "_lib", None)
    monkeypatch.setattr(wetsand, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        wetsand.load()


def test_binding_options_struct_matches_the_header():
    """The ctypes mirror of wts_opts lists the header's fields in order."""
    import re
    from paper_2404_12134_amd.wetsand import _Opts
    body = open(HEADER).read()
    struct = body[body.index("typedef struct {", body.index("WTS_DECISION_FP64")):]
    struct = struct[:struct.index("} wts_opts;")]
    fields = re.findall(r"^\s*(?:int32_t|double)\s+(\w+);", struct, re.M)
    assert fields == [f for f, _ in _Opts._fields_]
