"""Thin Python binding of libwetsand_mi.so (the C ABI in include/wetsand_mi.h).

Argument marshalling only: every step of the hot path runs in the HIP
kernels behind the C ABI.  PyTorch provides device memory (tensors) and the
stream (torch's current stream) -- nothing is computed with it here.
The library is required: if it is not built, every call raises.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwetsand_mi.so")

F32, F64 = 0, 1
COST_SQ, COST_EUCLID = 0, 1
(OP_ALIGN, OP_ALIGN_PATHS, OP_DBA, OP_SCORE, OP_SOFT_FWD, OP_SOFT_BWD, OP_MEDOID, OP_SUBDTW,
 OP_SOFT_GRAD_C) = range(9)
INIT_EUCLID_MEAN, INIT_NEAREST, INIT_COPY = 0, 1, 2
DECISION_FP64, DECISION_FP32 = 0, 1

_lib = None


class WtsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("wetsand_mi status %d: %s" % (status, msg))
        self.status = status


# status codes of include/wetsand_mi.h
(OK, E_ARG, E_SHAPE, E_DTYPE, E_WORKSPACE, E_CAPACITY, E_HIP, E_NONFINITE, E_UNSUPPORTED,
 E_DEVICE) = 0, -1, -2, -3, -4, -5, -6, -7, -8, -9


_WALKS = {"auto": 0, "strips": 1, "pairs": 2}


class _Opts(ctypes.Structure):
    _fields_ = [("cost", ctypes.c_int32), ("rho", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("validate", ctypes.c_int32), ("decision", ctypes.c_int32),
                ("band", ctypes.c_double), ("dense_e", ctypes.c_int32), ("walk", ctypes.c_int32)]


def load():
    """Open the shared library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libwetsand_mi.so is not built (python -m paper_2404_12134_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, SZ, D = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t,
                          ctypes.c_double)
    sig = {
        "wts_plan_create": [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, I32, I32, I32, P, I64,
                            ctypes.POINTER(_Opts)],
        "wts_workspace_bytes": [P, ctypes.c_int],
        "wts_dtw_align": [P, P, P, P, P, P, P, SZ, P],
        "wts_dba_iterate": [P, P, P, P, P, P, P, P, SZ, P],
        "wts_anomaly_score": [P, P, P, P, P, P, P, SZ, P],
        "wts_softdtw_forward": [P, P, P, D, P, P, SZ, P],
        "wts_softdtw_backward": [P, P, P, D, P, SZ, P, P, P, I32, P, SZ, P],
        "wts_medoid": [P, P, P, P, P, P, SZ, P],
        "wts_init_barycenter": [P, P, I32, I32, P, P, P],
        "wts_precond_step": [P, P, P, I64, I32, D, P],
        "wts_plan_timing": [P, I32],
        "wts_plan_sweep_ms": [P, ctypes.c_int, P, P],
        "wts_plan_bwd_tiles": [P, P, P],
        "wts_plan_walk": [P],
        "wts_plan_rho": [P, ctypes.c_int],
        "wts_subdtw": [P, P, P, P, P, P, P, SZ, P],
        "wts_softdtw_grad_cycles": [P, P, P, D, P, P, P, SZ, P],
        "wts_plan_status": [P, P],
        "wts_anomaly_score_noalloc": [P, P, P, P, P, P, P],
        "wts_barycenter_objective": [P, P, I32, I32, P, P],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.wts_workspace_bytes.restype = SZ
    L.wts_plan_destroy.argtypes = [P]
    L.wts_plan_destroy.restype = None
    L.wts_last_error.argtypes = []
    L.wts_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def exported_symbols():
    """Names the binding expects the library to export."""
    return ["wts_plan_create", "wts_plan_destroy", "wts_workspace_bytes", "wts_last_error",
            "wts_dtw_align", "wts_dba_iterate", "wts_anomaly_score", "wts_softdtw_forward",
            "wts_softdtw_backward", "wts_medoid", "wts_init_barycenter", "wts_precond_step",
            "wts_plan_timing", "wts_plan_sweep_ms", "wts_plan_rho", "wts_subdtw",
            "wts_softdtw_grad_cycles", "wts_plan_status", "wts_barycenter_objective",
            "wts_anomaly_score_noalloc", "wts_plan_bwd_tiles", "wts_plan_walk"]


def _check(rc: int):
    if rc != 0:
        raise WtsError(rc, load().wts_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# ---------------------------------------------------------- argument checks
# The C ABI takes raw device pointers and trusts their sizes: every tensor is
# checked here (dtype, device, contiguity, size) before its pointer is passed.

def _need(t, what: str, dtype, device, shape=None, numel=None, min_numel=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor, not %s" % (what, type(t).__name__))
    if t.dtype != dtype:
        raise ValueError("%s must be %s, not %s" % (what, dtype, t.dtype))
    if t.device != device:
        raise ValueError("%s must be on %s, not %s" % (what, device, t.device))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, not %s" % (what, tuple(shape), tuple(t.shape)))
    if numel is not None and t.numel() != numel:
        raise ValueError("%s must hold %d values, not %d" % (what, numel, t.numel()))
    if min_numel is not None and t.numel() < min_numel:
        raise ValueError("%s must hold at least %d values, not %d" % (what, min_numel, t.numel()))
    return t


def _device(plan) -> torch.device:
    return torch.device("cuda", plan.device)


def _bary_arg(plan, t, what: str = "bary"):
    """A float64 [L][d] barycenter (or reference) on the plan's device."""
    return _need(t, what, torch.float64, _device(plan), shape=(plan.L, plan.d))


def _cycles_arg(plan, t, what: str = "cycles"):
    """The packed [sum N][d] cycle values of the plan's storage dtype."""
    dt = torch.float32 if plan.dtype == "f32" else torch.float64
    return _need(t, what, dt, _device(plan), numel=int(plan.offsets[-1]) * plan.d)


def _vec_arg(plan, t, what: str, n: Optional[int] = None, dtype=torch.float64):
    """An optional [n] vector (None passes through)."""
    if t is None:
        return None
    return _need(t, what, dtype, _device(plan), numel=plan.n if n is None else n)


class Plan:
    """A plan binds the cycle lengths, the channel count, the storage dtype and
    the barycenter length L (L = 0: a plan for the medoid only).  band > 0
    restricts the Soft-DTW calls to a Sakoe-Chiba band of that fraction of
    the longer length (Table I).  dense_e=True makes the Soft-DTW backward
    sweep every tile, also those whose E entries are exactly zero (same
    results, more time).  walk picks the path recovery of the DBA and
    path calls: "strips" (entry tags, all strips walked at once), "pairs"
    (no tags, each pair walks its strips in turn) or "auto" (the library
    decides by the batch's size); the results are the same bits."""

    def __init__(self, offsets, d: int, dtype: str, L: int, device: int = 0, cost: str = "sq",
                 rho: int = 0, grid: int = 0, band: float = 0.0, validate: bool = False,
                 decision: str = "fp64", dense_e: bool = False, walk: str = "auto"):
        lib = load()
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        self.offsets = off
        self.n = int(off.size - 1)
        self.d = int(d)
        self.dtype = dtype
        self.L = int(L)
        self.device = int(device)
        if dtype not in ("f32", "f64"):
            raise ValueError("dtype must be 'f32' or 'f64'")
        if decision not in ("fp64", "fp32"):
            raise ValueError("decision must be 'fp64' or 'fp32'")
        if walk not in _WALKS:
            raise ValueError("walk must be 'auto', 'strips' or 'pairs'")
        self.decision = decision
        opts = _Opts(COST_EUCLID if cost == "euclid" else COST_SQ, int(rho), int(grid),
                     1 if validate else 0, DECISION_FP32 if decision == "fp32" else DECISION_FP64,
                     float(band), 1 if dense_e else 0, _WALKS[walk])
        h = ctypes.c_void_p()
        _check(lib.wts_plan_create(ctypes.byref(h), self.device, self.n, self.d,
                                   F32 if dtype == "f32" else F64,
                                   off.ctypes.data_as(ctypes.c_void_p), self.L,
                                   ctypes.byref(opts)))
        self._h = h
        self._ws = {}

    @property
    def handle(self):
        return self._h

    def workspace_bytes(self, op: int) -> int:
        return int(load().wts_workspace_bytes(self._h, op))

    def workspace(self, op: int) -> torch.Tensor:
        """A cached, 256-byte aligned device buffer for operation `op`."""
        nbytes = self.workspace_bytes(op)
        ws = self._ws.get(op)
        if ws is None or ws[1] < nbytes:
            raw = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda:%d" % self.device)
            shift = (-raw.data_ptr()) % 256
            ws = (raw, nbytes, raw[shift:shift + nbytes])
            self._ws[op] = ws
        return ws[2]

    def set_workspace(self, op: int, buf: torch.Tensor):
        """Installs a caller-owned buffer as the workspace of `op` (uint8 on
        the plan's device, 256-byte aligned, at least workspace_bytes(op)
        bytes), for instance a view of memory that other work ordered on the
        same stream also uses."""
        nbytes = self.workspace_bytes(op)
        if nbytes == 0:
            raise ValueError("this plan cannot run operation %d" % op)
        _buffer_arg(self, buf, "workspace", nbytes)
        self._ws[op] = (buf, nbytes, buf[:nbytes])

    def enable_timing(self, max_launches: int = 256):
        """Bracket every sweep kernel of this plan with HIP events (eager use only)."""
        _check(load().wts_plan_timing(self._h, int(max_launches)))

    def sweep_ms(self, op: int):
        """(total ms, launches) of the sweep kernels of `op` recorded since the last query."""
        tot = ctypes.c_double(0.0)
        cnt = ctypes.c_int32(0)
        _check(load().wts_plan_sweep_ms(self._h, int(op), ctypes.byref(tot), ctypes.byref(cnt)))
        return tot.value, cnt.value

    def walk(self) -> str:
        """The path recovery of this plan's barycenter calls: "strips" or "pairs"."""
        w = int(load().wts_plan_walk(self._h))
        _check(min(w, 0))
        return {1: "strips", 2: "pairs"}[w]

    def bwd_tiles(self):
        """(tiles swept, tiles in range) of the Soft-DTW backward kernels of this
        plan since the last query (waits for the device; eager use only)."""
        sw = ctypes.c_int64(0)
        tot = ctypes.c_int64(0)
        _check(load().wts_plan_bwd_tiles(self._h, ctypes.byref(sw), ctypes.byref(tot)))
        return sw.value, tot.value

    def rho(self, op: int) -> int:
        """Rows per lane of the sweeps `op` runs on this plan (names the kernel instance)."""
        r = int(load().wts_plan_rho(self._h, int(op)))
        _check(min(r, 0))
        return r

    def status(self) -> int:
        """Reads and clears the plan's device status word after synchronising
        the current stream: OK, E_NONFINITE (a validated call found a NaN or
        an infinity) or E_DEVICE (a strip gave up waiting, or inconsistent
        path tags)."""
        return int(load().wts_plan_status(self._h, _stream()))

    def check(self):
        """status(), raising WtsError unless it is OK."""
        _check(self.status())

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.wts_plan_destroy(self._h)
            self._h = None
        self._ws = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pack_cycles(cycles: Sequence[np.ndarray], device: int = 0, dtype: Optional[str] = None):
    """Host ragged cycles -> (device tensor [sum N][d], int64 offsets)."""
    lens = np.array([c.shape[0] for c in cycles], dtype=np.int64)
    off = np.zeros(len(cycles) + 1, dtype=np.int64)
    off[1:] = np.cumsum(lens)
    vals = np.concatenate([np.asarray(c).reshape(c.shape[0], -1) for c in cycles], axis=0)
    if dtype is None:
        dtype = "f32" if vals.dtype == np.float32 else "f64"
    vals = vals.astype(np.float32 if dtype == "f32" else np.float64, copy=False)
    t = torch.from_numpy(np.ascontiguousarray(vals)).to("cuda:%d" % device)
    return t, off, dtype


def _dev(plan: Plan):
    return "cuda:%d" % plan.device


def dtw_align(plan: Plan, bary: torch.Tensor, cycles: torch.Tensor, paths: bool = False):
    """Eq. 1 per cycle: (dist [n] f64, path_len [n] i64, paths or None).

    With paths=True the path rows of cycle k start at k*(L-1) + offsets[k]."""
    _bary_arg(plan, bary)
    _cycles_arg(plan, cycles)
    n = plan.n
    dist = torch.empty(n, dtype=torch.float64, device=_dev(plan))
    plen = torch.empty(n, dtype=torch.int64, device=_dev(plan))
    pth = None
    op = OP_ALIGN
    if paths:
        rows = n * (plan.L - 1) + int(plan.offsets[-1])
        pth = torch.empty((rows, 2), dtype=torch.int32, device=_dev(plan))
        op = OP_ALIGN_PATHS
    ws = plan.workspace(op)
    _check(load().wts_dtw_align(plan.handle, _ptr(bary), _ptr(cycles), _ptr(dist), _ptr(plen),
                                _ptr(pth), _ptr(ws), ws.numel(), _stream()))
    return dist, plen, pth


def path_of(plan: Plan, paths: torch.Tensor, path_len: torch.Tensor, k: int) -> np.ndarray:
    base = k * (plan.L - 1) + int(plan.offsets[k])
    return paths[base:base + int(path_len[k])].cpu().numpy()


def dba_iterate(plan: Plan, bary_in: torch.Tensor, cycles: torch.Tensor,
                weights: Optional[torch.Tensor] = None, bary_out: Optional[torch.Tensor] = None,
                counts: Optional[torch.Tensor] = None, dist: Optional[torch.Tensor] = None):
    """One DBA update: returns (bary_out [L][d] f64, counts [L] i64, dist [n] f64)."""
    _bary_arg(plan, bary_in, "bary_in")
    _cycles_arg(plan, cycles)
    _vec_arg(plan, weights, "weights")
    if bary_out is None:
        bary_out = torch.empty((plan.L, plan.d), dtype=torch.float64, device=_dev(plan))
    if counts is None:
        counts = torch.empty(plan.L, dtype=torch.int64, device=_dev(plan))
    if dist is None:
        dist = torch.empty(plan.n, dtype=torch.float64, device=_dev(plan))
    _bary_arg(plan, bary_out, "bary_out")
    _vec_arg(plan, counts, "counts", n=plan.L, dtype=torch.int64)
    _vec_arg(plan, dist, "dist")
    ws = plan.workspace(OP_DBA)
    _check(load().wts_dba_iterate(plan.handle, _ptr(bary_in), _ptr(cycles), _ptr(weights),
                                  _ptr(bary_out), _ptr(counts), _ptr(dist), _ptr(ws), ws.numel(),
                                  _stream()))
    return bary_out, counts, dist


def anomaly_score(plan: Plan, bary: torch.Tensor, cycles: torch.Tensor):
    """Eq. 8: (score [n], dist [n], path_len [n])."""
    _bary_arg(plan, bary)
    _cycles_arg(plan, cycles)
    n = plan.n
    score = torch.empty(n, dtype=torch.float64, device=_dev(plan))
    dist = torch.empty(n, dtype=torch.float64, device=_dev(plan))
    plen = torch.empty(n, dtype=torch.int64, device=_dev(plan))
    ws = plan.workspace(OP_SCORE)
    _check(load().wts_anomaly_score(plan.handle, _ptr(bary), _ptr(cycles), _ptr(score),
                                    _ptr(dist), _ptr(plen), _ptr(ws), ws.numel(), _stream()))
    return score, dist, plen


def anomaly_score_noalloc(plan: Plan, bary: torch.Tensor, cycles: torch.Tensor,
                          score: Optional[torch.Tensor] = None,
                          dist: Optional[torch.Tensor] = None,
                          path_len: Optional[torch.Tensor] = None):
    """Eq. 8 through the entry point that allocates nothing (its workspace is
    the library's static device scratch): (score [n], dist [n] or None,
    path_len [n] or None).  Outputs given by the caller are filled in place;
    a missing score is allocated here, on the caller's side of the call."""
    _bary_arg(plan, bary)
    _cycles_arg(plan, cycles)
    if score is None:
        score = torch.empty(plan.n, dtype=torch.float64, device=_dev(plan))
    _vec_arg(plan, score, "score")
    _vec_arg(plan, dist, "dist")
    _vec_arg(plan, path_len, "path_len", dtype=torch.int64)
    _check(load().wts_anomaly_score_noalloc(plan.handle, _ptr(bary), _ptr(cycles), _ptr(score),
                                            _ptr(dist), _ptr(path_len), _stream()))
    return score, dist, path_len


def subdtw(plan: Plan, x: torch.Tensor, windows: torch.Tensor):
    """Sec. III-B, Eq. 2: Sub-DTW of the reference x ([L][d] float64) against
    every window of the plan's batch: (value [n] f64, a* [n] i64, b* [n] i64),
    0-based columns of each window."""
    _bary_arg(plan, x, "x")
    _cycles_arg(plan, windows, "windows")
    n = plan.n
    value = torch.empty(n, dtype=torch.float64, device=_dev(plan))
    a = torch.empty(n, dtype=torch.int64, device=_dev(plan))
    b = torch.empty(n, dtype=torch.int64, device=_dev(plan))
    ws = plan.workspace(OP_SUBDTW)
    _check(load().wts_subdtw(plan.handle, _ptr(x), _ptr(windows), _ptr(value), _ptr(a), _ptr(b),
                             _ptr(ws), ws.numel(), _stream()))
    return value, a, b


def medoid(plan: Plan, cycles: torch.Tensor, with_matrix: bool = True):
    """All-pairs DTW: (medoid index tensor [1] i32, D [n][n] or None, totals [n])."""
    _cycles_arg(plan, cycles)
    n = plan.n
    Dm = torch.empty((n, n), dtype=torch.float64, device=_dev(plan)) if with_matrix else None
    tot = torch.empty(n, dtype=torch.float64, device=_dev(plan))
    k = torch.empty(1, dtype=torch.int32, device=_dev(plan))
    ws = plan.workspace(OP_MEDOID)
    _check(load().wts_medoid(plan.handle, _ptr(cycles), _ptr(Dm), _ptr(tot), _ptr(k), _ptr(ws),
                             ws.numel(), _stream()))
    return k, Dm, tot


def init_barycenter(plan: Plan, cycles: torch.Tensor, kind: int, index: int = 0):
    """(bary [L][d] f64, index of the cycle used or -1 for the mean)."""
    _cycles_arg(plan, cycles)
    out = torch.empty((plan.L, plan.d), dtype=torch.float64, device=_dev(plan))
    chosen = ctypes.c_int32(-2)
    _check(load().wts_init_barycenter(plan.handle, _ptr(cycles), int(kind), int(index), _ptr(out),
                                      ctypes.byref(chosen), _stream()))
    return out, int(chosen.value)


def aligned_buffer(nbytes: int, device) -> torch.Tensor:
    """A 256-byte aligned uint8 view of nbytes on `device` (the view keeps
    its allocation alive)."""
    raw = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    shift = (-raw.data_ptr()) % 256
    buf = raw[shift:shift + int(nbytes)]
    buf._wts_base = raw
    return buf


def _buffer_arg(plan, t, what: str, nbytes: int):
    _need(t, what, torch.uint8, _device(plan), min_numel=nbytes)
    if t.data_ptr() % 256:
        raise ValueError("%s must be 256-byte aligned" % what)
    return t


def softdtw_forward(plan: Plan, bary: torch.Tensor, cycles: torch.Tensor, gamma: float,
                    ckpt: Optional[torch.Tensor] = None, value: Optional[torch.Tensor] = None):
    """Eq. 3-5: (values [n] f64, checkpoint buffer for softdtw_backward).

    ckpt: a caller-owned uint8 buffer of at least
    plan.workspace_bytes(OP_SOFT_FWD) bytes, 256-byte aligned (else one is
    allocated); value: a float64 [n] output (else allocated)."""
    _bary_arg(plan, bary)
    _cycles_arg(plan, cycles)
    nbytes = plan.workspace_bytes(OP_SOFT_FWD)
    if ckpt is None:
        ckpt = aligned_buffer(nbytes, _dev(plan))
    _buffer_arg(plan, ckpt, "ckpt", nbytes)
    if value is None:
        value = torch.empty(plan.n, dtype=torch.float64, device=_dev(plan))
    _vec_arg(plan, value, "value")
    _check(load().wts_softdtw_forward(plan.handle, _ptr(bary), _ptr(cycles), float(gamma),
                                      _ptr(value), _ptr(ckpt), ckpt.numel(), _stream()))
    return value, ckpt


def softdtw_backward(plan: Plan, bary: torch.Tensor, cycles: torch.Tensor, gamma: float,
                     ckpt: torch.Tensor, grad_value: Optional[torch.Tensor] = None,
                     with_mass: bool = False, grad: Optional[torch.Tensor] = None,
                     mass: Optional[torch.Tensor] = None, accumulate: bool = False):
    """Eq. 6-7: grad_bary [L][d] = sum_k grad_value_k dSoft-DTW_k/dB (and row mass).

    grad / mass: caller-owned float64 outputs ([L][d], [L]); with
    accumulate=True the sums start from their contents (cycle groups)."""
    _bary_arg(plan, bary)
    _cycles_arg(plan, cycles)
    _buffer_arg(plan, ckpt, "ckpt", plan.workspace_bytes(OP_SOFT_FWD))
    _vec_arg(plan, grad_value, "grad_value")
    if grad is None:
        if accumulate:
            raise ValueError("accumulate needs the grad (and mass) to add to")
        grad = torch.empty((plan.L, plan.d), dtype=torch.float64, device=_dev(plan))
    _bary_arg(plan, grad, "grad")
    if with_mass and mass is None:
        if accumulate:
            raise ValueError("accumulate needs the grad (and mass) to add to")
        mass = torch.empty(plan.L, dtype=torch.float64, device=_dev(plan))
    _vec_arg(plan, mass, "mass", n=plan.L)
    ws = plan.workspace(OP_SOFT_BWD)
    _check(load().wts_softdtw_backward(plan.handle, _ptr(bary), _ptr(cycles), float(gamma),
                                       _ptr(ckpt), ckpt.numel(), _ptr(grad_value), _ptr(grad),
                                       _ptr(mass), 1 if accumulate else 0, _ptr(ws), ws.numel(),
                                       _stream()))
    return (grad, mass) if mass is not None else grad


def softdtw_grad_cycles(plan: Plan, bary: torch.Tensor, cycles: torch.Tensor, gamma: float,
                        grad_value: Optional[torch.Tensor] = None):
    """Eq. 6 for the cycles: grad [sum N][d] f64, row j of cycle k holding
    grad_value_k dSoft-DTW^gamma(B, C_k)/dc_kj (the sweeps run with the
    cycles on the rows; cycles of the plan's dtype are widened to float64
    first, float64 cycles are taken as they are)."""
    _bary_arg(plan, bary)
    if cycles.dtype == torch.float64:    # already widened (any plan dtype)
        _need(cycles, "cycles", torch.float64, _device(plan),
              numel=int(plan.offsets[-1]) * plan.d)
    else:
        _cycles_arg(plan, cycles)
    _vec_arg(plan, grad_value, "grad_value")
    c64 = cycles.to(torch.float64).contiguous()
    grad = torch.empty_like(c64)
    ws = plan.workspace(OP_SOFT_GRAD_C)
    _check(load().wts_softdtw_grad_cycles(plan.handle, _ptr(bary), _ptr(c64), float(gamma),
                                          _ptr(grad_value), _ptr(grad), _ptr(ws), ws.numel(),
                                          _stream()))
    return grad


def barycenter_objective(values: torch.Tensor, weights: Optional[torch.Tensor] = None,
                         out: Optional[torch.Tensor] = None, accumulate: bool = False):
    """Eq. 7: out [1] float64 = [out +] sum_k weights_k values_k (ascending k)."""
    dev = values.device
    n = values.numel()
    _need(values, "values", torch.float64, dev, numel=n)
    if weights is not None:
        _need(weights, "weights", torch.float64, dev, numel=n)
    if out is None:
        if accumulate:
            raise ValueError("accumulate needs the output to add to")
        out = torch.empty(1, dtype=torch.float64, device=dev)
    _need(out, "out", torch.float64, dev, numel=1)
    _check(load().wts_barycenter_objective(_ptr(values), _ptr(weights), int(n),
                                           1 if accumulate else 0, _ptr(out), _stream()))
    return out


class SoftDTW(torch.autograd.Function):
    """values[k] = Soft-DTW^gamma(B, C_k) with the hand-written E-matrix backward.

    Usage: SoftDTW.apply(bary, plan, cycles, gamma) with bary a float64 [L][d]
    tensor and cycles the packed [sum N][d] buffer of the plan; the
    checkpoints of the forward are kept for the backward.  Gradients flow to
    the barycenter and, when it requires them, to the cycle buffer.  The
    backward reads the plan's status word and raises on a device error."""

    @staticmethod
    def forward(ctx, bary, plan, cycles, gamma):
        bary_c = bary.detach().contiguous()
        cyc = cycles.detach()
        value, ckpt = softdtw_forward(plan, bary_c, cyc, gamma)
        ctx.plan, ctx.cycles, ctx.gamma, ctx.ckpt = plan, cyc, gamma, ckpt
        ctx.save_for_backward(bary_c)
        return value

    @staticmethod
    def backward(ctx, grad_value):
        (bary_c,) = ctx.saved_tensors
        gv = grad_value.to(torch.float64).contiguous()
        grad_b = grad_c = None
        if ctx.needs_input_grad[0]:
            grad_b = softdtw_backward(ctx.plan, bary_c, ctx.cycles, ctx.gamma, ctx.ckpt, gv)
        ctx.ckpt = None
        if ctx.needs_input_grad[2]:
            grad_c = softdtw_grad_cycles(ctx.plan, bary_c, ctx.cycles, ctx.gamma, gv)
            grad_c = grad_c.to(ctx.cycles.dtype)
        ctx.plan.check()
        return grad_b, None, grad_c, None


class SoftDTWObjective(torch.autograd.Function):
    """f = sum_k w_k Soft-DTW^gamma(B, C_k) (Eq. 7), as a device scalar: the
    forward sweep gives the values, wts_barycenter_objective folds them in
    ascending k, and the backward runs the E-matrix sweep with upstream
    weights w_k times the incoming gradient of f.

    Usage: SoftDTWObjective.apply(bary, plan, cycles, gamma, weights)."""

    @staticmethod
    def forward(ctx, bary, plan, cycles, gamma, weights):
        bary_c = bary.detach().contiguous()
        value, ckpt = softdtw_forward(plan, bary_c, cycles.detach(), gamma)
        f = barycenter_objective(value, weights)
        ctx.plan, ctx.cycles, ctx.gamma, ctx.ckpt, ctx.weights = (plan, cycles.detach(), gamma,
                                                                  ckpt, weights)
        ctx.save_for_backward(bary_c)
        return f.reshape(())

    @staticmethod
    def backward(ctx, grad_f):
        (bary_c,) = ctx.saved_tensors
        w = ctx.weights if ctx.weights is not None else torch.ones(
            ctx.plan.n, dtype=torch.float64, device=bary_c.device)
        gv = (w * grad_f.to(torch.float64)).contiguous()   # chain rule through the sum
        grad_b = softdtw_backward(ctx.plan, bary_c, ctx.cycles, ctx.gamma, ctx.ckpt, gv)
        ctx.ckpt = None
        ctx.plan.check()
        return grad_b, None, None, None, None


def precond_step(bary: torch.Tensor, grad: torch.Tensor, row_mass: torch.Tensor, eta: float):
    """In place: bary <- bary - eta * grad / (2 row_mass) (Soft-DTW barycenter descent)."""
    if bary.dim() != 2:
        raise ValueError("bary must be [L][d]")
    L, d = bary.shape
    _need(bary, "bary", torch.float64, bary.device)
    _need(grad, "grad", torch.float64, bary.device, shape=(L, d))
    _need(row_mass, "row_mass", torch.float64, bary.device, numel=L)
    _check(load().wts_precond_step(_ptr(bary), _ptr(grad), _ptr(row_mass), int(L), int(d),
                                   float(eta), _stream()))
    return bary


# ------------------------------------------------------------------ drivers

class DBARunner:
    """Runs DBA iterations on a fixed plan.  With graph=True the two
    ping-pong iterations (A -> B -> A) are captured once into a hipGraph
    (torch.cuda.CUDAGraph on the plan's device) and replayed; every kernel of
    an iteration, including the zeroing of the sweep's counters, is in it."""

    def __init__(self, plan: Plan, cycles: torch.Tensor, bary0: torch.Tensor,
                 weights: Optional[torch.Tensor] = None, graph: bool = True):
        _cycles_arg(plan, cycles)
        _vec_arg(plan, weights, "weights")
        self.plan, self.cycles, self.weights = plan, cycles, weights
        dev = _dev(plan)
        self.A = bary0.detach().to(device=dev, dtype=torch.float64).contiguous().clone()
        self.B = torch.empty_like(self.A)
        self.counts = torch.empty(plan.L, dtype=torch.int64, device=dev)
        self.dist = torch.empty(plan.n, dtype=torch.float64, device=dev)
        plan.workspace(OP_DBA)
        self.graph = None
        if graph:
            s = torch.cuda.Stream(device=dev)
            s.wait_stream(torch.cuda.current_stream(dev))
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                self._two()
            torch.cuda.current_stream(dev).wait_stream(s)
            self.graph = g

    def _two(self):
        dba_iterate(self.plan, self.A, self.cycles, self.weights, self.B, self.counts, self.dist)
        dba_iterate(self.plan, self.B, self.cycles, self.weights, self.A, self.counts, self.dist)

    def run(self, iters: int, check: bool = True) -> torch.Tensor:
        """Applies `iters` DBA iterations to the current barycenter; returns it.
        check=True then reads the plan's status word (a synchronisation)."""
        for _ in range(iters // 2):
            if self.graph is not None:
                self.graph.replay()
            else:
                self._two()
        if iters % 2:
            dba_iterate(self.plan, self.A, self.cycles, self.weights, self.B, self.counts,
                        self.dist)
            self.A, self.B = self.B, self.A
        if check:
            self.plan.check()
        return self.A


def subset_plans(offsets, d: int, dtype: str, L: int, max_ckpt_bytes: int, device: int = 0,
                 band: float = 0.0, grid: int = 0):
    """Splits a batch into consecutive cycle groups whose Soft-DTW checkpoint
    buffer stays below max_ckpt_bytes.  Returns [(first, last+1, plan)].

    Groups are grown greedily with a per-cycle size estimate (strip rows plus
    the 16-step sweep states) and then checked against the plan's own count."""
    off = np.asarray(offsets, dtype=np.int64)
    n = off.size - 1
    strips = -(-L // 128)

    def est(k):
        N = int(off[k + 1] - off[k])
        wt = -(-(N + 63) // 16)
        return strips * N * 8 + strips * wt * 3 * 64 * 8

    groups, a = [], 0
    while a < n:
        b, tot = a, 0
        while b < n and (b == a or tot + est(b) <= max_ckpt_bytes):
            tot += est(b)
            b += 1
        while True:
            plan = Plan(off[a:b + 1] - off[a], d, dtype, L, device=device, band=band, grid=grid)
            if b == a + 1 or plan.workspace_bytes(OP_SOFT_FWD) <= max_ckpt_bytes:
                break
            plan.close()
            b -= 1
        groups.append((a, b, plan))
        a = b
    return groups


class SoftDescent:
    """Preconditioned Soft-DTW descent steps (Eq. 7, weights w_k) over cycle
    groups whose checkpoints fit in memory: per group one forward and one
    backward (accumulating into one gradient and row mass, which gives
    bitwise the result of one call over all cycles), the Eq. 7 objective
    folded the same way, then bary <- bary - eta G / (2 h).

    Every buffer is allocated here, once: the checkpoint buffer is shared by
    the groups (ckpt: a caller-owned 256-byte aligned uint8 buffer of at
    least ckpt_bytes(groups) bytes, for instance one that other stream-ordered
    work also uses; else one is allocated), so step() allocates nothing and
    can be captured into a graph."""

    def __init__(self, groups, cycles: torch.Tensor, offsets, L: int, d: int, gamma: float,
                 grad_value: torch.Tensor, eta: float, ckpt: Optional[torch.Tensor] = None):
        self.groups = groups
        off = np.asarray(offsets, dtype=np.int64)
        dev = groups[0][2].device
        n = off.size - 1
        self.gamma, self.eta = float(gamma), float(eta)
        self.parts = []
        for a, b, plan in groups:
            Y = cycles[int(off[a]):int(off[b])]
            _cycles_arg(plan, Y, "cycles of group %d..%d" % (a, b))
            plan.workspace(OP_SOFT_BWD)
            self.parts.append((plan, Y, grad_value[a:b], a, b))
        need = self.ckpt_bytes(groups)
        self.ckpt = aligned_buffer(need, "cuda:%d" % dev) if ckpt is None else ckpt
        self.G = torch.empty((L, d), dtype=torch.float64, device="cuda:%d" % dev)
        self.H = torch.empty(L, dtype=torch.float64, device="cuda:%d" % dev)
        self.values = torch.empty(n, dtype=torch.float64, device="cuda:%d" % dev)
        self.objective = torch.empty(1, dtype=torch.float64, device="cuda:%d" % dev)
        self.grad_value = _need(grad_value, "grad_value", torch.float64, self.G.device, numel=n)

    @staticmethod
    def ckpt_bytes(groups) -> int:
        return max(plan.workspace_bytes(OP_SOFT_FWD) for _, _, plan in groups)

    def step(self, bary: torch.Tensor, check: bool = False) -> torch.Tensor:
        """One descent step on bary (in place); returns the values at the old
        bary.  The objective sum_k w_k value_k is left in self.objective."""
        for q, (plan, Y, gv, a, b) in enumerate(self.parts):
            ck = self.ckpt[:plan.workspace_bytes(OP_SOFT_FWD)]
            v, _ = softdtw_forward(plan, bary, Y, self.gamma, ckpt=ck, value=self.values[a:b])
            softdtw_backward(plan, bary, Y, self.gamma, ck, gv, grad=self.G, mass=self.H,
                             accumulate=q > 0)
            barycenter_objective(v, gv, out=self.objective, accumulate=q > 0)
        precond_step(bary, self.G, self.H, self.eta)
        if check:
            for _, _, plan in self.groups:
                plan.check()
        return self.values


def softdtw_descent_step(groups, cycles: torch.Tensor, offsets, bary: torch.Tensor,
                         gamma: float, grad_value: torch.Tensor, eta: float):
    """One preconditioned Soft-DTW descent step over cycle groups (see
    SoftDescent); returns the values at the old bary."""
    sd = SoftDescent(groups, cycles, offsets, bary.shape[0], bary.shape[1], gamma, grad_value, eta)
    return sd.step(bary, check=True)


def segment_alpha(M: int) -> int:
    """alpha = 0.15 M (Sec. III-B), in whole samples (rounded down)."""
    return int(0.15 * M)


def segment(x: torch.Tensor, streams: Sequence[torch.Tensor], dtype: str,
            alpha: Optional[int] = None, device: int = 0, decision: str = "fp64"):
    """The segmentation of Sec. III-B for several streams at once.

    Each stream s keeps a window start ws_s (0 at first).  Every round runs
    one Sub-DTW launch over the windows streams[s][ws_s : ws_s + 2M] of the
    streams not yet finished, records the cycle [ws_s + a*, ws_s + b*] of
    each, and moves ws_s to ws_s + b* - alpha -- or, where that would not
    move it forward, to ws_s + b* + 1 -- until ws_s reaches the end of its
    stream.  x: [M][d] float64 reference;
    streams: [N_s][d] tensors of the plans' storage dtype.  Returns, per
    stream, the list of (a*, b*, value) with absolute sample indices.

    Plans are cached by window lengths, so rounds in which every window is
    2M long reuse one plan.  decision: the plans' decision precision ("fp32"
    needs float32 streams)."""
    M, d = int(x.shape[0]), int(x.shape[1])
    if x.dtype != torch.float64 or not x.is_contiguous():
        raise ValueError("x must be a contiguous float64 [M][d] tensor")
    want = torch.float32 if dtype == "f32" else torch.float64
    for y in streams:
        if y.dtype != want or y.dim() != 2 or int(y.shape[1]) != d:
            raise ValueError("every stream must be a [N][%d] %s tensor" % (d, want))
    al = segment_alpha(M) if alpha is None else int(alpha)
    if al < 0:
        raise ValueError("alpha must be >= 0")
    ws = [0] * len(streams)
    out = [[] for _ in streams]
    plans = {}
    try:
        while True:
            live = [k for k, y in enumerate(streams) if ws[k] < y.shape[0]]
            if not live:
                break
            ends = [min(ws[k] + 2 * M, streams[k].shape[0]) for k in live]
            lens = tuple(e - ws[k] for k, e in zip(live, ends))
            plan = plans.get(lens)
            if plan is None:
                off = np.zeros(len(lens) + 1, dtype=np.int64)
                off[1:] = np.cumsum(lens)
                plan = plans[lens] = Plan(off, d, dtype, M, device=device, decision=decision)
            win = torch.cat([streams[k][ws[k]:e] for k, e in zip(live, ends)]).contiguous()
            v, a, b = subdtw(plan, x, win)
            v, a, b = v.cpu().numpy(), a.cpu().numpy(), b.cpu().numpy()
            for q, k in enumerate(live):
                out[k].append((ws[k] + int(a[q]), ws[k] + int(b[q]), float(v[q])))
                bq = int(b[q])
                ws[k] = ws[k] + bq - al if bq - al > 0 else ws[k] + bq + 1
    finally:
        for p in plans.values():
            p.close()
    return out


def lbfgs_barycenter(plan: Plan, cycles: torch.Tensor, bary0: torch.Tensor, gamma: float,
                     weights: Optional[torch.Tensor] = None, max_iter: int = 40,
                     max_eval: int = 200, tolerance_grad: float = 1e-8,
                     tolerance_change: float = 1e-5, history_size: int = 10):
    """Soft-DTW barycenter with the optimizer of the paper's Table I: L-BFGS
    on f(B) = sum_k w_k Soft-DTW^gamma(B, C_k) (Eq. 7 with w_k = lambda_k / m_k
    supplied by the caller; default 1), at most `max_iter` iterations and
    `max_eval` evaluations of f, stopping on a gradient of max-norm below
    `tolerance_grad` or a change of f or B below `tolerance_change`.  Every
    evaluation is one forward (checkpoints), the Eq. 7 sum and one E-matrix
    backward on the GPU (SoftDTWObjective); torch.optim.LBFGS (strong-Wolfe
    line search) only combines the resulting [L][d] gradients.  Returns
    (B, history of f values)."""
    B = bary0.detach().to(dtype=torch.float64).contiguous().clone().requires_grad_(True)
    w = (torch.ones(plan.n, dtype=torch.float64, device=B.device) if weights is None
         else weights.to(device=B.device, dtype=torch.float64).contiguous())
    opt = torch.optim.LBFGS([B], lr=1.0, max_iter=max_iter, max_eval=max_eval,
                            tolerance_grad=tolerance_grad, tolerance_change=tolerance_change,
                            history_size=history_size, line_search_fn="strong_wolfe")
    hist = []

    def closure():
        opt.zero_grad()
        f = SoftDTWObjective.apply(B, plan, cycles, gamma, w)
        f.backward()
        hist.append(float(f.detach()))
        return f.detach()

    opt.step(closure)
    return B.detach(), hist
