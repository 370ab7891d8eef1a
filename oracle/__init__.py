"""FP64 CPU oracle for the WETSAND hot path -- TEST INFRASTRUCTURE ONLY.

The hard-DTW programs (cost, DTW with its path, Sub-DTW) also run in float32
from the same C source (``fp32=True``, ``dtw32``, ``cost32``): the reference
of the float32-decision variant of the sweeps.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path
(``paper_2404_12134_amd``) never imports, links or calls it, and the two share
no code: the C source ``wts_oracle.c`` is a plain transcription of the
paper's definitions (Sec. III, Eq. 1-8) in FP64, and ``brute.py`` enumerates
every alignment path of tiny inputs to pin it.

``build()`` compiles ``wts_oracle.c`` with gcc (-O2 -ffp-contract=off,
OpenMP); ``lib()`` loads it, building it first if no library is there.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "wts_oracle.c")
SO = os.path.join(HERE, "libwts_oracle.so")

SQEUCLID, EUCLID = 0, 1

_lib = None


def build() -> str:
    """Compile the oracle shared library (always recompiles)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-o", SO + ".tmp", SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(SO + ".tmp", SO)
    return SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(SO):
            build()
        L = ctypes.CDLL(SO)
        P, I64, I32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        L.wts_o_cost.restype = D
        L.wts_o_cost.argtypes = [P, P, I32, I32]
        L.wts_o_cost32.restype = ctypes.c_float
        L.wts_o_cost32.argtypes = [P, P, I32, I32]
        L.wts_o_dtw.argtypes = [P, I64, P, I64, I32, I32, P, P, P, P]
        L.wts_o_dtw32.argtypes = [P, I64, P, I64, I32, I32, P, P, P, P]
        L.wts_o_dtw_batch.argtypes = [P, I64, P, P, I32, I32, I32, P, P, I32]
        L.wts_o_score_batch.argtypes = [P, I64, P, P, I32, I32, I32, P, P, P, I32]
        L.wts_o_dba_iterate.argtypes = [P, I64, P, P, I32, I32, P, P, P, P, P, I32]
        L.wts_o_softdtw.argtypes = [P, I64, P, I64, I32, D, P, P]
        L.wts_o_softdtw_band.argtypes = [P, I64, P, I64, I32, D, D, P, P]
        L.wts_o_softdtw_grad_band.argtypes = [P, I64, P, I64, I32, D, D, P, P, P, P]
        L.wts_o_softdtw_grad_ckpt.argtypes = [P, I64, P, I64, I32, D, D, P, P, P]
        L.wts_o_softdtw_batch_band.argtypes = [P, I64, P, P, I32, I32, D, D, P, P, P, P]
        L.wts_o_band_cols.argtypes = [I64, I64, D, I64, P, P]
        L.wts_o_band_cols.restype = None
        L.wts_o_softdtw_grad.argtypes = [P, I64, P, I64, I32, D, P, P, P, P]
        L.wts_o_softdtw_batch.argtypes = [P, I64, P, P, I32, I32, D, P, P, P, P]
        L.wts_o_medoid.argtypes = [P, P, I32, I32, P, P, I32]
        L.wts_o_subdtw.argtypes = [P, I64, P, I64, I32, I32, P, P, P]
        L.wts_o_subdtw32.argtypes = [P, I64, P, I64, I32, I32, P, P, P]
        L.wts_o_subdtw_batch.argtypes = [P, I64, P, P, I32, I32, I32, P, P, P, I32]
        L.wts_o_resample.argtypes = [P, I64, I32, I64, P]
        L.wts_o_resample.restype = None
        L.wts_o_euclid_mean.argtypes = [P, P, I32, I32, I64, P]
        L.wts_o_nearest_init.argtypes = [P, P, I32, I32, I64, P]
        for f in ("wts_o_dtw", "wts_o_dtw32", "wts_o_subdtw32", "wts_o_dtw_batch", "wts_o_score_batch", "wts_o_dba_iterate",
                  "wts_o_softdtw", "wts_o_softdtw_grad", "wts_o_softdtw_batch", "wts_o_medoid",
                  "wts_o_euclid_mean", "wts_o_nearest_init", "wts_o_num_threads",
                  "wts_o_subdtw", "wts_o_subdtw_batch", "wts_o_softdtw_band",
                  "wts_o_softdtw_grad_band", "wts_o_softdtw_batch_band",
                  "wts_o_softdtw_grad_ckpt"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _series(x):
    x = _f64(x)
    return x if x.ndim == 2 else x.reshape(-1, 1)


def _packed(cycles):
    cyc = [_series(c) for c in cycles]
    off = np.zeros(len(cyc) + 1, dtype=np.int64)
    off[1:] = np.cumsum([c.shape[0] for c in cyc])
    return _f64(np.concatenate(cyc, axis=0)), off


def _check(rc):
    if rc != 0:
        raise MemoryError("oracle allocation failed")


def num_threads() -> int:
    return int(lib().wts_o_num_threads())


def cost(x, y, kind=SQEUCLID) -> float:
    x, y = _f64(x).ravel(), _f64(y).ravel()
    return float(lib().wts_o_cost(_p(x), _p(y), x.size, kind))


def dtw(X, Y, kind=SQEUCLID, with_path=True, with_codes=False):
    """Eq. 1: returns (dist, |pi|, path [|pi|][2] or None, codes [M][N] or None)."""
    X, Y = _series(X), _series(Y)
    M, N, d = X.shape[0], Y.shape[0], X.shape[1]
    dist = np.zeros(1)
    plen = np.zeros(1, dtype=np.int64)
    path = np.zeros((M + N - 1, 2), dtype=np.int32) if with_path else None
    codes = np.zeros((M, N), dtype=np.uint8) if with_codes else None
    _check(lib().wts_o_dtw(_p(X), M, _p(Y), N, d, kind, _p(dist), _p(plen), _p(path),
                           _p(codes)))
    k = int(plen[0])
    return float(dist[0]), k, (path[:k].copy() if with_path else None), codes


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def cost32(x, y, kind=SQEUCLID) -> float:
    """Def. 3 evaluated in float32 on float32 inputs (the float32 program)."""
    x, y = _f32(x).ravel(), _f32(y).ravel()
    return float(lib().wts_o_cost32(_p(x), _p(y), x.size, kind))


def dtw32(X, Y, kind=SQEUCLID, with_path=True, with_codes=False):
    """Eq. 1 run in float32 on the inputs rounded to float32 (the reference
    of the float32-decision sweeps): returns (dist as float64, |pi|, path,
    codes) like dtw()."""
    X, Y = _f32(_series(X)), _f32(_series(Y))
    M, N, d = X.shape[0], Y.shape[0], X.shape[1]
    dist = np.zeros(1, dtype=np.float32)
    plen = np.zeros(1, dtype=np.int64)
    path = np.zeros((M + N - 1, 2), dtype=np.int32) if with_path else None
    codes = np.zeros((M, N), dtype=np.uint8) if with_codes else None
    _check(lib().wts_o_dtw32(_p(X), M, _p(Y), N, d, kind, _p(dist), _p(plen), _p(path),
                             _p(codes)))
    k = int(plen[0])
    return float(dist[0]), k, (path[:k].copy() if with_path else None), codes


def dtw_batch(X, cycles, kind=SQEUCLID, fp32=False):
    """Eq. 1 for every cycle: (dist, |pi|); fp32: float32 decisions."""
    X = _series(X)
    Y, off = _packed(cycles)
    n = len(cycles)
    dist = np.zeros(n)
    plen = np.zeros(n, dtype=np.int64)
    _check(lib().wts_o_dtw_batch(_p(X), X.shape[0], _p(Y), _p(off), n, X.shape[1], kind,
                                 _p(dist), _p(plen), int(bool(fp32))))
    return dist, plen


def score_batch(B, cycles, kind=SQEUCLID, fp32=False):
    """Eq. 8 for every cycle: returns (score, dist, |pi|); fp32: float32
    decisions."""
    B = _series(B)
    Y, off = _packed(cycles)
    n = len(cycles)
    score, dist = np.zeros(n), np.zeros(n)
    plen = np.zeros(n, dtype=np.int64)
    _check(lib().wts_o_score_batch(_p(B), B.shape[0], _p(Y), _p(off), n, B.shape[1], kind,
                                   _p(score), _p(dist), _p(plen), int(bool(fp32))))
    return score, dist, plen


def dba_iterate(B, cycles, weights=None, fp32=False):
    """One DBA iteration: returns (B', K counts, dist, |pi|); fp32: the paths
    from float32 decisions (sums and division in float64)."""
    B = _series(B)
    Y, off = _packed(cycles)
    n, L, d = len(cycles), B.shape[0], B.shape[1]
    w = None if weights is None else _f64(weights)
    Bout = np.zeros((L, d))
    counts = np.zeros(L, dtype=np.int64)
    dist = np.zeros(n)
    plen = np.zeros(n, dtype=np.int64)
    _check(lib().wts_o_dba_iterate(_p(B), L, _p(Y), _p(off), n, d, _p(w), _p(Bout), _p(counts),
                                   _p(dist), _p(plen), int(bool(fp32))))
    return Bout, counts, dist, plen


def band_cols(M: int, N: int, band: float, i: int):
    """Columns [jlo, jhi] of row i inside the Sakoe-Chiba band (Table I)."""
    lo = np.zeros(1, dtype=np.int64)
    hi = np.zeros(1, dtype=np.int64)
    lib().wts_o_band_cols(int(M), int(N), float(band), int(i), _p(lo), _p(hi))
    return int(lo[0]), int(hi[0])


def softdtw(X, Y, gamma, with_R=False, band=0.0):
    """Eq. 3-5 (band > 0: restricted to the Sakoe-Chiba band of Table I)."""
    X, Y = _series(X), _series(Y)
    M, N = X.shape[0], Y.shape[0]
    v = np.zeros(1)
    R = np.zeros((M, N)) if with_R else None
    _check(lib().wts_o_softdtw_band(_p(X), M, _p(Y), N, X.shape[1], float(gamma), float(band),
                                    _p(v), _p(R)))
    return (float(v[0]), R) if with_R else float(v[0])


def softdtw_grad(X, Y, gamma, with_E=False, band=0.0):
    """Eq. 6: returns (value, grad [M][d], rowmass [M], E [M][N] or None)."""
    X, Y = _series(X), _series(Y)
    M, N, d = X.shape[0], Y.shape[0], X.shape[1]
    v = np.zeros(1)
    g = np.zeros((M, d))
    h = np.zeros(M)
    E = np.zeros((M, N)) if with_E else None
    _check(lib().wts_o_softdtw_grad_band(_p(X), M, _p(Y), N, d, float(gamma), float(band),
                                         _p(v), _p(g), _p(h), _p(E)))
    return float(v[0]), g, h, E


def softdtw_grad_ckpt(X, Y, gamma, band=0.0):
    """Eq. 6 with square-root checkpointing of R (memory ~2 sqrt(M) N doubles,
    for pairs of 50k samples): returns (value, grad [M][d], rowmass [M]),
    bitwise those of softdtw_grad."""
    X, Y = _series(X), _series(Y)
    M, N, d = X.shape[0], Y.shape[0], X.shape[1]
    v = np.zeros(1)
    g = np.zeros((M, d))
    h = np.zeros(M)
    _check(lib().wts_o_softdtw_grad_ckpt(_p(X), M, _p(Y), N, d, float(gamma), float(band),
                                         _p(v), _p(g), _p(h)))
    return float(v[0]), g, h


def softdtw_grad_y(X, Y, gamma, band=0.0):
    """Eq. 6 taken with respect to the second series: the cost of cell (i, j)
    depends on y_j through ||x_i - y_j||^2, whose derivative is 2 (y_j - x_i),
    so d Soft-DTW / d y_j = sum_i e_ij 2 (y_j - x_i).  E comes from the
    oracle's own backward recursion; returns (value, grad [N][d])."""
    X, Y = _series(X), _series(Y)
    v, _, _, E = softdtw_grad(X, Y, gamma, with_E=True, band=band)
    colmass = E.sum(axis=0)
    return v, 2.0 * (colmass[:, None] * Y - E.T @ X)


def softdtw_batch(X, cycles, gamma, weights=None, grad=True, band=0.0):
    """Values [n] and, if grad, (sum_i w_i dSDTW_i/dX [M][d], sum_i w_i rowmass_i [M])."""
    X = _series(X)
    Y, off = _packed(cycles)
    n, M, d = len(cycles), X.shape[0], X.shape[1]
    w = None if weights is None else _f64(weights)
    vals = np.zeros(n)
    g = np.zeros((M, d)) if grad else None
    h = np.zeros(M) if grad else None
    _check(lib().wts_o_softdtw_batch_band(_p(X), M, _p(Y), _p(off), n, d, float(gamma),
                                          float(band), _p(w), _p(vals), _p(g), _p(h)))
    return (vals, g, h) if grad else vals


def medoid(cycles, fp32=False):
    Y, off = _packed(cycles)
    n, d = len(cycles), Y.shape[1]
    D = np.zeros((n, n))
    k = np.zeros(1, dtype=np.int32)
    _check(lib().wts_o_medoid(_p(Y), _p(off), n, d, _p(D), _p(k), int(bool(fp32))))
    return int(k[0]), D


def resample(Y, L):
    Y = _series(Y)
    out = np.zeros((L, Y.shape[1]))
    lib().wts_o_resample(_p(Y), Y.shape[0], Y.shape[1], L, _p(out))
    return out


def euclid_mean(cycles, L):
    Y, off = _packed(cycles)
    out = np.zeros((L, Y.shape[1]))
    _check(lib().wts_o_euclid_mean(_p(Y), _p(off), len(cycles), Y.shape[1], L, _p(out)))
    return out


def nearest_init(cycles, L):
    Y, off = _packed(cycles)
    out = np.zeros((L, Y.shape[1]))
    k = lib().wts_o_nearest_init(_p(Y), _p(off), len(cycles), Y.shape[1], L, _p(out))
    return int(k), out


def subdtw(X, Y, kind=SQEUCLID, fp32=False):
    """Sub-DTW (Sec. III-B, Eq. 2): (value, a*, b*), 0-based columns of Y;
    fp32: the same program in float32 on the inputs rounded to float32."""
    a = np.zeros(1, dtype=np.int64)
    b = np.zeros(1, dtype=np.int64)
    if fp32:
        X, Y = _f32(_series(X)), _f32(_series(Y))
        v = np.zeros(1, dtype=np.float32)
        _check(lib().wts_o_subdtw32(_p(X), X.shape[0], _p(Y), Y.shape[0], X.shape[1], kind,
                                    _p(v), _p(a), _p(b)))
    else:
        X, Y = _series(X), _series(Y)
        v = np.zeros(1)
        _check(lib().wts_o_subdtw(_p(X), X.shape[0], _p(Y), Y.shape[0], X.shape[1], kind,
                                  _p(v), _p(a), _p(b)))
    return float(v[0]), int(a[0]), int(b[0])


def subdtw_batch(X, windows, kind=SQEUCLID, fp32=False):
    """Sub-DTW of X against every window: (values, a*, b*) arrays; fp32:
    float32 decisions."""
    X = _series(X)
    Y, off = _packed(windows)
    n = len(windows)
    v = np.zeros(n)
    a = np.zeros(n, dtype=np.int64)
    b = np.zeros(n, dtype=np.int64)
    _check(lib().wts_o_subdtw_batch(_p(X), X.shape[0], _p(Y), _p(off), n, X.shape[1], kind,
                                    _p(v), _p(a), _p(b), int(bool(fp32))))
    return v, a, b


def segment_alpha(M: int) -> int:
    """alpha = 0.15 M (Sec. III-B), rounded down to whole samples."""
    return int(0.15 * M)


def segment(X, Y, kind=SQEUCLID, fp32=False):
    """The segmentation loop of Sec. III-B, 0-based and half-open windows:
    ws = 0; repeat: window Y[ws : min(ws + 2M, N)], (a*, b*) of its Sub-DTW
    made absolute, cycle Y[a* .. b*] kept, ws <- b* - alpha, while ws < N.
    Where b* - alpha would not move the window forward (the paper does not
    say what then), it restarts just past the match: ws <- b* + 1.
    Returns [(a*, b*, value)] in order.  fp32: each Sub-DTW with float32
    decisions."""
    X, Y = _series(X), _series(Y)
    M, N = X.shape[0], Y.shape[0]
    alpha = segment_alpha(M)
    out = []
    ws = 0
    while ws < N:
        we = min(ws + 2 * M, N)
        v, a, b = subdtw(X, Y[ws:we], kind, fp32=fp32)
        out.append((ws + a, ws + b, v))
        ws = ws + b - alpha if b - alpha > 0 else ws + b + 1
    return out
