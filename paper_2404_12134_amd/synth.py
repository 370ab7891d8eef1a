"""Seeded synthetic workloads standing in for the paper's robot joint cycles.

The paper evaluates on private robot recordings (Sec. IV-A: 217 cycles of one
robot, joint trajectories of about 16k-18k samples, d = 9 channels in total or
one joint at a time; Sec. III-A: samples with missing values are dropped, so
cycles have uneven lengths).  Those recordings are not available, so every
workload here is drawn from a seeded generator with the same structure:
quasi-periodic cycles that are time-warped copies of one template, with
additive noise, uneven lengths, optional injected drifts (the anomalies) and
optional dropped-sample gaps.

This module only draws signals.  It computes no DTW value, path, barycenter,
gradient or score, so both the oracle and the HIP path can take their inputs
from it without sharing any of the method's arithmetic.

Recipe (shared by all configurations):

* template ``f`` on ``t in [0, 1]``;
* per cycle a monotone piecewise-linear warp ``w`` with ``w(0)=0``, ``w(1)=1``
  and four interior knots at ``u = k/5`` moved to ``u + U(-0.08, 0.08)``
  (sorted, clipped to (0, 1));
* sample ``k`` of an ``N``-sample cycle sits at ``t = k/(N-1)`` and takes the
  value ``f(w(t)) + N(0, 0.05^2)`` independently per sample and channel.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

NOISE_STD = 0.05
WARP_JITTER = 0.08


@dataclasses.dataclass
class Workload:
    """One batch of cycles plus how the hot path is driven over it."""

    name: str
    cycles: List[np.ndarray]          # each [N_i][d], time-major
    dtype: str                        # "f32" or "f64": storage type of the cycles
    L: Optional[int]                  # barycenter length (None: length of the medoid)
    init: str                         # "medoid" | "nearest" | "euclid"
    dba_iters: int = 0
    soft_steps: int = 0
    gammas: Sequence[float] = ()
    scores: bool = False
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return len(self.cycles)

    @property
    def d(self) -> int:
        return int(self.cycles[0].shape[1])

    @property
    def lengths(self) -> np.ndarray:
        return np.array([c.shape[0] for c in self.cycles], dtype=np.int64)


def pack(cycles: Sequence[np.ndarray]):
    """Concatenate ragged cycles into one time-major buffer plus int64 offsets."""
    lens = np.array([c.shape[0] for c in cycles], dtype=np.int64)
    off = np.zeros(len(cycles) + 1, dtype=np.int64)
    off[1:] = np.cumsum(lens)
    vals = np.ascontiguousarray(np.concatenate(cycles, axis=0))
    return vals, off


def _warp(rng: np.random.Generator):
    u = np.arange(1, 5) / 5.0
    v = np.sort(np.clip(u + rng.uniform(-WARP_JITTER, WARP_JITTER, 4), 1e-6, 1 - 1e-6))
    xs = np.concatenate([[0.0], u, [1.0]])
    ys = np.concatenate([[0.0], v, [1.0]])
    return xs, ys


def _times(N: int) -> np.ndarray:
    return np.zeros(1) if N == 1 else np.arange(N, dtype=np.float64) / (N - 1)


def _sine_template(t: np.ndarray) -> np.ndarray:
    return (np.sin(2 * np.pi * t) + 0.5 * np.sin(6 * np.pi * t))[:, None]


class _FourierTemplate:
    """Random smooth template: 8 harmonics per channel, each channel unit-std."""

    def __init__(self, rng: np.random.Generator, d: int, harmonics: int = 8):
        k = np.arange(1, harmonics + 1, dtype=np.float64)
        self.k = k
        self.a = rng.standard_normal((d, harmonics)) / k
        self.phi = rng.uniform(0.0, 2 * np.pi, (d, harmonics))
        grid = np.arange(4096) / 4095.0
        raw = self._raw(grid)
        self.mu = raw.mean(axis=0)
        self.sd = raw.std(axis=0)

    def _raw(self, t: np.ndarray) -> np.ndarray:
        out = np.zeros((t.shape[0], self.a.shape[0]))
        for c in range(self.a.shape[0]):
            ang = 2 * np.pi * t[:, None] * self.k[None, :] + self.phi[c][None, :]
            out[:, c] = (np.sin(ang) * self.a[c][None, :]).sum(axis=1)
        return out

    def __call__(self, t: np.ndarray) -> np.ndarray:
        return (self._raw(t) - self.mu) / self.sd


def _cycle(rng, template, N: int, d: int) -> np.ndarray:
    xs, ys = _warp(rng)
    t = _times(N)
    x = template(np.interp(t, xs, ys))
    return x + rng.normal(0.0, NOISE_STD, (N, d))


def _with_gaps(rng, x: np.ndarray, frac: float = 0.01, gap_lo: int = 1, gap_hi: int = 50):
    """Drop about ``frac`` of the samples in non-overlapping gaps of 1..50 samples.

    Mirrors the paper's data preparation: samples with missing values are
    removed, leaving an irregularly sampled series whose timestamps the
    kernels never see.
    """
    N = x.shape[0]
    keep = np.ones(N, dtype=bool)
    target = int(math.ceil(frac * N))
    dropped = 0
    while dropped < target:
        g = int(rng.integers(gap_lo, gap_hi + 1))
        s = int(rng.integers(1, N - g - 1))           # never drop the first/last sample
        lo, hi = s - 1, s + g + 1                     # keep gaps non-adjacent
        if keep[lo:hi].all():
            keep[s:s + g] = False
            dropped += g
    stamps = np.nonzero(keep)[0].astype(np.float64) / (N - 1)
    return np.ascontiguousarray(x[keep]), stamps


def make(k: int, *, n: Optional[int] = None, len_range=None, L: Optional[int] = None,
         seed: Optional[int] = None) -> Workload:
    """Build workload ``k`` (1..5) with optional overrides for smaller test copies.

    ``len_range`` replaces the (lo, hi) length range; ``L`` the barycenter
    length; ``n`` the number of cycles.  The seed defaults to ``k``.
    """
    rng = np.random.Generator(np.random.PCG64(k if seed is None else seed))
    if k == 1:
        n = 8 if n is None else n
        lo, hi = len_range or (200, 256)
        lens = rng.integers(lo, hi + 1, n)
        cyc = [_cycle(rng, _sine_template, int(N), 1) for N in lens]
        return Workload("c1_sine_n%d_d1_f64" % n, cyc, "f64", L, "medoid", dba_iters=5)
    if k == 2:
        n = 64 if n is None else n
        lo, hi = len_range or (4000, 6000)
        tmpl = _FourierTemplate(rng, 3)
        lens = rng.integers(lo, hi + 1, n)
        cyc = [_cycle(rng, tmpl, int(N), 3) for N in lens]
        n_drift = min(3, n)
        drift_idx = sorted(int(i) for i in rng.choice(n, n_drift, replace=False))
        for i in drift_idx:
            t = _times(cyc[i].shape[0])
            t0 = rng.uniform(0.1, 0.7)
            cyc[i] = cyc[i] + 0.3 * np.clip((t - t0) / 0.2, 0.0, 1.0)[:, None]
        cyc = [c.astype(np.float32) for c in cyc]
        return Workload("c2_fourier_n%d_d3_f32" % n, cyc, "f32", L, "medoid", dba_iters=10,
                        scores=True, meta={"drift": drift_idx})
    if k == 3:
        n = 512 if n is None else n
        lo, hi = len_range or (1000, 20000)
        tmpl = _FourierTemplate(rng, 6)
        lens = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), n))).astype(np.int64)
        cyc = [_cycle(rng, tmpl, int(N), 6).astype(np.float32) for N in lens]
        L = 10000 if L is None else L
        return Workload("c3_uneven_n%d_d6_f32_L%d" % (n, L), cyc, "f32", L, "nearest",
                        dba_iters=10)
    if k == 4:
        n = 128 if n is None else n
        lo, hi = len_range or (18000, 22000)
        tmpl = _FourierTemplate(rng, 6)
        lens = rng.integers(lo, hi + 1, n)
        cyc = [_cycle(rng, tmpl, int(N), 6).astype(np.float32) for N in lens]
        L = 20000 if L is None else L
        return Workload("c4_soft_n%d_d6_f32_L%d" % (n, L), cyc, "f32", L, "euclid",
                        soft_steps=50, gammas=(0.1, 1.0))
    if k == 5:
        n = 256 if n is None else n
        lo, hi = len_range or (40000, 50000)
        tmpl = _FourierTemplate(rng, 6)
        lens = rng.integers(lo, hi + 1, n)
        cyc, stamps = [], []
        for N in lens:
            x, ts = _with_gaps(rng, _cycle(rng, tmpl, int(N), 6))
            cyc.append(x.astype(np.float32))
            stamps.append(ts)
        Lmax = max(c.shape[0] for c in cyc)
        L = Lmax if L is None else L
        return Workload("c5_gaps_n%d_d6_f32_L%d" % (n, L), cyc, "f32", L, "nearest",
                        dba_iters=10, soft_steps=10, gammas=(0.1,), scores=True,
                        meta={"timestamps": stamps})
    raise ValueError("workload index must be 1..5")


def make_stream(seed: int, n_cycles: int, len_range=(15000, 17500), d: int = 3,
                idle_frac=(0.0, 0.08), dtype: str = "f32", template_seed: Optional[int] = None):
    """A long quasi-periodic stream for the segmentation step (Sec. III-B,
    Sec. V-A: a robot repeating its task): ``n_cycles`` warped, noisy copies
    of one template, each with about 1 % of its samples dropped in gaps, and
    after each an idle stretch (the last value held, plus noise) of
    U(idle_frac) times the cycle length.  The reference cycle X is one more
    such cycle, as an operator would delimit it.  Streams drawn with the same
    ``template_seed`` (default: ``seed``) repeat the same task.  Returns
    (X, Y, bounds) with bounds[k] = (first, last) sample of cycle k in Y."""
    tmpl = _FourierTemplate(
        np.random.Generator(np.random.PCG64(seed if template_seed is None else template_seed)), d)
    rng = np.random.Generator(np.random.PCG64((seed, 1)))
    lo, hi = len_range
    X, _ = _with_gaps(rng, _cycle(rng, tmpl, int(rng.integers(lo, hi + 1)), d))
    parts, bounds, pos = [], [], 0
    for _ in range(n_cycles):
        c, _ = _with_gaps(rng, _cycle(rng, tmpl, int(rng.integers(lo, hi + 1)), d))
        idle_n = int(rng.uniform(*idle_frac) * c.shape[0])
        idle = c[-1][None, :] + rng.normal(0.0, NOISE_STD, (idle_n, d))
        bounds.append((pos, pos + c.shape[0] - 1))
        parts += [c, idle]
        pos += c.shape[0] + idle_n
    Y = np.concatenate(parts)
    t = np.float32 if dtype == "f32" else np.float64
    return X.astype(t), Y.astype(t), bounds


def integer_pair(rng: np.random.Generator, L: int, N: int, d: int, hi: int = 3):
    """Small-integer series: exact arithmetic and many tied optimal paths."""
    x = rng.integers(0, hi + 1, (L, d)).astype(np.float64)
    y = rng.integers(0, hi + 1, (N, d)).astype(np.float64)
    return x, y


def dyadic(rng: np.random.Generator, shape, bits: int = 10, lo: float = -2.0, hi: float = 2.0):
    """Values on a 2^-bits grid: sums of a few of them are exact in FP64."""
    q = 1 << bits
    return np.rint(rng.uniform(lo, hi, shape) * q) / q
