"""Brute force over every complete alignment path -- pins the oracle.

TEST INFRASTRUCTURE ONLY.  Pure Python, for series of length <= 6 or so.
It does not run a dynamic program: it lists every alignment path of
Def. 1 (steps (0,1), (1,0), (1,1) from (1,1) to (M,N)) and evaluates the
definitions directly:

* DTW (Eq. 1): the minimum over paths of <A, Delta>.
* Soft-DTW (Eq. 4): -gamma log sum_paths exp(-<A, Delta> / gamma).
* E (the matrix of Eq. 6): the Gibbs expectation of the alignment matrix,
  sum_paths A * p(path) with p proportional to exp(-<A, Delta> / gamma).
  This is the derivative of Soft-DTW with respect to Delta.
* the optimal path under the tie-break that the oracle's backtrack applies:
  among the paths of minimal cost, the one whose backward step sequence
  (from (M, N) towards (1, 1)) is lexicographically smallest with
  diag < up < left.

The number of complete paths of an M x N grid is the Delannoy number
D(M-1, N-1) = sum_k C(M-1, k) C(N-1, k) 2^k.

Float32 arithmetic (for the float32-decision program): every operation is
evaluated exactly on rationals and rounded once to the nearest float32
(ties to even), so a path's cost is its cost summed in float32 in path
order.  Rounding to nearest is monotone, so the minimum over paths of these
sums is what a float32 dynamic program computes.
"""

from __future__ import annotations

import math
from fractions import Fraction
from functools import lru_cache
from typing import List, Tuple

import numpy as np

DIAG, UP, LEFT = 0, 1, 2


def delannoy(m: int, n: int) -> int:
    return sum(math.comb(m, k) * math.comb(n, k) * (1 << k) for k in range(min(m, n) + 1))


def all_paths(M: int, N: int) -> List[List[Tuple[int, int]]]:
    """Every complete alignment path of an M x N grid, 0-based, forward order."""

    @lru_cache(maxsize=None)
    def from_cell(i, j):
        if i == M - 1 and j == N - 1:
            return [((i, j),)]
        out = []
        for di, dj in ((0, 1), (1, 0), (1, 1)):
            a, b = i + di, j + dj
            if a < M and b < N:
                out.extend(((i, j),) + rest for rest in from_cell(a, b))
        return out

    return [list(p) for p in from_cell(0, 0)]


def fma(a: float, b: float, c: float) -> float:
    """a*b + c rounded once (exact rational arithmetic, then one rounding)."""
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def delta(x, y, kind="sq"):
    """Def. 3, squared Euclidean (or its square root), same operation order
    as the oracle: e_0*e_0, then fma(e_c, e_c, s)."""
    x = np.asarray(x, dtype=np.float64).ravel()
    y = np.asarray(y, dtype=np.float64).ravel()
    e = float(x[0] - y[0])
    s = e * e
    for c in range(1, x.size):
        e = float(x[c] - y[c])
        s = fma(e, e, s)
    return math.sqrt(s) if kind == "l2" else s


def path_cost(X, Y, path, kind="sq") -> float:
    """<A, Delta> accumulated along the path from (1,1), c = delta + c."""
    c = 0.0
    for i, j in path:
        c = delta(X[i], Y[j], kind) + c
    return c


def backward_steps(path) -> Tuple[int, ...]:
    steps = []
    for (i0, j0), (i1, j1) in zip(path[-2::-1], path[::-1]):
        di, dj = i1 - i0, j1 - j0
        steps.append(DIAG if (di, dj) == (1, 1) else UP if (di, dj) == (1, 0) else LEFT)
    return tuple(steps)


def _series(a):
    a = np.asarray(a, dtype=np.float64)
    return a.reshape(-1, 1) if a.ndim == 1 else a


def dtw(X, Y, kind="sq"):
    """Returns (min cost, tie-broken optimal path, number of optimal paths)."""
    X, Y = _series(X), _series(Y)
    paths = all_paths(X.shape[0], Y.shape[0])
    costs = [path_cost(X, Y, p, kind) for p in paths]
    best = min(costs)
    opt = [p for p, c in zip(paths, costs) if c == best]
    chosen = min(opt, key=backward_steps)
    return best, chosen, len(opt)


def subdtw(X, Y, kind="sq"):
    """Sub-DTW by enumeration: every complete path of X against every
    subsequence Y[a..b].  Returns (min cost, a*, b*) where b* is the lowest
    end column of an optimal path and a* the start of the optimal path ending
    there whose backward steps, followed by the entry from the row above
    (ranked as a diagonal step), are lexicographically smallest."""
    X, Y = _series(X), _series(Y)
    M, N = X.shape[0], Y.shape[0]
    cands = []
    for a in range(N):
        for b in range(a, N):
            for p in all_paths(M, b - a + 1):
                path = [(i, j + a) for i, j in p]
                cands.append((path_cost(X, Y, path, kind), b, path))
    best = min(c for c, _, _ in cands)
    b_star = min(b for c, b, _ in cands if c == best)
    opt = [p for c, b, p in cands if c == best and b == b_star]
    chosen = min(opt, key=lambda p: backward_steps(p) + (DIAG,))
    return best, chosen[0][1], b_star


def in_band(i: int, j: int, M: int, N: int, w: float) -> bool:
    """Sakoe-Chiba band of Table I, as the oracle reads it: a band of radius
    R = ceil(w max(M, N)) around the diagonal from (0, 0) to (M-1, N-1),
    measured along the longer side (R at least ceil(max(M-1, N-1) /
    min(M-1, N-1))); w <= 0 is no band."""
    if w <= 0 or M == 1 or N == 1:
        return True
    a, b = M - 1, N - 1
    R = max(math.ceil(w * max(M, N)), -(-max(a, b) // min(a, b)))
    return abs(i * b - j * a) <= R * min(a, b)


def band_paths(M: int, N: int, w: float):
    return [p for p in all_paths(M, N) if all(in_band(i, j, M, N, w) for i, j in p)]


def softdtw(X, Y, gamma, band=0.0):
    X, Y = _series(X), _series(Y)
    costs = np.array([path_cost(X, Y, p) for p in band_paths(X.shape[0], Y.shape[0], band)])
    m = costs.min()
    return float(m - gamma * math.log(math.fsum(np.exp(-(costs - m) / gamma))))


def gibbs_E(X, Y, gamma, band=0.0):
    """E = sum over paths (inside the band) of A(path) * p(path)."""
    X, Y = _series(X), _series(Y)
    M, N = X.shape[0], Y.shape[0]
    paths = band_paths(M, N, band)
    costs = np.array([path_cost(X, Y, p) for p in paths])
    wts = np.exp(-(costs - costs.min()) / gamma)
    wts = wts / math.fsum(wts)
    E = np.zeros((M, N))
    for p, w in zip(paths, wts):
        for i, j in p:
            E[i, j] += w
    return E


def dba_iterate(B, cycles, weights=None):
    """One DBA step computed from brute-force optimal paths, summed in the
    order a backtrack visits each row (descending j), then ascending cycle."""
    B = _series(B)
    L, d = B.shape
    n = len(cycles)
    w = [1.0] * n if weights is None else [float(v) for v in weights]
    psum = np.zeros((n, L, d))
    pcnt = np.zeros((n, L), dtype=np.int64)
    for p, Y in enumerate(cycles):
        Y = _series(Y)
        _, path, _ = dtw(B, Y)
        for i, j in reversed(path):
            for c in range(d):
                psum[p, i, c] = psum[p, i, c] + Y[j, c]
            pcnt[p, i] += 1
    out = np.zeros((L, d))
    K = pcnt.sum(axis=0)
    for l in range(L):
        C = 0.0
        for p in range(n):
            C = C + w[p] * float(pcnt[p, l])
        for c in range(d):
            S = 0.0
            for p in range(n):
                S = S + w[p] * psum[p, l, c]
            out[l, c] = S / C
    return out, K


# ------------------------------------------------------- float32 arithmetic

def round_f32(q) -> float:
    """The float32 nearest to the rational q (ties to even), as a float."""
    q = Fraction(q)
    if q == 0:
        return 0.0
    sign = -1 if q < 0 else 1
    a = abs(q)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1                        # now 2^e <= a < 2^(e+1)
    e = max(e, -126)                  # subnormals share the smallest exponent
    ulp = Fraction(2) ** (e - 23)
    m = a / ulp                       # 2^23 <= m < 2^24 for normal numbers
    lo = m.numerator // m.denominator
    rem = m - lo
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and lo % 2 == 1):
        lo += 1
    v = lo * ulp
    if v >= Fraction(2) ** 128:
        return sign * math.inf
    return sign * float(v)            # exact: v has at most 24 significant bits


def delta32(x, y):
    """Def. 3 in float32, the oracle's operation order: e_c = x_c - y_c,
    s = e_0 * e_0, s = fma(e_c, e_c, s), each rounded once to float32."""
    x = [Fraction(float(v)) for v in np.asarray(x, dtype=np.float32).ravel()]
    y = [Fraction(float(v)) for v in np.asarray(y, dtype=np.float32).ravel()]
    e = Fraction(round_f32(x[0] - y[0]))
    s = Fraction(round_f32(e * e))
    for c in range(1, len(x)):
        e = Fraction(round_f32(x[c] - y[c]))
        s = Fraction(round_f32(e * e + s))
    return float(s)


def path_cost32(X, Y, path) -> float:
    """The path's cost summed in float32 from (1,1): c = delta + c."""
    c = Fraction(0)
    for i, j in path:
        c = Fraction(round_f32(Fraction(delta32(X[i], Y[j])) + c))
    return float(c)


def dtw32_value(X, Y) -> float:
    """Eq. 1 in float32 arithmetic: the minimum over paths of path_cost32."""
    X, Y = _series(X), _series(Y)
    return min(path_cost32(X, Y, p) for p in all_paths(X.shape[0], Y.shape[0]))


def subdtw32_value(X, Y) -> float:
    """Sub-DTW in float32 arithmetic: the minimum over every subsequence
    Y[a..b] and every path of X against it of path_cost32."""
    X, Y = _series(X), _series(Y)
    M, N = X.shape[0], Y.shape[0]
    best = math.inf
    for a in range(N):
        for b in range(a, N):
            for p in all_paths(M, b - a + 1):
                best = min(best, path_cost32(X, Y, [(i, j + a) for i, j in p]))
    return best
