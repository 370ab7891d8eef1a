"""Detection thresholds on the similarity scores (Sec. V-C) -- host helpers.

The scores d_score = DTW(B, C_k) / |pi| come from the GPU (anomaly_score);
choosing a threshold is left to the user by the paper, which evaluates two:

* the 2-sigma threshold: mean + k * standard deviation of the scores
  (k = 2; the population standard deviation);
* the boxplot threshold: Q_max = q3 + 1.5 |q3 - q1| with q1, q3 the first and
  third quartiles (linear interpolation between order statistics).

Detections are scored with the F_beta measure, beta = 2 (recall weighted
above precision, as the paper does).
"""

from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np


def two_sigma_threshold(scores: Sequence[float], k: float = 2.0) -> float:
    s = np.asarray(scores, dtype=np.float64)
    return float(s.mean() + k * s.std())


def boxplot_threshold(scores: Sequence[float]) -> float:
    s = np.asarray(scores, dtype=np.float64)
    q1, q3 = np.percentile(s, [25.0, 75.0])
    return float(q3 + 1.5 * abs(q3 - q1))


def flag(scores: Sequence[float], threshold: float) -> np.ndarray:
    """True where a cycle is declared abnormal (score above the threshold)."""
    return np.asarray(scores, dtype=np.float64) > threshold


def confusion(pred: Sequence[bool], truth: Sequence[bool]) -> Tuple[int, int, int, int]:
    """(true positives, false negatives, false positives, true negatives)."""
    p = np.asarray(pred, dtype=bool)
    t = np.asarray(truth, dtype=bool)
    return (int((p & t).sum()), int((~p & t).sum()), int((p & ~t).sum()), int((~p & ~t).sum()))


def f_beta(tp: int, fn: int, fp: int, beta: float = 2.0) -> float:
    """(1 + b^2) P R / (b^2 P + R); 0 when nothing is detected correctly."""
    if tp == 0:
        return 0.0
    prec = tp / (tp + fp)
    rec = tp / (tp + fn)
    b2 = beta * beta
    return (1 + b2) * prec * rec / (b2 * prec + rec)
