"""Host helpers of the detection step (Sec. V-C): thresholds and F2."""

import json
import os

import numpy as np

from paper_2404_12134_amd import detect

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "detection_confusion.json")


def test_f2_reproduces_the_paper_from_its_confusion_matrices():
    g = json.load(open(GOLDEN))
    for key in ("two_sigma", "boxplot"):
        c = g[key]
        assert round(detect.f_beta(c["tp"], c["fn"], c["fp"]), 2) == c["f2"]


def test_two_sigma_closed_form():
    s = [1.0, 2.0, 3.0, 4.0, 5.0]
    assert detect.two_sigma_threshold(s) == 3.0 + 2.0 * np.sqrt(2.0)
    assert detect.two_sigma_threshold(s, k=3.0) == 3.0 + 3.0 * np.sqrt(2.0)


def test_boxplot_closed_form():
    # quartiles of 1..8 by linear interpolation: 2.75 and 6.25
    assert detect.boxplot_threshold(np.arange(1, 9)) == 6.25 + 1.5 * 3.5


def test_confusion_and_flags():
    scores = [0.1, 0.2, 5.0, 0.3, 9.0]
    pred = detect.flag(scores, 1.0)
    assert pred.tolist() == [False, False, True, False, True]
    assert detect.confusion(pred, [False, True, True, False, True]) == (2, 1, 0, 2)
    assert detect.f_beta(0, 3, 2) == 0.0
