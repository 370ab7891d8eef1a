"""Writes tests/golden/c5_longest_pair_softdtw.npz: the oracle's Soft-DTW
value, gradient and row mass (Eq. 4-6, gamma = 0.1) of one full-size pair of
the 256-cycle workload (6 channels, lengths 40,000..50,000 with 1 % of the
samples dropped in gaps; seed 5): the Euclidean-mean barycenter at
L = max N (the paper's preferred initialisation, Table I) against the longest
cycle.  The oracle keeps square-root checkpoints of R (a 49k x 49k R would be
20 GB); it takes about six minutes on one core.

Only oracle/ and the seeded generator are called.  The file also stores the
SHA-256 of both float64 inputs, so a test can confirm it regenerated the same
pair.

    python tests/golden/make_c5_pair.py
"""

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2404_12134_amd import synth  # noqa: E402

OUT = os.path.join(HERE, "c5_longest_pair_softdtw.npz")
GAMMA = 0.1


def pair():
    """(B [L][6] float64, Y [N][6] float64, index of Y) of the fixture."""
    w = synth.make(5)
    B = oracle.euclid_mean([np.asarray(c, dtype=np.float64) for c in w.cycles], w.L)
    k = int(np.argmax(w.lengths))          # lowest index among the longest
    return B, np.asarray(w.cycles[k], dtype=np.float64), k


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float64).tobytes()).hexdigest()


def main():
    B, Y, k = pair()
    t0 = time.time()
    v, g, h = oracle.softdtw_grad_ckpt(B, Y, GAMMA)
    print("pair (L=%d, N=%d, cycle %d): value %.17g in %.0f s" % (B.shape[0], Y.shape[0], k, v,
                                                                 time.time() - t0))
    np.savez_compressed(OUT, value=np.array([v]), grad=g, rowmass=h, gamma=np.array([GAMMA]),
                        cycle=np.array([k]), sha_b=np.array(sha(B)), sha_y=np.array(sha(Y)))


if __name__ == "__main__":
    main()
