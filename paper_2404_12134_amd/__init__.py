"""WETSAND hot path on MI355X (gfx950): DTW barycenters and DTW anomaly scores.

The compute path lives in ``csrc/`` (HIP kernels behind a C ABI declared in
``include/wetsand_mi.h``); :mod:`paper_2404_12134_amd.wetsand` is the thin
ctypes binding over it.  :mod:`paper_2404_12134_amd.synth` holds the seeded
synthetic workloads and nothing of the method's arithmetic.

Importing this package loads nothing native: the shared library is opened on
first use by :mod:`paper_2404_12134_amd.wetsand`, which raises if it is missing.
"""

__all__ = ["synth", "wetsand"]
