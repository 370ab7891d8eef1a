"""Host-side parts of the sweep-shape autotuner (no GPU needed)."""

import json

import pytest

from paper_2404_12134_amd import autotune


def test_length_signature_rounds_to_two_digits():
    n, p10, p50, p90 = autotune.length_signature([4000, 4100, 5000, 5900, 6000])
    assert n == 5
    assert p50 == 5000 and p10 == 4000 and p90 == 6000
    # batches differing only in detail share a signature
    assert autotune.length_signature([4012, 4991, 5988]) == autotune.length_signature([4009, 4990, 5991])


def test_cache_key_separates_shapes():
    k1 = autotune.cache_key("gfx950-256cu", "dba", 3, "f32", 4077, [5000] * 64)
    assert k1 != autotune.cache_key("gfx950-304cu", "dba", 3, "f32", 4077, [5000] * 64)
    assert k1 != autotune.cache_key("gfx942-256cu", "dba", 3, "f32", 4077, [5000] * 64)
    k1 = autotune.cache_key("dev", "dba", 3, "f32", 4077, [5000] * 64)
    assert k1 == autotune.cache_key("dev", "dba", 3, "f32", 4077, [5000] * 64)
    assert k1 != autotune.cache_key("dev", "score", 3, "f32", 4077, [5000] * 64)
    assert k1 != autotune.cache_key("dev", "dba", 3, "f32", 4078, [5000] * 64)
    assert k1 != autotune.cache_key("dev", "dba", 3, "f32", 4077, [5000] * 65)


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert autotune.load_cache(path) == {}
    autotune.store_cache(path, "a", {"rho": 5, "grid": 0, "ms": 1.5, "table": [[5, 0, 1.5]]})
    autotune.store_cache(path, "b", {"rho": 4, "grid": 0, "ms": 2.0, "table": []})
    data = json.load(open(path))
    assert data["a"]["rho"] == 5 and data["b"]["rho"] == 4


def test_candidates_cover_the_supported_shapes():
    for op in ("dba", "medoid", "score"):
        shapes = list(autotune.candidates(op, 256))
        assert sorted({r for r, _ in shapes}) == [2, 4, 5]
        # every rows-per-lane choice with every grid: the default and fewer waves
        assert sorted(shapes) == sorted((r, g) for r in (2, 4, 5) for g in (0, 16 * 256, 8 * 256))
    # the Soft-DTW sweeps are built for 2 rows per lane: only their grid is tuned
    soft = list(autotune.candidates("soft", 304))
    assert soft == [(2, 0), (2, 12 * 304), (2, 6 * 304)]


def test_tune_rejects_op_plan_mismatch_before_any_gpu_call():
    with pytest.raises(ValueError):
        autotune.tune([0, 5], 1, "f64", 0, op="dba")
    with pytest.raises(ValueError):
        autotune.tune([0, 5], 1, "f64", 4, op="medoid")
    with pytest.raises(ValueError):
        autotune.tune([0, 5], 1, "f64", 4, op="nope")
